/*
 * ibmlb_oracle.c — plain FP64 CPU oracle of the IB-LB droplet timestep.
 *
 * TEST INFRASTRUCTURE ONLY: it checks the HIP library and is never on the
 * product path. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load it. It shares nothing with the HIP library.
 *
 * Every routine is the plain definition or the algorithm's steps in the
 * paper's order (arXiv 2403.01161), in FP64, with a fixed summation order:
 * vertices ascending, triangles ascending, nodes z-major then y then x.
 * The lattice sweeps (and the indicator) are split over z-planes with
 * OpenMP on boxes of 32768 nodes or more; each node is computed by one
 * thread alone, so results do not depend on the thread count.
 *
 * Readings of the paper taken here (the paper is silent or inconsistent):
 *  - Eq. (equilibriumLB) prints the velocity-squared term as u.u/cs^2; that
 *    breaks sum_i f_eq = rho. The standard second-order form with
 *    u.u/(2 cs^2) is used (the form of the reference the paper cites).
 *  - The moving walls use the link-wise velocity bounce-back of
 *    Eq. (standard BB), f_out = f_in + 2 w_i rho0 c_i.u_w / cs^2 (which is
 *    rho0/3 c_i.u_w on axis links), applied to every link that leaves the
 *    box, with walls half a spacing outside the outermost nodes and u_w
 *    from Eq. (velo_facce_cubo_da_gradiente) at the link midpoint. The
 *    wet-node counter-slip corrections for faces, edges and corners are not
 *    part of this step.
 *  - The nodal force of Pi = sigma I_2 (Eq. pi_drop) is taken as
 *    phi_k = -sigma dA_surface/dr_k: a uniform isotropic tension on the
 *    deformed surface.
 *  - The interpolated velocity (Eq. ibm_force_d, second line) is the
 *    half-force-corrected u of Eq. (density_velocity_LB).
 *  - Sub-step order in one step: forces, spread, moments, interpolate,
 *    collide, stream, Euler move (Eq. fwd_euler), smoothing. All sub-steps
 *    use the same u^n.
 *  - In the smoothing correction (Eq. HC_algo_full) the neighbour mean of b
 *    enters with reg_sign (+1 by default, the sign of Vollmer's HC scheme
 *    that the paper follows; -1 reproduces the printed sign).
 *    Smoothing runs after every step with an iteration cap.
 *  - S is (5/V) times the second moment of the enclosed volume about its
 *    centroid, so S = R^2 I for a sphere and the eigenvalues of an
 *    ellipsoid are the squared semi-axes (Sec. 2 takes the root of the
 *    largest eigenvalue as the major semi-axis).
 *  - Initial state: f_eq(rho0, A0 (x - x_c)) plus its Chapman-Enskog
 *    non-equilibrium part -3 tau w_i rho0 (c_i c_i - I/3):A0, with the outer
 *    tau everywhere.
 *  - Viscosity ratio chi (Sec. 2): one density, and nodes inside the mesh
 *    (winding number above 1/2) relax with tau_in = 1/2 + chi (tau - 1/2),
 *    both in the BGK rate and the Guo factor; the indicator of a step is
 *    that of the mesh the step's forces come from.
 */
#include "ibmlb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* D3Q19 velocities and weights (Sec. 3.1: w_0 = 1/3, w_1..6 = 1/18,
 * w_7..18 = 1/36). Index 0 is the rest population. */
static const int CV[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double weight(int i)
{
    int n2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
    if (n2 == 0) return 1.0 / 3.0;
    if (n2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static int opposite(int i)
{
    for (int j = 0; j < 19; ++j)
        if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2]) return j;
    return -1;
}

void ibo_lattice(int c[19 * 3], double w[19], int opp[19])
{
    for (int i = 0; i < 19; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = CV[i][a];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* Peskin 4-point stencil, Sec. 3.1. */
double ibo_phi(double r)
{
    double a = fabs(r);
    if (a < 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a < 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

/* Second-order equilibrium, Eq. (equilibriumLB) with cs^2 = 1/3 and the
 * velocity-squared term u.u/(2 cs^2). */
void ibo_equilibrium(double rho, const double u[3], double feq[19])
{
    const double cs2 = 1.0 / 3.0;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 19; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        feq[i] = weight(i) * rho *
                 (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
}

/* Guo forcing source, Sec. 3.1:
 * S_i = (1 - 1/(2 tau)) w_i/cs^2 [ ((c_i.u)/cs^2 + 1) c_i - u ] . F. */
void ibo_guo_source(double tau, const double u[3], const double F[3], double S[19])
{
    const double cs2 = 1.0 / 3.0;
    for (int i = 0; i < 19; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += ((cu / cs2 + 1.0) * CV[i][a] - u[a]) * F[a];
        S[i] = (1.0 - 1.0 / (2.0 * tau)) * weight(i) / cs2 * s;
    }
}

/* Multiple-relaxation-time collision (the paper mentions it as an option for
 * stability and for separating bulk viscosity; d'Humieres et al., 2002).
 * Moments m = M f over the orthogonal D3Q19 basis of that reference, with
 * c2 = |c|^2: rho; e = 19 c2 - 30; eps = (21 c2^2 - 53 c2 + 24)/2; j_a = c_a;
 * q_a = (5 c2 - 9) c_a; 3p_xx = 3 c_x^2 - c2; 3pi_xx = (3 c_x^2 - c2)(3 c2 - 5);
 * p_ww = c_y^2 - c_z^2; pi_ww = (c_y^2 - c_z^2)(3 c2 - 5); p_xy, p_yz, p_xz =
 * c_a c_b; m_x = (c_y^2 - c_z^2) c_x, m_y = (c_z^2 - c_x^2) c_y,
 * m_z = (c_x^2 - c_y^2) c_z. Order: rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z,
 * 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z. */
void ibo_mrt_basis(double M[19 * 19], double norm2[19])
{
    for (int i = 0; i < 19; ++i) {
        const double cx = CV[i][0], cy = CV[i][1], cz = CV[i][2];
        const double c2 = cx * cx + cy * cy + cz * cz;
        const double row[19] = {1.0,
                                19.0 * c2 - 30.0,
                                (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0,
                                cx, (5.0 * c2 - 9.0) * cx,
                                cy, (5.0 * c2 - 9.0) * cy,
                                cz, (5.0 * c2 - 9.0) * cz,
                                3.0 * cx * cx - c2, (3.0 * cx * cx - c2) * (3.0 * c2 - 5.0),
                                cy * cy - cz * cz, (cy * cy - cz * cz) * (3.0 * c2 - 5.0),
                                cx * cy, cy * cz, cx * cz,
                                (cy * cy - cz * cz) * cx, (cz * cz - cx * cx) * cy, (cx * cx - cy * cy) * cz};
        for (int k = 0; k < 19; ++k) M[19 * k + i] = row[k];
    }
    for (int k = 0; k < 19; ++k) {
        norm2[k] = 0.0;
        for (int i = 0; i < 19; ++i) norm2[k] += M[19 * k + i] * M[19 * k + i];
    }
}

/* ------------------------------------------------------------------ */
/* Surface-tension nodal forces, Eq. (pi_drop): phi_k = -sigma dA/dr_k.
 * For triangle (a, b, c) with unit normal n = (b-a)x(c-a)/|(b-a)x(c-a)|,
 * dA/da = n x (c - b)/2, dA/db = n x (a - c)/2, dA/dc = n x (b - a)/2. */
static void cross(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

void ibo_forces(int nv, const double* r, int nt, const int* tris, double sigma, double* phi)
{
    for (int k = 0; k < 3 * nv; ++k) phi[k] = 0.0;
    for (int t = 0; t < nt; ++t) {
        const int* v = tris + 3 * t;
        double e1[3], e2[3], n[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = r[3 * v[1] + a] - r[3 * v[0] + a];
            e2[a] = r[3 * v[2] + a] - r[3 * v[0] + a];
        }
        cross(e1, e2, n);
        double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (len == 0.0) continue;
        for (int a = 0; a < 3; ++a) n[a] /= len;
        for (int j = 0; j < 3; ++j) {
            int k = v[j], nxt = v[(j + 1) % 3], prv = v[(j + 2) % 3];
            double d[3], g[3];
            for (int a = 0; a < 3; ++a) d[a] = r[3 * prv + a] - r[3 * nxt + a];
            cross(n, d, g);
            for (int a = 0; a < 3; ++a) phi[3 * k + a] -= sigma * 0.5 * g[a];
        }
    }
}

/* Stencil node along one axis; -1 if it falls outside a wall axis. */
static long axis_node(long j, int L, int periodic)
{
    if (periodic) {
        long m = j % L;
        return m < 0 ? m + L : m;
    }
    if (j < 0 || j >= L) return -1;
    return j;
}

/* Spreading, Eq. (ibm_force_d) first line, with Delta = phi(x)phi(y)phi(z)
 * over the 4x4x4 nodes floor(r)-1 .. floor(r)+2. F is [N][3] and is added to. */
int ibo_spread(const int L[3], const int periodic[3], int nv, const double* r,
               const double* phi, double* F)
{
    for (int k = 0; k < nv; ++k) {
        const double* rk = r + 3 * k;
        if (!isfinite(rk[0]) || !isfinite(rk[1]) || !isfinite(rk[2])) return IBO_ENONFINITE;
        long base[3];
        for (int a = 0; a < 3; ++a) base[a] = (long)floor(rk[a]);
        for (long dz = -1; dz <= 2; ++dz)
            for (long dy = -1; dy <= 2; ++dy)
                for (long dx = -1; dx <= 2; ++dx) {
                    long j[3] = {base[0] + dx, base[1] + dy, base[2] + dz};
                    long n[3];
                    for (int a = 0; a < 3; ++a) {
                        n[a] = axis_node(j[a], L[a], periodic[a]);
                        if (n[a] < 0) return IBO_EDOMAIN;
                    }
                    double wgt = ibo_phi(rk[0] - j[0]) * ibo_phi(rk[1] - j[1]) * ibo_phi(rk[2] - j[2]);
                    long node = n[0] + (long)L[0] * (n[1] + (long)L[1] * n[2]);
                    for (int a = 0; a < 3; ++a) F[3 * node + a] += phi[3 * k + a] * wgt;
                }
    }
    return IBO_OK;
}

/* Interpolation, Eq. (ibm_force_d) second line: U_k = sum_x u(x) Delta(r_k - x). */
int ibo_interp(const int L[3], const int periodic[3], int nv, const double* r,
               const double* u, double* U)
{
    for (int k = 0; k < nv; ++k) {
        const double* rk = r + 3 * k;
        if (!isfinite(rk[0]) || !isfinite(rk[1]) || !isfinite(rk[2])) return IBO_ENONFINITE;
        long base[3];
        for (int a = 0; a < 3; ++a) base[a] = (long)floor(rk[a]);
        double acc[3] = {0.0, 0.0, 0.0};
        for (long dz = -1; dz <= 2; ++dz)
            for (long dy = -1; dy <= 2; ++dy)
                for (long dx = -1; dx <= 2; ++dx) {
                    long j[3] = {base[0] + dx, base[1] + dy, base[2] + dz};
                    long n[3];
                    for (int a = 0; a < 3; ++a) {
                        n[a] = axis_node(j[a], L[a], periodic[a]);
                        if (n[a] < 0) return IBO_EDOMAIN;
                    }
                    double wgt = ibo_phi(rk[0] - j[0]) * ibo_phi(rk[1] - j[1]) * ibo_phi(rk[2] - j[2]);
                    long node = n[0] + (long)L[0] * (n[1] + (long)L[1] * n[2]);
                    for (int a = 0; a < 3; ++a) acc[a] += u[3 * node + a] * wgt;
                }
        for (int a = 0; a < 3; ++a) U[3 * k + a] = acc[a];
    }
    return IBO_OK;
}

/* ------------------------------------------------------------------ */
/* One-ring neighbours (edge-connected vertices), sorted ascending. */
typedef struct {
    int* start; /* [nv+1] */
    int* list;
} ring_t;

static int cmp_int(const void* a, const void* b)
{
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

static int build_ring(int nv, int nt, const int* tris, ring_t* ring)
{
    int* cnt = calloc((size_t)nv + 1, sizeof(int));
    int* pairs = malloc(sizeof(int) * 12 * (size_t)(nt > 0 ? nt : 1));
    if (!cnt || !pairs) { free(cnt); free(pairs); return IBO_ENOMEM; }
    /* every directed edge of every triangle, both directions */
    int np = 0;
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j) {
            int a = tris[3 * t + j], b = tris[3 * t + (j + 1) % 3];
            pairs[2 * np] = a; pairs[2 * np + 1] = b; ++np;
            pairs[2 * np] = b; pairs[2 * np + 1] = a; ++np;
        }
    int** lists = calloc((size_t)nv, sizeof(int*));
    int* fill = calloc((size_t)nv, sizeof(int));
    for (int p = 0; p < np; ++p) cnt[pairs[2 * p]]++;
    for (int v = 0; v < nv; ++v) lists[v] = malloc(sizeof(int) * (size_t)(cnt[v] > 0 ? cnt[v] : 1));
    for (int p = 0; p < np; ++p) {
        int a = pairs[2 * p];
        lists[a][fill[a]++] = pairs[2 * p + 1];
    }
    ring->start = malloc(sizeof(int) * ((size_t)nv + 1));
    ring->list = malloc(sizeof(int) * (size_t)(np > 0 ? np : 1));
    int pos = 0;
    for (int v = 0; v < nv; ++v) {
        qsort(lists[v], (size_t)fill[v], sizeof(int), cmp_int);
        ring->start[v] = pos;
        for (int q = 0; q < fill[v]; ++q)
            if (q == 0 || lists[v][q] != lists[v][q - 1]) ring->list[pos++] = lists[v][q];
        free(lists[v]);
    }
    ring->start[nv] = pos;
    free(lists); free(fill); free(cnt); free(pairs);
    return IBO_OK;
}

static void free_ring(ring_t* ring)
{
    free(ring->start);
    free(ring->list);
    ring->start = ring->list = NULL;
}

/* HC smoothing, Sec. 3.3, with x_o the positions after the Euler move:
 *   x_p = x_o; repeat { x_q = x_p;
 *     x_p^i = alpha x_o^i + (1-alpha)/N_i sum_j x_q^j;
 *     x_b^i = x_p^i - [alpha x_o^i + (1-alpha) x_q^i];
 *     x_p^i -= gamma x_b^i + sign (1-gamma)/N_i sum_j x_b^j;
 *   } until max_i |x_p^i - x_q^i| < tol (or max_iter iterations).
 * r holds x_o on entry and the smoothed x_p on exit. Returns the iteration
 * count; *capped is set if the cap was reached without convergence. */
static int hc_run(int nv, const ring_t* ring, double alpha, double gamma, double tol,
                  int max_iter, int sign, double* r, int* capped)
{
    *capped = 0;
    if (max_iter <= 0 || nv == 0) return 0;
    size_t bytes = sizeof(double) * 3 * (size_t)nv;
    double* o = malloc(bytes);
    double* q = malloc(bytes);
    double* p = malloc(bytes);
    double* b = malloc(bytes);
    memcpy(o, r, bytes);
    memcpy(p, r, bytes);
    int it = 0;
    for (;;) {
        ++it;
        memcpy(q, p, bytes);
        for (int i = 0; i < nv; ++i) {
            int s0 = ring->start[i], s1 = ring->start[i + 1];
            double sum[3] = {0.0, 0.0, 0.0};
            for (int e = s0; e < s1; ++e)
                for (int a = 0; a < 3; ++a) sum[a] += q[3 * ring->list[e] + a];
            double Ni = (double)(s1 - s0);
            for (int a = 0; a < 3; ++a)
                p[3 * i + a] = alpha * o[3 * i + a] + (1.0 - alpha) / Ni * sum[a];
        }
        for (int i = 0; i < nv; ++i)
            for (int a = 0; a < 3; ++a)
                b[3 * i + a] = p[3 * i + a] - (alpha * o[3 * i + a] + (1.0 - alpha) * q[3 * i + a]);
        for (int i = 0; i < nv; ++i) {
            int s0 = ring->start[i], s1 = ring->start[i + 1];
            double sum[3] = {0.0, 0.0, 0.0};
            for (int e = s0; e < s1; ++e)
                for (int a = 0; a < 3; ++a) sum[a] += b[3 * ring->list[e] + a];
            double Ni = (double)(s1 - s0);
            for (int a = 0; a < 3; ++a)
                p[3 * i + a] -= gamma * b[3 * i + a] + (double)sign * (1.0 - gamma) / Ni * sum[a];
        }
        double dmax = 0.0;
        for (int i = 0; i < nv; ++i) {
            double d0 = p[3 * i] - q[3 * i], d1 = p[3 * i + 1] - q[3 * i + 1], d2 = p[3 * i + 2] - q[3 * i + 2];
            double d = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            if (d > dmax) dmax = d;
        }
        if (dmax < tol) break;
        if (it >= max_iter) { *capped = 1; break; }
    }
    memcpy(r, p, bytes);
    free(o); free(q); free(p); free(b);
    return it;
}

int ibo_hc(int nv, int nt, const int* tris, double alpha, double gamma, double tol,
           int max_iter, int sign, double* r, int* capped)
{
    ring_t ring;
    int rc = build_ring(nv, nt, tris, &ring);
    if (rc) return rc;
    int it = hc_run(nv, &ring, alpha, gamma, tol, max_iter, sign, r, capped);
    free_ring(&ring);
    return it;
}

/* ------------------------------------------------------------------ */
/* Symmetric 3x3 eigen-decomposition by the cyclic Jacobi method.
 * evals descending; evecs row k is the unit eigenvector of evals[k], with its
 * largest-magnitude component made positive. */
void ibo_eig3(const double S[9], double evals[3], double evecs[9])
{
    double a[3][3], v[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a[i][j] = 0.5 * (S[3 * i + j] + S[3 * j + i]);
            v[i][j] = (i == j) ? 1.0 : 0.0;
        }
    double scale = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]) +
                   fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        if (off <= 1e-15 * scale || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with J the rotation in the (p, q) plane */
                for (int k = 0; k < 3; ++k) {
                    double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double vkp = v[k][p], vkq = v[k][q];
                    v[k][p] = c * vkp - s * vkq;
                    v[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int order[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (a[order[j]][order[j]] > a[order[i]][order[i]]) {
                int tmp = order[i]; order[i] = order[j]; order[j] = tmp;
            }
    for (int k = 0; k < 3; ++k) {
        int col = order[k];
        evals[k] = a[col][col];
        int big = 0;
        for (int i = 1; i < 3; ++i)
            if (fabs(v[i][col]) > fabs(v[big][col])) big = i;
        double sgn = v[big][col] < 0.0 ? -1.0 : 1.0;
        for (int i = 0; i < 3; ++i) evecs[3 * k + i] = sgn * v[i][col];
    }
}

/* Droplet shape observables (Sec. 2): volume, centroid, morphological tensor
 * S = (5/V) int (x - xbar)(x - xbar)^T dV, eigenpairs, Taylor deformation
 * D = (sqrt(l1) - sqrt(l3))/(sqrt(l1) + sqrt(l3)), Eq. (beta) with
 * E = (A + A^T)/2, and theta = atan2(v_y, v_x) folded into (-90, 90] deg.
 * Volume integrals are sums over the signed tetrahedra (o, a, b, c) of each
 * triangle with o the mean vertex position:
 *   V_t = a.(b x c)/6, int x dV = V_t (a+b+c)/4,
 *   int x x^T dV = V_t/20 (aa^T + bb^T + cc^T + (a+b+c)(a+b+c)^T).
 * Mesh quality (the loosening and clustering of elements that the smoothing
 * of Sec. 3.3 prevents): the smallest interior angle of any triangle,
 * angle(u, v) = atan2(|u x v|, u.v) at each corner, and the shortest and
 * longest edge; out[35..37]. */
int ibo_shape(int nv, const double* r, int nt, const int* tris, const double A[9],
              double radius, double out[IBO_OBS_N])
{
    for (int k = 0; k < IBO_OBS_N; ++k) out[k] = 0.0;
    if (nv <= 0 || nt <= 0) return IBO_EINVAL;
    double o[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < nv; ++k)
        for (int a = 0; a < 3; ++a) o[a] += r[3 * k + a];
    for (int a = 0; a < 3; ++a) o[a] /= (double)nv;
    double V = 0.0, m1[3] = {0.0, 0.0, 0.0}, m2[3][3] = {{0.0}};
    double min_angle = INFINITY, emin = INFINITY, emax = 0.0;
    for (int t = 0; t < nt; ++t) {
        double p[3][3];
        for (int j = 0; j < 3; ++j)
            for (int a = 0; a < 3; ++a) p[j][a] = r[3 * tris[3 * t + j] + a] - o[a];
        for (int j = 0; j < 3; ++j) {
            double u[3], w[3], uxw[3];
            for (int a = 0; a < 3; ++a) {
                u[a] = p[(j + 1) % 3][a] - p[j][a];
                w[a] = p[(j + 2) % 3][a] - p[j][a];
            }
            cross(u, w, uxw);
            const double ang = atan2(sqrt(uxw[0] * uxw[0] + uxw[1] * uxw[1] + uxw[2] * uxw[2]),
                                     u[0] * w[0] + u[1] * w[1] + u[2] * w[2]);
            if (ang < min_angle) min_angle = ang;
            const double len = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (len < emin) emin = len;
            if (len > emax) emax = len;
        }
        double bxc[3];
        cross(p[1], p[2], bxc);
        double Vt = (p[0][0] * bxc[0] + p[0][1] * bxc[1] + p[0][2] * bxc[2]) / 6.0;
        double s[3];
        for (int a = 0; a < 3; ++a) s[a] = p[0][a] + p[1][a] + p[2][a];
        V += Vt;
        for (int a = 0; a < 3; ++a) m1[a] += Vt * s[a] / 4.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                m2[a][b] += Vt / 20.0 *
                            (p[0][a] * p[0][b] + p[1][a] * p[1][b] + p[2][a] * p[2][b] + s[a] * s[b]);
    }
    if (!(V > 0.0)) return IBO_EINVAL;
    double xbar[3];
    for (int a = 0; a < 3; ++a) xbar[a] = m1[a] / V;
    double S[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[3 * a + b] = 5.0 / V * (m2[a][b] - V * xbar[a] * xbar[b]);
    double ev[3], vec[9];
    ibo_eig3(S, ev, vec);
    double D = (sqrt(ev[0]) - sqrt(ev[2])) / (sqrt(ev[0]) + sqrt(ev[2]));
    int flags = 0;
    double beta = NAN, theta = NAN;
    double E[9], En = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            E[3 * a + b] = 0.5 * (A[3 * a + b] + A[3 * b + a]);
            En += E[3 * a + b] * E[3 * a + b];
        }
    En = sqrt(En);
    if (ev[0] - ev[1] < 1e-12 * radius * radius) flags |= IBO_FLAG_DEGENERATE;
    if (En == 0.0) flags |= IBO_FLAG_E_ZERO;
    if (!(flags & IBO_FLAG_DEGENERATE)) {
        const double* v1 = vec;
        theta = atan2(v1[1], v1[0]) * 180.0 / M_PI;
        if (theta > 90.0) theta -= 180.0;
        if (theta <= -90.0) theta += 180.0;
        if (!(flags & IBO_FLAG_E_ZERO)) {
            double q = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) q += v1[a] * E[3 * a + b] * v1[b];
            beta = q / En;
        }
    }
    out[35] = min_angle * 180.0 / M_PI;
    out[36] = emin;
    out[37] = emax;
    out[1] = V;
    for (int a = 0; a < 3; ++a) out[2 + a] = o[a] + xbar[a];
    for (int k = 0; k < 9; ++k) out[5 + k] = S[k];
    for (int k = 0; k < 3; ++k) out[14 + k] = ev[k];
    for (int k = 0; k < 9; ++k) out[17 + k] = vec[k];
    out[26] = D;
    out[27] = beta;
    out[28] = theta;
    out[34] = (double)flags;
    return IBO_OK;
}

/* Viscosity ratio (Sec. 2: the droplet phase has viscosity chi mu). A node
 * takes the inner relaxation time when it lies inside the closed surface.
 * Inside is defined by the winding number: the solid angles that the
 * triangles subtend at the point, summed with their orientation and divided
 * by 4 pi, are 1 inside an outward-oriented closed surface and 0 outside.
 * Each solid angle follows Van Oosterom and Strackee (1983):
 * tan(Omega/2) = a.(b x c) / (|a||b||c| + (a.b)|c| + (a.c)|b| + (b.c)|a|),
 * a, b, c the vertices relative to the point. */
double ibo_winding(int nv, const double* r, int nt, const int* tris, const double p[3])
{
    (void)nv;
    double sum = 0.0;
    for (int t = 0; t < nt; ++t) {
        double a[3], b[3], c[3], bc[3];
        for (int k = 0; k < 3; ++k) {
            a[k] = r[3 * tris[3 * t] + k] - p[k];
            b[k] = r[3 * tris[3 * t + 1] + k] - p[k];
            c[k] = r[3 * tris[3 * t + 2] + k] - p[k];
        }
        cross(b, c, bc);
        double la = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        double lb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        double lc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        double num = a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2];
        double den = la * lb * lc + (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) * lc +
                     (a[0] * c[0] + a[1] * c[1] + a[2] * c[2]) * lb + (b[0] * c[0] + b[1] * c[1] + b[2] * c[2]) * la;
        sum += 2.0 * atan2(num, den);
    }
    return sum / (4.0 * M_PI);
}

void ibo_indicator(const int L[3], int nv, const double* r, int nt, const int* tris, unsigned char* out)
{
    const long N = (long)L[0] * L[1] * L[2];
    memset(out, 0, (size_t)N);
    if (nv == 0 || nt == 0) return;
    long lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        double mn = r[a], mx = r[a];
        for (int k = 1; k < nv; ++k) {
            if (r[3 * k + a] < mn) mn = r[3 * k + a];
            if (r[3 * k + a] > mx) mx = r[3 * k + a];
        }
        lo[a] = (long)ceil(mn);
        hi[a] = (long)floor(mx);
        if (lo[a] < 0) lo[a] = 0;
        if (hi[a] > L[a] - 1) hi[a] = L[a] - 1;
    }
#pragma omp parallel for schedule(dynamic)
    for (long z = lo[2]; z <= hi[2]; ++z)
        for (long y = lo[1]; y <= hi[1]; ++y)
            for (long x = lo[0]; x <= hi[0]; ++x) {
                double p[3] = {(double)x, (double)y, (double)z};
                out[x + L[0] * (y + (long)L[1] * z)] = ibo_winding(nv, r, nt, tris, p) > 0.5;
            }
}

/* ------------------------------------------------------------------ */
struct ibo_sim {
    int L[3], per[3];
    long N;
    double tau, sigma, radius, rho0;
    double xc[3];
    double *f, *fpost;      /* [N][19] */
    double *F, *rho, *u;    /* [N][3], [N], [N][3] */
    int nv, nt;
    double *r, *phi, *U;    /* [nv][3] */
    int* tris;
    ring_t ring;
    double reg_alpha, reg_gamma, reg_tol;
    int reg_max_iter, reg_sign;
    long step;
    int last_iters;
    int cap_hits;
    double A_last[9];
    int* sched;             /* frozen smoothing iteration counts, see ibo_freeze_iters */
    int sched_n, sched_pos;
    int wall_bc;            /* 0 link bounce-back, 1 wet-node velocity walls, 2 the same with the
                               edge and corner rules as printed */
    int collision;          /* 0 BGK, 1 MRT */
    double mrt_M[19 * 19], mrt_n2[19], mrt_s[19];  /* basis, squared norms, rate per moment */
    double tau_in;          /* relaxation time inside the droplet (tau when chi = 1) */
    unsigned char* ind;     /* [N] inside indicator of the step's mesh, when tau_in != tau */
};

long ibo_nodes(const ibo_sim* s) { return s->N; }

void ibo_destroy(ibo_sim* s)
{
    if (!s) return;
    free(s->f); free(s->fpost); free(s->F); free(s->rho); free(s->u);
    free(s->r); free(s->phi); free(s->U); free(s->tris);
    free(s->sched);
    free(s->ind);
    free_ring(&s->ring);
    free(s);
}

int ibo_create(const ibo_params* p, ibo_sim** out)
{
    *out = NULL;
    if (!p) return IBO_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (p->L[a] < 4) return IBO_EINVAL;
    if (!(p->tau > 0.5) || !(p->sigma >= 0.0) || !(p->rho0 > 0.0)) return IBO_EINVAL;
    if (p->collision < 0 || p->collision > 1) return IBO_EINVAL;
    if (p->wall_bc < 0 || p->wall_bc > 2) return IBO_EINVAL;
    for (int k = 0; k < 5; ++k)
        if (!(p->mrt_s[k] >= 0.0 && p->mrt_s[k] < 2.0)) return IBO_EINVAL;
    if (!(p->chi >= 0.0) || (p->chi != 0.0 && p->chi != 1.0 && p->collision != 0)) return IBO_EINVAL;
    if (p->nv < 0 || p->nt < 0 || (p->nv > 0 && (!p->verts || !p->tris || p->nt == 0)))
        return IBO_EINVAL;
    for (int t = 0; t < 3 * p->nt; ++t)
        if (p->tris[t] < 0 || p->tris[t] >= p->nv) return IBO_EINVAL;
    ibo_sim* s = calloc(1, sizeof(ibo_sim));
    if (!s) return IBO_ENOMEM;
    for (int a = 0; a < 3; ++a) {
        s->L[a] = p->L[a];
        s->per[a] = p->periodic[a] ? 1 : 0;
        s->xc[a] = (p->L[a] - 1) / 2.0;
    }
    s->N = (long)p->L[0] * p->L[1] * p->L[2];
    s->tau = p->tau; s->sigma = p->sigma; s->radius = p->radius; s->rho0 = p->rho0;
    s->nv = p->nv; s->nt = p->nt;
    s->reg_alpha = p->reg_alpha; s->reg_gamma = p->reg_gamma; s->reg_tol = p->reg_tol;
    s->reg_max_iter = p->reg_max_iter; s->reg_sign = p->reg_sign >= 0 ? 1 : -1;
    s->wall_bc = p->wall_bc;
    {
        const double chi = p->chi == 0.0 ? 1.0 : p->chi;
        s->tau_in = chi == 1.0 ? p->tau : 0.5 + chi * (p->tau - 0.5);
    }
    s->collision = p->collision;
    if (s->collision == 1) {
        /* rate per moment: conserved rho and j at 1/tau (their non-equilibrium
         * and source parts cancel), the five stress moments at 1/tau (the
         * viscosity), the others from mrt_s */
        static const double dflt[5] = {1.19, 1.4, 1.2, 1.4, 1.98};
        double r[5];
        for (int k = 0; k < 5; ++k) r[k] = p->mrt_s[k] > 0.0 ? p->mrt_s[k] : dflt[k];
        const double sv = 1.0 / p->tau;
        const double rate[19] = {sv, r[0], r[1], sv, r[2], sv, r[2], sv, r[2],
                                 sv, r[3], sv, r[3], sv, sv, sv, r[4], r[4], r[4]};
        memcpy(s->mrt_s, rate, sizeof(rate));
        ibo_mrt_basis(s->mrt_M, s->mrt_n2);
    }
    s->f = malloc(sizeof(double) * 19 * (size_t)s->N);
    s->fpost = malloc(sizeof(double) * 19 * (size_t)s->N);
    s->F = calloc(3 * (size_t)s->N, sizeof(double));
    s->rho = malloc(sizeof(double) * (size_t)s->N);
    s->u = malloc(sizeof(double) * 3 * (size_t)s->N);
    size_t nvb = 3 * (size_t)(s->nv > 0 ? s->nv : 1);
    s->r = malloc(sizeof(double) * nvb);
    s->phi = malloc(sizeof(double) * nvb);
    s->U = malloc(sizeof(double) * nvb);
    s->tris = malloc(sizeof(int) * 3 * (size_t)(s->nt > 0 ? s->nt : 1));
    if (s->tau_in != s->tau) s->ind = calloc((size_t)s->N, 1);
    if (!s->f || !s->fpost || !s->F || !s->rho || !s->u || !s->r || !s->phi || !s->U || !s->tris ||
        (s->tau_in != s->tau && !s->ind)) {
        ibo_destroy(s);
        return IBO_ENOMEM;
    }
    if (s->nv) memcpy(s->r, p->verts, sizeof(double) * 3 * (size_t)s->nv);
    if (s->nt) memcpy(s->tris, p->tris, sizeof(int) * 3 * (size_t)s->nt);
    if (build_ring(s->nv, s->nt, s->tris, &s->ring)) {
        ibo_destroy(s);
        return IBO_ENOMEM;
    }
    for (int k = 0; k < 9; ++k) s->A_last[k] = p->A0[k];
    /* Initial populations. */
    double trA = p->A0[0] + p->A0[4] + p->A0[8];
    for (long z = 0; z < s->L[2]; ++z)
        for (long y = 0; y < s->L[1]; ++y)
            for (long x = 0; x < s->L[0]; ++x) {
                long n = x + s->L[0] * (y + (long)s->L[1] * z);
                double* fn = s->f + 19 * n;
                if (p->init_rest) {
                    for (int i = 0; i < 19; ++i) fn[i] = weight(i) * s->rho0;
                    continue;
                }
                double d[3] = {x - s->xc[0], y - s->xc[1], z - s->xc[2]}, u[3];
                for (int a = 0; a < 3; ++a)
                    u[a] = p->A0[3 * a] * d[0] + p->A0[3 * a + 1] * d[1] + p->A0[3 * a + 2] * d[2];
                ibo_equilibrium(s->rho0, u, fn);
                for (int i = 0; i < 19; ++i) {
                    double cAc = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) cAc += CV[i][a] * p->A0[3 * a + b] * CV[i][b];
                    fn[i] -= 3.0 * s->tau * weight(i) * s->rho0 * (cAc - trA / 3.0);
                }
            }
    *out = s;
    return IBO_OK;
}

/* Forces from the current mesh, spread onto F (zeroed first). */
static int force_field(ibo_sim* s)
{
    memset(s->F, 0, sizeof(double) * 3 * (size_t)s->N);
    if (s->nv == 0) return IBO_OK;
    ibo_forces(s->nv, s->r, s->nt, s->tris, s->sigma, s->phi);
    return ibo_spread(s->L, s->per, s->nv, s->r, s->phi, s->F);
}

/* Moments, Eq. (density_velocity_LB): rho = sum f, rho u = sum c f + F/2. */
static void moments(ibo_sim* s)
{
#pragma omp parallel for schedule(static) if (s->N >= 32768)
    for (long z = 0; z < s->L[2]; ++z)
        for (long y = 0; y < s->L[1]; ++y)
            for (long x = 0; x < s->L[0]; ++x) {
                long n = x + s->L[0] * (y + (long)s->L[1] * z);
                const double* fn = s->f + 19 * n;
                double rho = 0.0, m[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < 19; ++i) {
                    rho += fn[i];
                    for (int a = 0; a < 3; ++a) m[a] += CV[i][a] * fn[i];
                }
                s->rho[n] = rho;
                for (int a = 0; a < 3; ++a) s->u[3 * n + a] = (m[a] + 0.5 * s->F[3 * n + a]) / rho;
            }
}

/* BGK collision with Guo source, Eqs. (LBMEQ), (collision):
 * f*_i = f_i - (f_i - f_i^eq)/tau + S_i.
 * MRT: f* = f - M^-1 [ S M (f - f_eq) - (I - S/2) M G ] with G the Guo term
 * without its (1 - 1/(2 tau)) factor and S the diagonal of rates; the basis
 * is orthogonal, so M^-1 = M^T diag(1/|M_k|^2). With every rate 1/tau this is
 * the BGK step. */
static void collide(ibo_sim* s)
{
#pragma omp parallel for schedule(static) if (s->N >= 32768)
    for (long z = 0; z < s->L[2]; ++z)
        for (long y = 0; y < s->L[1]; ++y)
            for (long x = 0; x < s->L[0]; ++x) {
                long n = x + s->L[0] * (y + (long)s->L[1] * z);
                double feq[19], S[19];
                ibo_equilibrium(s->rho[n], s->u + 3 * n, feq);
                if (s->collision == 1) {
                    double G[19], mn[19], mg[19];
                    ibo_guo_source(1.0, s->u + 3 * n, s->F + 3 * n, G);
                    for (int i = 0; i < 19; ++i) G[i] *= 2.0;  /* the source at tau = 1 is G / 2 */
                    for (int k = 0; k < 19; ++k) {
                        mn[k] = mg[k] = 0.0;
                        for (int i = 0; i < 19; ++i) {
                            mn[k] += s->mrt_M[19 * k + i] * (s->f[19 * n + i] - feq[i]);
                            mg[k] += s->mrt_M[19 * k + i] * G[i];
                        }
                    }
                    for (int i = 0; i < 19; ++i) {
                        double d = 0.0;
                        for (int k = 0; k < 19; ++k)
                            d += s->mrt_M[19 * k + i] *
                                 (s->mrt_s[k] * mn[k] - (1.0 - 0.5 * s->mrt_s[k]) * mg[k]) / s->mrt_n2[k];
                        s->fpost[19 * n + i] = s->f[19 * n + i] - d;
                    }
                    continue;
                }
                /* the node's relaxation time: tau_in inside the droplet */
                const double tn = s->ind && s->ind[n] ? s->tau_in : s->tau;
                ibo_guo_source(tn, s->u + 3 * n, s->F + 3 * n, S);
                for (int i = 0; i < 19; ++i)
                    s->fpost[19 * n + i] = s->f[19 * n + i] - (s->f[19 * n + i] - feq[i]) / tn + S[i];
            }
}

/* Streaming, left side of Eq. (LBMEQ): f_i(x, t+1) = f*_i(x - c_i, t).
 * A link whose source x - c_i lies beyond a wall reflects the opposite
 * population at x with the moving-wall term of Eq. (standard BB):
 * f_i(x) = f*_{-i}(x) + 2 w_i rho0 (c_i.u_w)/cs^2, u_w = A (x - c_i/2 - x_c). */
static void stream(ibo_sim* s, const double A[9])
{
    const double cs2 = 1.0 / 3.0;
#pragma omp parallel for schedule(static) if (s->N >= 32768)
    for (long z = 0; z < s->L[2]; ++z)
        for (long y = 0; y < s->L[1]; ++y)
            for (long x = 0; x < s->L[0]; ++x) {
                long n = x + s->L[0] * (y + (long)s->L[1] * z);
                long xyz[3] = {x, y, z};
                for (int i = 0; i < 19; ++i) {
                    long src[3];
                    int wall = 0;
                    for (int a = 0; a < 3; ++a) {
                        long j = xyz[a] - CV[i][a];
                        src[a] = axis_node(j, s->L[a], s->per[a]);
                        if (src[a] < 0) wall = 1;
                    }
                    if (!wall) {
                        long m = src[0] + s->L[0] * (src[1] + (long)s->L[1] * src[2]);
                        s->f[19 * n + i] = s->fpost[19 * m + i];
                    } else {
                        double pw[3], uw[3];
                        for (int a = 0; a < 3; ++a) pw[a] = xyz[a] - 0.5 * CV[i][a] - s->xc[a];
                        for (int a = 0; a < 3; ++a)
                            uw[a] = A[3 * a] * pw[0] + A[3 * a + 1] * pw[1] + A[3 * a + 2] * pw[2];
                        double cu = CV[i][0] * uw[0] + CV[i][1] * uw[1] + CV[i][2] * uw[2];
                        s->f[19 * n + i] = s->fpost[19 * n + opposite(i)] + 2.0 * weight(i) * s->rho0 * cu / cs2;
                    }
                }
            }
}

/* Edges and corners as printed (Sec. 3.1, Eqs. ZH_edges,
 * zh-buried-links-edges, zh-buried-links-corners): no wall-velocity term;
 * the unknowns of a corner whose opposite is known by plain reflection. */
static void wet_corner_printed(double* f, int nw, int nrm[3][3], const int unknown[19], const int buried[19])
{
    int N[3];
    for (int a = 0; a < 3; ++a) N[a] = nrm[0][a] + nrm[1][a] + (nw == 3 ? nrm[2][a] : 0);
    double fn[19];
    memcpy(fn, f, sizeof(fn));
    for (int j = 0; j < 19; ++j) {
        if (!unknown[j] || buried[j]) continue;
        const int i = opposite(j);
        if (nw == 3) {
            fn[j] = f[i];
            continue;
        }
        double t[3], corr = 0.0;
        const int* n1 = nrm[0];
        const int* n2 = nrm[1];
        const int c1 = CV[i][0] * n1[0] + CV[i][1] * n1[1] + CV[i][2] * n1[2];
        const int c2 = CV[i][0] * n2[0] + CV[i][1] * n2[1] + CV[i][2] * n2[2];
        for (int a = 0; a < 3; ++a) t[a] = CV[i][a] - c1 * n1[a] - c2 * n2[a];
        for (int k = 0; k < 19; ++k) {
            int k1 = CV[k][0] * n1[0] + CV[k][1] * n1[1] + CV[k][2] * n1[2];
            int k2 = CV[k][0] * n2[0] + CV[k][1] * n2[1] + CV[k][2] * n2[2];
            double tc = t[0] * CV[k][0] + t[1] * CV[k][1] + t[2] * CV[k][2];
            corr += f[k] * tc * (1.0 - abs(k1)) * (1.0 - abs(k2));
        }
        fn[j] = f[i] - 0.25 * corr;
    }
    memcpy(f, fn, sizeof(fn));
    double fb = 0.0;
    if (nw == 2) {
        const int* n1 = nrm[0];
        const int* n2 = nrm[1];
        const int cr[3] = {n1[1] * n2[2] - n1[2] * n2[1], n1[2] * n2[0] - n1[0] * n2[2],
                           n1[0] * n2[1] - n1[1] * n2[0]};
        for (int i = 1; i < 19; ++i) {
            const double c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
            const double a1 = abs(CV[i][0] * cr[0] + CV[i][1] * cr[1] + CV[i][2] * cr[2]);
            const double a2 = abs(CV[i][0] * N[0] + CV[i][1] * N[1] + CV[i][2] * N[2]) / c2;
            fb += f[i] * (1.0 - (1.0 - a1) * (1.0 - a2));
        }
        fb /= 22.0;
    } else {
        for (int i = 1; i < 19; ++i) {
            const double c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
            fb += f[i] * abs(CV[i][0] * N[0] + CV[i][1] * N[1] + CV[i][2] * N[2]) / c2;
        }
        fb /= 18.0;
    }
    for (int j = 0; j < 19; ++j)
        if (buried[j]) f[j] = fb;
    f[0] = 12.0 * fb;
}

/* Wet-node velocity walls (Sec. 3.1): the walls pass through the boundary
 * nodes, each with the velocity u_w = A (x - x_c) of Eq.
 * (velo_facce_cubo_da_gradiente) at the node. After streaming, a population
 * f_j whose source x - c_j lies outside the box is unknown; with n the
 * inward normal of a wall plane through x and i the opposite of j:
 *  (a) one wall: rho = (sum_{c.n=0} f + 2 sum_{c.n<0} f) / (1 - u_w.n) (mass
 *      and normal momentum) and Eq. (ZH_bulk),
 *      f_j = f_i - (2 - |t_i|) rho/6 c_i.u_w - rho/3 t_i.u_w
 *            + 1/2 sum_k f_k (t_i.c_k)(1 - |c_k.n|),  t_i = c_i - (c_i.n) n;
 *  (b) two walls (an edge, inward normals n1, n2, t_i = c_i minus its
 *      components along n1 and n2): Eq. (ZH_edges) for the unknowns whose
 *      opposite is known, then the two buried links c = +-(n1 - n2) by
 *      Eq. (zh-buried-links-edges) and f_0 = 12 f_b;
 *  (c) three walls (a corner): the unknowns whose opposite is known by
 *      reflection (the text gives no rule for them), then the six buried
 *      links c.(n1 + n2 + n3) = 0 by Eq. (zh-buried-links-corners) and
 *      f_0 = 12 f_b.
 * The edge and corner rules as printed carry no wall-velocity term, and the
 * printed sign of the edge correction adds the along-edge momentum of the
 * resting populations +-e a second time where the face rule's correction
 * removes it; a linear flow then stays wrong at first order in A. Mode 2
 * (printed = 1) applies them as printed. Mode 1 applies the reading in which
 * an edge or corner node carries the wall velocity and the wall's linear
 * field, the conditions from which Eq. (ZH_bulk) follows on a face (the same
 * derivation gives Eq. (ZH_bulk) back):
 *  - an unknown j whose opposite i is known: Eq. (standard BB) for any link,
 *    f_j = f_i - 6 w_i rho c_i.u_w, and at an edge also the correction of
 *    Eq. (ZH_edges) with the sign of Eq. (ZH_bulk)'s and its velocity term,
 *    - rho/12 t_i.u_w + 1/4 sum_k f_k (t_i.c_k)(1 - |c_k.n1|)(1 - |c_k.n2|);
 *  - the buried links and the rest population, which the paper resets,
 *    take the equilibrium at (rho, u_w) plus the non-equilibrium part of the
 *    linear field, -3 tau w_j rho (c_j c_j - I/3):A (as the initial state);
 *  - rho is the node's density: sum_j f_j = rho solved for rho (every
 *    population above is linear in rho).
 * The node then holds density rho and momentum rho u_w exactly, and the
 * linear field's populations up to second order in A. At rest both modes
 * give the rest weights. */
static void wet_walls(ibo_sim* s, const double A[9], int printed)
{
#pragma omp parallel for schedule(static) if (s->N >= 32768)
    for (long z = 0; z < s->L[2]; ++z)
        for (long y = 0; y < s->L[1]; ++y)
            for (long x = 0; x < s->L[0]; ++x) {
                const long xyz[3] = {x, y, z};
                int nw = 0;
                int nrm[3][3];
                for (int a = 0; a < 3; ++a) {
                    if (s->per[a]) continue;
                    int dir = xyz[a] == 0 ? 1 : (xyz[a] == s->L[a] - 1 ? -1 : 0);
                    if (!dir) continue;
                    for (int b = 0; b < 3; ++b) nrm[nw][b] = b == a ? dir : 0;
                    ++nw;
                }
                if (!nw) continue;
                double* f = s->f + 19 * (x + s->L[0] * (y + (long)s->L[1] * z));
                double u[3];
                for (int a = 0; a < 3; ++a) {
                    u[a] = 0.0;
                    for (int b = 0; b < 3; ++b) u[a] += A[3 * a + b] * (xyz[b] - s->xc[b]);
                }
                int unknown[19];
                for (int j = 0; j < 19; ++j) {
                    unknown[j] = 0;
                    for (int k = 0; k < nw; ++k) {
                        int cn = CV[j][0] * nrm[k][0] + CV[j][1] * nrm[k][1] + CV[j][2] * nrm[k][2];
                        if (cn > 0) unknown[j] = 1;
                    }
                }
                if (nw == 1) {
                    const int* n = nrm[0];
                    double s0 = 0.0, sm = 0.0;
                    for (int k = 0; k < 19; ++k) {
                        int cn = CV[k][0] * n[0] + CV[k][1] * n[1] + CV[k][2] * n[2];
                        if (cn == 0) s0 += f[k];
                        if (cn < 0) sm += f[k];
                    }
                    const double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
                    const double rho = (s0 + 2.0 * sm) / (1.0 - un);
                    double fn[19];
                    memcpy(fn, f, sizeof(fn));
                    for (int j = 0; j < 19; ++j) {
                        if (!unknown[j]) continue;
                        const int i = opposite(j);
                        const int ci_n = CV[i][0] * n[0] + CV[i][1] * n[1] + CV[i][2] * n[2];
                        double t[3], tt = 0.0, cu = 0.0, tu = 0.0, corr = 0.0;
                        for (int a = 0; a < 3; ++a) {
                            t[a] = CV[i][a] - ci_n * n[a];
                            tt += t[a] * t[a];
                            cu += CV[i][a] * u[a];
                            tu += t[a] * u[a];
                        }
                        for (int k = 0; k < 19; ++k) {
                            int ck_n = CV[k][0] * n[0] + CV[k][1] * n[1] + CV[k][2] * n[2];
                            double tc = t[0] * CV[k][0] + t[1] * CV[k][1] + t[2] * CV[k][2];
                            corr += f[k] * tc * (1.0 - abs(ck_n));
                        }
                        fn[j] = f[i] - (2.0 - sqrt(tt)) * rho / 6.0 * cu - rho / 3.0 * tu + 0.5 * corr;
                    }
                    memcpy(f, fn, sizeof(fn));
                    continue;
                }
                int buried[19];
                for (int j = 0; j < 19; ++j) buried[j] = unknown[j] && unknown[opposite(j)];
                if (printed) {
                    wet_corner_printed(f, nw, nrm, unknown, buried);
                    continue;
                }
                /* populations reset from (rho, u_w, A): rho g_j */
                double g[19];
                const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                for (int j = 0; j < 19; ++j) {
                    g[j] = 0.0;
                    if (j != 0 && !buried[j]) continue;
                    const double cu = CV[j][0] * u[0] + CV[j][1] * u[1] + CV[j][2] * u[2];
                    double cAc = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) cAc += CV[j][a] * A[3 * a + b] * CV[j][b];
                    const double trA = A[0] + A[4] + A[8];
                    g[j] = weight(j) * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu) -
                           3.0 * s->tau * weight(j) * (cAc - trA / 3.0);
                }
                /* density: sum_j f_j = rho over the completed node */
                double known = 0.0, lin = 1.0;
                for (int j = 0; j < 19; ++j) {
                    if (j == 0 || buried[j]) {
                        lin -= g[j];
                    } else if (unknown[j]) {
                        const int i = opposite(j);
                        known += 2.0 * f[i];
                        lin += 6.0 * weight(i) * (CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2]);
                    } else if (!unknown[opposite(j)]) {
                        known += f[j]; /* neither it nor its opposite crosses a wall */
                    }
                }
                const double rho = known / lin;
                double fn[19];
                memcpy(fn, f, sizeof(fn));
                for (int j = 0; j < 19; ++j) {
                    if (j == 0 || buried[j]) {
                        fn[j] = rho * g[j];
                        continue;
                    }
                    if (!unknown[j]) continue;
                    const int i = opposite(j);
                    const double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
                    fn[j] = f[i] - 6.0 * weight(i) * rho * cu;
                    if (nw == 3) continue;
                    const int* n1 = nrm[0];
                    const int* n2 = nrm[1];
                    const int c1 = CV[i][0] * n1[0] + CV[i][1] * n1[1] + CV[i][2] * n1[2];
                    const int c2 = CV[i][0] * n2[0] + CV[i][1] * n2[1] + CV[i][2] * n2[2];
                    double t[3], corr = 0.0;
                    for (int a = 0; a < 3; ++a) t[a] = CV[i][a] - c1 * n1[a] - c2 * n2[a];
                    for (int k = 0; k < 19; ++k) {
                        int k1 = CV[k][0] * n1[0] + CV[k][1] * n1[1] + CV[k][2] * n1[2];
                        int k2 = CV[k][0] * n2[0] + CV[k][1] * n2[1] + CV[k][2] * n2[2];
                        double tc = t[0] * CV[k][0] + t[1] * CV[k][1] + t[2] * CV[k][2];
                        corr += f[k] * tc * (1.0 - abs(k1)) * (1.0 - abs(k2));
                    }
                    const double tu = t[0] * u[0] + t[1] * u[1] + t[2] * u[2];
                    fn[j] += -rho / 12.0 * tu + 0.25 * corr;
                }
                memcpy(f, fn, sizeof(fn));
            }
}

static int one_step(ibo_sim* s, const double A[9])
{
    int rc = force_field(s);                                   /* phi, F */
    if (rc) return rc;
    if (s->ind) ibo_indicator(s->L, s->nv, s->r, s->nt, s->tris, s->ind); /* tau per node */
    moments(s);                                                /* rho, u */
    if (s->nv) {
        rc = ibo_interp(s->L, s->per, s->nv, s->r, s->u, s->U); /* U */
        if (rc) return rc;
    }
    collide(s);
    stream(s, A);
    if (s->wall_bc) wet_walls(s, A, s->wall_bc == 2);
    for (int k = 0; k < 3 * s->nv; ++k) s->r[k] += s->U[k];   /* Eq. (fwd_euler) */
    int capped = 0;
    if (s->sched_pos < s->sched_n) {
        /* frozen count: exactly m iterations, no convergence test (a negative
         * tolerance is never met, so the loop ends at its cap m) */
        int m = s->sched[s->sched_pos++];
        s->last_iters = hc_run(s->nv, &s->ring, s->reg_alpha, s->reg_gamma, -1.0, m, s->reg_sign,
                               s->r, &capped);
    } else {
        s->last_iters = hc_run(s->nv, &s->ring, s->reg_alpha, s->reg_gamma, s->reg_tol,
                               s->reg_max_iter, s->reg_sign, s->r, &capped);
        if (capped) s->cap_hits++;
    }
    for (int k = 0; k < 9; ++k) s->A_last[k] = A[k];
    s->step++;
    for (int k = 0; k < 3 * s->nv; ++k)
        if (!isfinite(s->r[k])) return IBO_ENONFINITE;
    return IBO_OK;
}

int ibo_step(ibo_sim* s, const double* A, int nsteps, int stride)
{
    if (!s || !A || nsteps < 0) return IBO_EINVAL;
    for (int n = 0; n < nsteps; ++n) {
        int rc = one_step(s, A + 9 * (long)n * (stride ? 1 : 0));
        if (rc) return rc;
    }
    return IBO_OK;
}

int ibo_observables(ibo_sim* s, double out[IBO_OBS_N])
{
    for (int k = 0; k < IBO_OBS_N; ++k) out[k] = 0.0;
    int rc = IBO_OK;
    if (s->nv > 0) rc = ibo_shape(s->nv, s->r, s->nt, s->tris, s->A_last, s->radius, out);
    double mass = 0.0, mom[3] = {0.0, 0.0, 0.0};
    for (long n = 0; n < s->N; ++n)
        for (int i = 0; i < 19; ++i) {
            mass += s->f[19 * n + i];
            for (int a = 0; a < 3; ++a) mom[a] += CV[i][a] * s->f[19 * n + i];
        }
    out[0] = (double)s->step;
    out[29] = mass;
    for (int a = 0; a < 3; ++a) out[30 + a] = mom[a];
    out[33] = (double)s->last_iters;
    int flags = (int)out[34];
    if (s->cap_hits) flags |= IBO_FLAG_REG_CAP;
    out[34] = (double)flags;
    s->cap_hits = 0;
    return rc;
}

int ibo_freeze_iters(ibo_sim* s, const int* counts, int n)
{
    if (!s || n < 0 || (n > 0 && !counts)) return IBO_EINVAL;
    for (int j = 0; j < n; ++j)
        if (counts[j] < 0) return IBO_EINVAL;
    free(s->sched);
    s->sched = NULL;
    s->sched_n = s->sched_pos = 0;
    if (n == 0) return IBO_OK;
    s->sched = malloc(sizeof(int) * (size_t)n);
    if (!s->sched) return IBO_ENOMEM;
    memcpy(s->sched, counts, sizeof(int) * (size_t)n);
    s->sched_n = n;
    return IBO_OK;
}

int ibo_last_iters(const ibo_sim* s) { return s->last_iters; }

int ibo_get_vertices(const ibo_sim* s, double* r)
{
    memcpy(r, s->r, sizeof(double) * 3 * (size_t)s->nv);
    return IBO_OK;
}

int ibo_set_vertices(ibo_sim* s, const double* r)
{
    memcpy(s->r, r, sizeof(double) * 3 * (size_t)s->nv);
    return IBO_OK;
}

int ibo_fields(ibo_sim* s, double* rho, double* u)
{
    int rc = force_field(s);
    if (rc) return rc;
    moments(s);
    memcpy(rho, s->rho, sizeof(double) * (size_t)s->N);
    memcpy(u, s->u, sizeof(double) * 3 * (size_t)s->N);
    return IBO_OK;
}

int ibo_get_indicator(const ibo_sim* s, unsigned char* out)
{
    if (!s || !out) return IBO_EINVAL;
    ibo_indicator(s->L, s->nv, s->r, s->nt, s->tris, out);
    return IBO_OK;
}

int ibo_get_populations(const ibo_sim* s, double* f)
{
    memcpy(f, s->f, sizeof(double) * 19 * (size_t)s->N);
    return IBO_OK;
}

int ibo_set_populations(ibo_sim* s, const double* f)
{
    memcpy(s->f, f, sizeof(double) * 19 * (size_t)s->N);
    return IBO_OK;
}
