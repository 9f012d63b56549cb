// Discrete adjoint (reverse-mode derivative) of the IB-LB droplet timestep.
//
// The forward step n -> n+1 (Sec. 3.1 and Sec. 3.3) is, with the HC iteration
// count of the step frozen, a smooth map of (f^n, r^n, sigma, A^n):
//   phi   = -sigma dA_surf/dr                      Eq. (pi_drop)
//   F     = sum_k phi_k Delta(r_k - x)             Eq. (ibm_force_d), line 1
//   rho, u from f and F/2                          Eq. (density_velocity_LB)
//   U_k   = sum_x u(x) Delta(r_k - x)              Eq. (ibm_force_d), line 2
//   f*    = f - (f - f^eq)/tau + S                 Eqs. (LBMEQ), (collision)
//   f^{n+1} = stream f* with moving-wall bounce-back, Eq. (standard BB)
//   o     = r + U                                  Eq. (fwd_euler)
//   r^{n+1} = m_n HC iterations on o               Eq. (HC_algo_full)
// The kernels below apply the transpose of each of these linearised maps, in
// reverse order, to the adjoint state (fbar, rbar) and accumulate the
// derivatives of the objective with respect to sigma and to the gradient
// rows A^n. All adjoint arithmetic is FP64 whatever the population storage;
// the forward quantities it needs (rho, u, F on every node, positions and
// iteration counts of every step) are recorded during a recompute of the
// segment from its checkpoint.
#include <math.h>

#include "lattice_common.h"

namespace ibmlb {

__device__ inline double4 d4(double x, double y, double z) { return make_double4(x, y, z, 0.0); }
__device__ inline double4 operator+(double4 a, double4 b) { return d4(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline double4 operator-(double4 a, double4 b) { return d4(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline double4 operator*(double s, double4 a) { return d4(s * a.x, s * a.y, s * a.z); }
__device__ inline double dot3(double4 a, double4 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline double4 cross3(double4 a, double4 b) {
    return d4(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// ---------------------------------------------------------------- recording
// rho, u (with F/2) and F of the current populations on every node: the
// state the lattice kernel of this step will see. The work-groups after the
// node range record the vertex positions, and the first of them the
// previous step's smoothing iteration count (when prev_iters is not null).
template <class C>
__global__ __launch_bounds__(256) void k_rec_fields(Geom g, LatticeParams lp, const typename C::store_t* __restrict__ fin,
                                                    const typename C::real* __restrict__ F,
                                                    const int* __restrict__ mark, const Ctl* __restrict__ ctl, int ib,
                                                    double* __restrict__ rho, double* __restrict__ u,
                                                    double* __restrict__ Fo, int nv,
                                                    const V4<typename C::real>* __restrict__ r,
                                                    double4* __restrict__ pos, int* __restrict__ prev_iters) {
    const long long nbN = (g.N + 255) / 256;
    if ((long long)blockIdx.x >= nbN) {
        const int k = int(((long long)blockIdx.x - nbN) * 256) + threadIdx.x;
        if (k < nv) {
            const V4<typename C::real> p = r[k];
            pos[k] = d4(double(p.x), double(p.y), double(p.z));
        }
        if (k == 0 && prev_iters) *prev_iters = ctl->iters;
        return;
    }
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const long long N = g.N;
    double dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double v = double(dec<C>(fin[i * N + n], lp.inv_scale));
        dr += v;
        jx += CX[i] * v;
        jy += CY[i] * v;
        jz += CZ[i] * v;
    }
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    if (ib) {
        const int LxLy = g.Lx * g.Ly;
        const int z = int(n / LxLy), rem = int(n - (long long)z * LxLy), y = rem / g.Lx, x = rem - y * g.Lx;
        const int tile = (x >> TILE_SHIFT) + g.TX * ((y >> TILE_SHIFT) + g.TY * (z >> TILE_SHIFT));
        if (mark[tile] == ctl->epoch) {
            Fx = double(F[n]);
            Fy = double(F[N + n]);
            Fz = double(F[2 * N + n]);
        }
    }
    const double rh = lp.rho0 + dr;
    rho[n] = rh;
    u[n] = (jx + 0.5 * Fx) / rh;
    u[N + n] = (jy + 0.5 * Fy) / rh;
    u[2 * N + n] = (jz + 0.5 * Fz) / rh;
    Fo[n] = Fx;
    Fo[N + n] = Fy;
    Fo[2 * N + n] = Fz;
}

__global__ void k_rec_iters(const Ctl* ctl, int* slot) {
    if (threadIdx.x == 0) *slot = ctl->iters;
}

// ---------------------------------------------------------------- HC transpose
// Forward iteration (o fixed, M the one-ring mean, s the sign):
//   p' = a o + (1-a) M q,  b = p' - a o - (1-a) q,  p = p' - g b - s (1-g) M b.
// Transpose for an incoming pbar:
//   bbar = -g pbar - s (1-g) M^T pbar,   p'bar = pbar + bbar,
//   obar += a pbar,   qbar = -(1-a) bbar + (1-a) M^T p'bar,
// with (M^T y)_j = sum_{k in ring(j)} y_k / m_k. The sweep starts from
// pbar = rbar with obar = 0, and after the m iterations (q_0 = o) obar +=
// qbar. PS and PpS hold P / m and P' / m.
__device__ inline double4 ring_total(const int4* fan, const double4* X, int k, int* m_out) {
    int nb[MAXV];
    const int m = load_fan(fan, k, nb);
    double4 s = d4(0.0, 0.0, 0.0);
#pragma unroll
    for (int j = 0; j < MAXV; ++j)
        if (j < m) s = s + X[nb[j]];
    *m_out = m;
    return s;
}

__global__ void k_adj_hc_a(int nv, const int4* __restrict__ fan, double alpha, double gamma, double sgn,
                           const double4* __restrict__ P, const double4* __restrict__ PS, double4* __restrict__ Pp,
                           double4* __restrict__ PpS, double4* __restrict__ Ob, double4* __restrict__ Qp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    int m;
    const double4 s = ring_total(fan, PS, k, &m);
    const double4 p = P[k];
    const double4 bb = (-gamma) * p - (sgn * (1.0 - gamma)) * s;
    const double4 pp = p + bb;
    Pp[k] = pp;
    PpS[k] = (1.0 / double(m)) * pp;
    Ob[k] = Ob[k] + alpha * p;  // a bbar + a p'bar - a bbar
    Qp[k] = (-(1.0 - alpha)) * bb;
}

__global__ void k_adj_hc_b(int nv, const int4* __restrict__ fan, double alpha, const double4* __restrict__ PpS,
                           const double4* __restrict__ Qp, double4* __restrict__ P, double4* __restrict__ PS) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    int m;
    const double4 s = ring_total(fan, PpS, k, &m);
    const double4 q = Qp[k] + (1.0 - alpha) * s;
    P[k] = q;
    PS[k] = (1.0 / double(m)) * q;
}

// The first iteration's pass a with the initialisation folded in (P = rbar,
// PS = rbar / m, obar = 0 before it). The last iteration's pass b, with the
// final obar += qbar, runs at the start of the interpolation transpose
// (k_adj_spread), in the same operations and order.
__global__ void k_adj_hc_a_first(int nv, const int4* __restrict__ fan, double alpha, double gamma, double sgn,
                                 const double4* __restrict__ rb, double4* __restrict__ Pp, double4* __restrict__ PpS,
                                 double4* __restrict__ Ob, double4* __restrict__ Qp) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    int nb[MAXV];
    const int m = load_fan(fan, k, nb);
    double4 s = d4(0.0, 0.0, 0.0);
#pragma unroll
    for (int j = 0; j < MAXV; ++j)
        if (j < m) s = s + (1.0 / double(fan[4 * nb[j]].x)) * rb[nb[j]];
    const double4 p = rb[k];
    const double4 bb = (-gamma) * p - (sgn * (1.0 - gamma)) * s;
    const double4 pp = p + bb;
    Pp[k] = pp;
    PpS[k] = (1.0 / double(m)) * pp;
    Ob[k] = alpha * p;
    Qp[k] = (-(1.0 - alpha)) * bb;
}

// ---------------------------------------------------------------- stencils (FP64)
// Peskin 4-point weights and their derivatives with respect to the vertex
// coordinate, for fractional part f: with q = sqrt(1 + 4f - 4f^2),
// dq/df = (2 - 4f)/q.
__device__ inline void peskin4_d(double f, double w[4], double dw[4]) {
    const double q = sqrt(1.0 + 4.0 * f - 4.0 * f * f);
    const double dq = (2.0 - 4.0 * f) / q;
    w[0] = (3.0 - 2.0 * f - q) * 0.125;
    w[1] = (3.0 - 2.0 * f + q) * 0.125;
    w[2] = (1.0 + 2.0 * f + q) * 0.125;
    w[3] = (1.0 + 2.0 * f - q) * 0.125;
    dw[0] = (-2.0 - dq) * 0.125;
    dw[1] = (-2.0 + dq) * 0.125;
    dw[2] = (2.0 + dq) * 0.125;
    dw[3] = (2.0 - dq) * 0.125;
}

__device__ inline bool stencil_d(const Geom& g, double4 p, int f[3], double w[3][4], double dw[3][4]) {
    double fr[3];
    const bool ok = stencil_base(p.x, g.xci[0], g.xcf[0], g.Lx, g.px, &f[0], &fr[0]) &&
                    stencil_base(p.y, g.xci[1], g.xcf[1], g.Ly, g.py, &f[1], &fr[1]) &&
                    stencil_base(p.z, g.xci[2], g.xcf[2], g.Lz, g.pz, &f[2], &fr[2]);
    if (ok)
        for (int d = 0; d < 3; ++d) peskin4_d(fr[d], w[d], dw[d]);
    return ok;
}

// Transpose of the interpolation U_k = sum_x u(x) Delta(r_k - x): ubar(x) +=
// Ubar_k Delta(r_k - x). One work-group per surface patch of IB_PATCH
// consecutive vertices (the internal order numbers the vertices patch by
// patch): the patch's 64 stencil contributions per vertex are summed in an
// FP64 LDS window over the patch's stencils (one lane per stencil node, each
// wave taking every fourth vertex), then every touched node takes one global
// atomic add per component. A patch whose window exceeds ADJ_WCAP nodes adds
// its contributions straight to global memory.
constexpr int ADJ_WCAP = 2048;

//
// The work-group's first wave first finishes obar of its vertices, for every
// vertex whether or not its stencil lies in the box: with HC the last
// smoothing iteration's pass b (obar += qbar, qbar = Qp + (1 - alpha) M^T
// p'bar); without smoothing in the forward step obar = rbar.
template <bool HC>
__global__ __launch_bounds__(256) void k_adj_spread(Geom g, int nv, const double4* __restrict__ pos,
                                                    const int4* __restrict__ fan, double alpha,
                                                    const double4* __restrict__ PpS, const double4* __restrict__ Qp,
                                                    const double4* __restrict__ rb, double4* __restrict__ Ob,
                                                    double* __restrict__ ubar) {
    __shared__ int sf[IB_PATCH][3];
    __shared__ double sw[IB_PATCH][3][4];
    __shared__ double sv[IB_PATCH][3];
    __shared__ int sok[IB_PATCH];
    __shared__ int red[6][4];
    __shared__ double win[3 * ADJ_WCAP];
    const int t = threadIdx.x;
    const int k = blockIdx.x * IB_PATCH + t;
    int f[3] = {0, 0, 0};
    bool ok = false;
    if (t < IB_PATCH && k < nv) {
        double4 v;
        if constexpr (HC) {
            int m;
            const double4 sr = ring_total(fan, PpS, k, &m);
            const double4 q = Qp[k] + (1.0 - alpha) * sr;
            v = Ob[k] + q;
        } else {
            v = rb[k];
        }
        Ob[k] = v;
        double w[3][4], dw[3][4];
        ok = stencil_d(g, pos[k], f, w, dw);
        if (ok) {
            for (int d = 0; d < 3; ++d)
                for (int j = 0; j < 4; ++j) sw[t][d][j] = w[d][j];
            sv[t][0] = v.x;
            sv[t][1] = v.y;
            sv[t][2] = v.z;
        }
    }
    if (t < IB_PATCH) {
        for (int d = 0; d < 3; ++d) sf[t][d] = f[d];
        sok[t] = ok ? 1 : 0;
    }
    // window: origin and extent of the active stencils
    int mn[3], mx[3];
    for (int d = 0; d < 3; ++d) {
        mn[d] = ok ? f[d] : 0x3fffffff;
        mx[d] = ok ? f[d] : -0x3fffffff;
    }
    for (int off = 32; off > 0; off >>= 1)
        for (int d = 0; d < 3; ++d) {
            mn[d] = min(mn[d], __shfl_xor(mn[d], off, 64));
            mx[d] = max(mx[d], __shfl_xor(mx[d], off, 64));
        }
    if ((t & 63) == 0)
        for (int d = 0; d < 3; ++d) {
            red[d][t >> 6] = mn[d];
            red[3 + d][t >> 6] = mx[d];
        }
    __syncthreads();
    int o[3], e[3];
    long long vol = 1;
    bool any = true;
    for (int d = 0; d < 3; ++d) {
        int lo = red[d][0], hi = red[3 + d][0];
        for (int q = 1; q < 4; ++q) {
            lo = min(lo, red[d][q]);
            hi = max(hi, red[3 + d][q]);
        }
        any = any && lo <= hi;
        o[d] = lo;
        e[d] = any ? hi - lo + 4 : 0;
        vol *= e[d];
    }
    if (!any) return;
    const long long N = g.N;
    const int lane = t & 63, jx = lane & 3, jy = (lane >> 2) & 3, jz = lane >> 4;
    if (vol > ADJ_WCAP) {
        for (int v = t >> 6; v < IB_PATCH; v += 4) {
            if (!sok[v]) continue;
            const double wt = sw[v][0][jx] * sw[v][1][jy] * sw[v][2][jz];
            const long long n = node_index(g, sf[v][0] + jx, sf[v][1] + jy, sf[v][2] + jz);
            unsafeAtomicAdd(ubar + n, sv[v][0] * wt);
            unsafeAtomicAdd(ubar + N + n, sv[v][1] * wt);
            unsafeAtomicAdd(ubar + 2 * N + n, sv[v][2] * wt);
        }
        return;
    }
    const int nw = int(vol);
    for (int i = t; i < 3 * nw; i += 256) win[i] = 0.0;
    __syncthreads();
    for (int v = t >> 6; v < IB_PATCH; v += 4) {
        if (!sok[v]) continue;
        const double wt = sw[v][0][jx] * sw[v][1][jy] * sw[v][2][jz];
        const int cell = (sf[v][0] + jx - o[0]) + e[0] * ((sf[v][1] + jy - o[1]) + e[1] * (sf[v][2] + jz - o[2]));
        atomicAdd(&win[cell], sv[v][0] * wt);
        atomicAdd(&win[nw + cell], sv[v][1] * wt);
        atomicAdd(&win[2 * nw + cell], sv[v][2] * wt);
    }
    __syncthreads();
    for (int i = t; i < nw; i += 256) {
        const double vx = win[i], vy = win[nw + i], vz = win[2 * nw + i];
        if (vx == 0.0 && vy == 0.0 && vz == 0.0) continue;
        const int lx = i % e[0], rest = i / e[0];
        const int ly = rest % e[1], lz = rest / e[1];
        const long long n = node_index(g, o[0] + lx, o[1] + ly, o[2] + lz);
        unsafeAtomicAdd(ubar + n, vx);
        unsafeAtomicAdd(ubar + N + n, vy);
        unsafeAtomicAdd(ubar + 2 * N + n, vz);
    }
}

// ---------------------------------------------------------------- lattice adjoint
// One thread per node x. Streaming transpose (pull): gbar_i(x) = fbar_i(x +
// c_i), or fbar_{-i}(x) when x + c_i lies beyond a wall. Collision and
// moments transpose with the recorded rho, u, F:
//   rhobar = omega sum_i gbar_i f^eq_i / rho
//   ubar   = ubar_ext + sum_i gbar_i [omega df^eq_i/du + dS_i/du]
//   Fbar   = sum_i gbar_i dS_i/dF + ubar / (2 rho)
//   fbar_j = (1 - omega) gbar_j + rhobar + ubar.(c_j - u) / rho.
// ubar_ext (the transposed interpolation) is cleared once read. Afterwards a
// boundary node adds the moving-wall terms' share of dJ/dA from its pulled
// values: the forward reflected f*_i(x) into slot -i with the term
// -6 w_i rho0 c_i . A (x + c_i/2 - x_c), so dJ/dA += fbar_{-i}(x)
// (-6 w_i rho0) c_i (x + c_i/2 - x_c)^T; each work-group writes its 9 sums to
// part[block][9] (fixed order).
__device__ __forceinline__ void adj_lattice_node(const Geom& g, const LatticeParams& lp, const double* __restrict__ fbin,
                                                 double* __restrict__ fbout, const double* __restrict__ rho_,
                                                 const double* __restrict__ u_, const double* __restrict__ F_,
                                                 double* __restrict__ ubar, double* __restrict__ Fbar, long long n,
                                                 int x, int y, int z, double dA[9]) {
    const long long N = g.N;
    const int LxLy = g.Lx * g.Ly;
    double gb[Q];
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        // the pull source x + c_i, moved back across a periodic side
        long long src = n + CX[i] + (long long)CY[i] * g.Lx + (long long)CZ[i] * LxLy;
        bool wall = false;
        if (CX[i] == 1 && x == g.Lx - 1) { if (g.px) src -= g.Lx; else wall = true; }
        if (CX[i] == -1 && x == 0) { if (g.px) src += g.Lx; else wall = true; }
        if (CY[i] == 1 && y == g.Ly - 1) { if (g.py) src -= LxLy; else wall = true; }
        if (CY[i] == -1 && y == 0) { if (g.py) src += LxLy; else wall = true; }
        if (CZ[i] == 1 && z == g.Lz - 1) { if (g.pz) src -= N; else wall = true; }
        if (CZ[i] == -1 && z == 0) { if (g.pz) src += N; else wall = true; }
        gb[i] = wall ? fbin[opp(i) * N + n] : fbin[i * N + src];
    });
    const double rho = rho_[n];
    const double ux = u_[n], uy = u_[N + n], uz = u_[2 * N + n];
    const double Fx = F_[n], Fy = F_[N + n], Fz = F_[2 * N + n];
    double ex = ubar[n], ey = ubar[N + n], ez = ubar[2 * N + n];
    if (ex != 0.0 || ey != 0.0 || ez != 0.0) {
        ubar[n] = 0.0;
        ubar[N + n] = 0.0;
        ubar[2 * N + n] = 0.0;
    }
    // the sums over i reduce to weighted moments of gbar: G0 = sum w_i g_i,
    // G1 = sum w_i g_i c_i, G2 = sum w_i g_i c_i c_i (c.u = c_i.u, c.F = c_i.F):
    //   rhobar / omega = G0 + 3 G1.u + 9/2 u.G2.u - 3/2 (u.u) G0
    //   ubar - ubar_ext = omega rho (3 G1 + 9 G2 u - 3 u G0) + kg (9 G2 F - 3 F G0)
    //   Fbar_S = kg (3 G1 + 9 G2 u - 3 u G0)
    double G0 = 0.0, G1x = 0.0, G1y = 0.0, G1z = 0.0;
    double Gxx = 0.0, Gyy = 0.0, Gzz = 0.0, Gxy = 0.0, Gxz = 0.0, Gyz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double wg = wgt<double>(i) * gb[i];
        G0 += wg;
        if (CX[i]) G1x += CX[i] * wg;
        if (CY[i]) G1y += CY[i] * wg;
        if (CZ[i]) G1z += CZ[i] * wg;
        if (CX[i]) Gxx += wg;
        if (CY[i]) Gyy += wg;
        if (CZ[i]) Gzz += wg;
        if (CX[i] * CY[i]) Gxy += CX[i] * CY[i] * wg;
        if (CX[i] * CZ[i]) Gxz += CX[i] * CZ[i] * wg;
        if (CY[i] * CZ[i]) Gyz += CY[i] * CZ[i] * wg;
    }
    const double om = lp.omega, kg = lp.kguo;
    const double uu = ux * ux + uy * uy + uz * uz;
    const double Gux = Gxx * ux + Gxy * uy + Gxz * uz;
    const double Guy = Gxy * ux + Gyy * uy + Gyz * uz;
    const double Guz = Gxz * ux + Gyz * uy + Gzz * uz;
    const double GFx = Gxx * Fx + Gxy * Fy + Gxz * Fz;
    const double GFy = Gxy * Fx + Gyy * Fy + Gyz * Fz;
    const double GFz = Gxz * Fx + Gyz * Fy + Gzz * Fz;
    double rb = G0 + 3.0 * (G1x * ux + G1y * uy + G1z * uz) + 4.5 * (ux * Gux + uy * Guy + uz * Guz) - 1.5 * uu * G0;
    const double sx = 3.0 * G1x + 9.0 * Gux - 3.0 * ux * G0;
    const double sy = 3.0 * G1y + 9.0 * Guy - 3.0 * uy * G0;
    const double sz = 3.0 * G1z + 9.0 * Guz - 3.0 * uz * G0;
    const double ubx = ex + om * rho * sx + kg * (9.0 * GFx - 3.0 * Fx * G0);
    const double uby = ey + om * rho * sy + kg * (9.0 * GFy - 3.0 * Fy * G0);
    const double ubz = ez + om * rho * sz + kg * (9.0 * GFz - 3.0 * Fz * G0);
    const double fbx = kg * sx, fby = kg * sy, fbz = kg * sz;
    rb *= om;
    const double inv = 1.0 / rho;
    const double ubu = ubx * ux + uby * uy + ubz * uz;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const double ubc = ubx * CX[j] + uby * CY[j] + ubz * CZ[j];
        fbout[j * N + n] = (1.0 - om) * gb[j] + rb + (ubc - ubu) * inv;
    }
    Fbar[n] = fbx + 0.5 * ubx * inv;
    Fbar[N + n] = fby + 0.5 * uby * inv;
    Fbar[2 * N + n] = fbz + 0.5 * ubz * inv;
    // the moving-wall terms' share of dJ/dA on a boundary node, from the
    // pulled values of its wall links (gbar_i = fbar_{-i}(x) there)
    const bool bnd = (!g.px && (x == 0 || x == g.Lx - 1)) || (!g.py && (y == 0 || y == g.Ly - 1)) ||
                     (!g.pz && (z == 0 || z == g.Lz - 1));
    if (bnd) {
        const double xr = double(x - g.xci[0]) - g.xcf[0];
        const double yr = double(y - g.xci[1]) - g.xcf[1];
        const double zr = double(z - g.xci[2]) - g.xcf[2];
        static_for<1, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const bool wall = (!g.px && ((CX[i] == 1 && x == g.Lx - 1) || (CX[i] == -1 && x == 0))) ||
                              (!g.py && ((CY[i] == 1 && y == g.Ly - 1) || (CY[i] == -1 && y == 0))) ||
                              (!g.pz && ((CZ[i] == 1 && z == g.Lz - 1) || (CZ[i] == -1 && z == 0)));
            if (!wall) return;
            const double sv = -6.0 * wgt<double>(i) * lp.rho0 * gb[i];
            const double wv[3] = {xr + 0.5 * CX[i], yr + 0.5 * CY[i], zr + 0.5 * CZ[i]};
            const int ci[3] = {CX[i], CY[i], CZ[i]};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) dA[3 * a + b] += sv * ci[a] * wv[b];
        });
    }
}

__global__ __launch_bounds__(256) void k_adj_lattice(Geom g, LatticeParams lp, const double* __restrict__ fbin,
                                                     double* __restrict__ fbout, const double* __restrict__ rho_,
                                                     const double* __restrict__ u_, const double* __restrict__ F_,
                                                     double* __restrict__ ubar, double* __restrict__ Fbar,
                                                     double* __restrict__ part) {
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long N = g.N;
    double dA[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) dA[c] = 0.0;
    if (n < N) {
        const int LxLy = g.Lx * g.Ly;
        const int z = int(n / LxLy);
        const int rem = int(n - (long long)z * LxLy);
        const int y = rem / g.Lx;
        const int x = rem - y * g.Lx;
        adj_lattice_node(g, lp, fbin, fbout, rho_, u_, F_, ubar, Fbar, n, x, y, z, dA);
    }
    // fixed-order work-group sums through LDS: 72 threads add runs of 32
    // nodes, then 9 threads add the 8 runs
    __shared__ double red[9][256];
    __shared__ double run[9][8];
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < 9; ++c) red[c][t] = dA[c];
    __syncthreads();
    if (t < 72) {
        const int c = t >> 3, r0 = (t & 7) * 32;
        double acc = 0.0;
#pragma unroll 8
        for (int i = 0; i < 32; ++i) acc += red[c][r0 + i];
        run[c][t & 7] = acc;
    }
    __syncthreads();
    if (t < 9) {
        double acc = run[t][0];
        for (int r = 1; r < 8; ++r) acc += run[t][r];
        part[(long long)blockIdx.x * 9 + t] = acc;
    }
}

// ---------------------------------------------------------------- vertex adjoints
// Transposes of spreading and interpolation with respect to the forces and
// the positions. One wave per vertex, one lane per stencil node:
//   phibar_k = sum_x Fbar(x) Delta(r_k - x)
//   rt_k     = Ob_k + sum_x [Fbar(x).phi_k + u(x).Ubar_k] grad Delta(r_k - x)
// (Ob = Ubar is also the direct term of the Euler move o = r + U.) The
// vertex's force phi_k is recomputed (FP64) from the recorded positions by
// the forward's rule, phi_k = -sigma sum_t n_t x (r_{n_{j+1}} - r_{n_j}) / 2,
// one lane per triangle of the fan.
__global__ __launch_bounds__(256) void k_adj_interp(Geom g, int nv, const int4* __restrict__ fan, double sigma,
                                                    const double4* __restrict__ pos, const double4* __restrict__ Ob,
                                                    const double* __restrict__ Fbar, const double* __restrict__ u_,
                                                    double4* __restrict__ phib, double4* __restrict__ rt) {
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= nv) return;
    double4 phi;
    {
        // the fan holds 16 ints per vertex: the valence, then the ordered ring
        const int* fi = reinterpret_cast<const int*>(fan) + 4 * 4 * (long long)k;
        const int m = fi[0];
        double4 term = d4(0.0, 0.0, 0.0);
        if (lane < m) {
            const double4 pk = pos[k], pa = pos[fi[1 + lane]], pb = pos[fi[1 + (lane + 1 < m ? lane + 1 : 0)]];
            const double4 nn = cross3(pa - pk, pb - pk);
            const double len = sqrt(dot3(nn, nn));
            if (len > 0.0) term = (-0.5 * sigma / len) * cross3(nn, pb - pa);
        }
        phi = d4(wave_sum(term.x), wave_sum(term.y), wave_sum(term.z));
    }
    int f[3];
    double w[3][4], dw[3][4];
    const double4 ub = Ob[k];
    if (!stencil_d(g, pos[k], f, w, dw)) {
        if (lane == 0) {
            phib[k] = d4(0.0, 0.0, 0.0);
            rt[k] = ub;
        }
        return;
    }
    const int jx = lane & 3, jy = (lane >> 2) & 3, jz = lane >> 4;
    const long long n = node_index(g, f[0] + jx, f[1] + jy, f[2] + jz);
    const long long N = g.N;
    const double W = w[0][jx] * w[1][jy] * w[2][jz];
    const double Gx = dw[0][jx] * w[1][jy] * w[2][jz];
    const double Gy = w[0][jx] * dw[1][jy] * w[2][jz];
    const double Gz = w[0][jx] * w[1][jy] * dw[2][jz];
    const double4 fb = d4(Fbar[n], Fbar[N + n], Fbar[2 * N + n]);
    const double4 uu = d4(u_[n], u_[N + n], u_[2 * N + n]);
    const double s = dot3(fb, phi) + dot3(uu, ub);
    const double px = wave_sum(fb.x * W), py = wave_sum(fb.y * W), pz = wave_sum(fb.z * W);
    const double rx = wave_sum(s * Gx), ry = wave_sum(s * Gy), rz = wave_sum(s * Gz);
    if (lane == 0) {
        phib[k] = d4(px, py, pz);
        rt[k] = ub + d4(rx, ry, rz);
    }
}

// Transpose of the forces with respect to the positions and to sigma. For
// the triangle t = (k, a, b) with e1 = r_a - r_k, e2 = r_b - r_k, n = e1 x e2,
// the force adjoint is the directional derivative of its area along phibar,
//   g_t = n^.(de1 x e2 + e1 x de2) / 2,  de1 = phibar_a - phibar_k, ...
// whose position gradient at r_k is -(dg/de1 + dg/de2) with
//   dg/de1 = (e2 x w + de2 x n^)/2,  dg/de2 = (w x e1 + n^ x de1)/2,
//   w = (dn - (n^.dn) n^)/|n|,  dn = de1 x e2 + e1 x de2.
// rbar_k = rt_k - sigma sum_t dg_t/dr_k; dJ/dsigma gets -sum_t g_t, each
// triangle counted at its lowest vertex index (block partials in part).
__global__ __launch_bounds__(256) void k_adj_hess(int nv, const int4* __restrict__ fan, double sigma,
                                                  const double4* __restrict__ pos, const double4* __restrict__ phib,
                                                  const double4* __restrict__ rt, double4* __restrict__ rb,
                                                  double* __restrict__ part) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    double gs = 0.0;
    if (k < nv) {
        int nb[MAXV];
        const int m = load_fan(fan, k, nb);
        const double4 pk = pos[k], qk = phib[k];
        double4 acc = d4(0.0, 0.0, 0.0);
        for (int j = 0; j < m; ++j) {
            const int a = nb[j], b = nb[j + 1 < m ? j + 1 : 0];
            const double4 e1 = pos[a] - pk, e2 = pos[b] - pk;
            const double4 nn = cross3(e1, e2);
            const double len = sqrt(dot3(nn, nn));
            if (!(len > 0.0)) continue;
            const double4 nh = (1.0 / len) * nn;
            const double4 de1 = phib[a] - qk, de2 = phib[b] - qk;
            const double4 dn = cross3(de1, e2) + cross3(e1, de2);
            const double nd = dot3(nh, dn);
            const double4 wv = (1.0 / len) * (dn - nd * nh);
            const double4 g1 = 0.5 * (cross3(e2, wv) + cross3(de2, nh));
            const double4 g2 = 0.5 * (cross3(wv, e1) + cross3(nh, de1));
            acc = acc - (g1 + g2);
            if (k < a && k < b) gs += 0.5 * nd;
        }
        rb[k] = rt[k] - sigma * acc;
    }
    __shared__ double red[4];
    const double v = wave_sum(-gs);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Per-step block partials -> dJ/dA rows (overwritten) and dJ/dsigma
// (accumulated). One work-group per step: each thread sums a fixed strided
// subset of the partials, then a fixed-order tree in LDS; the result does not
// depend on scheduling.
__global__ __launch_bounds__(256) void k_adj_reduce_A(int nbl, const double* __restrict__ Apart,
                                                      double* __restrict__ dA) {
    __shared__ double red[9][256];
    const int j = blockIdx.x, t = threadIdx.x;
    double s[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) s[c] = 0.0;
    for (int b = t; b < nbl; b += 256)
#pragma unroll
        for (int c = 0; c < 9; ++c) s[c] += Apart[((long long)j * nbl + b) * 9 + c];
#pragma unroll
    for (int c = 0; c < 9; ++c) red[c][t] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int c = 0; c < 9; ++c) red[c][t] += red[c][t + w];
        __syncthreads();
    }
    if (t < 9) dA[9 * j + t] = red[t][0];
}

__global__ __launch_bounds__(256) void k_adj_reduce_sigma(long long n, const double* __restrict__ spart,
                                                          double* __restrict__ dsigma) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    double s = 0.0;
    for (long long i = t; i < n; i += 256) s += spart[i];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) *dsigma += red[0];
}

// ---------------------------------------------------------------- objective
// J = D = (sqrt(l1) - sqrt(l3)) / (sqrt(l1) + sqrt(l3)) of S = (5/V)(M - V xb xb^T)
// (Sec. 2). dD/dl1 = c/(a (a+c)^2), dD/dl3 = -a/(c (a+c)^2) with a = sqrt(l1),
// c = sqrt(l3), and dl_i/dS = v_i v_i^T, so Sbar = dD/dl1 v1 v1^T + dD/dl3 v3 v3^T.
// Through S = 5M/V - 5 P P^T / V^2 (P = V xb):
//   Mbar = 5 Sbar / V,  Pbar = -10 Sbar xb / V,  Vbar = (-Sbar:S + 5 xb.Sbar xb) / V.
// Other objectives: J = lambda_max, Sbar = v1 v1^T; J = beta = v1^T E v1 / |E|
// (Eq. beta; its direct dependence on the last row, through E, is added on
// the host), through the eigenvector
// derivative dv1 = sum_{j > 1} v_j (v_j^T dS v1) / (l1 - l_j):
// Sbar = sum_{j > 1} 2 (v1^T E v_j) / (|E| (l1 - l_j)) (v_j v1^T + v1 v_j^T) / 2.
// obs: the observables record (0 V, 1..3 xb relative to x_c, 4..12 S,
// 13..15 eigenvalues, 16..24 eigenvectors by rows). Arow: the last gradient.
// which: 0 D, 1 lambda_max, 2 beta. coef: Vbar, Pbar[3], Mbar[9].
__global__ void k_adj_seed_coef(const double* __restrict__ obs, const double* __restrict__ Arow, int which,
                                double* __restrict__ coef) {
    if (threadIdx.x != 0) return;
    const double V = obs[0];
    const double xb[3] = {obs[1], obs[2], obs[3]};
    const double* S = obs + 4;
    const double* v1 = obs + 16;
    const double* v3 = obs + 22;
    double Sb[9];
    if (which == 0) {
        const double a = sqrt(obs[13]), c = sqrt(obs[15]);
        const double d1 = c / (a * (a + c) * (a + c)), d3 = -a / (c * (a + c) * (a + c));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Sb[3 * i + j] = d1 * v1[i] * v1[j] + d3 * v3[i] * v3[j];
    } else if (which == 1) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) Sb[3 * i + j] = v1[i] * v1[j];
    } else {
        double E[9], En = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                E[3 * i + j] = 0.5 * (Arow[3 * i + j] + Arow[3 * j + i]);
                En += E[3 * i + j] * E[3 * i + j];
            }
        En = sqrt(En);
        for (int k = 0; k < 9; ++k) Sb[k] = 0.0;
        for (int jj = 1; jj < 3; ++jj) {
            const double* vj = obs + 16 + 3 * jj;
            double q = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) q += v1[i] * E[3 * i + j] * vj[j];
            const double cj = 2.0 * q / (En * (obs[13] - obs[13 + jj]));
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Sb[3 * i + j] += 0.5 * cj * (vj[i] * v1[j] + v1[i] * vj[j]);
        }
    }
    double SbS = 0.0, xSx = 0.0, Sx[3];
    for (int i = 0; i < 3; ++i) {
        Sx[i] = 0.0;
        for (int j = 0; j < 3; ++j) {
            SbS += Sb[3 * i + j] * S[3 * i + j];
            Sx[i] += Sb[3 * i + j] * xb[j];
        }
        xSx += xb[i] * Sx[i];
    }
    coef[0] = (-SbS + 5.0 * xSx) / V;
    for (int i = 0; i < 3; ++i) coef[1 + i] = -10.0 * Sx[i] / V;
    for (int k = 0; k < 9; ++k) coef[4 + k] = 5.0 * Sb[k] / V;
}

// dJ/dr_k from the tetrahedra (x_c, r_k, b, c) of the fan triangles (k, b, c):
//   V_t = r_k.(b x c)/6, s = r_k + b + c, Q = r_k r_k^T + b b^T + c c^T + s s^T,
//   dJ/dr_k = sum_t [Vbar + Pbar.s/4 + Mbar:Q/20] (b x c)/6 + V_t [Pbar/4 + Mbar (r_k + s)/10].
__device__ inline double qform(const double* M, double4 v) {
    return v.x * (M[0] * v.x + M[1] * v.y + M[2] * v.z) + v.y * (M[3] * v.x + M[4] * v.y + M[5] * v.z) +
           v.z * (M[6] * v.x + M[7] * v.y + M[8] * v.z);
}

template <class R>
__global__ void k_adj_seed(int nv, const int4* __restrict__ fan, const V4<R>* __restrict__ r,
                           const double* __restrict__ coef, double4* __restrict__ rb) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    const double Vb = coef[0];
    const double4 Pb = d4(coef[1], coef[2], coef[3]);
    const double* Mb = coef + 4;
    int nb[MAXV];
    const int m = load_fan(fan, k, nb);
    const V4<R> pk = r[k];
    const double4 a = d4(double(pk.x), double(pk.y), double(pk.z));
    double4 g = d4(0.0, 0.0, 0.0);
    for (int j = 0; j < m; ++j) {
        const V4<R> qb = r[nb[j]], qc = r[nb[j + 1 < m ? j + 1 : 0]];
        const double4 b = d4(double(qb.x), double(qb.y), double(qb.z));
        const double4 c = d4(double(qc.x), double(qc.y), double(qc.z));
        const double4 bxc = cross3(b, c);
        const double Vt = dot3(a, bxc) / 6.0;
        const double4 s = a + b + c;
        const double MQ = qform(Mb, a) + qform(Mb, b) + qform(Mb, c) + qform(Mb, s);
        const double4 as = a + s;
        const double4 Mas = d4(Mb[0] * as.x + Mb[1] * as.y + Mb[2] * as.z, Mb[3] * as.x + Mb[4] * as.y + Mb[5] * as.z,
                               Mb[6] * as.x + Mb[7] * as.y + Mb[8] * as.z);
        g = g + ((Vb + 0.25 * dot3(Pb, s) + MQ / 20.0) / 6.0) * bxc + Vt * (0.25 * Pb + 0.1 * Mas);
    }
    rb[k] = g;
}

// ---------------------------------------------------------------- vertex order
// perm[k] = caller index of internal vertex k.
__global__ void k_adj_perm_in(int nv, const int* __restrict__ perm, const double* __restrict__ user,
                              double4* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    const int p = perm[k];
    out[k] = d4(user[3 * p], user[3 * p + 1], user[3 * p + 2]);
}

__global__ void k_adj_perm_out(int nv, const int* __restrict__ perm, const double4* __restrict__ in,
                               double* __restrict__ user) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    const int p = perm[k];
    const double4 v = in[k];
    user[3 * p] = v.x;
    user[3 * p + 1] = v.y;
    user[3 * p + 2] = v.z;
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblk(long long n, int bs) { return unsigned((n + bs - 1) / bs); }

#define ADJ_DISPATCH_STORAGE(storage, C, ...)                                \
    switch (storage) {                                                      \
        case IBM_LB_F64: { using C = SF64; __VA_ARGS__; break; }            \
        case IBM_LB_F32: { using C = SF32; __VA_ARGS__; break; }            \
        case IBM_LB_F16DEV: { using C = SF16; __VA_ARGS__; break; }         \
        default: { using C = SBF16; __VA_ARGS__; break; }                   \
    }

hipError_t launch_adj_record(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur,
                             int nv, const AdjStep& st, int* prev_iters, hipStream_t s) {
    ADJ_DISPATCH_STORAGE(storage, C, {
        using R = typename C::real;
        const unsigned nbv = nv > 0 ? nblk(nv, 256) : (prev_iters ? 1u : 0u);
        hipLaunchKernelGGL(k_rec_fields<C>, dim3(nblk(g.N, 256) + nbv), dim3(256), 0, s, g, lp,
                           (const typename C::store_t*)d.f[cur], (const R*)d.F, d.mark, d.ctl, nv > 0 ? 1 : 0,
                           st.rho, st.u, st.F, nv, (const V4<R>*)d.r, st.pos, prev_iters);
    });
    return hipGetLastError();
}

hipError_t launch_adj_record_iters(const DevPtrs& d, int* slot, hipStream_t s) {
    hipLaunchKernelGGL(k_rec_iters, dim3(1), dim3(64), 0, s, d.ctl, slot);
    return hipGetLastError();
}

hipError_t launch_adj_hc(int nv, const int4* fan, const SmoothParams& sp, int iters, const AdjVerts& v,
                         hipStream_t s) {
    const unsigned nb = nblk(nv, 256);
    for (int it = 0; it < iters; ++it) {
        if (it == 0)
            hipLaunchKernelGGL(k_adj_hc_a_first, dim3(nb), dim3(256), 0, s, nv, fan, sp.alpha, sp.gamma,
                               double(sp.sign), v.rb, v.Pp, v.PpS, v.Ob, v.Qp);
        else
            hipLaunchKernelGGL(k_adj_hc_a, dim3(nb), dim3(256), 0, s, nv, fan, sp.alpha, sp.gamma, double(sp.sign),
                               v.P, v.PS, v.Pp, v.PpS, v.Ob, v.Qp);
        if (it < iters - 1)
            hipLaunchKernelGGL(k_adj_hc_b, dim3(nb), dim3(256), 0, s, nv, fan, sp.alpha, v.PpS, v.Qp, v.P, v.PS);
    }
    return hipGetLastError();
}

hipError_t launch_adj_ib_spread(const Geom& g, int nv, const int4* fan, double alpha, int iters,
                                const double4* pos, const AdjVerts& v, double* ubar, hipStream_t s) {
    if (iters > 0)
        hipLaunchKernelGGL(k_adj_spread<true>, dim3(nblk(nv, IB_PATCH)), dim3(256), 0, s, g, nv, pos, fan, alpha,
                           v.PpS, v.Qp, v.rb, v.Ob, ubar);
    else
        hipLaunchKernelGGL(k_adj_spread<false>, dim3(nblk(nv, IB_PATCH)), dim3(256), 0, s, g, nv, pos, fan, alpha,
                           v.PpS, v.Qp, v.rb, v.Ob, ubar);
    return hipGetLastError();
}

int adj_lattice_blocks(long long N) { return (int)nblk(N, 256); }
int adj_vertex_blocks(int nv) { return (int)nblk(nv, 256); }

hipError_t launch_adj_lattice(const Geom& g, const LatticeParams& lp, const double* fbin, double* fbout,
                              const AdjStep& st, double* ubar, double* Fbar, double* Apart, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_lattice, dim3(nblk(g.N, 256)), dim3(256), 0, s, g, lp, fbin, fbout, st.rho, st.u, st.F,
                       ubar, Fbar, Apart);
    return hipGetLastError();
}

hipError_t launch_adj_ib_back(const Geom& g, int nv, const int4* fan, double sigma, const AdjStep& st,
                              const double* Fbar, const AdjVerts& v, double* spart, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_interp, dim3(nblk(nv, 4)), dim3(256), 0, s, g, nv, fan, sigma, st.pos, v.Ob, Fbar, st.u,
                       v.phib, v.rt);
    hipLaunchKernelGGL(k_adj_hess, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, fan, sigma, st.pos, v.phib, v.rt, v.rb,
                       spart);
    return hipGetLastError();
}

hipError_t launch_adj_reduce(int nsteps, int nbl, const double* Apart, int nbv, const double* spart, double* dA,
                             double* dsigma, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_reduce_A, dim3(nsteps), dim3(256), 0, s, nbl, Apart, dA);
    if (nbv > 0)
        hipLaunchKernelGGL(k_adj_reduce_sigma, dim3(1), dim3(256), 0, s, (long long)nsteps * nbv, spart, dsigma);
    return hipGetLastError();
}

hipError_t launch_adj_seed(int storage, int nv, const DevPtrs& d, double* coef, double4* rb, hipStream_t s,
                           int which) {
    hipLaunchKernelGGL(k_adj_seed_coef, dim3(1), dim3(64), 0, s, d.obs_out, d.Abuf + 9ll * ACAP, which, coef);
    if (storage == IBM_LB_F64)
        hipLaunchKernelGGL(k_adj_seed<double>, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, d.fan,
                           (const V4<double>*)d.r, coef, rb);
    else
        hipLaunchKernelGGL(k_adj_seed<float>, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, d.fan, (const V4<float>*)d.r,
                           coef, rb);
    return hipGetLastError();
}

hipError_t launch_adj_perm_in(int nv, const int* perm, const double* user, double4* out, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_perm_in, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, perm, user, out);
    return hipGetLastError();
}

// dJ/dA0 through the initial populations (linear initial state):
//   f_i^0 - w_i rho0 = w_i rho0 [3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u.u] - 3 tau w_i rho0 (c_i c_i - I/3):A0,
//   u = A0 (x - x_c), so with d = x - x_c
//   d f_i^0 / d A0_ab = w_i rho0 [(3 c_ia + 9 (c_i.u) c_ia - 3 u_a) d_b - 3 tau (c_ia c_ib - delta_ab / 3)].
// Each work-group sums fbar_i(x) times that over its nodes (grid-stride) into
// part[block][9]; the host adds the blocks in order.
struct Mat9 {
    double a[9];
};

__global__ __launch_bounds__(256) void k_adj_init_A0(Geom g, LatticeParams lp, Mat9 A0, const double* __restrict__ fbar,
                                                     double* __restrict__ part) {
    __shared__ double red[9][256];
    const long long N = g.N;
    const int LxLy = g.Lx * g.Ly;
    double acc[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] = 0.0;
    for (long long n = (long long)blockIdx.x * 256 + threadIdx.x; n < N; n += (long long)gridDim.x * 256) {
        const int z = int(n / LxLy), rem = int(n - (long long)z * LxLy), y = rem / g.Lx, x = rem - y * g.Lx;
        const double dv[3] = {double(x - g.xci[0]) - g.xcf[0], double(y - g.xci[1]) - g.xcf[1],
                              double(z - g.xci[2]) - g.xcf[2]};
        double u[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = A0.a[3 * a] * dv[0] + A0.a[3 * a + 1] * dv[1] + A0.a[3 * a + 2] * dv[2];
        double G[3] = {0.0, 0.0, 0.0}, H[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) H[c] = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double wf = wgt<double>(i) * fbar[(long long)i * N + n];
            const int ci[3] = {CX[i], CY[i], CZ[i]};
            const double cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                G[a] += wf * ((3.0 + 9.0 * cu) * ci[a] - 3.0 * u[a]);
#pragma unroll
                for (int b = 0; b < 3; ++b) H[3 * a + b] += wf * (ci[a] * ci[b] - (a == b ? 1.0 / 3.0 : 0.0));
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) acc[3 * a + b] += lp.rho0 * (G[a] * dv[b] - 3.0 * lp.tau * H[3 * a + b]);
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 9; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 9) part[9ll * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_adj_init_A0(const Geom& g, const LatticeParams& lp, const double A0[9], const double* fbar,
                              double* part, int nblocks, hipStream_t s) {
    Mat9 m;
    for (int c = 0; c < 9; ++c) m.a[c] = A0[c];
    hipLaunchKernelGGL(k_adj_init_A0, dim3(nblocks), dim3(256), 0, s, g, lp, m, fbar, part);
    return hipGetLastError();
}

hipError_t launch_adj_perm_out(int nv, const int* perm, const double4* in, double* user, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_perm_out, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, perm, in, user);
    return hipGetLastError();
}

}  // namespace ibmlb
