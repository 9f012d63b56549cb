// HIP kernels of the IB-LB droplet step for gfx950 (wave64).
//
// Method: arXiv 2403.01161 (Taglienti, Guglietta & Sbragaglia), Sec. 3.1
// (D3Q19 BGK + Guo forcing, Peskin 4-point immersed boundary, moving walls)
// and Sec. 3.3 (HC mesh smoothing); observables of Sec. 2.
//
// Layout: populations are SoA planes f[i][z][y][x] holding deviations
// d_i = f_i - w_i rho0 from the rest equilibrium; force and velocity fields
// are SoA [3][z][y][x] and are only touched inside the 8^3 tiles marked for
// the current step; vertex data are AoS V4 records relative to the box centre.
#include <hip/hip_ext.h>
#include <math.h>

#include "lattice_kernels.h"

namespace ibmlb {

// The per-storage lattice launchers are compiled in lattice_{f64,f32,f16,bf16}.hip.
#define IBMLB_LATTICE_EXTERN(C)                                                                                   \
    extern template hipError_t launch_lattice_c<C>(const Geom&, const LatticeParams&, const DevPtrs&, int, bool,    \
                                                   const double*, int, int, hipStream_t, hipEvent_t, hipEvent_t,     \
                                                   const MrtRates*, const ChiRates*);                                \
    extern template hipError_t launch_lattice_batch_c<C>(const LatDesc*, const int2*, const int*, const int*,       \
                                                         const int*, int, long long, int, bool, hipStream_t);
IBMLB_LATTICE_EXTERN(SF64)
IBMLB_LATTICE_EXTERN(SF32)
IBMLB_LATTICE_EXTERN(SF16)
IBMLB_LATTICE_EXTERN(SBF16)
#undef IBMLB_LATTICE_EXTERN

// ---------------------------------------------------------------- initial state
template <class C>
__global__ __launch_bounds__(256) void k_init(Geom g, LatticeParams lp, typename C::store_t* f,
                                              const double* A0, int rest) {
    long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    if (rest) {
#pragma unroll
        for (int i = 0; i < Q; ++i) f[i * g.N + n] = enc<C>(typename C::real(0), lp.scale);
        return;
    }
    int LxLy = g.Lx * g.Ly;
    int z = int(n / LxLy), rem = int(n - (long long)z * LxLy), y = rem / g.Lx, x = rem - y * g.Lx;
    double dx = x - (g.xci[0] + g.xcf[0]), dy = y - (g.xci[1] + g.xcf[1]),
           dz = z - (g.xci[2] + g.xcf[2]);
    double ux = A0[0] * dx + A0[1] * dy + A0[2] * dz;
    double uy = A0[3] * dx + A0[4] * dy + A0[5] * dz;
    double uz = A0[6] * dx + A0[7] * dy + A0[8] * dz;
    double uu = ux * ux + uy * uy + uz * uz, tr = A0[0] + A0[4] + A0[8];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        double cAc = 0.0;
        const int c[3] = {CX[i], CY[i], CZ[i]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) cAc += c[a] * A0[3 * a + b] * c[b];
        double w = wgt<double>(i);
        // f_eq(rho0, u) - w rho0 plus the Chapman-Enskog non-equilibrium part
        double dv = w * lp.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu) -
                    3.0 * lp.tau * w * lp.rho0 * (cAc - tr / 3.0);
        f[i * g.N + n] = enc<C>(typename C::real(dv), lp.scale);
    }
}

// Diagnostic moments: rho and u (with F/2) of the current populations; the
// force field is the one already spread for the coming step (read only).
template <class C>
__global__ __launch_bounds__(256) void k_moments(Geom g, LatticeParams lp,
                                                 const typename C::store_t* __restrict__ fin,
                                                 const typename C::real* __restrict__ F,
                                                 const int* __restrict__ mark, const Ctl* ctl,
                                                 int ib, double* rho_out, double* u_out) {
    using R = typename C::real;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.N) return;
    const long long N = g.N;
    const int LxLy = g.Lx * g.Ly;
    const int z = int(n / LxLy), rem = int(n - (long long)z * LxLy), y = rem / g.Lx, x = rem - y * g.Lx;
    R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        R v = dec<C>(fin[i * N + n], lp.inv_scale);
        drho += v;
        jx += R(CX[i]) * v;
        jy += R(CY[i]) * v;
        jz += R(CZ[i]) * v;
    }
    R Fx = R(0), Fy = R(0), Fz = R(0);
    if (ib) {
        const int tile = (x >> TILE_SHIFT) + g.TX * ((y >> TILE_SHIFT) + g.TY * (z >> TILE_SHIFT));
        if (mark[tile] == ctl->epoch) {
            Fx = F[n]; Fy = F[N + n]; Fz = F[2 * N + n];
        }
    }
    const R rho = R(lp.rho0) + drho;
    rho_out[n] = double(rho);
    u_out[n] = double((jx + R(0.5) * Fx) / rho);
    u_out[N + n] = double((jy + R(0.5) * Fy) / rho);
    u_out[2 * N + n] = double((jz + R(0.5) * Fz) / rho);
}

// FP64 mass and momentum partial sums (sum of deviations; the host adds N rho0).
template <class C>
__global__ __launch_bounds__(256) void k_mass(Geom g, LatticeParams lp,
                                              const typename C::store_t* __restrict__ fin,
                                              double* part) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < g.N;
         n += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            double v = double(dec<C>(fin[i * g.N + n], lp.inv_scale));
            s[0] += v;
            s[1] += CX[i] * v;
            s[2] += CY[i] * v;
            s[3] += CZ[i] * v;
        }
    }
    __shared__ double red[4][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double v = wave_sum(s[k]);
        if (lane == 0) red[k][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        int k = threadIdx.x;
        part[blockIdx.x * 4 + k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
    }
}

__global__ void k_bump_epoch(Ctl* ctl) {
    if (threadIdx.x == 0) ctl->epoch += 1;
}

template <class R>
__global__ void k_clear(R* F, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        F[i] = R(0);
}

// ---------------------------------------------------------------- wet-node walls
// Velocity walls through the boundary nodes (Sec. 3.1, the Zou-He conditions
// in the 3D form of Hecht and Harting), applied to the streamed populations
// of f: every population whose source lies outside the box is rebuilt from
// the known ones and the wall velocity u_w = A (x - x_c) at the node. With n
// the inward normal of a wall through the node and i the opposite of an
// unknown j (deviations d = f - w rho0; the rest-weight parts cancel):
//   one wall (Eq. ZH_bulk): rho = (rho0 + sum_{c.n=0} d + 2 sum_{c.n<0} d) / (1 - u_w.n),
//     d_j = d_i - (2 - |t_i|) rho/6 c_i.u_w - rho/3 t_i.u_w + 1/2 sum_k d_k (t_i.c_k)(1 - |c_k.n|),
//     t_i = c_i - (c_i.n) n;
//   two or three walls (an edge or a corner; inward normals n1, n2 (, n3)):
//     the node takes density rho and momentum rho u_w, and the linear field's
//     populations up to second order in A. An unknown j whose opposite i is
//     known bounces back with the moving-wall term of Eq. (standard BB) for
//     any link, d_j = d_i - 6 w_i rho c_i.u_w; at an edge it also takes the
//     along-edge correction of Eq. (ZH_edges), with the sign of Eq. (ZH_bulk)'s
//     and its velocity term: - rho/12 t_i.u_w
//     + 1/4 sum_k d_k (t_i.c_k)(1 - |c_k.n1|)(1 - |c_k.n2|). The buried links
//     (c.(n1 + n2 (+ n3)) = 0 with both c and -c unknown) and the rest
//     population are reset (as Eqs. zh-buried-links-edges and -corners
//     reset them) to the equilibrium at (rho, u_w) plus the linear field's
//     non-equilibrium part: d_j = w_j (rho - rho0) + rho h_j,
//     h_j = w_j (3 c.u + 9/2 (c.u)^2 - 3/2 u.u) - 3 tau w_j (c c - I/3):A.
//     rho follows from sum_j f_j = rho: with D the sum of d over the known
//     populations outside the bounce-back pairs plus twice d_i over the pairs,
//     S6 = sum_pairs 6 w_i c_i.u_w, H = sum over the reset populations of h_j
//     and W their weight, rho - rho0 = (D - rho0 S6 + rho0 H) / (1 + S6 - W - H).
//     (As printed, the edge and corner rules carry no wall-velocity term and
//     the edge correction has the opposite sign; a linear flow then stays
//     wrong at first order in A.)
// Thread t takes node t of the concatenated non-periodic face planes, the
// lower in-plane axis fastest (so the y and z faces read whole x-rows); a
// node on several faces is rebuilt by the first of them (order x-, x+, y-,
// y+, z-, z+). With (wx, wy, wz) the inward normal components of the walls
// through the node, every rule above is generic: t_i is c_i without its wall
// components, the products (1 - |c.n|) run over the walls, n1 + n2 (+ n3) is
// (wx, wy, wz), and n1 x n2 points along the axis without a wall.
// Face nodes of the non-periodic axes, concatenated.
__host__ __device__ inline long long wall_nodes(const Geom& g) {
    long long total = 0;
    if (!g.px) total += 2ll * g.Ly * g.Lz;
    if (!g.py) total += 2ll * g.Lx * g.Lz;
    if (!g.pz) total += 2ll * g.Lx * g.Ly;
    return total;
}

// Face node r (< wall_nodes(g)) of the walls above; f plain or global-space.
template <class C, class PF, class PA>
__device__ __forceinline__ void wet_wall_node(const Geom& g, const LatticeParams& lp, PF f, PA Arow, long long r) {
    using R = typename C::real;
    // the face of this thread and its node (faces of periodic axes absent)
    int x = 0, y = 0, z = 0, face = -1;
    const long long ax = (long long)g.Ly * g.Lz, ay = (long long)g.Lx * g.Lz, az = (long long)g.Lx * g.Ly;
    if (!g.px) {
        if (r < 2 * ax) {
            face = r < ax ? 0 : 1;
            const long long q = r - (face & 1) * ax;
            x = face == 0 ? 0 : g.Lx - 1;
            y = int(q % g.Ly);
            z = int(q / g.Ly);
        } else {
            r -= 2 * ax;
        }
    }
    if (face < 0 && !g.py) {
        if (r < 2 * ay) {
            face = r < ay ? 2 : 3;
            const long long q = r - (face & 1) * ay;
            y = face == 2 ? 0 : g.Ly - 1;
            x = int(q % g.Lx);
            z = int(q / g.Lx);
        } else {
            r -= 2 * ay;
        }
    }
    if (face < 0 && !g.pz) {
        if (r < 2 * az) {
            face = r < az ? 4 : 5;
            const long long q = r - (face & 1) * az;
            z = face == 4 ? 0 : g.Lz - 1;
            x = int(q % g.Lx);
            y = int(q / g.Lx);
        }
    }
    if (face < 0) return;
    // inward normal components of the walls through the node (0: no wall on that axis)
    const int wx = g.px ? 0 : (x == 0 ? 1 : (x == g.Lx - 1 ? -1 : 0));
    const int wy = g.py ? 0 : (y == 0 ? 1 : (y == g.Ly - 1 ? -1 : 0));
    const int wz = g.pz ? 0 : (z == 0 ? 1 : (z == g.Lz - 1 ? -1 : 0));
    const int first = wx ? (wx > 0 ? 0 : 1) : (wy ? (wy > 0 ? 2 : 3) : (wz > 0 ? 4 : 5));
    if (first != face) return;  // another face's thread rebuilds this node
    const int nw = (wx != 0) + (wy != 0) + (wz != 0);
    const long long N = g.N;
    const long long n = x + (long long)g.Lx * (y + (long long)g.Ly * z);
    R d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = dec<C>(f[i * N + n], lp.inv_scale);
    const double rx = x - g.xci[0] - g.xcf[0], ry = y - g.xci[1] - g.xcf[1], rz = z - g.xci[2] - g.xcf[2];
    const R u0 = R(Arow[0] * rx + Arow[1] * ry + Arow[2] * rz);
    const R u1 = R(Arow[3] * rx + Arow[4] * ry + Arow[5] * rz);
    const R u2 = R(Arow[6] * rx + Arow[7] * ry + Arow[8] * rz);
    // per population: unknown (from outside), c.(sum of the normals), and the
    // product over the walls of (1 - |c.n|)
    auto unk = [&](int j) { return wx * CX[j] > 0 || wy * CY[j] > 0 || wz * CZ[j] > 0; };
    auto cN = [&](int j) { return wx * CX[j] + wy * CY[j] + wz * CZ[j]; };
    auto tang = [&](int k) {
        return (1 - abs(wx * CX[k])) * (1 - abs(wy * CY[k])) * (1 - abs(wz * CZ[k]));
    };
    R out[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) out[j] = d[j];
    if (nw == 1) {
        R s0 = R(0), sm = R(0);
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const int cn = cN(k);
            s0 += cn == 0 ? d[k] : R(0);
            sm += cn < 0 ? d[k] : R(0);
        }
        const R un = u0 * R(wx) + u1 * R(wy) + u2 * R(wz);
        const R rho = (R(lp.rho0) + s0 + R(2) * sm) / (R(1) - un);
#pragma unroll
        for (int j = 1; j < Q; ++j) {
            if (!unk(j)) continue;
            const int i = opp(j);
            // t_i: c_i without its component along the normal
            const int tx = wx ? 0 : CX[i], ty = wy ? 0 : CY[i], tz = wz ? 0 : CZ[i];
            const R tn = R(tx * tx + ty * ty + tz * tz);  // |t| is 0 or 1
            const R cu = R(CX[i]) * u0 + R(CY[i]) * u1 + R(CZ[i]) * u2;
            const R tu = R(tx) * u0 + R(ty) * u1 + R(tz) * u2;
            R corr = R(0);
#pragma unroll
            for (int k = 1; k < Q; ++k) corr += R(tang(k) * (tx * CX[k] + ty * CY[k] + tz * CZ[k])) * d[k];
            out[j] = d[i] - (R(2) - tn) * rho / R(6) * cu - rho / R(3) * tu + R(0.5) * corr;
        }
    } else {
        // reset populations (buried links and rest): h_j, their weight W and sum H
        const R uu = u0 * u0 + u1 * u1 + u2 * u2;
        const double trA3 = (Arow[0] + Arow[4] + Arow[8]) / 3.0;
        const R tau3 = R(3.0 * lp.tau);
        R h[Q];
        R W = R(0), H = R(0), S6 = R(0), D = R(0);
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const bool reset = j == 0 || (unk(j) && unk(opp(j)));
            h[j] = R(0);
            if (reset) {
                const R cu = R(CX[j]) * u0 + R(CY[j]) * u1 + R(CZ[j]) * u2;
                double cAc = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b2 = 0; b2 < 3; ++b2) {
                        const int ca = a == 0 ? CX[j] : (a == 1 ? CY[j] : CZ[j]);
                        const int cb = b2 == 0 ? CX[j] : (b2 == 1 ? CY[j] : CZ[j]);
                        if (ca * cb) cAc += double(ca * cb) * Arow[3 * a + b2];
                    }
                h[j] = wgt<R>(j) * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * uu - tau3 * R(cAc - trA3));
                W += wgt<R>(j);
                H += h[j];
            } else if (unk(j)) {
                const int i = opp(j);
                S6 += (R(6) * wgt<R>(i)) * (R(CX[i]) * u0 + R(CY[i]) * u1 + R(CZ[i]) * u2);
                D += R(2) * d[i];
            } else if (!unk(opp(j))) {
                D += d[j];  // neither it nor its opposite crosses a wall
            }
        }
        const R r0 = R(lp.rho0);
        const R drho = (D - r0 * S6 + r0 * H) / (R(1) + S6 - W - H);
        const R rho = r0 + drho;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            if (j == 0 || (unk(j) && unk(opp(j)))) {
                out[j] = wgt<R>(j) * drho + rho * h[j];
                continue;
            }
            if (!unk(j)) continue;
            const int i = opp(j);
            const R cu = R(CX[i]) * u0 + R(CY[i]) * u1 + R(CZ[i]) * u2;
            out[j] = d[i] - (R(6) * wgt<R>(i)) * rho * cu;
            if (nw == 3) continue;
            const int tx = wx ? 0 : CX[i], ty = wy ? 0 : CY[i], tz = wz ? 0 : CZ[i];
            const R tu = R(tx) * u0 + R(ty) * u1 + R(tz) * u2;
            R corr = R(0);
#pragma unroll
            for (int k = 1; k < Q; ++k) corr += R(tang(k) * (tx * CX[k] + ty * CY[k] + tz * CZ[k])) * d[k];
            out[j] += R(0.25) * corr - rho / R(12) * tu;
        }
    }
#pragma unroll
    for (int j = 0; j < Q; ++j)
        if ((j > 0 && unk(j)) || (j == 0 && nw > 1)) f[j * N + n] = enc<C>(out[j], lp.scale);
}

template <class C>
__global__ __launch_bounds__(256) void k_wet_walls(Geom g, LatticeParams lp, typename C::store_t* __restrict__ f,
                                                   const double* __restrict__ Arow, long long total) {
    const long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= total) return;
    wet_wall_node<C>(g, lp, f, Arow, r);
}

// Ensemble form: work-group b takes block map[b].y of the face nodes of
// member map[b].x, on the copy its lattice launch (input copy cur) wrote,
// with the gradient row at A + arow.
template <class C>
__global__ __launch_bounds__(256) void k_wet_walls_batch(const LatDesc* __restrict__ desc,
                                                         const int2* __restrict__ map, int cur, long long arow) {
    const int2 e = map[blockIdx.x];
    const MemberView<C> M(desc[e.x], cur);
    const long long r = (long long)e.y * 256 + threadIdx.x;
    if (r >= wall_nodes(M.g)) return;
    wet_wall_node<C>(M.g, M.lp, M.fout, M.A + arow, r);
}

// ---------------------------------------------------------------- observables (FP64)
// Signed tetrahedra (x_c, a, b, c) of every triangle: V_t = a.(b x c)/6,
// int x dV = V_t (a+b+c)/4, int x x^T dV = V_t/20 (aa^T+bb^T+cc^T+ss^T).
// Mesh quality: the smallest corner angle atan2(|u x v|, u.v) and the
// shortest and longest edge (block slots 10, 11, 12).
template <class R>
__global__ __launch_bounds__(256) void k_obs_partial(int nt, const int4* __restrict__ tris,
                                                     const V4<R>* __restrict__ r, double* part) {
    double s[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) s[k] = 0.0;
    double amin = __builtin_inf(), emin = __builtin_inf(), emax = 0.0;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
        const int4 tr = tris[t];
        const V4<R> pa = r[tr.x], pb = r[tr.y], pc = r[tr.z];
        const double a[3] = {double(pa.x), double(pa.y), double(pa.z)};
        const double b[3] = {double(pb.x), double(pb.y), double(pb.z)};
        const double c[3] = {double(pc.x), double(pc.y), double(pc.z)};
        const double bxc0 = b[1] * c[2] - b[2] * c[1], bxc1 = b[2] * c[0] - b[0] * c[2],
                     bxc2 = b[0] * c[1] - b[1] * c[0];
        const double V = (a[0] * bxc0 + a[1] * bxc1 + a[2] * bxc2) / 6.0;
        const double sx = a[0] + b[0] + c[0], sy = a[1] + b[1] + c[1], sz = a[2] + b[2] + c[2];
        s[0] += V;
        s[1] += V * sx * 0.25;
        s[2] += V * sy * 0.25;
        s[3] += V * sz * 0.25;
        const double v20 = V / 20.0;
        s[4] += v20 * (a[0] * a[0] + b[0] * b[0] + c[0] * c[0] + sx * sx);
        s[5] += v20 * (a[1] * a[1] + b[1] * b[1] + c[1] * c[1] + sy * sy);
        s[6] += v20 * (a[2] * a[2] + b[2] * b[2] + c[2] * c[2] + sz * sz);
        s[7] += v20 * (a[0] * a[1] + b[0] * b[1] + c[0] * c[1] + sx * sy);
        s[8] += v20 * (a[0] * a[2] + b[0] * b[2] + c[0] * c[2] + sx * sz);
        s[9] += v20 * (a[1] * a[2] + b[1] * b[2] + c[1] * c[2] + sy * sz);
        const double* P[3] = {a, b, c};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double* p0 = P[j];
            const double* p1 = P[(j + 1) % 3];
            const double* p2 = P[(j + 2) % 3];
            const double u0 = p1[0] - p0[0], u1 = p1[1] - p0[1], u2 = p1[2] - p0[2];
            const double w0 = p2[0] - p0[0], w1 = p2[1] - p0[1], w2 = p2[2] - p0[2];
            const double x0 = u1 * w2 - u2 * w1, x1 = u2 * w0 - u0 * w2, x2 = u0 * w1 - u1 * w0;
            amin = fmin(amin, atan2(sqrt(x0 * x0 + x1 * x1 + x2 * x2), u0 * w0 + u1 * w1 + u2 * w2));
            const double len = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
            emin = fmin(emin, len);
            emax = fmax(emax, len);
        }
    }
    __shared__ double red[13][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 10; ++k) {
        double v = wave_sum(s[k]);
        if (lane == 0) red[k][wv] = v;
    }
    for (int m = 32; m > 0; m >>= 1) {
        amin = fmin(amin, __shfl_xor(amin, m, 64));
        emin = fmin(emin, __shfl_xor(emin, m, 64));
        emax = fmax(emax, __shfl_xor(emax, m, 64));
    }
    if (lane == 0) {
        red[10][wv] = amin;
        red[11][wv] = emin;
        red[12][wv] = emax;
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        const int k = threadIdx.x;
        part[blockIdx.x * 16 + k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
    } else if (threadIdx.x < 13) {
        const int k = threadIdx.x;
        double v = red[k][0];
        for (int w = 1; w < 4; ++w) v = k == 12 ? fmax(v, red[k][w]) : fmin(v, red[k][w]);
        part[blockIdx.x * 16 + k] = v;
    }
}

// Symmetric 3x3 eigenpairs by cyclic Jacobi rotations (FP64), descending, each
// eigenvector with its largest-magnitude component positive.
__device__ __forceinline__ void jacobi3(const double S[9], double ev[3], double vec[9]) {
    double a[3][3], v[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a[i][j] = 0.5 * (S[3 * i + j] + S[3 * j + i]);
            v[i][j] = i == j ? 1.0 : 0.0;
        }
    const double scale = fabs(a[0][0]) + fabs(a[1][1]) + fabs(a[2][2]) + fabs(a[0][1]) +
                         fabs(a[0][2]) + fabs(a[1][2]);
    for (int sweep = 0; sweep < 100; ++sweep) {
        const double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        if (off == 0.0 || off <= 1e-15 * scale) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {
                    const double x = a[k][p], y = a[k][q];
                    a[k][p] = c * x - s * y;
                    a[k][q] = s * x + c * y;
                }
                for (int k = 0; k < 3; ++k) {
                    const double x = a[p][k], y = a[q][k];
                    a[p][k] = c * x - s * y;
                    a[q][k] = s * x + c * y;
                }
                for (int k = 0; k < 3; ++k) {
                    const double x = v[k][p], y = v[k][q];
                    v[k][p] = c * x - s * y;
                    v[k][q] = s * x + c * y;
                }
            }
    }
    // eigenpairs by decreasing eigenvalue: compare-exchanges (0, 1), (0, 2),
    // (1, 2) of the diagonal that carry the columns of v along (constant
    // indices throughout, so the arrays stay in registers)
    double e[3] = {a[0][0], a[1][1], a[2][2]};
    double c[3][3];
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) c[k][i] = v[i][k];
    auto cx = [&](int i, int j) {
        if (e[j] > e[i]) {
            const double t = e[i];
            e[i] = e[j];
            e[j] = t;
            for (int m = 0; m < 3; ++m) {
                const double u = c[i][m];
                c[i][m] = c[j][m];
                c[j][m] = u;
            }
        }
    };
    cx(0, 1);
    cx(0, 2);
    cx(1, 2);
    for (int k = 0; k < 3; ++k) {
        ev[k] = e[k];
        // sign: the largest component (the first of equal ones) positive
        double big = c[k][0];
        if (fabs(c[k][1]) > fabs(big)) big = c[k][1];
        if (fabs(c[k][2]) > fabs(big)) big = c[k][2];
        const double sg = big < 0.0 ? -1.0 : 1.0;
        for (int i = 0; i < 3; ++i) vec[3 * k + i] = sg * c[k][i];
    }
}

// Output layout (doubles): 0 volume, 1..3 centroid (relative to x_c),
// 4..12 S, 13..15 eigval, 16..24 eigvec, 25 D, 26 beta, 27 theta_deg,
// 28 flags, 29 sum of deviations, 30..32 momentum, 33 iters, 34 cap hits,
// 35 smallest triangle angle (degrees), 36 shortest edge, 37 longest edge.
// The block partials are reduced by 256 threads in a fixed order (thread t
// takes partials t, t + 256, ... in turn, then a fixed pairwise tree in LDS),
// so the result is the same on every run; thread 0 finishes.
constexpr int OBS_FINAL_THREADS = 256;
__global__ __launch_bounds__(OBS_FINAL_THREADS) void k_obs_final(int nblocks, const double* part, int mblocks,
                                                                 const double* mpart, const double* Arow,
                                                                 double radius, int has_mesh, Ctl* ctl,
                                                                 double* out) {
    // slots 0-3 mass and momentum, 4-13 volume moments, 14 smallest angle,
    // 15 shortest edge, 16 longest edge
    constexpr int NS = 17;
    __shared__ double red[NS][OBS_FINAL_THREADS];
    const int t = threadIdx.x;
    double v[NS];
    for (int k = 0; k < 14; ++k) v[k] = 0.0;
    v[14] = __builtin_inf();
    v[15] = __builtin_inf();
    v[16] = 0.0;
    for (int b = t; b < mblocks; b += OBS_FINAL_THREADS)
        for (int k = 0; k < 4; ++k) v[k] += mpart[4 * b + k];
    if (has_mesh)
        for (int b = t; b < nblocks; b += OBS_FINAL_THREADS) {
            for (int k = 0; k < 10; ++k) v[4 + k] += part[16 * b + k];
            v[14] = fmin(v[14], part[16 * b + 10]);
            v[15] = fmin(v[15], part[16 * b + 11]);
            v[16] = fmax(v[16], part[16 * b + 12]);
        }
    for (int k = 0; k < NS; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int h = OBS_FINAL_THREADS / 2; h > 0; h >>= 1) {
        if (t < h) {
            for (int k = 0; k < 14; ++k) red[k][t] += red[k][t + h];
            red[14][t] = fmin(red[14][t], red[14][t + h]);
            red[15][t] = fmin(red[15][t], red[15][t + h]);
            red[16][t] = fmax(red[16][t], red[16][t + h]);
        }
        __syncthreads();
    }
    if (t != 0) return;
    for (int k = 0; k < OBS_OUT_N; ++k) out[k] = 0.0;
    out[29] = red[0][0];
    out[30] = red[1][0];
    out[31] = red[2][0];
    out[32] = red[3][0];
    out[33] = ctl->iters;
    out[34] = ctl->cap_hits;
    ctl->cap_hits = 0;
    if (!has_mesh) return;
    double s[10];
    for (int k = 0; k < 10; ++k) s[k] = red[4 + k][0];
    out[35] = red[14][0] * (180.0 / 3.14159265358979323846);
    out[36] = red[15][0];
    out[37] = red[16][0];
    const double V = s[0];
    const double xb[3] = {s[1] / V, s[2] / V, s[3] / V};
    const double M[9] = {s[4], s[7], s[8], s[7], s[5], s[9], s[8], s[9], s[6]};
    double S[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[3 * a + b] = 5.0 / V * (M[3 * a + b] - V * xb[a] * xb[b]);
    double ev[3], vec[9];
    jacobi3(S, ev, vec);
    const double D = (sqrt(ev[0]) - sqrt(ev[2])) / (sqrt(ev[0]) + sqrt(ev[2]));
    double E[9], En = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            E[3 * a + b] = 0.5 * (Arow[3 * a + b] + Arow[3 * b + a]);
            En += E[3 * a + b] * E[3 * a + b];
        }
    En = sqrt(En);
    int flags = 0;
    if (ev[0] - ev[1] < 1e-12 * radius * radius) flags |= IBM_LB_OBS_DEGENERATE;
    if (En == 0.0) flags |= IBM_LB_OBS_E_ZERO;
    double beta = __builtin_nan(""), theta = __builtin_nan("");
    if (!(flags & IBM_LB_OBS_DEGENERATE)) {
        theta = atan2(vec[1], vec[0]) * (180.0 / 3.14159265358979323846);
        if (theta > 90.0) theta -= 180.0;
        if (theta <= -90.0) theta += 180.0;
        if (!(flags & IBM_LB_OBS_E_ZERO)) {
            double q = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) q += vec[a] * E[3 * a + b] * vec[b];
            beta = q / En;
        }
    }
    out[0] = V;
    for (int a = 0; a < 3; ++a) out[1 + a] = xb[a];
    for (int k = 0; k < 9; ++k) out[4 + k] = S[k];
    for (int k = 0; k < 3; ++k) out[13 + k] = ev[k];
    for (int k = 0; k < 9; ++k) out[16 + k] = vec[k];
    out[25] = D;
    out[26] = beta;
    out[27] = theta;
    out[28] = flags;
}

// ---------------------------------------------------------------- position transfer
template <class R>
__global__ void k_pos_to_abs(Geom g, int nv, const V4<R>* r, double* out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    const V4<R> p = r[k];
    out[3 * k + 0] = double(p.x) + (g.xci[0] + g.xcf[0]);
    out[3 * k + 1] = double(p.y) + (g.xci[1] + g.xcf[1]);
    out[3 * k + 2] = double(p.z) + (g.xci[2] + g.xcf[2]);
}

template <class R>
__global__ void k_pos_from_abs(Geom g, int nv, const double* in, V4<R>* r) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    r[k] = V4<R>{R(in[3 * k + 0] - (g.xci[0] + g.xcf[0])), R(in[3 * k + 1] - (g.xci[1] + g.xcf[1])),
                 R(in[3 * k + 2] - (g.xci[2] + g.xcf[2])), R(0)};
}

// ---------------------------------------------------------------- launchers
size_t storage_bytes(int storage) {
    switch (storage) {
        case IBM_LB_F64: return 8;
        case IBM_LB_F32: return 4;
        default: return 2;
    }
}
size_t real_bytes(int storage) { return storage == IBM_LB_F64 ? 8 : 4; }



hipError_t launch_init(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d,
                       const double* A0, int rest, hipStream_t s) {
    DISPATCH_STORAGE(storage, C, {
        hipLaunchKernelGGL(k_init<C>, dim3(blocks_for(g.N, 256)), dim3(256), 0, s, g, lp,
                           (typename C::store_t*)d.f[0], A0, rest);
    });
    return hipGetLastError();
}

// Launched with hipExtLaunchKernelGGL so that optional timing events are
// stamped by the dispatch itself (no separate event packets around it).
hipError_t launch_aa_settle(int storage, const Geom& g, const DevPtrs& d, int cur, hipStream_t s) {
    DISPATCH_STORAGE(storage, C, {
        using S = typename C::store_t;
        hipLaunchKernelGGL(k_aa_settle<C>, dim3(blocks_for(g.N, 256)), dim3(256), 0, s, g, (S*)d.f[cur]);
    });
    return hipGetLastError();
}

int lattice_rows_per_block(int variant, int Lx) {
    if (!(variant & VAR_ROWS) || Lx < 1 || Lx > ROWS_MAX_T) return 0;
    const int want = LAT_BS[(variant >> 1) & 3];
    const int r = want / Lx;
    return r < 1 ? 1 : r;
}

int lattice_variant_ok(int variant, const Geom& g) {
    if (variant < 0 || variant >= STEP_VARIANTS) return 0;
    if ((variant & VAR_AA) && (variant & VAR_ROWS)) return 0;
    if (variant & VAR_ROWS) return lattice_rows_per_block(variant, g.Lx) > 0;
    return 1;
}

hipError_t launch_lattice(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d,
                          int cur, bool ib, const double* A_row, int variant, int parity, hipStream_t s,
                          hipEvent_t e0, hipEvent_t e1, const MrtRates* mrt, const ChiRates* chi) {
    if (!lattice_variant_ok(variant, g)) return hipErrorInvalidValue;
    if (mrt && chi) return hipErrorInvalidValue;
    switch (storage) {
        case IBM_LB_F64: return launch_lattice_c<SF64>(g, lp, d, cur, ib, A_row, variant, parity, s, e0, e1, mrt, chi);
        case IBM_LB_F32: return launch_lattice_c<SF32>(g, lp, d, cur, ib, A_row, variant, parity, s, e0, e1, mrt, chi);
        case IBM_LB_F16DEV:
            return launch_lattice_c<SF16>(g, lp, d, cur, ib, A_row, variant, parity, s, e0, e1, mrt, chi);
        default: return launch_lattice_c<SBF16>(g, lp, d, cur, ib, A_row, variant, parity, s, e0, e1, mrt, chi);
    }
}

hipError_t launch_lattice_batch(int storage, const LatDesc* desc, const int2* maps, const int moff[8],
                                const int nblocks[8], const int nib[8], int cur, long long step, int variant,
                                bool mrt, hipStream_t s) {
    if (variant < 0 || variant >= STEP_VARIANTS) return hipErrorInvalidValue;
    switch (storage) {
        case IBM_LB_F64: return launch_lattice_batch_c<SF64>(desc, maps, moff, nblocks, nib, cur, step, variant, mrt, s);
        case IBM_LB_F32: return launch_lattice_batch_c<SF32>(desc, maps, moff, nblocks, nib, cur, step, variant, mrt, s);
        case IBM_LB_F16DEV:
            return launch_lattice_batch_c<SF16>(desc, maps, moff, nblocks, nib, cur, step, variant, mrt, s);
        default: return launch_lattice_batch_c<SBF16>(desc, maps, moff, nblocks, nib, cur, step, variant, mrt, s);
    }
}

// Point every member's gradient rows at base + i * stride (graph replays of
// the batched step read rows 0, 1, ... from there).
__global__ void k_set_rows(LatDesc* desc, int n, const double* base, long long stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) desc[i].A = base + (long long)i * stride;
}

hipError_t launch_set_rows(LatDesc* desc, int n, const double* base, long long stride, hipStream_t s) {
    hipLaunchKernelGGL(k_set_rows, dim3((n + 63) / 64), dim3(64), 0, s, desc, n, base, stride);
    return hipGetLastError();
}

#define DISPATCH_REAL(storage, R, ...)                                   \
    if ((storage) == IBM_LB_F64) { using R = double; __VA_ARGS__; }     \
    else { using R = float; __VA_ARGS__; }

long long wall_node_count(const Geom& g) { return wall_nodes(g); }

hipError_t launch_wet_walls_batch(int storage, const LatDesc* desc, const int2* map, int nblocks, int cur,
                                  long long arow, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    DISPATCH_STORAGE(storage, C, {
        hipLaunchKernelGGL(k_wet_walls_batch<C>, dim3(nblocks), dim3(256), 0, s, desc, map, cur, arow);
    });
    return hipGetLastError();
}

hipError_t launch_wet_walls(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur,
                            const double* A_row, hipStream_t s) {
    const long long total = wall_nodes(g);
    if (total == 0) return hipSuccess;
    DISPATCH_STORAGE(storage, C, {
        using S = typename C::store_t;
        hipLaunchKernelGGL(k_wet_walls<C>, dim3(blocks_for(total, 256)), dim3(256), 0, s, g, lp, (S*)d.f[cur], A_row,
                           total);
    });
    return hipGetLastError();
}

hipError_t launch_bump_epoch(const DevPtrs& d, hipStream_t s) {
    hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(64), 0, s, d.ctl);
    return hipGetLastError();
}

hipError_t launch_clear_force(int storage, const Geom& g, const DevPtrs& d, hipStream_t s) {
    DISPATCH_REAL(storage, R, {
        hipLaunchKernelGGL(k_clear<R>, dim3(1024), dim3(256), 0, s, (R*)d.F, 3 * g.N);
    });
    return hipGetLastError();
}

hipError_t launch_moments(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d,
                          int cur, bool ib, double* rho_out, double* u_out, hipStream_t s) {
    DISPATCH_STORAGE(storage, C, {
        using R = typename C::real;
        hipLaunchKernelGGL(k_moments<C>, dim3(blocks_for(g.N, 256)), dim3(256), 0, s, g, lp,
                           (const typename C::store_t*)d.f[cur], (const R*)d.F, d.mark, d.ctl, ib ? 1 : 0,
                           rho_out, u_out);
    });
    return hipGetLastError();
}

hipError_t launch_observables(int storage, const Geom& g, const LatticeParams& lp,
                              const DevPtrs& d, int cur, int nv, int nt, double radius,
                              const double* A_row, hipStream_t s) {
    DISPATCH_STORAGE(storage, C, {
        hipLaunchKernelGGL(k_mass<C>, dim3(MASS_BLOCKS), dim3(256), 0, s, g, lp,
                           (const typename C::store_t*)d.f[cur], d.mass_part);
    });
    if (nv > 0) {
        DISPATCH_REAL(storage, R, {
            hipLaunchKernelGGL(k_obs_partial<R>, dim3(OBS_BLOCKS), dim3(256), 0, s, nt, d.tris,
                               (const V4<R>*)d.r, d.obs_part);
        });
    }
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(OBS_FINAL_THREADS), 0, s, OBS_BLOCKS, d.obs_part, MASS_BLOCKS,
                       d.mass_part, A_row, radius, nv > 0 ? 1 : 0, d.ctl, d.obs_out);
    return hipGetLastError();
}

hipError_t launch_positions_to_abs(int storage, const Geom& g, const DevPtrs& d, int nv,
                                   double* out, hipStream_t s) {
    DISPATCH_REAL(storage, R, {
        hipLaunchKernelGGL(k_pos_to_abs<R>, dim3(blocks_for(nv, 256)), dim3(256), 0, s, g, nv,
                           (const V4<R>*)d.r, out);
    });
    return hipGetLastError();
}

hipError_t launch_positions_from_abs(int storage, const Geom& g, const DevPtrs& d, int nv,
                                     const double* in, hipStream_t s) {
    DISPATCH_REAL(storage, R, {
        hipLaunchKernelGGL(k_pos_from_abs<R>, dim3(blocks_for(nv, 256)), dim3(256), 0, s, g, nv, in,
                           (V4<R>*)d.r);
    });
    return hipGetLastError();
}

}  // namespace ibmlb
