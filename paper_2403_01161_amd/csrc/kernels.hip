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

#include "lattice_common.h"

namespace ibmlb {

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

// ---------------------------------------------------------------- fused lattice step
// One thread per node: load the 19 deviations (coalesced), form rho and the
// half-force-corrected u, relax with BGK plus the Guo source, and push each
// post-collision population to its neighbour. A population whose target lies
// beyond a wall is reflected into the opposite slot of the same node with
// the moving-wall term -2 w_i rho0 c_i.u_w / cs^2, u_w = A (x + c_i/2 - x_c).
//
// Two store layouts, chosen per configuration by the autotuner:
//   * linear (k_lattice): work-group b owns nodes [b BS, (b+1) BS) and writes
//     every population straight to its target; the ten populations that move
//     along x land one element off the thread's own node, so their stores
//     straddle cache lines shared with the neighbouring work-group. Optional
//     XCD grouping gives each XCD a contiguous range of the lattice, so that
//     such shared lines meet in one L2 (pays when the two population copies
//     nearly fit the last-level cache);
//   * rows (k_lattice_rows): a work-group owns whole x-rows; the populations
//     that move along x are handed to their target thread through LDS, so
//     every global store is at the storing thread's own x (row-aligned).
//     Pays for footprints well beyond the last-level cache.
// Further options: non-temporal population loads, non-temporal population
// stores (rows) and the work-group size.

// Rank of population i among the ten that move along x (their LDS slot).
__host__ __device__ constexpr int xslot(int i) {
    int k = 0;
    for (int j = 0; j < i; ++j) k += CX[j] != 0 ? 1 : 0;
    return k;
}
constexpr int NXMOVE = xslot(Q);

// Block order grouped by XCD: consecutive work-groups are dispatched to the
// eight XCDs in turn; this sends the first eighth of the lattice to XCD 0,
// the next eighth to XCD 1, and so on (a tail of nb mod 8 blocks keeps its
// place).
__device__ inline unsigned xcd_order(unsigned b, unsigned nb) {
    const unsigned per = nb >> 3;
    return b < (per << 3) ? (b & 7u) * per + (b >> 3) : b;
}

template <bool NTS, class P, class V>
__device__ __forceinline__ void put(P p, V v) {
    if (NTS) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Node coordinates from the linear index (32-bit division below 2^31 nodes).
__device__ __forceinline__ void node_xyz(const Geom& g, long long n, int& x, int& y, int& z) {
    const int LxLy = g.Lx * g.Ly;
    int r;
    if (g.N <= 0x7fffffffll) {
        const int m = int(n);
        z = m / LxLy;
        r = m - z * LxLy;
    } else {
        z = int(n / LxLy);
        r = int(n - (long long)z * LxLy);
    }
    y = r / g.Lx;
    x = r - y * g.Lx;
}

// Target of population i pushed from node n = (x, y, z): n + c_i . (1, Lx,
// Lx Ly), moved back across a periodic side; *wall when it leaves through a
// wall instead.
template <int I>
__device__ __forceinline__ long long push_target(const Geom& g, long long n, int x, int y, int z, bool* wall) {
    const long long LxLy = (long long)g.Lx * g.Ly;
    long long t = n + CX[I] + (long long)CY[I] * g.Lx + (long long)CZ[I] * LxLy;
    bool w = false;
    if (CX[I] == 1 && x == g.Lx - 1) { if (g.px) t -= g.Lx; else w = true; }
    if (CX[I] == -1 && x == 0) { if (g.px) t += g.Lx; else w = true; }
    if (CY[I] == 1 && y == g.Ly - 1) { if (g.py) t -= LxLy; else w = true; }
    if (CY[I] == -1 && y == 0) { if (g.py) t += LxLy; else w = true; }
    if (CZ[I] == 1 && z == g.Lz - 1) { if (g.pz) t -= g.N; else w = true; }
    if (CZ[I] == -1 && z == 0) { if (g.pz) t += g.N; else w = true; }
    *wall = w;
    return t;
}

// In-place streaming in two alternating steps (one population copy):
//   even step: node x reads its own populations f_i(x) and stores its
//     post-collision f*_i(x) in slot opp(i) of x itself, the moving-wall
//     term already applied when the link leaves through a wall;
//   odd step: node x reads f_i(x) = f*_i(x - c_i) from slot opp(i) of
//     x - c_i (from slot i of x itself when x - c_i lies beyond a wall),
//     and stores f*_i(x) in slot i of x + c_i (slot opp(i) of x, with the
//     wall term, through a wall).
// Each thread reads and writes the same set of locations in either step, so
// no two threads touch one location. After an odd step the copy holds the
// populations in natural order again; after an even step they are read with
// the odd step's mapping (aa_settle).
//
// Where population i of node (x, y, z) is read in the odd step: *slot and
// the node index.
template <int I>
__device__ __forceinline__ long long pull_source(const Geom& g, long long n, int x, int y, int z, int* slot) {
    const long long LxLy = (long long)g.Lx * g.Ly;
    long long s = n - CX[I] - (long long)CY[I] * g.Lx - (long long)CZ[I] * LxLy;
    bool w = false;
    if (CX[I] == -1 && x == g.Lx - 1) { if (g.px) s -= g.Lx; else w = true; }
    if (CX[I] == 1 && x == 0) { if (g.px) s += g.Lx; else w = true; }
    if (CY[I] == -1 && y == g.Ly - 1) { if (g.py) s -= LxLy; else w = true; }
    if (CY[I] == 1 && y == 0) { if (g.py) s += LxLy; else w = true; }
    if (CZ[I] == -1 && z == g.Lz - 1) { if (g.pz) s -= g.N; else w = true; }
    if (CZ[I] == 1 && z == 0) { if (g.pz) s += g.N; else w = true; }
    *slot = w ? I : opp(I);
    return w ? n : s;
}

// ROWS: x-moving populations that stay in the box go to stage[xslot(i) T + t]
// instead of global memory (t: the thread's slot, T: slots per plane).
// The pointer parameters are plain pointers, or global-address-space
// pointers where the caller read them from memory (so that the accesses
// compile to global rather than flat instructions).
// AREG: read the gradient row into registers before any store (for
// pointers the compiler cannot tell apart from the stores' targets);
// otherwise it is read where a reflection needs it.
// AA: 0 two copies (read fin, push into fout), 1 even in-place step, 2 odd
// in-place step (fin and fout the same copy).
// MRT: the multiple-relaxation-time collision with the rates *mr instead of
// BGK: f* = f - M^-1 [S M (f - f_eq) - (I - S/2) M G], G the Guo term without
// its (1 - 1/(2 tau)) factor (with every rate 1/tau, the BGK step).
// CHI: a node whose indicator byte ind[n] is set (inside the droplet) relaxes
// with the rates *ch instead of lp's; the byte is cleared for the next
// step's indicator. Only marked tiles hold inside nodes, so only they read it.
template <class C, bool IB, bool NTL, bool ROWS, bool NTS, bool AREG, int AA, bool MRT = false, bool CHI = false,
          class PIn, class POut, class PR, class PM, class PC, class PA>
__device__ __forceinline__ void lattice_node(const Geom& g, const LatticeParams& lp, PIn fin, POut fout, PR F,
                                             PR U, PM mark, PC ctl, PA Arow,
                                             const long long n, const int x, const int y, const int z,
                                             typename C::store_t* stage, int t, int T,
                                             const MrtRates* mr = nullptr, unsigned char* ind = nullptr,
                                             const ChiRates* ch = nullptr) {
    using R = typename C::real;
    using S = typename C::store_t;
    const long long N = g.N;

    R d[Q];
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        int slot = i;
        const long long src = AA == 2 ? pull_source<i>(g, n, x, y, z, &slot) : n;
        if (NTL) d[i] = dec<C>(__builtin_nontemporal_load(&fin[slot * N + src]), lp.inv_scale);
        else d[i] = dec<C>(fin[slot * N + src], lp.inv_scale);
    });

    R drho = R(0), jx = R(0), jy = R(0), jz = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        drho += d[i];
        if (CX[i] == 1) jx += d[i];
        if (CX[i] == -1) jx -= d[i];
        if (CY[i] == 1) jy += d[i];
        if (CY[i] == -1) jy -= d[i];
        if (CZ[i] == 1) jz += d[i];
        if (CZ[i] == -1) jz -= d[i];
    }

    R Fx = R(0), Fy = R(0), Fz = R(0);
    bool marked = false;
    if (IB) {
        const int tile = (x >> TILE_SHIFT) + g.TX * ((y >> TILE_SHIFT) + g.TY * (z >> TILE_SHIFT));
        marked = mark[tile] == ctl->epoch;
        if (marked) {
            Fx = F[n];
            Fy = F[N + n];
            Fz = F[2 * N + n];
            // leave the force field zero for the next step's spreading
            F[n] = R(0);
            F[N + n] = R(0);
            F[2 * N + n] = R(0);
        }
    }
    const R rho = R(lp.rho0) + drho;
    const R inv = R(1) / rho;
    const R ux = (jx + R(0.5) * Fx) * inv;
    const R uy = (jy + R(0.5) * Fy) * inv;
    const R uz = (jz + R(0.5) * Fz) * inv;
    if (IB && marked) {
        U[n] = ux;
        U[N + n] = uy;
        U[2 * N + n] = uz;
    }
    if (!(rho > R(0)) || !isfinite(ux + uy + uz)) atomicOr((int*)&ctl->flags, DFLAG_NONFINITE);

    R omega = R(lp.omega), kg = R(lp.kguo);
    const R rho0 = R(lp.rho0);
    if constexpr (CHI) {
        // inside nodes lie in marked tiles only (the indicator build marks them)
        if (marked && ind[n]) {
            omega = R(ch->omega_in);
            kg = R(ch->kguo_in);
            ind[n] = 0;
        }
    }
    const R usq = ux * ux + uy * uy + uz * uz;
    const R uF = ux * Fx + uy * Fy + uz * Fz;

    // Moving-wall term of a reflected population: 6 w_i rho0 c_i . u_w with
    // the wall velocity u_w = A (x - x_c + c_i / 2) at the link midpoint.
    double Ad[9];  // uniform: scalar registers
    if constexpr (AREG) {
#pragma unroll
        for (int k = 0; k < 9; ++k) Ad[k] = Arow[k];
    }
    auto wall_term = [&](int i) {
        R A[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) A[k] = R(AREG ? Ad[k] : double(Arow[k]));
        const R xr = R(x - g.xci[0]) - R(g.xcf[0]);
        const R yr = R(y - g.xci[1]) - R(g.xcf[1]);
        const R zr = R(z - g.xci[2]) - R(g.xcf[2]);
        const R cx = R(CX[i]), cy = R(CY[i]), cz = R(CZ[i]);
        const R ax = A[0] * (xr + R(0.5) * cx) + A[1] * (yr + R(0.5) * cy) + A[2] * (zr + R(0.5) * cz);
        const R ay = A[3] * (xr + R(0.5) * cx) + A[4] * (yr + R(0.5) * cy) + A[5] * (zr + R(0.5) * cz);
        const R az = A[6] * (xr + R(0.5) * cx) + A[7] * (yr + R(0.5) * cy) + A[8] * (zr + R(0.5) * cz);
        return R(6) * wgt<R>(i) * rho0 * (cx * ax + cy * ay + cz * az);
    };

    auto push = [&](auto ic, R val) {
        constexpr int i = decltype(ic)::value;
        bool wall;
        const long long tg = push_target<i>(g, n, x, y, z, &wall);
        if (AA == 1) {
            put<NTS>(&fout[opp(i) * N + n], enc<C>(wall ? val - wall_term(i) : val, lp.scale));
        } else if (!wall) {
            if (ROWS && CX[i] != 0) stage[xslot(i) * T + t] = enc<C>(val, lp.scale);
            else put<NTS>(&fout[i * N + tg], enc<C>(val, lp.scale));
        } else {
            put<NTS>(&fout[opp(i) * N + n], enc<C>(val - wall_term(i), lp.scale));
        }
    };

    if constexpr (MRT) {
        R nq[Q], gq[Q];
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const R w = wgt<R>(i);
            const R cu = R(CX[i]) * ux + R(CY[i]) * uy + R(CZ[i]) * uz;
            const R cF = R(CX[i]) * Fx + R(CY[i]) * Fy + R(CZ[i]) * Fz;
            nq[i] = d[i] - w * (drho + rho * (R(4.5) * cu * cu + R(3) * cu - R(1.5) * usq));
            gq[i] = w * (R(3) * (cF - uF) + R(9) * cu * cF);
        });
        static_for<0, Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            R mn = R(0), mg = R(0);
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int m = mrt_m(k, i);
                if constexpr (m != 0) {
                    mn += R(m) * nq[i];
                    mg += R(m) * gq[i];
                }
            });
            const R sk = R(mr->s[k]);
            const R r = (sk * mn - (R(1) - R(0.5) * sk) * mg) * (R(1) / R(mrt_norm2(k)));
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int m = mrt_m(k, i);
                if constexpr (m != 0) d[i] -= R(m) * r;
            });
        });
        put<NTS>(&fout[n], enc<C>(d[0], lp.scale));
        static_for<1, Q>([&](auto ic) { push(ic, d[decltype(ic)::value]); });
        return;
    }
    {   // rest population
        const R w = wgt<R>(0);
        const R deq = w * (drho + rho * (R(-1.5) * usq));
        const R S0 = kg * w * (R(-3) * uF);
        put<NTS>(&fout[n], enc<C>(d[0] - omega * (d[0] - deq) + S0, lp.scale));
    }
    static_for<1, 10>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        constexpr int i = 2 * p - 1, j = 2 * p;
        const R w = wgt<R>(i);
        const R cu = R(CX[i]) * ux + R(CY[i]) * uy + R(CZ[i]) * uz;
        const R cF = R(CX[i]) * Fx + R(CY[i]) * Fy + R(CZ[i]) * Fz;
        const R sym = w * (drho + rho * (R(4.5) * cu * cu - R(1.5) * usq));
        const R anti = w * rho * R(3) * cu;
        const R Ssym = kg * w * (R(9) * cu * cF - R(3) * uF);
        const R Santi = kg * w * R(3) * cF;
        push(std::integral_constant<int, i>{}, d[i] - omega * (d[i] - (sym + anti)) + Ssym + Santi);
        push(std::integral_constant<int, j>{}, d[j] - omega * (d[j] - (sym - anti)) + Ssym - Santi);
    });
}

// Second half of the row layout: thread t (node n, coordinates x, y, z)
// stores, at its own x, every x-moving population arriving from x - c_x in
// its row (x - c_x wrapped on a periodic axis; nothing arrives through a
// wall, and nothing whose row shift crosses a wall, both having been
// reflected at the source).
template <class C, bool NTS, class POut>
__device__ __forceinline__ void rows_receive(const Geom& g, POut fout, const typename C::store_t* stage, long long n,
                                             int x, int y, int z, int t, int T) {
    const long long N = g.N;
    const long long LxLy = (long long)g.Lx * g.Ly;
    const int row0 = t - x;  // slot of x = 0 in this row
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if (CX[i] == 0) return;
        int xs = x - CX[i];
        if (xs < 0 || xs >= g.Lx) {
            if (!g.px) return;
            xs = wrap(xs, g.Lx);
        }
        long long tg = n + (long long)CY[i] * g.Lx + (long long)CZ[i] * LxLy;
        if (CY[i] == 1 && y == g.Ly - 1) { if (!g.py) return; tg -= LxLy; }
        if (CY[i] == -1 && y == 0) { if (!g.py) return; tg += LxLy; }
        if (CZ[i] == 1 && z == g.Lz - 1) { if (!g.pz) return; tg -= N; }
        if (CZ[i] == -1 && z == 0) { if (!g.pz) return; tg += N; }
        put<NTS>(&fout[i * N + tg], stage[xslot(i) * T + row0 + xs]);
    });
}

template <class C, bool IB, bool NTL, int BS>
__global__ __launch_bounds__(BS) void k_lattice(Geom g, LatticeParams lp,
                                                 const typename C::store_t* __restrict__ fin,
                                                 typename C::store_t* __restrict__ fout,
                                                 typename C::real* __restrict__ F,
                                                 typename C::real* __restrict__ U,
                                                 const int* __restrict__ mark, Ctl* ctl,
                                                 const double* __restrict__ Arow, int xcd) {
    const unsigned b = xcd ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
    const long long n = (long long)b * BS + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    lattice_node<C, IB, NTL, false, false, false, 0>(g, lp, fin, fout, F, U, mark, ctl, Arow, n, x, y, z, nullptr, 0,
                                                  0);
}

// MRT collision, linear layout with two copies.
template <class C, bool IB, bool NTL, int BS>
__global__ __launch_bounds__(BS) void k_lattice_mrt(Geom g, LatticeParams lp,
                                                     const typename C::store_t* __restrict__ fin,
                                                     typename C::store_t* __restrict__ fout,
                                                     typename C::real* __restrict__ F,
                                                     typename C::real* __restrict__ U,
                                                     const int* __restrict__ mark, Ctl* ctl,
                                                     const double* __restrict__ Arow, int xcd, MrtRates mr) {
    const unsigned b = xcd ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
    const long long n = (long long)b * BS + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    lattice_node<C, IB, NTL, false, false, false, 0, true>(g, lp, fin, fout, F, U, mark, ctl, Arow, n, x, y, z,
                                                        nullptr, 0, 0, &mr);
}

// Viscosity ratio: BGK with the inner rates on the nodes the indicator marks,
// linear layout with two copies.
template <class C, bool IB, bool NTL, int BS>
__global__ __launch_bounds__(BS) void k_lattice_chi(Geom g, LatticeParams lp,
                                                     const typename C::store_t* __restrict__ fin,
                                                     typename C::store_t* __restrict__ fout,
                                                     typename C::real* __restrict__ F,
                                                     typename C::real* __restrict__ U,
                                                     const int* __restrict__ mark, Ctl* ctl,
                                                     const double* __restrict__ Arow, int xcd,
                                                     unsigned char* __restrict__ ind, ChiRates ch) {
    const unsigned b = xcd ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
    const long long n = (long long)b * BS + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    lattice_node<C, IB, NTL, false, false, false, 0, false, true>(g, lp, fin, fout, F, U, mark, ctl, Arow, n, x, y,
                                                               z, nullptr, 0, 0, nullptr, ind, &ch);
}

// In-place (single-copy) form, linear layout: ODD selects the step parity.
// CHI: the viscosity ratio's inner rates on the nodes the indicator marks.
template <class C, bool IB, bool NTL, int BS, bool ODD, bool CHI = false>
__global__ __launch_bounds__(BS) void k_lattice_aa(Geom g, LatticeParams lp, typename C::store_t* f,
                                                    typename C::real* __restrict__ F,
                                                    typename C::real* __restrict__ U,
                                                    const int* __restrict__ mark, Ctl* ctl,
                                                    const double* __restrict__ Arow, int xcd,
                                                    unsigned char* __restrict__ ind = nullptr,
                                                    ChiRates ch = ChiRates{}) {
    const unsigned b = xcd ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
    const long long n = (long long)b * BS + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    lattice_node<C, IB, NTL, false, false, false, ODD ? 2 : 1, false, CHI>(
        g, lp, (const typename C::store_t*)f, f, F, U, mark, ctl, Arow, n, x, y, z, nullptr, 0, 0, nullptr, ind, &ch);
}

// After an even in-place step, back to natural order in place. In the odd
// mapping f_i(x) sits in slot opp(i) of x - c_i, and slot i of x holds
// f_opp(i)(x - c_i): the two swap. Node x swaps this pair for the directions
// of odd index (each pair of opposite directions is (2p - 1, 2p)), so every
// location belongs to one pair handled by one thread; where x - c_i lies
// beyond a wall both populations are already in place.
template <class C>
__global__ __launch_bounds__(256) void k_aa_settle(Geom g, typename C::store_t* __restrict__ f) {
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    const long long N = g.N;
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (i & 1) {
            static_assert(opp(i) == i + 1, "opposite directions are paired (2p - 1, 2p)");
            int slot;
            const long long src = pull_source<i>(g, n, x, y, z, &slot);
            if (slot != i) {
                const typename C::store_t a = f[i * N + n], b = f[opp(i) * N + src];
                f[i * N + n] = b;
                f[opp(i) * N + src] = a;
            }
        }
    });
}

// Row layout: `rows` whole x-rows per work-group (blockDim = rows * Lx <= 512).
// CHI: the viscosity ratio's inner rates on the nodes the indicator marks;
// MRT: the multiple-relaxation-time collision with the rates mr.
constexpr int ROWS_MAX_T = 512;

template <class C, bool IB, bool NTL, bool NTS, bool CHI = false, bool MRT = false>
__global__ __launch_bounds__(ROWS_MAX_T) void k_lattice_rows(Geom g, LatticeParams lp,
                                                             const typename C::store_t* __restrict__ fin,
                                                             typename C::store_t* __restrict__ fout,
                                                             typename C::real* __restrict__ F,
                                                             typename C::real* __restrict__ U,
                                                             const int* __restrict__ mark, Ctl* ctl,
                                                             const double* __restrict__ Arow, int rows,
                                                             unsigned char* __restrict__ ind = nullptr,
                                                             ChiRates ch = ChiRates{}, MrtRates mr = MrtRates{}) {
    using S = typename C::store_t;
    extern __shared__ __align__(16) unsigned char dyn[];
    S* stage = reinterpret_cast<S*>(dyn);
    const int T = rows * g.Lx;
    const int t = threadIdx.x;
    // rows of Lx nodes: row index from the work-group, x from the thread
    const int rl = t / g.Lx;
    const int x = t - rl * g.Lx;
    const int row = int(blockIdx.x) * rows + rl;
    const int z = row / g.Ly, y = row - z * g.Ly;
    const long long n = (long long)row * g.Lx + x;
    const bool act = n < g.N;
    if (act)
        lattice_node<C, IB, NTL, true, NTS, false, 0, MRT, CHI>(g, lp, fin, fout, F, U, mark, ctl, Arow, n, x, y,
                                                             z, stage, t, T, &mr, ind, &ch);
    __syncthreads();
    if (act) rows_receive<C, NTS>(g, fout, stage, n, x, y, z, t, T);
}

// Ensemble forms: one launch covers every member's lattice; work-group b
// updates block map[b].y of member map[b].x (linear: BS nodes per block;
// rows: floor(blockDim / Lx) whole rows of that member per block).
template <class T>
using gptr = __attribute__((address_space(1))) T*;

// A member's descriptor in registers, its pointers in the global address
// space.
template <class C>
struct MemberView {
    using S = typename C::store_t;
    using R = typename C::real;
    Geom g;
    LatticeParams lp;
    gptr<const S> fin;
    gptr<S> fout;
    gptr<R> F, U;
    gptr<const int> mark;
    gptr<Ctl> ctl;
    gptr<const double> A;
    __device__ MemberView(const LatDesc& D, int cur)
        : g(D.g), lp(D.lp), fin((gptr<const S>)D.f[cur]), fout((gptr<S>)D.f[cur ^ 1]), F((gptr<R>)D.F),
          U((gptr<R>)D.u), mark((gptr<const int>)D.mark), ctl((gptr<Ctl>)D.ctl), A((gptr<const double>)D.A) {}
};

// Waves per SIMD the batched kernel is compiled for: six fit the 16- and
// 32-bit forms in 80 registers without spills; FP64 takes what it needs.
template <class C>
constexpr int batch_waves = 6;
template <>
constexpr int batch_waves<SF64> = 1;

// IB: every member the launch covers carries a droplet, or none does.
template <class C, bool IB, bool NTL, int BS>
__global__ __launch_bounds__(BS, batch_waves<C>) void k_lattice_batch(const LatDesc* __restrict__ desc, const int2* __restrict__ map,
                                                       int cur, long long arow, int xcd) {
    const int2 e = map[xcd ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x];
    const MemberView<C> M(desc[e.x], cur);
    const long long n = (long long)e.y * BS + threadIdx.x;
    if (n >= M.g.N) return;
    int x, y, z;
    node_xyz(M.g, n, x, y, z);
    const gptr<const double> Arow = M.A + arow;
    lattice_node<C, IB, NTL, false, false, true, 0>(M.g, M.lp, M.fin, M.fout, M.F, M.U, M.mark, M.ctl, Arow, n, x, y, z,
                                           nullptr, 0, 0);
}

template <class C, bool IB, bool NTL, bool NTS>
__global__ __launch_bounds__(ROWS_MAX_T) void k_lattice_rows_batch(const LatDesc* __restrict__ desc,
                                                                   const int2* __restrict__ map, int cur,
                                                                   long long arow) {
    using S = typename C::store_t;
    extern __shared__ __align__(16) unsigned char dyn[];
    S* stage = reinterpret_cast<S*>(dyn);
    const int2 e = map[blockIdx.x];
    const MemberView<C> M(desc[e.x], cur);
    const int rows = int(blockDim.x) / M.g.Lx;
    const int T = rows * M.g.Lx;
    const int t = threadIdx.x;
    const int rl = t / M.g.Lx;
    const int x = t - rl * M.g.Lx;
    const int row = e.y * rows + rl;
    const int z = row / M.g.Ly, y = row - z * M.g.Ly;
    const long long n = (long long)row * M.g.Lx + x;
    const bool act = t < T && n < M.g.N;
    const gptr<const double> Arow = M.A + arow;
    if (act)
        lattice_node<C, IB, NTL, true, NTS, true, 0>(M.g, M.lp, M.fin, M.fout, M.F, M.U, M.mark, M.ctl, Arow, n, x, y, z,
                                            stage, t, T);
    __syncthreads();
    if (act) rows_receive<C, NTS>(M.g, M.fout, stage, n, x, y, z, t, T);
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
template <class C>
__global__ __launch_bounds__(256) void k_wet_walls(Geom g, LatticeParams lp, typename C::store_t* __restrict__ f,
                                                   const double* __restrict__ Arow, long long total) {
    using R = typename C::real;
    long long r = (long long)blockIdx.x * 256 + threadIdx.x;
    if (r >= total) return;
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
__device__ void jacobi3(const double S[9], double ev[3], double vec[9]) {
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
    int o[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (a[o[j]][o[j]] > a[o[i]][o[i]]) {
                const int t = o[i];
                o[i] = o[j];
                o[j] = t;
            }
    for (int k = 0; k < 3; ++k) {
        const int col = o[k];
        ev[k] = a[col][col];
        int big = 0;
        for (int i = 1; i < 3; ++i)
            if (fabs(v[i][col]) > fabs(v[big][col])) big = i;
        const double sg = v[big][col] < 0.0 ? -1.0 : 1.0;
        for (int i = 0; i < 3; ++i) vec[3 * k + i] = sg * v[i][col];
    }
}

// Output layout (doubles): 0 volume, 1..3 centroid (relative to x_c),
// 4..12 S, 13..15 eigval, 16..24 eigvec, 25 D, 26 beta, 27 theta_deg,
// 28 flags, 29 sum of deviations, 30..32 momentum, 33 iters, 34 cap hits,
// 35 smallest triangle angle (degrees), 36 shortest edge, 37 longest edge.
__global__ void k_obs_final(int nblocks, const double* part, int mblocks, const double* mpart,
                            const double* Arow, double radius, int has_mesh, Ctl* ctl,
                            double* out) {
    if (threadIdx.x != 0) return;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < mblocks; ++b)
        for (int k = 0; k < 4; ++k) m[k] += mpart[4 * b + k];
    for (int k = 0; k < OBS_OUT_N; ++k) out[k] = 0.0;
    out[29] = m[0];
    out[30] = m[1];
    out[31] = m[2];
    out[32] = m[3];
    out[33] = ctl->iters;
    out[34] = ctl->cap_hits;
    ctl->cap_hits = 0;
    if (!has_mesh) return;
    double s[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double amin = __builtin_inf(), emin = __builtin_inf(), emax = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        for (int k = 0; k < 10; ++k) s[k] += part[16 * b + k];
        amin = fmin(amin, part[16 * b + 10]);
        emin = fmin(emin, part[16 * b + 11]);
        emax = fmax(emax, part[16 * b + 12]);
    }
    out[35] = amin * (180.0 / 3.14159265358979323846);
    out[36] = emin;
    out[37] = emax;
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

static inline unsigned blocks_for(long long n, int bs) { return unsigned((n + bs - 1) / bs); }

#define DISPATCH_STORAGE(storage, C, ...)                  \
    switch (storage) {                                     \
        case IBM_LB_F64: { using C = SF64; __VA_ARGS__; break; }  \
        case IBM_LB_F32: { using C = SF32; __VA_ARGS__; break; }  \
        case IBM_LB_F16DEV: { using C = SF16; __VA_ARGS__; break; } \
        default: { using C = SBF16; __VA_ARGS__; break; }  \
    }

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
template <class C, bool IB, bool NTL, int BS>
static void lattice_launch(const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur, const double* A_row,
                           int xcd, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    using R = typename C::real;
    using S = typename C::store_t;
    hipExtLaunchKernelGGL((k_lattice<C, IB, NTL, BS>), dim3(blocks_for(g.N, BS)), dim3(BS), 0, s, e0, e1, 0, g, lp,
                          (const S*)d.f[cur], (S*)d.f[cur ^ 1], (R*)d.F, (R*)d.u, (const int*)d.mark, d.ctl, A_row,
                          xcd);
}

template <class C, bool IB, bool NTL, int BS>
static void mrt_launch(const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur, const double* A_row,
                       int xcd, const MrtRates& mr, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    using R = typename C::real;
    using S = typename C::store_t;
    hipExtLaunchKernelGGL((k_lattice_mrt<C, IB, NTL, BS>), dim3(blocks_for(g.N, BS)), dim3(BS), 0, s, e0, e1, 0, g,
                          lp, (const S*)d.f[cur], (S*)d.f[cur ^ 1], (R*)d.F, (R*)d.u, (const int*)d.mark, d.ctl,
                          A_row, xcd, mr);
}

template <class C, bool IB, bool NTL>
static void launch_mrt_v(int variant, const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur,
                         const double* A_row, const MrtRates& mr, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int xcd = (variant & VAR_X) ? 1 : 0;
    switch ((variant >> 1) & 3) {
        case 0: mrt_launch<C, IB, NTL, LAT_BS[0]>(g, lp, d, cur, A_row, xcd, mr, s, e0, e1); break;
        case 1: mrt_launch<C, IB, NTL, LAT_BS[1]>(g, lp, d, cur, A_row, xcd, mr, s, e0, e1); break;
        case 2: mrt_launch<C, IB, NTL, LAT_BS[2]>(g, lp, d, cur, A_row, xcd, mr, s, e0, e1); break;
        default: mrt_launch<C, IB, NTL, LAT_BS[3]>(g, lp, d, cur, A_row, xcd, mr, s, e0, e1); break;
    }
}

template <class C, bool IB, bool NTL, int BS>
static void chi_launch(const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur, const double* A_row,
                       int xcd, const ChiRates& ch, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    using R = typename C::real;
    using S = typename C::store_t;
    hipExtLaunchKernelGGL((k_lattice_chi<C, IB, NTL, BS>), dim3(blocks_for(g.N, BS)), dim3(BS), 0, s, e0, e1, 0, g,
                          lp, (const S*)d.f[cur], (S*)d.f[cur ^ 1], (R*)d.F, (R*)d.u, (const int*)d.mark, d.ctl,
                          A_row, xcd, d.ind, ch);
}

template <class C, bool IB, bool NTL>
static void launch_chi_v(int variant, const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur,
                         const double* A_row, const ChiRates& ch, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const int xcd = (variant & VAR_X) ? 1 : 0;
    switch ((variant >> 1) & 3) {
        case 0: chi_launch<C, IB, NTL, LAT_BS[0]>(g, lp, d, cur, A_row, xcd, ch, s, e0, e1); break;
        case 1: chi_launch<C, IB, NTL, LAT_BS[1]>(g, lp, d, cur, A_row, xcd, ch, s, e0, e1); break;
        case 2: chi_launch<C, IB, NTL, LAT_BS[2]>(g, lp, d, cur, A_row, xcd, ch, s, e0, e1); break;
        default: chi_launch<C, IB, NTL, LAT_BS[3]>(g, lp, d, cur, A_row, xcd, ch, s, e0, e1); break;
    }
}

template <class C, bool IB, bool NTL, int BS, bool CHI = false>
static void aa_launch(const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur, const double* A_row, int xcd,
                      int parity, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const ChiRates* ch = nullptr) {
    using R = typename C::real;
    using S = typename C::store_t;
    unsigned char* ind = CHI ? d.ind : nullptr;
    const ChiRates cr = ch ? *ch : ChiRates{};
    if (parity)
        hipExtLaunchKernelGGL((k_lattice_aa<C, IB, NTL, BS, true, CHI>), dim3(blocks_for(g.N, BS)), dim3(BS), 0, s, e0,
                              e1, 0, g, lp, (S*)d.f[cur], (R*)d.F, (R*)d.u, (const int*)d.mark, d.ctl, A_row, xcd,
                              ind, cr);
    else
        hipExtLaunchKernelGGL((k_lattice_aa<C, IB, NTL, BS, false, CHI>), dim3(blocks_for(g.N, BS)), dim3(BS), 0, s,
                              e0, e1, 0, g, lp, (S*)d.f[cur], (R*)d.F, (R*)d.u, (const int*)d.mark, d.ctl, A_row,
                              xcd, ind, cr);
}

hipError_t launch_aa_settle(int storage, const Geom& g, const DevPtrs& d, int cur, hipStream_t s) {
    DISPATCH_STORAGE(storage, C, {
        using S = typename C::store_t;
        hipLaunchKernelGGL(k_aa_settle<C>, dim3(blocks_for(g.N, 256)), dim3(256), 0, s, g, (S*)d.f[cur]);
    });
    return hipGetLastError();
}

template <class C, bool IB, bool NTL, bool NTS, bool CHI = false, bool MRT = false>
static void rows_launch(const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur, const double* A_row,
                        int rows, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const ChiRates* ch = nullptr,
                        const MrtRates* mr = nullptr) {
    using R = typename C::real;
    using S = typename C::store_t;
    const int T = rows * g.Lx;
    const long long nrows = (long long)g.Ly * g.Lz;
    const unsigned nb = unsigned((nrows + rows - 1) / rows);
    hipExtLaunchKernelGGL((k_lattice_rows<C, IB, NTL, NTS, CHI, MRT>), dim3(nb), dim3(T),
                          uint32_t(NXMOVE * T * sizeof(S)), s, e0, e1, 0, g, lp, (const S*)d.f[cur],
                          (S*)d.f[cur ^ 1], (R*)d.F, (R*)d.u, (const int*)d.mark, d.ctl, A_row, rows,
                          CHI ? d.ind : nullptr, ch ? *ch : ChiRates{}, mr ? *mr : MrtRates{});
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

template <class C, bool IB, bool NTL>
static void launch_lattice_v(int variant, const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur,
                             const double* A_row, int parity, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (variant & VAR_AA) {
        const int xcd = (variant & VAR_X) ? 1 : 0;
        switch ((variant >> 1) & 3) {
            case 0: aa_launch<C, IB, NTL, LAT_BS[0]>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1); break;
            case 1: aa_launch<C, IB, NTL, LAT_BS[1]>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1); break;
            case 2: aa_launch<C, IB, NTL, LAT_BS[2]>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1); break;
            default: aa_launch<C, IB, NTL, LAT_BS[3]>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1); break;
        }
        return;
    }
    if (variant & VAR_ROWS) {
        const int rows = lattice_rows_per_block(variant, g.Lx);
        if (variant & VAR_X) rows_launch<C, IB, NTL, true>(g, lp, d, cur, A_row, rows, s, e0, e1);
        else rows_launch<C, IB, NTL, false>(g, lp, d, cur, A_row, rows, s, e0, e1);
        return;
    }
    const int xcd = (variant & VAR_X) ? 1 : 0;
    switch ((variant >> 1) & 3) {
        case 0: lattice_launch<C, IB, NTL, LAT_BS[0]>(g, lp, d, cur, A_row, xcd, s, e0, e1); break;
        case 1: lattice_launch<C, IB, NTL, LAT_BS[1]>(g, lp, d, cur, A_row, xcd, s, e0, e1); break;
        case 2: lattice_launch<C, IB, NTL, LAT_BS[2]>(g, lp, d, cur, A_row, xcd, s, e0, e1); break;
        default: lattice_launch<C, IB, NTL, LAT_BS[3]>(g, lp, d, cur, A_row, xcd, s, e0, e1); break;
    }
}

hipError_t launch_lattice(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d,
                          int cur, bool ib, const double* A_row, int variant, int parity, hipStream_t s,
                          hipEvent_t e0, hipEvent_t e1, const MrtRates* mrt, const ChiRates* chi) {
    if (!lattice_variant_ok(variant, g)) return hipErrorInvalidValue;
    if (mrt && chi) return hipErrorInvalidValue;
    if (chi) {
        // the indicator exists only with a droplet
        if (!ib || !d.ind) return hipErrorInvalidValue;
        if (variant & VAR_AA) {
            const int xcd = (variant & VAR_X) ? 1 : 0;
#define CHI_AA(NTLV)                                                                                               \
    do {                                                                                                           \
        switch ((variant >> 1) & 3) {                                                                              \
            case 0: aa_launch<C, true, NTLV, LAT_BS[0], true>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1, chi); break; \
            case 1: aa_launch<C, true, NTLV, LAT_BS[1], true>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1, chi); break; \
            case 2: aa_launch<C, true, NTLV, LAT_BS[2], true>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1, chi); break; \
            default: aa_launch<C, true, NTLV, LAT_BS[3], true>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1, chi); break; \
        }                                                                                                          \
    } while (0)
            DISPATCH_STORAGE(storage, C, {
                if (variant & 1) CHI_AA(true);
                else CHI_AA(false);
            });
#undef CHI_AA
            return hipGetLastError();
        }
        if (variant & VAR_ROWS) {
            const int rows = lattice_rows_per_block(variant, g.Lx);
            const bool nts = (variant & VAR_X) != 0;
            DISPATCH_STORAGE(storage, C, {
                if (variant & 1) {
                    if (nts) rows_launch<C, true, true, true, true>(g, lp, d, cur, A_row, rows, s, e0, e1, chi);
                    else rows_launch<C, true, true, false, true>(g, lp, d, cur, A_row, rows, s, e0, e1, chi);
                } else {
                    if (nts) rows_launch<C, true, false, true, true>(g, lp, d, cur, A_row, rows, s, e0, e1, chi);
                    else rows_launch<C, true, false, false, true>(g, lp, d, cur, A_row, rows, s, e0, e1, chi);
                }
            });
            return hipGetLastError();
        }
        DISPATCH_STORAGE(storage, C, {
            if (variant & 1) launch_chi_v<C, true, true>(variant, g, lp, d, cur, A_row, *chi, s, e0, e1);
            else launch_chi_v<C, true, false>(variant, g, lp, d, cur, A_row, *chi, s, e0, e1);
        });
        return hipGetLastError();
    }
    if (mrt) {
        if (variant & VAR_AA) return hipErrorInvalidValue;
        if (variant & VAR_ROWS) {
            const int rows = lattice_rows_per_block(variant, g.Lx);
            const bool nts = (variant & VAR_X) != 0;
#define MRT_ROWS(IBV, NTLV)                                                                                   \
    do {                                                                                                      \
        if (nts) rows_launch<C, IBV, NTLV, true, false, true>(g, lp, d, cur, A_row, rows, s, e0, e1, nullptr, mrt); \
        else rows_launch<C, IBV, NTLV, false, false, true>(g, lp, d, cur, A_row, rows, s, e0, e1, nullptr, mrt);  \
    } while (0)
            DISPATCH_STORAGE(storage, C, {
                if (ib) {
                    if (variant & 1) MRT_ROWS(true, true);
                    else MRT_ROWS(true, false);
                } else {
                    if (variant & 1) MRT_ROWS(false, true);
                    else MRT_ROWS(false, false);
                }
            });
#undef MRT_ROWS
            return hipGetLastError();
        }
        DISPATCH_STORAGE(storage, C, {
            if (ib) {
                if (variant & 1) launch_mrt_v<C, true, true>(variant, g, lp, d, cur, A_row, *mrt, s, e0, e1);
                else launch_mrt_v<C, true, false>(variant, g, lp, d, cur, A_row, *mrt, s, e0, e1);
            } else {
                if (variant & 1) launch_mrt_v<C, false, true>(variant, g, lp, d, cur, A_row, *mrt, s, e0, e1);
                else launch_mrt_v<C, false, false>(variant, g, lp, d, cur, A_row, *mrt, s, e0, e1);
            }
        });
        return hipGetLastError();
    }
    DISPATCH_STORAGE(storage, C, {
        if (ib) {
            if (variant & 1) launch_lattice_v<C, true, true>(variant, g, lp, d, cur, A_row, parity, s, e0, e1);
            else launch_lattice_v<C, true, false>(variant, g, lp, d, cur, A_row, parity, s, e0, e1);
        } else {
            if (variant & 1) launch_lattice_v<C, false, true>(variant, g, lp, d, cur, A_row, parity, s, e0, e1);
            else launch_lattice_v<C, false, false>(variant, g, lp, d, cur, A_row, parity, s, e0, e1);
        }
    });
    return hipGetLastError();
}

template <class C, bool IB, bool NTL>
static void launch_batch_v(int bsi, const LatDesc* desc, const int2* map, int nblocks, int cur, long long step,
                           int xcd, hipStream_t s) {
    if (nblocks <= 0) return;
    switch (bsi) {
        case 0:
            hipLaunchKernelGGL((k_lattice_batch<C, IB, NTL, LAT_BS[0]>), dim3(nblocks), dim3(LAT_BS[0]), 0, s, desc,
                               map, cur, step, xcd);
            break;
        case 1:
            hipLaunchKernelGGL((k_lattice_batch<C, IB, NTL, LAT_BS[1]>), dim3(nblocks), dim3(LAT_BS[1]), 0, s, desc,
                               map, cur, step, xcd);
            break;
        case 2:
            hipLaunchKernelGGL((k_lattice_batch<C, IB, NTL, LAT_BS[2]>), dim3(nblocks), dim3(LAT_BS[2]), 0, s, desc,
                               map, cur, step, xcd);
            break;
        default:
            hipLaunchKernelGGL((k_lattice_batch<C, IB, NTL, LAT_BS[3]>), dim3(nblocks), dim3(LAT_BS[3]), 0, s, desc,
                               map, cur, step, xcd);
            break;
    }
}

template <class C, bool IB, bool NTL, bool NTS>
static void launch_rows_batch(int T, const LatDesc* desc, const int2* map, int nblocks, int cur, long long step,
                              hipStream_t s) {
    if (nblocks <= 0) return;
    using S = typename C::store_t;
    hipLaunchKernelGGL((k_lattice_rows_batch<C, IB, NTL, NTS>), dim3(nblocks), dim3(T),
                       size_t(NXMOVE) * T * sizeof(S), s, desc, map, cur, step);
}

template <class C, bool NTL, bool NTS>
static void launch_rows_both(int T, const LatDesc* desc, const int2* map, int nblocks, int nib, int cur,
                             long long step, hipStream_t s) {
    launch_rows_batch<C, true, NTL, NTS>(T, desc, map, nib, cur, step, s);
    launch_rows_batch<C, false, NTL, NTS>(T, desc, map + nib, nblocks - nib, cur, step, s);
}

template <class C, bool NTL>
static void launch_batch_both(int bsi, const LatDesc* desc, const int2* map, int nblocks, int nib, int cur,
                              long long step, int xcd, hipStream_t s) {
    launch_batch_v<C, true, NTL>(bsi, desc, map, nib, cur, step, xcd, s);
    launch_batch_v<C, false, NTL>(bsi, desc, map + nib, nblocks - nib, cur, step, xcd, s);
}

hipError_t launch_lattice_batch(int storage, const LatDesc* desc, const int2* maps, const int moff[8],
                                const int nblocks[8], const int nib[8], int cur, long long step, int variant,
                                hipStream_t s) {
    if (variant < 0 || variant >= STEP_VARIANTS) return hipErrorInvalidValue;
    const int bsi = (variant >> 1) & 3;
    const int xb = variant & VAR_X ? 1 : 0;
    if (variant & VAR_ROWS) {
        const int q = 4 + bsi;
        if (nblocks[q] <= 0) return hipErrorInvalidValue;
        const int T = LAT_BS[bsi];
        DISPATCH_STORAGE(storage, C, {
            if (variant & 1) {
                if (xb) launch_rows_both<C, true, true>(T, desc, maps + moff[q], nblocks[q], nib[q], cur, step, s);
                else launch_rows_both<C, true, false>(T, desc, maps + moff[q], nblocks[q], nib[q], cur, step, s);
            } else {
                if (xb) launch_rows_both<C, false, true>(T, desc, maps + moff[q], nblocks[q], nib[q], cur, step, s);
                else launch_rows_both<C, false, false>(T, desc, maps + moff[q], nblocks[q], nib[q], cur, step, s);
            }
        });
        return hipGetLastError();
    }
    DISPATCH_STORAGE(storage, C, {
        if (variant & 1)
            launch_batch_both<C, true>(bsi, desc, maps + moff[bsi], nblocks[bsi], nib[bsi], cur, step, xb, s);
        else
            launch_batch_both<C, false>(bsi, desc, maps + moff[bsi], nblocks[bsi], nib[bsi], cur, step, xb, s);
    });
    return hipGetLastError();
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

hipError_t launch_wet_walls(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur,
                            const double* A_row, hipStream_t s) {
    long long total = 0;
    if (!g.px) total += 2ll * g.Ly * g.Lz;
    if (!g.py) total += 2ll * g.Lx * g.Lz;
    if (!g.pz) total += 2ll * g.Lx * g.Ly;
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
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(64), 0, s, OBS_BLOCKS, d.obs_part, MASS_BLOCKS,
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
