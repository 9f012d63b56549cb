// Fused lattice kernels (the collide-stream step of Sec. 3.1 in every
// layout and collision) and their launchers, per population storage type C.
// Included by the per-storage translation units lattice_f64.hip,
// lattice_f32.hip, lattice_f16.hip and lattice_bf16.hip, which instantiate
// launch_lattice_c<C> and launch_lattice_batch_c<C>, and by kernels.hip for
// the shared device helpers.
#pragma once

#include <hip/hip_ext.h>
#include <math.h>

#include "lattice_common.h"

namespace ibmlb {

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
        // Moment k of the non-equilibrium part and of the Guo term. The
        // equilibrium deviation w_i (drho - 1.5 rho u.u + 3 rho c_i.u + 4.5 rho
        // (c_i.u)^2) and the Guo term w_i (3 c_i.F - 3 u.F + 9 (c_i.u)(c_i.F))
        // are quadratic in c_i, so their moments come from the basis rows'
        // weighted moments (compile-time integers, most of them zero); only
        // the populations' moments sum over i. The basis is orthogonal, so
        // the updates of the other moments leave sum_i m_ki d_i unchanged and
        // d can be updated moment by moment.
        const R uv[3] = {ux, uy, uz}, Fv[3] = {Fx, Fy, Fz};
        const R e0 = drho - R(1.5) * rho * usq;
        static_for<0, Q>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            R md = R(0);
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int m = mrt_m(k, i);
                if constexpr (m != 0) md += R(m) * d[i];
            });
            R meq = R(0), mg = R(0);
            if constexpr (mrt_w0(k) != 0) {
                meq += R(mrt_w0(k)) * e0;
                mg -= R(3 * mrt_w0(k)) * uF;
            }
            static_for<0, 3>([&](auto ac) {
                constexpr int a = decltype(ac)::value;
                if constexpr (mrt_w1(k, a) != 0) {
                    meq += R(3 * mrt_w1(k, a)) * rho * uv[a];
                    mg += R(3 * mrt_w1(k, a)) * Fv[a];
                }
                static_for<0, 3>([&](auto bc) {
                    constexpr int b = decltype(bc)::value;
                    if constexpr (mrt_w2(k, a, b) != 0) {
                        meq += R(4.5) * R(mrt_w2(k, a, b)) * rho * uv[a] * uv[b];
                        mg += R(9 * mrt_w2(k, a, b)) * uv[a] * Fv[b];
                    }
                });
            });
            const R mn = md - meq * R(1.0 / 36.0);
            const R sk = R(mr->s[k]);
            const R r = (sk * mn - (R(1) - R(0.5) * sk) * (mg * R(1.0 / 36.0))) * (R(1) / R(mrt_norm2(k)));
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
// CHI: the viscosity ratio's inner rates on the nodes the indicator marks;
// MRT: the multiple-relaxation-time collision with the rates mr.
template <class C, bool IB, bool NTL, int BS, bool ODD, bool CHI = false, bool MRT = false>
__global__ __launch_bounds__(BS) void k_lattice_aa(Geom g, LatticeParams lp, typename C::store_t* f,
                                                    typename C::real* __restrict__ F,
                                                    typename C::real* __restrict__ U,
                                                    const int* __restrict__ mark, Ctl* ctl,
                                                    const double* __restrict__ Arow, int xcd,
                                                    unsigned char* __restrict__ ind = nullptr,
                                                    ChiRates ch = ChiRates{}, MrtRates mr = MrtRates{}) {
    const unsigned b = xcd ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
    const long long n = (long long)b * BS + threadIdx.x;
    if (n >= g.N) return;
    int x, y, z;
    node_xyz(g, n, x, y, z);
    lattice_node<C, IB, NTL, false, false, false, ODD ? 2 : 1, MRT, CHI>(
        g, lp, (const typename C::store_t*)f, f, F, U, mark, ctl, Arow, n, x, y, z, nullptr, 0, 0, &mr, ind, &ch);
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
    gptr<const double> mrt;
    __device__ MemberView(const LatDesc& D, int cur)
        : g(D.g), lp(D.lp), fin((gptr<const S>)D.f[cur]), fout((gptr<S>)D.f[cur ^ 1]), F((gptr<R>)D.F),
          U((gptr<R>)D.u), mark((gptr<const int>)D.mark), ctl((gptr<Ctl>)D.ctl), A((gptr<const double>)D.A),
          mrt((gptr<const double>)D.mrt) {}
    // the member's MRT rates, read into registers (uniform: scalar loads)
    __device__ MrtRates rates() const {
        MrtRates r;
#pragma unroll
        for (int k = 0; k < Q; ++k) r.s[k] = mrt[k];
        return r;
    }
};

// Waves per SIMD the batched kernel is compiled for: six fit the 16- and
// 32-bit forms in 80 registers without spills; FP64 takes what it needs.
template <class C>
inline constexpr int batch_waves = 6;
template <>
inline constexpr int batch_waves<SF64> = 1;

// IB: every member the launch covers carries a droplet, or none does.
// MRT: every member runs the MRT collision (with its own rates), or none does.
template <class C, bool IB, bool NTL, int BS, bool MRT = false>
__global__ __launch_bounds__(BS, batch_waves<C>) void k_lattice_batch(const LatDesc* __restrict__ desc, const int2* __restrict__ map,
                                                       int cur, long long arow, int xcd) {
    const int2 e = map[xcd ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x];
    const MemberView<C> M(desc[e.x], cur);
    const long long n = (long long)e.y * BS + threadIdx.x;
    if (n >= M.g.N) return;
    int x, y, z;
    node_xyz(M.g, n, x, y, z);
    const gptr<const double> Arow = M.A + arow;
    MrtRates mr;
    if constexpr (MRT) mr = M.rates();
    lattice_node<C, IB, NTL, false, false, true, 0, MRT>(M.g, M.lp, M.fin, M.fout, M.F, M.U, M.mark, M.ctl, Arow, n, x,
                                                     y, z, nullptr, 0, 0, &mr);
}

template <class C, bool IB, bool NTL, bool NTS, bool MRT = false>
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
    MrtRates mr;
    if constexpr (MRT) mr = M.rates();
    if (act)
        lattice_node<C, IB, NTL, true, NTS, true, 0, MRT>(M.g, M.lp, M.fin, M.fout, M.F, M.U, M.mark, M.ctl, Arow, n, x,
                                                      y, z, stage, t, T, &mr);
    __syncthreads();
    if (act) rows_receive<C, NTS>(M.g, M.fout, stage, n, x, y, z, t, T);
}

// ---------------------------------------------------------------- launchers
static inline unsigned blocks_for(long long n, int bs) { return unsigned((n + bs - 1) / bs); }

#define DISPATCH_STORAGE(storage, C, ...)                  \
    switch (storage) {                                     \
        case IBM_LB_F64: { using C = SF64; __VA_ARGS__; break; }  \
        case IBM_LB_F32: { using C = SF32; __VA_ARGS__; break; }  \
        case IBM_LB_F16DEV: { using C = SF16; __VA_ARGS__; break; } \
        default: { using C = SBF16; __VA_ARGS__; break; }  \
    }

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

template <class C, bool IB, bool NTL, int BS, bool CHI = false, bool MRT = false>
static void aa_launch(const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur, const double* A_row, int xcd,
                      int parity, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const ChiRates* ch = nullptr,
                      const MrtRates* mr = nullptr) {
    using R = typename C::real;
    using S = typename C::store_t;
    unsigned char* ind = CHI ? d.ind : nullptr;
    const ChiRates cr = ch ? *ch : ChiRates{};
    const MrtRates mrr = mr ? *mr : MrtRates{};
    if (parity)
        hipExtLaunchKernelGGL((k_lattice_aa<C, IB, NTL, BS, true, CHI, MRT>), dim3(blocks_for(g.N, BS)), dim3(BS), 0,
                              s, e0, e1, 0, g, lp, (S*)d.f[cur], (R*)d.F, (R*)d.u, (const int*)d.mark, d.ctl, A_row,
                              xcd, ind, cr, mrr);
    else
        hipExtLaunchKernelGGL((k_lattice_aa<C, IB, NTL, BS, false, CHI, MRT>), dim3(blocks_for(g.N, BS)), dim3(BS), 0,
                              s, e0, e1, 0, g, lp, (S*)d.f[cur], (R*)d.F, (R*)d.u, (const int*)d.mark, d.ctl, A_row,
                              xcd, ind, cr, mrr);
}

// MRT, in place (one copy), linear layout.
template <class C, bool IB, bool NTL>
static void launch_mrt_aa(int variant, const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur,
                          const double* A_row, int parity, const MrtRates* mr, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1) {
    const int xcd = (variant & VAR_X) ? 1 : 0;
    switch ((variant >> 1) & 3) {
        case 0: aa_launch<C, IB, NTL, LAT_BS[0], false, true>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1, nullptr, mr); break;
        case 1: aa_launch<C, IB, NTL, LAT_BS[1], false, true>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1, nullptr, mr); break;
        case 2: aa_launch<C, IB, NTL, LAT_BS[2], false, true>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1, nullptr, mr); break;
        default: aa_launch<C, IB, NTL, LAT_BS[3], false, true>(g, lp, d, cur, A_row, xcd, parity, s, e0, e1, nullptr, mr); break;
    }
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

template <class C>
hipError_t launch_lattice_c(const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur, bool ib,
                            const double* A_row, int variant, int parity, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1, const MrtRates* mrt, const ChiRates* chi) {
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
            {
                if (variant & 1) CHI_AA(true);
                else CHI_AA(false);
            }
#undef CHI_AA
            return hipGetLastError();
        }
        if (variant & VAR_ROWS) {
            const int rows = lattice_rows_per_block(variant, g.Lx);
            const bool nts = (variant & VAR_X) != 0;
            {
                if (variant & 1) {
                    if (nts) rows_launch<C, true, true, true, true>(g, lp, d, cur, A_row, rows, s, e0, e1, chi);
                    else rows_launch<C, true, true, false, true>(g, lp, d, cur, A_row, rows, s, e0, e1, chi);
                } else {
                    if (nts) rows_launch<C, true, false, true, true>(g, lp, d, cur, A_row, rows, s, e0, e1, chi);
                    else rows_launch<C, true, false, false, true>(g, lp, d, cur, A_row, rows, s, e0, e1, chi);
                }
            }
            return hipGetLastError();
        }
        {
            if (variant & 1) launch_chi_v<C, true, true>(variant, g, lp, d, cur, A_row, *chi, s, e0, e1);
            else launch_chi_v<C, true, false>(variant, g, lp, d, cur, A_row, *chi, s, e0, e1);
        }
        return hipGetLastError();
    }
    if (mrt) {
        if (variant & VAR_AA) {
            if (ib) {
                if (variant & 1) launch_mrt_aa<C, true, true>(variant, g, lp, d, cur, A_row, parity, mrt, s, e0, e1);
                else launch_mrt_aa<C, true, false>(variant, g, lp, d, cur, A_row, parity, mrt, s, e0, e1);
            } else {
                if (variant & 1) launch_mrt_aa<C, false, true>(variant, g, lp, d, cur, A_row, parity, mrt, s, e0, e1);
                else launch_mrt_aa<C, false, false>(variant, g, lp, d, cur, A_row, parity, mrt, s, e0, e1);
            }
            return hipGetLastError();
        }
        if (variant & VAR_ROWS) {
            const int rows = lattice_rows_per_block(variant, g.Lx);
            const bool nts = (variant & VAR_X) != 0;
#define MRT_ROWS(IBV, NTLV)                                                                                   \
    do {                                                                                                      \
        if (nts) rows_launch<C, IBV, NTLV, true, false, true>(g, lp, d, cur, A_row, rows, s, e0, e1, nullptr, mrt); \
        else rows_launch<C, IBV, NTLV, false, false, true>(g, lp, d, cur, A_row, rows, s, e0, e1, nullptr, mrt);  \
    } while (0)
            {
                if (ib) {
                    if (variant & 1) MRT_ROWS(true, true);
                    else MRT_ROWS(true, false);
                } else {
                    if (variant & 1) MRT_ROWS(false, true);
                    else MRT_ROWS(false, false);
                }
            }
#undef MRT_ROWS
            return hipGetLastError();
        }
        {
            if (ib) {
                if (variant & 1) launch_mrt_v<C, true, true>(variant, g, lp, d, cur, A_row, *mrt, s, e0, e1);
                else launch_mrt_v<C, true, false>(variant, g, lp, d, cur, A_row, *mrt, s, e0, e1);
            } else {
                if (variant & 1) launch_mrt_v<C, false, true>(variant, g, lp, d, cur, A_row, *mrt, s, e0, e1);
                else launch_mrt_v<C, false, false>(variant, g, lp, d, cur, A_row, *mrt, s, e0, e1);
            }
        }
        return hipGetLastError();
    }
    {
        if (ib) {
            if (variant & 1) launch_lattice_v<C, true, true>(variant, g, lp, d, cur, A_row, parity, s, e0, e1);
            else launch_lattice_v<C, true, false>(variant, g, lp, d, cur, A_row, parity, s, e0, e1);
        } else {
            if (variant & 1) launch_lattice_v<C, false, true>(variant, g, lp, d, cur, A_row, parity, s, e0, e1);
            else launch_lattice_v<C, false, false>(variant, g, lp, d, cur, A_row, parity, s, e0, e1);
        }
    }
    return hipGetLastError();
}


template <class C, bool IB, bool NTL, bool MRT>
static void launch_batch_v(int bsi, const LatDesc* desc, const int2* map, int nblocks, int cur, long long step,
                           int xcd, hipStream_t s) {
    if (nblocks <= 0) return;
    switch (bsi) {
        case 0:
            hipLaunchKernelGGL((k_lattice_batch<C, IB, NTL, LAT_BS[0], MRT>), dim3(nblocks), dim3(LAT_BS[0]), 0, s,
                               desc, map, cur, step, xcd);
            break;
        case 1:
            hipLaunchKernelGGL((k_lattice_batch<C, IB, NTL, LAT_BS[1], MRT>), dim3(nblocks), dim3(LAT_BS[1]), 0, s,
                               desc, map, cur, step, xcd);
            break;
        case 2:
            hipLaunchKernelGGL((k_lattice_batch<C, IB, NTL, LAT_BS[2], MRT>), dim3(nblocks), dim3(LAT_BS[2]), 0, s,
                               desc, map, cur, step, xcd);
            break;
        default:
            hipLaunchKernelGGL((k_lattice_batch<C, IB, NTL, LAT_BS[3], MRT>), dim3(nblocks), dim3(LAT_BS[3]), 0, s,
                               desc, map, cur, step, xcd);
            break;
    }
}

template <class C, bool IB, bool NTL, bool NTS, bool MRT>
static void launch_rows_batch(int T, const LatDesc* desc, const int2* map, int nblocks, int cur, long long step,
                              hipStream_t s) {
    if (nblocks <= 0) return;
    using S = typename C::store_t;
    hipLaunchKernelGGL((k_lattice_rows_batch<C, IB, NTL, NTS, MRT>), dim3(nblocks), dim3(T),
                       size_t(NXMOVE) * T * sizeof(S), s, desc, map, cur, step);
}

template <class C, bool NTL, bool NTS, bool MRT>
static void launch_rows_both(int T, const LatDesc* desc, const int2* map, int nblocks, int nib, int cur,
                             long long step, hipStream_t s) {
    launch_rows_batch<C, true, NTL, NTS, MRT>(T, desc, map, nib, cur, step, s);
    launch_rows_batch<C, false, NTL, NTS, MRT>(T, desc, map + nib, nblocks - nib, cur, step, s);
}

template <class C, bool NTL, bool MRT>
static void launch_batch_both(int bsi, const LatDesc* desc, const int2* map, int nblocks, int nib, int cur,
                              long long step, int xcd, hipStream_t s) {
    launch_batch_v<C, true, NTL, MRT>(bsi, desc, map, nib, cur, step, xcd, s);
    launch_batch_v<C, false, NTL, MRT>(bsi, desc, map + nib, nblocks - nib, cur, step, xcd, s);
}

template <class C, bool MRT>
static hipError_t launch_batch_c(const LatDesc* desc, const int2* maps, const int moff[8], const int nblocks[8],
                                 const int nib[8], int cur, long long step, int variant, hipStream_t s) {
    const int bsi = (variant >> 1) & 3;
    const int xb = variant & VAR_X ? 1 : 0;
    if (variant & VAR_ROWS) {
        const int q = 4 + bsi;
        if (nblocks[q] <= 0) return hipErrorInvalidValue;
        const int T = LAT_BS[bsi];
        if (variant & 1) {
            if (xb) launch_rows_both<C, true, true, MRT>(T, desc, maps + moff[q], nblocks[q], nib[q], cur, step, s);
            else launch_rows_both<C, true, false, MRT>(T, desc, maps + moff[q], nblocks[q], nib[q], cur, step, s);
        } else {
            if (xb) launch_rows_both<C, false, true, MRT>(T, desc, maps + moff[q], nblocks[q], nib[q], cur, step, s);
            else launch_rows_both<C, false, false, MRT>(T, desc, maps + moff[q], nblocks[q], nib[q], cur, step, s);
        }
        return hipGetLastError();
    }
    if (variant & 1)
        launch_batch_both<C, true, MRT>(bsi, desc, maps + moff[bsi], nblocks[bsi], nib[bsi], cur, step, xb, s);
    else
        launch_batch_both<C, false, MRT>(bsi, desc, maps + moff[bsi], nblocks[bsi], nib[bsi], cur, step, xb, s);
    return hipGetLastError();
}

template <class C>
hipError_t launch_lattice_batch_c(const LatDesc* desc, const int2* maps, const int moff[8],
                                  const int nblocks[8], const int nib[8], int cur, long long step, int variant,
                                  bool mrt, hipStream_t s) {
    if (mrt) return launch_batch_c<C, true>(desc, maps, moff, nblocks, nib, cur, step, variant, s);
    return launch_batch_c<C, false>(desc, maps, moff, nblocks, nib, cur, step, variant, s);
}


}  // namespace ibmlb
