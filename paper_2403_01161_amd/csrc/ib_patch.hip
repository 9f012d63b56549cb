// Immersed-boundary half of the timestep, organised by surface patches.
//
// At set-up the vertices are renumbered by recursive bisection of their
// positions so that every run of PATCH (64) consecutive vertices is a compact
// patch of the droplet surface; one work-group (one wave) owns one patch and
// one lane one vertex. Small patches put the LDS work of the IB kernels on
// many compute units (a 10k-vertex droplet gives 161 work-groups). The
// lattice window covered by a patch's 4x4x4 stencils is staged in LDS:
//   * spreading (Sec. 3.1, Eq. ibm_force_d, first line): each of the four
//     waves takes every fourth vertex, one lane per stencil node, and adds its
//     64 contributions into an FP64 LDS window with LDS atomics (distinct
//     addresses within each instruction); the window is flushed to F with one
//     global atomic per touched node;
//   * interpolation (Eq. ibm_force_d, second line): the window of u is loaded
//     once and each vertex gathers its 64 nodes from LDS.
// A window beyond the LDS capacity falls back to direct global access.
//
// Topology is the ordered one-ring ("fan") of each vertex: valence m and
// neighbours n_0 .. n_{m-1} counter-clockwise, so (k, n_j, n_{j+1}) are the
// triangles around k. Forces and smoothing need two dependent loads per
// vertex: the fan, then the neighbour positions.
//
// Kernels of one step, after the fused lattice kernel:
//   k_interp_patch  interpolation + Euler move (Eq. fwd_euler): o = r + U
//   k_hc_fused      HC iteration 1 per patch (its halo's p' and b staged in
//                   LDS), grid-wide max |p - q|; the last work-group to finish
//                   runs the rare further iterations, records the count and
//                   advances the step epoch
//   k_fs_patch      next step's surface-tension forces (Eq. pi_drop), tile
//                   marks and spreading; with a viscosity ratio its idle
//                   waves also cross the patch's triangles with the lattice
//                   x-rows (first half of the inside indicator); the
//                   marks and spreading, from the final positions
#include <hip/hip_ext.h>

#include "device_common.h"
#include "indicator_common.h"

namespace ibmlb {

constexpr int PATCH = IB_PATCH;
constexpr int IBT = 256;  // threads of a patch work-group: lanes of the first wave own the vertices

// Pointer of address space AS: 0 = generic (kernel arguments, which the
// compiler proves global), 1 = global (records read from memory, whose
// pointers the compiler would otherwise access with flat instructions).
template <class T, int AS>
struct PtrT {
    using type = T*;
};
template <class T>
struct PtrT<T, 1> {
    using type = __attribute__((address_space(1))) T*;
};
template <class T, int AS>
using Ptr = typename PtrT<T, AS>::type;

// Deterministic spreading: the staged stencil of a vertex, written by the
// force kernel for the gather that follows it.
template <class R>
struct DetRec {
    int fw[3];  // first stencil node, wrapped into the box
    int ok;     // 0: no valid stencil (the error flag is raised)
    R w[3][4];  // Peskin weights per axis
    R val[3];   // force
};

template <class R, int AS = 0>
struct IbArgs {
    Geom g;
    int nv;
    R sigma;
    SmoothParams sp;
    Ptr<V4<R>, AS> r;      // positions at the start of the step (relative to x_c)
    Ptr<V4<R>, AS> o;      // after the Euler move
    Ptr<V4<R>, AS> qa;     // smoothing iterates; qa holds the final positions
    Ptr<V4<R>, AS> qb;
    Ptr<V4<R>, AS> pp;
    Ptr<V4<R>, AS> bb;
    Ptr<const int4, AS> fan;     // [nv][4]
    Ptr<const int4, AS> lfan;    // [nv][4] fan in patch-local slots
    Ptr<const int, AS> hstart;   // [npatch + 1]
    Ptr<const int, AS> hids;     // halo vertices of each patch
    Ptr<R, AS> F;                // [3][N]
    Ptr<const R, AS> U;          // [3][N]
    Ptr<int, AS> mark;
    Ptr<Ctl, AS> ctl;
    Ptr<unsigned long long, AS> red;  // grid-wide max of |p - q| (bit pattern of a non-negative real)
    Ptr<DetRec<R>, AS> det;      // [nv] staged stencils for the deterministic spreading, or null
    Ptr<int, AS> pbox;           // [npatch][8] window of each patch (origin, extent), with det
    int wcap;                    // LDS window capacity in nodes
};

// A record read from memory, with its pointers in the global space.
template <class R>
__device__ inline IbArgs<R, 1> to_global(const IbArgs<R, 0>& a) {
    IbArgs<R, 1> b;
    b.g = a.g;
    b.nv = a.nv;
    b.sigma = a.sigma;
    b.sp = a.sp;
    b.r = (Ptr<V4<R>, 1>)a.r;
    b.o = (Ptr<V4<R>, 1>)a.o;
    b.qa = (Ptr<V4<R>, 1>)a.qa;
    b.qb = (Ptr<V4<R>, 1>)a.qb;
    b.pp = (Ptr<V4<R>, 1>)a.pp;
    b.bb = (Ptr<V4<R>, 1>)a.bb;
    b.fan = (Ptr<const int4, 1>)a.fan;
    b.lfan = (Ptr<const int4, 1>)a.lfan;
    b.hstart = (Ptr<const int, 1>)a.hstart;
    b.hids = (Ptr<const int, 1>)a.hids;
    b.F = (Ptr<R, 1>)a.F;
    b.U = (Ptr<const R, 1>)a.U;
    b.mark = (Ptr<int, 1>)a.mark;
    b.ctl = (Ptr<Ctl, 1>)a.ctl;
    b.red = (Ptr<unsigned long long, 1>)a.red;
    b.det = (Ptr<DetRec<R>, 1>)a.det;
    b.pbox = (Ptr<int, 1>)a.pbox;
    b.wcap = a.wcap;
    return b;
}

// Relaxed device-scope atomics on generic or global pointers (no return).
template <class T>
__device__ inline void atom_add(T* p, T v) { unsafeAtomicAdd(p, v); }
template <class T>
__device__ inline void atom_add(__attribute__((address_space(1))) T* p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void atom_or(int* p, int v) { atomicOr(p, v); }
__device__ inline void atom_or(__attribute__((address_space(1))) int* p, int v) {
    __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long atom_inc(unsigned long long* p) { return atomicAdd(p, 1ull); }
__device__ inline unsigned long long atom_inc(__attribute__((address_space(1))) unsigned long long* p) {
    return __hip_atomic_fetch_add(p, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void atom_max(unsigned long long* p, unsigned long long v) { atomicMax(p, v); }
__device__ inline void atom_max(__attribute__((address_space(1))) unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- forces
// Surface-tension force of vertex k at positions P: Eq. (pi_drop) read as
// phi_k = -sigma dA/dr_k, with dA/dr_k = n_t x (r_{n_{j+1}} - r_{n_j}) / 2
// for the triangle t = (k, n_j, n_{j+1}) of unit normal n_t.
// Positions in P of the m fan neighbours nb of a vertex.
template <class R, int AS>
__device__ inline void fan_positions(Ptr<const V4<R>, AS> P, int m, const int nb[MAXV], V4<R> pn[MAXV]) {
#pragma unroll
    for (int j = 0; j < MAXV; ++j)
        if (j < m) pn[j] = ld4<V4<R>>(P + nb[j]);
}

template <class R, int AS>
__device__ inline void force_sum(const IbArgs<R, AS>& a, int m, const V4<R> pn[MAXV], const V4<R>& pk, R& fx, R& fy,
                                 R& fz) {
    fx = fy = fz = R(0);
#pragma unroll
    for (int j = 0; j < MAXV; ++j) {
        if (j < m) {
            const V4<R> pa = pn[j];
            const V4<R> pb = (j + 1 < MAXV && j + 1 < m) ? pn[j + 1 < MAXV ? j + 1 : 0] : pn[0];
            const R ax = pa.x - pk.x, ay = pa.y - pk.y, az = pa.z - pk.z;
            const R bx = pb.x - pk.x, by = pb.y - pk.y, bz = pb.z - pk.z;
            R nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
            const R len = sqrt(nx * nx + ny * ny + nz * nz);
            if (len > R(0)) {
                nx /= len; ny /= len; nz /= len;
                const R dx = pb.x - pa.x, dy = pb.y - pa.y, dz = pb.z - pa.z;
                fx -= a.sigma * R(0.5) * (ny * dz - nz * dy);
                fy -= a.sigma * R(0.5) * (nz * dx - nx * dz);
                fz -= a.sigma * R(0.5) * (nx * dy - ny * dx);
            }
        }
    }
}

// Surface-tension force of vertex k at positions P: Eq. (pi_drop) read as
// phi_k = -sigma dA/dr_k, with dA/dr_k = n_t x (r_{n_{j+1}} - r_{n_j}) / 2
// for the triangle t = (k, n_j, n_{j+1}) of unit normal n_t.
template <class R, int AS>
__device__ inline void force_of(const IbArgs<R, AS>& a, Ptr<const V4<R>, AS> P, int k, const V4<R>& pk, R& fx,
                                R& fy, R& fz) {
    int nb[MAXV];
    const int m = load_fan(a.fan, k, nb);
    V4<R> pn[MAXV];
    fan_positions<R, AS>(P, m, nb, pn);
    force_sum(a, m, pn, pk, fx, fy, fz);
}

// A vertex's position and its fan (valence and neighbours), loaded ahead of
// the force.
template <class R>
struct FanPre {
    V4<R> pos;
    int nb[MAXV];
    int m;
};

// Tiles touched by a stencil starting at unwrapped `first`, marked with `ep`.
template <class R, int AS>
__device__ inline void mark_tiles(const IbArgs<R, AS>& a, const int first[3], int ep) {
    const int L[3] = {a.g.Lx, a.g.Ly, a.g.Lz};
    int t0[3], t1[3], t2[3];
    for (int d = 0; d < 3; ++d) {
        // four consecutive nodes cover at most three tiles (three only when a
        // periodic stencil wraps around a side that is not a tile multiple)
        t0[d] = wrap_any(first[d], L[d]) >> TILE_SHIFT;
        t1[d] = wrap_any(first[d] + 3, L[d]) >> TILE_SHIFT;
        t2[d] = t0[d];
        for (int j = 1; j < 3; ++j) {
            const int t = wrap_any(first[d] + j, L[d]) >> TILE_SHIFT;
            if (t != t0[d] && t != t1[d]) t2[d] = t;
        }
    }
    for (int cz = 0; cz < 3; ++cz) {
        const int tz = cz == 0 ? t0[2] : (cz == 1 ? t1[2] : t2[2]);
        if (cz > 0 && (tz == t0[2] || (cz == 2 && tz == t1[2]))) continue;
        for (int cy = 0; cy < 3; ++cy) {
            const int ty = cy == 0 ? t0[1] : (cy == 1 ? t1[1] : t2[1]);
            if (cy > 0 && (ty == t0[1] || (cy == 2 && ty == t1[1]))) continue;
            for (int cx = 0; cx < 3; ++cx) {
                const int tx = cx == 0 ? t0[0] : (cx == 1 ? t1[0] : t2[0]);
                if (cx > 0 && (tx == t0[0] || (cx == 2 && tx == t1[0]))) continue;
                a.mark[tx + a.g.TX * (ty + a.g.TY * tz)] = ep;
            }
        }
    }
}

// Stencil of a vertex at p: unwrapped first nodes and Peskin weights. False
// (and the device flag raised) for a non-finite position or a stencil
// through a wall.
template <class R, int AS>
__device__ inline bool stencil_of(const IbArgs<R, AS>& a, const V4<R>& p, int f[3], R w[3][4]) {
    R fr[3];
    const bool fin = isfinite(p.x) && isfinite(p.y) && isfinite(p.z);
    const bool ok = fin && stencil_base(p.x, a.g.xci[0], a.g.xcf[0], a.g.Lx, a.g.px, &f[0], &fr[0]) &&
                    stencil_base(p.y, a.g.xci[1], a.g.xcf[1], a.g.Ly, a.g.py, &f[1], &fr[1]) &&
                    stencil_base(p.z, a.g.xci[2], a.g.xcf[2], a.g.Lz, a.g.pz, &f[2], &fr[2]);
    if (!fin) atom_or(&a.ctl->flags, DFLAG_NONFINITE);
    else if (!ok) atom_or(&a.ctl->flags, DFLAG_DOMAIN);
    if (ok)
        for (int d = 0; d < 3; ++d) peskin4(fr[d], w[d]);
    return ok;
}

// Block-wide window (origin, extent in unwrapped nodes) of the active
// threads' stencils.
struct Win {
    int o[3], e[3], vol;
    bool fits;
};

__device__ inline Win block_window(bool active, const int f[3], int wcap) {
    __shared__ int red[6][IBT / 64];
    const int t = threadIdx.x;
    int mn[3], mx[3];
    for (int d = 0; d < 3; ++d) {
        mn[d] = active ? f[d] : 0x3fffffff;
        mx[d] = active ? f[d] : -0x3fffffff;
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
    Win w;
    bool any = true;
    long long vol = 1;
    for (int d = 0; d < 3; ++d) {
        int lo = red[d][0], hi = red[3 + d][0];
        for (int k = 1; k < IBT / 64; ++k) {
            lo = min(lo, red[d][k]);
            hi = max(hi, red[3 + d][k]);
        }
        any = any && lo <= hi;
        w.o[d] = lo;
        w.e[d] = any ? hi - lo + 4 : 0;
        vol *= w.e[d];
    }
    __syncthreads();
    w.fits = any && vol <= wcap;
    w.vol = w.fits ? int(vol) : 0;
    return w;
}

// ---------------------------------------------------------------- forces + spreading
// Staged stencils of a patch. The spreading window accumulates in FP64: LDS
// atomic adds on doubles run at integer speed on this device, while FP32 LDS
// atomic adds are about twenty times slower.
template <class R>
struct Stage {
    int first[PATCH][3];
    R w[PATCH][3][4];
    R val[PATCH][3];
    int ok[PATCH];
};

// Nodes of the FP64 spreading window: 3 x 1456 x 8 B = 34,944 B of dynamic
// LDS, so that with the force kernel's static LDS (about 5 KB in FP32) four
// work-groups fit in a CU's 160 KB, as many as the batched kernel's registers
// allow (the single-droplet kernel's allow three in FP32). A patch's
// window (the box of its vertices' stencils) holds 300-900 nodes on average
// for the benchmark meshes, up to about 1400 for a 2562-vertex droplet of
// radius 12 stretched to D = 0.3; a larger one falls back to direct atomics.
constexpr int SPREAD_WCAP = 1456;

// Accumulate the staged vertices [lo_v, hi_v) into an LDS window and flush
// each touched node once to F; false if their window exceeds the capacity.
template <class R, int AS>
__device__ bool spread_window(const IbArgs<R, AS>& a, const Stage<R>& st, double* win, int lo_v, int hi_v) {
    const int t = threadIdx.x;
    const bool in = t >= lo_v && t < hi_v && st.ok[t];
    const int tv = t < PATCH ? t : 0;
    const int f[3] = {st.first[tv][0], st.first[tv][1], st.first[tv][2]};
    const Win w = block_window(in, f, SPREAD_WCAP);
    if (!w.fits) return false;
    const int lane = t & 63, jx = lane & 3, jy = (lane >> 2) & 3, jz = lane >> 4;
    const long long N = a.g.N;
    for (int i = t; i < 3 * w.vol; i += IBT) win[i] = 0.0;
    __syncthreads();
    // wave t/64 takes vertices t/64, t/64 + 4, ...: first all their staged data
    // into registers, then the atomics back to back (LDS operations complete
    // in order, so interleaving the reads would wait on every atomic)
    constexpr int VW = PATCH / (IBT / 64);
    double cx[VW], cy[VW], cz[VW];
    int cell[VW];
#pragma unroll
    for (int j = 0; j < VW; ++j) {
        const int v = (t >> 6) + j * (IBT / 64);
        const bool use = v >= lo_v && v < hi_v && st.ok[v];
        const double wt = use ? double(st.w[v][0][jx]) * double(st.w[v][1][jy]) * double(st.w[v][2][jz]) : 0.0;
        const int lx = st.first[v][0] + jx - w.o[0];
        const int ly = st.first[v][1] + jy - w.o[1];
        const int lz = st.first[v][2] + jz - w.o[2];
        cell[j] = use ? lx + w.e[0] * (ly + w.e[1] * lz) : -1;
        cx[j] = double(st.val[v][0]) * wt;
        cy[j] = double(st.val[v][1]) * wt;
        cz[j] = double(st.val[v][2]) * wt;
    }
#pragma unroll
    for (int j = 0; j < VW; ++j) {
        if (cell[j] < 0) continue;
        atomicAdd(&win[cell[j]], cx[j]);
        atomicAdd(&win[w.vol + cell[j]], cy[j]);
        atomicAdd(&win[2 * w.vol + cell[j]], cz[j]);
    }
    __syncthreads();
    for (int i = t; i < w.vol; i += IBT) {
        const double vx = win[i], vy = win[w.vol + i], vz = win[2 * w.vol + i];
        if (vx == 0.0 && vy == 0.0 && vz == 0.0) continue;
        const int lx = i % w.e[0], rest = i / w.e[0];
        const int ly = rest % w.e[1], lz = rest / w.e[1];
        const long long n = node_index(a.g, w.o[0] + lx, w.o[1] + ly, w.o[2] + lz);
        atom_add(a.F + n, R(vx));
        atom_add(a.F + N + n, R(vy));
        atom_add(a.F + 2 * N + n, R(vz));
    }
    __syncthreads();
    return true;
}

// Deterministic spreading, first half: the patch's staged stencils and its
// window go to memory instead of into the atomics.
template <class R, int AS>
__device__ void det_stage(const IbArgs<R, AS>& a, int p, const Stage<R>& st) {
    const int t = threadIdx.x;
    const int k = p * PATCH + t;
    const bool own = t < PATCH && k < a.nv;
    const int tv = t < PATCH ? t : 0;
    const int f[3] = {st.first[tv][0], st.first[tv][1], st.first[tv][2]};
    const Win w = block_window(own && st.ok[tv], f, 0x7fffffff);
    if (own) {
        const int L[3] = {a.g.Lx, a.g.Ly, a.g.Lz};
        const int ok = st.ok[t];
        auto rec = a.det + k;
        for (int d = 0; d < 3; ++d) {
            rec->fw[d] = wrap_any(f[d], L[d]);
            for (int j = 0; j < 4; ++j) rec->w[d][j] = ok ? st.w[t][d][j] : R(0);
            rec->val[d] = ok ? st.val[t][d] : R(0);
        }
        rec->ok = ok;
    }
    if (t < 3) {  // selected, not indexed: a per-thread index would put the window in scratch
        a.pbox[8 * p + t] = t == 0 ? w.o[0] : (t == 1 ? w.o[1] : w.o[2]);
        a.pbox[8 * p + 3 + t] = t == 0 ? w.e[0] : (t == 1 ? w.e[1] : w.e[2]);
    }
}

// The triangles each patch crosses with the lattice rows (viscosity ratio
// only): those whose lowest vertex id lies in the patch, listed patch by
// patch, and the indicator's toggle words and row ranges.
struct IndArgs {
    const int4* ptris;    // [nt], grouped by patch
    const int* ptstart;   // [npatch + 1]
    unsigned* words;      // indicator bytes as 32-bit words
    int* lo;              // [Ly Lz] row ranges
    int* hi;
    int* flags;           // the control block's error flags
};

// Forces, tile marks and spreading of patch p from positions P. With
// `commit`, P (the final smoothed positions) also becomes the state r.
// CHI: waves 1-3, idle while the first wave computes the forces, cross the
// patch's triangles (positions P) with the lattice rows.
// `pre` holds this thread's vertex position in P and its fan (for a thread
// that owns a vertex).
template <class R, int AS, bool CHI = false>
__device__ void fs_patch(const IbArgs<R, AS>& a, int p, Ptr<const V4<R>, AS> P, int commit, Stage<R>& st, double* win,
                         const IndArgs* ia, const FanPre<R>& pre) {
    const int t = threadIdx.x;
    const int k = p * PATCH + t;
    const int ep = a.ctl->epoch;
    const long long N = a.g.N;
    int f[3] = {0, 0, 0};
    R w[3][4];
    bool ok = false;
    if (t < PATCH && k < a.nv) {
        const V4<R> pos = pre.pos;
        if (commit) st4(a.r + k, pos);
        ok = stencil_of(a, pos, f, w);
        if (ok) {
            R fx, fy, fz;
            V4<R> pn[MAXV];
            fan_positions<R, AS>(P, pre.m, pre.nb, pn);
            force_sum(a, pre.m, pn, pos, fx, fy, fz);
            mark_tiles(a, f, ep);
            st.val[t][0] = fx;
            st.val[t][1] = fy;
            st.val[t][2] = fz;
            for (int d = 0; d < 3; ++d)
                for (int j = 0; j < 4; ++j) st.w[t][d][j] = w[d][j];
        }
    }
    if (t < PATCH) {
        for (int d = 0; d < 3; ++d) st.first[t][d] = f[d];
        st.ok[t] = ok ? 1 : 0;
    }
    if constexpr (CHI) {
        if (t >= 64) {
            const double xc[3] = {a.g.xci[0] + a.g.xcf[0], a.g.xci[1] + a.g.xcf[1], a.g.xci[2] + a.g.xcf[2]};
            for (int q = ia->ptstart[p] + t - 64; q < ia->ptstart[p + 1]; q += IBT - 64) {
                const int4 tv = ia->ptris[q];
                const int id[3] = {tv.x, tv.y, tv.z};
                double Pd[3][3];
                for (int c = 0; c < 3; ++c) {
                    const V4<R> pc = ld4<V4<R>>(P + id[c]);
                    Pd[c][0] = double(pc.x) + xc[0];
                    Pd[c][1] = double(pc.y) + xc[1];
                    Pd[c][2] = double(pc.z) + xc[2];
                }
                triangle_row_crossings(a.g, id, Pd, ia->words, ia->lo, ia->hi, ia->flags);
            }
        }
    }
    __syncthreads();
    if (a.det) {
        det_stage(a, p, st);
        return;
    }
    if (spread_window(a, st, win, 0, PATCH)) return;
    // a patch too spread out for the window: direct global atomics
    const int lane = t & 63, jx = lane & 3, jy = (lane >> 2) & 3, jz = lane >> 4;
    for (int v = t >> 6; v < PATCH; v += IBT / 64) {
        if (!st.ok[v]) continue;
        const R wt = st.w[v][0][jx] * st.w[v][1][jy] * st.w[v][2][jz];
        const long long n = node_index(a.g, st.first[v][0] + jx, st.first[v][1] + jy, st.first[v][2] + jz);
        atom_add(a.F + n, st.val[v][0] * wt);
        atom_add(a.F + N + n, st.val[v][1] * wt);
        atom_add(a.F + 2 * N + n, st.val[v][2] * wt);
    }
}

template <class R>
__device__ inline R from_bits(unsigned long long b);
template <>
__device__ inline float from_bits<float>(unsigned long long b) { return __uint_as_float((unsigned)b); }
template <>
__device__ inline double from_bits<double>(unsigned long long b) { return __longlong_as_double((long long)b); }

// The step's largest |p - q| so far: the maximum over the reduction slots,
// one slot a lane, folded across the wave (every lane of the calling wave
// active; each wave gets the value).
template <class R>
__device__ inline R slot_max(unsigned long long v) {
    for (int m = 32; m > 0; m >>= 1) {
        const unsigned long long o = __shfl_xor(v, m, 64);
        v = o > v ? o : v;
    }
    return from_bits<R>(v);
}

template <class R, int AS>
__device__ inline R red_max(const IbArgs<R, AS>& a) {
    return slot_max<R>(a.red[threadIdx.x & (RED_SLOTS - 1)]);
}

// Zero the reduction slots and the arrival count (the first wave of a
// work-group).
template <class R, int AS>
__device__ inline void red_clear(const IbArgs<R, AS>& a) {
    if (threadIdx.x < RED_SLOTS) a.red[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) a.red[RED_SLOTS] = 0ull;
}

template <class R, int AS>
__device__ int hc_more_iterations(const IbArgs<R, AS>& a, bool* capped);

// Forces, tile marks and spreading of every vertex by one work-group (the
// rare path below), 256 vertices at a time: one thread per vertex computes
// its stencil and force into LDS records (in the dynamic window's memory),
// then one wave per vertex adds its 64 contributions with direct global
// atomics, one lane per stencil node. With CHI, the viscosity ratio's row
// crossings of every triangle follow.
template <class R, bool CHI>
__device__ void fs_all_vertices(const IbArgs<R>& a, const V4<R>* P, int commit, const IndArgs* ia, int npatch,
                                double* win) {
    const int t = threadIdx.x, lane = t & 63;
    const int ep = a.ctl->epoch;
    const long long N = a.g.N;
    static_assert(IBT * sizeof(DetRec<R>) <= 3 * SPREAD_WCAP * sizeof(double), "records fit the window's LDS");
    DetRec<R>* rec = reinterpret_cast<DetRec<R>*>(win);  // IBT records, within the window's LDS
    const int jx = lane & 3, jy = (lane >> 2) & 3, jz = lane >> 4;
    for (int c0 = 0; c0 < a.nv; c0 += IBT) {
        const int k = c0 + t;
        int ok = 0;
        if (k < a.nv) {
            const V4<R> pos = ld4<V4<R>>(P + k);
            if (commit) st4(a.r + k, pos);
            int f[3];
            R w[3][4];
            if (stencil_of(a, pos, f, w)) {
                ok = 1;
                R fx, fy, fz;
                force_of(a, P, k, pos, fx, fy, fz);
                mark_tiles(a, f, ep);
                for (int d = 0; d < 3; ++d) {
                    rec[t].fw[d] = f[d];
                    for (int j = 0; j < 4; ++j) rec[t].w[d][j] = w[d][j];
                }
                rec[t].val[0] = fx;
                rec[t].val[1] = fy;
                rec[t].val[2] = fz;
            }
        }
        rec[t].ok = ok;
        __syncthreads();
        const int nc = min(IBT, a.nv - c0);
        for (int v = t >> 6; v < nc; v += IBT / 64) {
            if (!rec[v].ok) continue;
            const R wt = rec[v].w[0][jx] * rec[v].w[1][jy] * rec[v].w[2][jz];
            const long long n = node_index(a.g, rec[v].fw[0] + jx, rec[v].fw[1] + jy, rec[v].fw[2] + jz);
            atom_add(a.F + n, rec[v].val[0] * wt);
            atom_add(a.F + N + n, rec[v].val[1] * wt);
            atom_add(a.F + 2 * N + n, rec[v].val[2] * wt);
        }
        __syncthreads();
    }
    if constexpr (CHI) {
        const double xc[3] = {a.g.xci[0] + a.g.xcf[0], a.g.xci[1] + a.g.xcf[1], a.g.xci[2] + a.g.xcf[2]};
        for (int q = t; q < ia->ptstart[npatch]; q += IBT) {
            const int4 tv = ia->ptris[q];
            const int id[3] = {tv.x, tv.y, tv.z};
            double Pd[3][3];
            for (int c = 0; c < 3; ++c) {
                const V4<R> pc = ld4<V4<R>>(P + id[c]);
                Pd[c][0] = double(pc.x) + xc[0];
                Pd[c][1] = double(pc.y) + xc[1];
                Pd[c][2] = double(pc.z) + xc[2];
            }
            triangle_row_crossings(a.g, id, Pd, ia->words, ia->lo, ia->hi, ia->flags);
        }
    }
}

// The smoothing's finish folded into the force kernel (bit 5 of the step
// variant; not with the deterministic spreading). Every work-group takes the
// same decision from the reduction slots that the first smoothing iteration
// filled: when that iteration converged, hit the iteration cap or smoothing
// is off, work-group 0 records the count and every work-group treats its own
// patch; otherwise (rare) work-group 0 alone runs the further iterations,
// records the count and then treats every vertex with direct atomics, while
// the others return. The step epoch was advanced and the reduction slots
// cleared by the interpolation launch of the step.
template <class R, bool CHI>
__device__ void fs_step(const IbArgs<R>& a, int fold, int npatch, const V4<R>* P, int commit, Stage<R>& st,
                        double* win, const IndArgs* ia) {
    const int t = threadIdx.x;
    // the reduction slot, this thread's vertex position and its fan are
    // loaded together, before the decision that needs the slot (a path that
    // runs further iterations drops the vertex data)
    const bool test = fold && a.sp.max_iter > 0;
    const unsigned long long slot = test ? a.red[t & (RED_SLOTS - 1)] : 0ull;
    const int k0 = blockIdx.x * PATCH + t;
    FanPre<R> pre;
    pre.m = 0;
    pre.pos = V4<R>{};
    if (t < PATCH && k0 < a.nv) {
        pre.pos = ld4<V4<R>>(P + k0);
        pre.m = load_fan(a.fan, k0, pre.nb);
    }
    if (fold) {
        bool more = false, capped = false;
        if (test) {
            const bool converged = slot_max<R>(slot) < R(a.sp.tol);
            capped = !converged && a.sp.max_iter <= 1;
            more = !converged && !capped;
        }
        if (more) {
            if (blockIdx.x != 0) return;
            const int it = hc_more_iterations(a, &capped);
            if (t == 0) {
                a.ctl->iters = it;
                if (capped) a.ctl->cap_hits += 1;
            }
            __syncthreads();  // the final positions in qa, written by this work-group
            fs_all_vertices<R, CHI>(a, P, commit, ia, npatch, win);
            return;
        }
        if (blockIdx.x == 0 && t == 0) {
            a.ctl->iters = a.sp.max_iter > 0 ? 1 : 0;
            if (capped) a.ctl->cap_hits += 1;
        }
    }
    fs_patch<R, 0, CHI>(a, blockIdx.x, P, commit, st, win, ia, pre);
}

template <class R>
__global__ __launch_bounds__(IBT) void k_fs_patch(IbArgs<R> a, const V4<R>* P, int commit, int fold, int npatch) {
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ Stage<R> st;
    fs_step<R, false>(a, fold, npatch, P, commit, st, reinterpret_cast<double*>(dyn), nullptr);
}

// The same with the row crossings of the viscosity ratio's indicator.
template <class R>
__global__ __launch_bounds__(IBT) void k_fs_patch_ind(IbArgs<R> a, const V4<R>* P, int commit, IndArgs ia, int fold,
                                                      int npatch) {
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ Stage<R> st;
    fs_step<R, true>(a, fold, npatch, P, commit, st, reinterpret_cast<double*>(dyn), &ia);
}

// Deterministic spreading, second half (Eq. ibm_force_d, first line, as a
// gather): one single-wave work-group per z-slice of an 8^3 tile, one lane
// per node of the 8 x 8 slice. A tile marked for this step goes through the
// patches 64 at a time; those whose windows meet the slice are taken in
// increasing patch order, DET_CB at a time (lane v loads vertex v of each,
// all loads in flight together). For each patch in turn, the vertices whose
// stencils reach the slice are listed in LDS in increasing order (a ballot
// and prefix count), and every lane adds their contributions to its node in
// that order, in FP64. F is stored once per
// node. Each node's sum is therefore taken in one order (increasing vertex
// index) whatever the scheduling, and a run repeats bit for bit. The window
// atomics above differ from it only by the order of their additions (and,
// for FP32, by rounding each patch's part to FP32).
static_assert(TILE_SHIFT == 3, "the gather maps one wave onto an 8 x 8 slice of an 8^3 tile");
constexpr int DET_SLICES = 8;

__device__ inline int pmod(int a, int L) {
    const int m = a % L;
    return m < 0 ? m + L : m;
}

// Does the window origin o, extent e (unwrapped) cover any of the nodes
// t0 .. t0 + n - 1 of an axis of L nodes?
__device__ inline bool covers(int o, int e, int t0, int n, int L) {
    return e > 0 && (pmod(t0 - o, L) < e || pmod(o - t0, L) < n);
}

constexpr int DET_CB = 4;  // candidate patches loaded per round

template <class R>
__global__ __launch_bounds__(64) void k_spread_det(IbArgs<R> a, int npatch) {
    // the vertices of one candidate patch that reach the slice, compacted in
    // increasing order
    __shared__ int4 sfw[PATCH];     // first stencil node (folded)
    __shared__ R sw[PATCH][3][4];   // weights
    __shared__ R sval[PATCH][3];    // forces
    const int tile = blockIdx.x / DET_SLICES, zs = blockIdx.x % DET_SLICES;
    if (a.mark[tile] != a.ctl->epoch) return;
    const int lane = threadIdx.x;
    const int L[3] = {a.g.Lx, a.g.Ly, a.g.Lz};
    const int T0[3] = {(tile % a.g.TX) << TILE_SHIFT, ((tile / a.g.TX) % a.g.TY) << TILE_SHIFT,
                       ((tile / (a.g.TX * a.g.TY)) << TILE_SHIFT) + zs};
    if (T0[2] >= L[2]) return;  // a slice beyond a ragged z end
    const int cnt[3] = {min(8, L[0] - T0[0]), min(8, L[1] - T0[1]), 1};
    const int x = T0[0] + (lane & 7), y = T0[1] + (lane >> 3), z = T0[2];
    const bool act = x < L[0] && y < L[1];
    const unsigned long long below = (1ull << lane) - 1ull;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int base = 0; base < npatch; base += 64) {
        // lane l tests patch base + l
        const int p = base + lane;
        bool meet = p < npatch;
        if (meet)
            for (int d = 0; d < 3; ++d)
                meet = meet && covers(a.pbox[8 * p + d], a.pbox[8 * p + 3 + d], T0[d], cnt[d], L[d]);
        unsigned long long m = __ballot(meet);
        while (m) {
            // the next DET_CB candidates in increasing order; lane v loads
            // vertex v of each (all loads in flight together)
            int qc[DET_CB];
            int nc = 0;
#pragma unroll
            for (int c = 0; c < DET_CB; ++c) {
                qc[c] = -1;
                if (m) {
                    qc[c] = base + __ffsll((long long)m) - 1;
                    m &= m - 1;
                    nc = c + 1;
                }
            }
            int fw[DET_CB][3], ok[DET_CB];
            R w[DET_CB][3][4], val[DET_CB][3];
#pragma unroll
            for (int c = 0; c < DET_CB; ++c) {
                const int k = qc[c] * PATCH + lane;
                ok[c] = 0;
                if (qc[c] >= 0 && k < a.nv) {
                    const DetRec<R>* r = a.det + k;
                    ok[c] = r->ok;
                    for (int d = 0; d < 3; ++d) {
                        fw[c][d] = r->fw[d];
                        val[c][d] = r->val[d];
                        for (int j = 0; j < 4; ++j) w[c][d][j] = r->w[d][j];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < DET_CB; ++c) {
                if (c >= nc) break;
                // does this lane's vertex reach the slice? (its stencil covers
                // z and meets the slice's x and y ranges)
                bool rel = ok[c] != 0;
                if (rel) {
                    int dz = z - fw[c][2];
                    dz += dz < 0 ? L[2] : 0;
                    rel = dz <= 3 && covers(fw[c][0], 4, T0[0], cnt[0], L[0]) && covers(fw[c][1], 4, T0[1], cnt[1], L[1]);
                }
                const unsigned long long rm = __ballot(rel);
                if (rm == 0ull) continue;
                __syncthreads();  // the previous candidate's list is consumed
                if (rel) {
                    const int slot = __popcll(rm & below);
                    sfw[slot] = make_int4(fw[c][0], fw[c][1], fw[c][2], 0);
                    for (int d = 0; d < 3; ++d) {
                        for (int j = 0; j < 4; ++j) sw[slot][d][j] = w[c][d][j];
                        sval[slot][d] = val[c][d];
                    }
                }
                __syncthreads();
                const int nrel = __popcll(rm);
                if (!act) continue;
                for (int v = 0; v < nrel; ++v) {
                    const int4 f = sfw[v];
                    // offsets into the stencil; a node before the first one
                    // folds to at least 4 (walls: the stencil ends 4 nodes
                    // inside; periodic: the box has at least 8 nodes)
                    int dx = x - f.x, dy = y - f.y, dz = z - f.z;
                    dx += dx < 0 ? L[0] : 0;
                    dy += dy < 0 ? L[1] : 0;
                    dz += dz < 0 ? L[2] : 0;
                    if (dx > 3 || dy > 3 || dz > 3) continue;
                    const double wt = double(sw[v][0][dx]) * double(sw[v][1][dy]) * double(sw[v][2][dz]);
                    acc[0] += double(sval[v][0]) * wt;
                    acc[1] += double(sval[v][1]) * wt;
                    acc[2] += double(sval[v][2]) * wt;
                }
            }
        }
    }
    if (act) {
        const long long N = a.g.N;
        const long long n = x + (long long)L[0] * (y + (long long)L[1] * z);
        a.F[n] = R(acc[0]);
        a.F[N + n] = R(acc[1]);
        a.F[2 * N + n] = R(acc[2]);
    }
}

size_t det_rec_bytes(int storage) {
    return storage == IBM_LB_F64 ? sizeof(DetRec<double>) : sizeof(DetRec<float>);
}

// ---------------------------------------------------------------- interpolation
template <class R, int AS>
__device__ void interp_patch(const IbArgs<R, AS>& a, int patch, R* win) {
    const int t = threadIdx.x;
    const int k = patch * PATCH + t;
    const long long N = a.g.N;
    int f[3] = {0, 0, 0};
    R w[3][4];
    bool ok = false;
    V4<R> p = V4<R>{R(0), R(0), R(0), R(0)};
    if (t < PATCH && k < a.nv) {
        p = ld4<V4<R>>(a.r + k);
        ok = stencil_of(a, p, f, w);
    }
    const Win wn = block_window(ok, f, a.wcap);
    if (wn.fits) {
        for (int i = t; i < wn.vol; i += IBT) {
            const int lx = i % wn.e[0], rest = i / wn.e[0];
            const int ly = rest % wn.e[1], lz = rest / wn.e[1];
            const long long n = node_index(a.g, wn.o[0] + lx, wn.o[1] + ly, wn.o[2] + lz);
            win[i] = a.U[n];
            win[wn.vol + i] = a.U[N + n];
            win[2 * wn.vol + i] = a.U[2 * N + n];
        }
        __syncthreads();
    }
    if (t >= PATCH || k >= a.nv) return;
    R ux = R(0), uy = R(0), uz = R(0);
    if (ok) {
        if (wn.fits) {
            const int lx = f[0] - wn.o[0];
            for (int jz = 0; jz < 4; ++jz)
                for (int jy = 0; jy < 4; ++jy) {
                    const int base = lx + wn.e[0] * ((f[1] - wn.o[1] + jy) + wn.e[1] * (f[2] - wn.o[2] + jz));
                    const R wyz = w[1][jy] * w[2][jz];
#pragma unroll
                    for (int jx = 0; jx < 4; ++jx) {
                        const R wt = w[0][jx] * wyz;
                        ux += win[base + jx] * wt;
                        uy += win[wn.vol + base + jx] * wt;
                        uz += win[2 * wn.vol + base + jx] * wt;
                    }
                }
        } else {
            for (int jz = 0; jz < 4; ++jz)
                for (int jy = 0; jy < 4; ++jy) {
                    const R wyz = w[1][jy] * w[2][jz];
#pragma unroll
                    for (int jx = 0; jx < 4; ++jx) {
                        const R wt = w[0][jx] * wyz;
                        const long long n = node_index(a.g, f[0] + jx, f[1] + jy, f[2] + jz);
                        ux += a.U[n] * wt;
                        uy += a.U[N + n] * wt;
                        uz += a.U[2 * N + n] * wt;
                    }
                }
        }
    }
    st4(a.o + k, V4<R>{p.x + ux, p.y + uy, p.z + uz, R(0)});
}

template <class R>
__global__ __launch_bounds__(IBT) void k_interp_patch(IbArgs<R> a, int fold) {
    extern __shared__ __align__(16) unsigned char dyn[];
    // the step's reduction slots start at zero; with the smoothing's finish
    // folded into the force kernel, the step epoch advances here (nothing
    // between this launch and the force kernel reads it)
    if (blockIdx.x == 0) {
        red_clear(a);
        if (fold && threadIdx.x == 0) a.ctl->epoch += 1;
    }
    interp_patch(a, blockIdx.x, reinterpret_cast<R*>(dyn));
}

// ---------------------------------------------------------------- HC smoothing
// Sec. 3.3 with x_o = o: x_q = x_p; x_p = alpha x_o + (1-alpha) mean_nb(x_q);
// x_b = x_p - (alpha x_o + (1-alpha) x_q); x_p -= gamma x_b + sign (1-gamma)
// mean_nb(x_b); stop when max |x_p - x_q| < tol.
template <class R, int AS>
__device__ inline V4<R> ring_sum(const IbArgs<R, AS>& a, Ptr<const V4<R>, AS> X, int k, int* m_out) {
    int nb[MAXV];
    const int m = load_fan(a.fan, k, nb);
    R sx = R(0), sy = R(0), sz = R(0);
#pragma unroll
    for (int j = 0; j < MAXV; ++j) {
        if (j < m) {
            const V4<R> v = ld4<V4<R>>(X + nb[j]);
            sx += v.x; sy += v.y; sz += v.z;
        }
    }
    *m_out = m;
    return V4<R>{sx, sy, sz, R(0)};
}

template <class R, int AS>
__device__ inline void hc_first(const IbArgs<R, AS>& a, Ptr<const V4<R>, AS> q, int k, R alpha) {
    int m;
    const V4<R> s = ring_sum(a, q, k, &m);
    const R c = (R(1) - alpha) / R(m);
    const V4<R> ok = ld4<V4<R>>(a.o + k), qk = ld4<V4<R>>(q + k);
    const R px = alpha * ok.x + c * s.x, py = alpha * ok.y + c * s.y, pz = alpha * ok.z + c * s.z;
    st4(a.pp + k, V4<R>{px, py, pz, R(0)});
    st4(a.bb + k, V4<R>{px - (alpha * ok.x + (R(1) - alpha) * qk.x), py - (alpha * ok.y + (R(1) - alpha) * qk.y),
                    pz - (alpha * ok.z + (R(1) - alpha) * qk.z), R(0)});
}

template <class R, int AS>
__device__ inline R hc_second(const IbArgs<R, AS>& a, Ptr<const V4<R>, AS> q, Ptr<V4<R>, AS> qn, int k, R gamma, R sgn) {
    int m;
    const V4<R> s = ring_sum(a, a.bb, k, &m);
    const R c = sgn * (R(1) - gamma) / R(m);
    const V4<R> bk = ld4<V4<R>>(a.bb + k), pk = ld4<V4<R>>(a.pp + k), qk = ld4<V4<R>>(q + k);
    const R nx = pk.x - (gamma * bk.x + c * s.x);
    const R ny = pk.y - (gamma * bk.y + c * s.y);
    const R nz = pk.z - (gamma * bk.z + c * s.z);
    st4(qn + k, V4<R>{nx, ny, nz, R(0)});
    const R dx = nx - qk.x, dy = ny - qk.y, dz = nz - qk.z;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

template <class R>
__device__ inline unsigned long long max_bits(R v);
template <>
__device__ inline unsigned long long max_bits<float>(float v) { return (unsigned long long)__float_as_uint(v); }
template <>
__device__ inline unsigned long long max_bits<double>(double v) {
    return (unsigned long long)__double_as_longlong(v);
}
template <class R, int AS>
__device__ void hc_finish(const IbArgs<R, AS>& a);

// Smoothing of one step in one launch, one work-group per surface patch.
// Phase 1: p' and b of iteration 1 (q = o) for the patch's vertices and its
// halo (ring neighbours outside the patch) from the rings of o, into LDS.
// Phase 2: p of the patch's vertices from the b of their rings (LDS), into
// qa, and max |p - o| folded into its reduction slot. The last work-group to
// arrive (counted in the second slot) sees every patch's result and finishes
// the step: the convergence test, further iterations in the rare case they
// are needed, the iteration count and the epoch. The arithmetic is that of a
// pass computing every p' and b followed by a pass computing every p.
constexpr int HALO_CAP = MAXV * PATCH;  // no patch can have more halo vertices

// split: no arrival count; a later launch (k_hc_finish_batch) finishes the
// step from the reduction slots. This spares every work-group the
// device-scope release that must precede its arrival (on this device a
// write-back of its XCD's L2), which costs more than a launch once there are
// thousands of work-groups.
template <class R, int AS>
__device__ void hc_fused(const IbArgs<R, AS>& a, int p, int npatch, bool split) {
    __shared__ V4<R> sb[PATCH + HALO_CAP];
    __shared__ V4<R> spp[PATCH], so[PATCH];
    __shared__ R bred[IBT / 64];
    __shared__ int last;
    const int t = threadIdx.x;
    const bool on = a.sp.max_iter > 0;
    const int base = p * PATCH;
    const int nown = min(PATCH, a.nv - base);
    const R alpha = R(a.sp.alpha), gamma = R(a.sp.gamma), sgn = R(a.sp.sign);
    R d = R(0);
    if (on) {
        // the patch-local fan of this thread's own vertex, loaded before the
        // first phase so that its latency overlaps that phase's loads
        int lnb[MAXV];
        const int lm = t < nown ? load_fan(a.lfan, base + t, lnb) : 0;
        const int h0 = a.hstart[p], nh = a.hstart[p + 1] - h0;
        for (int i = t; i < PATCH + nh; i += IBT) {
            if (i >= nown && i < PATCH) continue;
            const int v = i < PATCH ? base + i : a.hids[h0 + i - PATCH];
            int m;
            const V4<R> sum = ring_sum(a, a.o, v, &m);
            const V4<R> ov = ld4<V4<R>>(a.o + v);
            const R c = (R(1) - alpha) / R(m);
            const R px = alpha * ov.x + c * sum.x, py = alpha * ov.y + c * sum.y, pz = alpha * ov.z + c * sum.z;
            sb[i] = V4<R>{px - (alpha * ov.x + (R(1) - alpha) * ov.x), py - (alpha * ov.y + (R(1) - alpha) * ov.y),
                          pz - (alpha * ov.z + (R(1) - alpha) * ov.z), R(0)};
            if (i < PATCH) {
                spp[i] = V4<R>{px, py, pz, R(0)};
                so[i] = ov;
            }
        }
        __syncthreads();
        if (t < nown) {
            const int m = lm;
            R sx = R(0), sy = R(0), sz = R(0);
#pragma unroll
            for (int j = 0; j < MAXV; ++j) {
                if (j < m) {
                    const V4<R> v = sb[lnb[j]];
                    sx += v.x;
                    sy += v.y;
                    sz += v.z;
                }
            }
            const R c = sgn * (R(1) - gamma) / R(m);
            const V4<R> bk = sb[t], pk = spp[t], ok = so[t];
            const R nx = pk.x - (gamma * bk.x + c * sx);
            const R ny = pk.y - (gamma * bk.y + c * sy);
            const R nz = pk.z - (gamma * bk.z + c * sz);
            st4(a.qa + base + t, V4<R>{nx, ny, nz, R(0)});
            const R dx = nx - ok.x, dy = ny - ok.y, dz = nz - ok.z;
            d = sqrt(dx * dx + dy * dy + dz * dz);
        }
    }
    for (int m = 32; m > 0; m >>= 1) d = fmax(d, __shfl_xor(d, m, 64));
    if ((t & 63) == 0) bred[t >> 6] = d;
    __syncthreads();
    if (split) {
        if (t == 0 && on) {
            R b = bred[0];
            for (int w = 1; w < IBT / 64; ++w) b = fmax(b, bred[w]);
            atom_max(a.red + (p & (RED_SLOTS - 1)), max_bits(b));
        }
        return;
    }
    if (t == 0) {
        R b = bred[0];
        for (int w = 1; w < IBT / 64; ++w) b = fmax(b, bred[w]);
        if (on) atom_max(a.red + (p & (RED_SLOTS - 1)), max_bits(b));
        __threadfence();
        last = atom_inc(a.red + RED_SLOTS) == (unsigned long long)(npatch - 1);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    hc_finish(a);
}

template <class R>
__global__ __launch_bounds__(IBT) void k_hc_fused(IbArgs<R> a, int npatch, int split) {
    hc_fused(a, blockIdx.x, npatch, split != 0);
}

// Split smoothing of one droplet with the deterministic spreading: the finish
// as a launch of its own.
template <class R>
__global__ __launch_bounds__(1024) void k_hc_finish(IbArgs<R> a) {
    hc_finish(a);
}

// One work-group, after iteration 1 is in qa and its maximum in the
// reduction slots (smoothing on): continue while not converged (rare) and
// leave the final positions in qa. Returns the iteration count; *capped_out
// tells whether the cap ended it.
template <class R, int AS>
__device__ int hc_more_iterations(const IbArgs<R, AS>& a, bool* capped_out) {
    __shared__ R bred[16];
    __shared__ int more;
    const int t = threadIdx.x, nth = blockDim.x;
    const R alpha = R(a.sp.alpha), gamma = R(a.sp.gamma), tol = R(a.sp.tol), sgn = R(a.sp.sign);
    const R dmax = red_max(a);
    int it = 1;
    bool capped = false;
    bool converged = dmax < tol;
    if (!converged && it >= a.sp.max_iter) capped = true;
    Ptr<V4<R>, AS> q = a.qa;
    Ptr<V4<R>, AS> qn = a.qb;
    while (!converged && !capped) {
        ++it;
        for (int k = t; k < a.nv; k += nth) hc_first(a, q, k, alpha);
        __syncthreads();
        R d = R(0);
        for (int k = t; k < a.nv; k += nth) d = fmax(d, hc_second(a, q, qn, k, gamma, sgn));
        for (int m = 32; m > 0; m >>= 1) d = fmax(d, __shfl_xor(d, m, 64));
        if ((t & 63) == 0) bred[t >> 6] = d;
        __syncthreads();
        if (t == 0) {
            R bmax = bred[0];
            for (int w = 1; w < (nth + 63) / 64; ++w) bmax = fmax(bmax, bred[w]);
            more = bmax < tol ? 0 : (it >= a.sp.max_iter ? 2 : 1);
        }
        __syncthreads();
        converged = more == 0;
        capped = more == 2;
        Ptr<V4<R>, AS> tmp = q;
        q = qn;
        qn = tmp;
    }
    // the newest iterate is in q
    if (q != a.qa)
        for (int k = t; k < a.nv; k += nth) st4(a.qa + k, ld4<V4<R>>(q + k));
    *capped_out = capped;
    return it;
}

// The finish of a step's smoothing in one work-group (the last smoothing
// work-group to arrive, or one per ensemble member): further iterations if
// needed, the iteration count, the epoch, and the reduction slots reset.
template <class R, int AS>
__device__ void hc_finish(const IbArgs<R, AS>& a) {
    const int t = threadIdx.x;
    if (a.sp.max_iter <= 0) {
        if (t == 0) {
            a.ctl->iters = 0;
            a.ctl->epoch += 1;
            a.red[RED_SLOTS] = 0ull;
        }
        return;
    }
    bool capped = false;
    const int it = hc_more_iterations(a, &capped);
    if (t == 0) {
        a.ctl->iters = it;
        if (capped) a.ctl->cap_hits += 1;
        a.ctl->epoch += 1;
    }
    red_clear(a);
}

// ---------------------------------------------------------------- ensemble forms
// Work-group b of a batched launch takes patch map[b].y of member map[b].x.
// The member's record is read from memory and its pointers are taken as
// global ones.
// Registers bounded for six waves per SIMD: left free, the compiler took 127
// (four waves), although the single-droplet form needs 71.
template <class R>
__global__ __launch_bounds__(IBT, 6) void k_interp_batch(const IbArgs<R>* __restrict__ args,
                                                       const int2* __restrict__ map) {
    extern __shared__ __align__(16) unsigned char dyn[];
    const int2 e = map[blockIdx.x];
    const IbArgs<R, 1> a = to_global(args[e.x]);
    interp_patch(a, e.y, reinterpret_cast<R*>(dyn));
}

template <class R>
__global__ __launch_bounds__(IBT) void k_hc_fused_batch(const IbArgs<R>* __restrict__ args,
                                                        const int2* __restrict__ map) {
    const int2 e = map[blockIdx.x];
    const IbArgs<R, 1> a = to_global(args[e.x]);
    hc_fused(a, e.y, (a.nv + PATCH - 1) / PATCH, true);
}

// One work-group per member, after k_hc_fused_batch: the convergence test,
// the further iterations when iteration 1 did not converge (1024 threads),
// the iteration count and the epoch.
template <class R>
__global__ __launch_bounds__(1024) void k_hc_finish_batch(const IbArgs<R>* __restrict__ args) {
    const IbArgs<R, 1> a = to_global(args[blockIdx.x]);
    if (a.nv == 0) return;
    hc_finish(a);
}

template <class R>
__global__ __launch_bounds__(IBT) void k_fs_batch(const IbArgs<R>* __restrict__ args, const int2* __restrict__ map,
                                                   int commit) {
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ Stage<R> st;
    const int2 e = map[blockIdx.x];
    const IbArgs<R, 1> a = to_global(args[e.x]);
    const Ptr<const V4<R>, 1> P = commit ? (a.sp.max_iter > 0 ? a.qa : a.o) : a.r;
    const int k = e.y * PATCH + int(threadIdx.x);
    FanPre<R> pre;
    pre.m = 0;
    pre.pos = V4<R>{};
    if (threadIdx.x < PATCH && k < a.nv) {
        pre.pos = ld4<V4<R>>(P + k);
        pre.m = load_fan(a.fan, k, pre.nb);
    }
    fs_patch(a, e.y, P, commit, st, reinterpret_cast<double*>(dyn), nullptr, pre);
}

// ---------------------------------------------------------------- launchers
int patch_window_nodes(int) { return 2048; }

static size_t dyn_lds(int storage) { return 3 * (size_t)patch_window_nodes(storage) * real_bytes(storage); }
static size_t dyn_lds_spread() { return 3 * (size_t)SPREAD_WCAP * sizeof(double); }

template <class R>
static IbArgs<R> make_args(const Geom& g, const DevPtrs& d, int nv, double sigma, const SmoothParams& sp) {
    IbArgs<R> a{};
    a.g = g;
    a.nv = nv;
    a.sigma = R(sigma);
    a.sp = sp;
    a.r = (V4<R>*)d.r;
    a.o = (V4<R>*)d.o;
    a.qa = (V4<R>*)d.qa;
    a.qb = (V4<R>*)d.qb;
    a.pp = (V4<R>*)d.pp;
    a.bb = (V4<R>*)d.bb;
    a.fan = d.fan;
    a.lfan = d.lfan;
    a.hstart = d.hstart;
    a.hids = d.hids;
    a.F = (R*)d.F;
    a.U = (const R*)d.u;
    a.mark = d.mark;
    a.ctl = d.ctl;
    a.red = d.red;
    a.det = (DetRec<R>*)d.det;
    a.pbox = d.pbox;
    a.wcap = patch_window_nodes(sizeof(R) == 8 ? IBM_LB_F64 : IBM_LB_F32);
    return a;
}

static IndArgs ind_args(const Geom& g, const DevPtrs& d) {
    return IndArgs{d.ptris, d.ptstart, (unsigned*)d.ind, d.ind_lines, d.ind_lines + (long long)g.Ly * g.Lz,
                   &d.ctl->flags};
}

hipError_t patch_setup(int storage) {
    const int lds = (int)dyn_lds(storage);
    hipError_t e;
    const int lds_s = (int)dyn_lds_spread();
    if (storage == IBM_LB_F64) {
        e = hipFuncSetAttribute((const void*)k_fs_patch<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_s);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_fs_patch_ind<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    lds_s);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_fs_batch<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_s);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_interp_patch<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_interp_batch<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    lds);
    } else {
        e = hipFuncSetAttribute((const void*)k_fs_patch<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_s);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_fs_patch_ind<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    lds_s);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_fs_batch<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_s);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_interp_patch<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_interp_batch<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    lds);
    }
    return e;
}

template <class R>
static hipError_t launch_step_t(const Geom& g, const DevPtrs& d, int nv, double sigma, const SmoothParams& sp,
                                hipStream_t s, size_t lds, hipEvent_t done, bool hc_split) {
    IbArgs<R> a = make_args<R>(g, d, nv, sigma, sp);
    const unsigned npatch = (nv + PATCH - 1) / PATCH;
    // split smoothing: its finish folded into the force kernel, or (with the
    // deterministic spreading) a launch of its own
    const int fold = hc_split && !d.det ? 1 : 0;
    hipLaunchKernelGGL(k_interp_patch<R>, dim3(npatch), dim3(IBT), lds, s, a, fold);
    const V4<R>* final_pos = sp.max_iter > 0 ? a.qa : a.o;
    hipLaunchKernelGGL(k_hc_fused<R>, dim3(npatch), dim3(IBT), 0, s, a, (int)npatch, hc_split ? 1 : 0);
    if (hc_split && !fold) hipLaunchKernelGGL(k_hc_finish<R>, dim3(1), dim3(1024), 0, s, a);
    // the stop event of the last launch before the next lattice kernel
    hipEvent_t fs_done = d.det ? nullptr : done;
    if (d.ind)
        hipExtLaunchKernelGGL(k_fs_patch_ind<R>, dim3(npatch), dim3(IBT), uint32_t(dyn_lds_spread()), s, nullptr,
                              fs_done, 0, a, final_pos, 1, ind_args(g, d), fold, (int)npatch);
    else
        hipExtLaunchKernelGGL(k_fs_patch<R>, dim3(npatch), dim3(IBT), uint32_t(dyn_lds_spread()), s, nullptr,
                              fs_done, 0, a, final_pos, 1, fold, (int)npatch);
    if (d.det)
        hipExtLaunchKernelGGL(k_spread_det<R>, dim3(g.TX * g.TY * g.TZ * DET_SLICES), dim3(64), 0, s, nullptr, done,
                              0, a, (int)npatch);
    return hipGetLastError();
}

size_t ib_args_bytes(int storage) { return storage == IBM_LB_F64 ? sizeof(IbArgs<double>) : sizeof(IbArgs<float>); }

void fill_ib_args(int storage, const Geom& g, const DevPtrs& d, int nv, double sigma, const SmoothParams& sp,
                  void* out) {
    if (storage == IBM_LB_F64) *(IbArgs<double>*)out = make_args<double>(g, d, nv, sigma, sp);
    else *(IbArgs<float>*)out = make_args<float>(g, d, nv, sigma, sp);
}

template <class R>
static hipError_t batch_step_t(const void* args, const int2* map, int npatch_total, int ndrop, hipStream_t s) {
    if (npatch_total == 0) return hipSuccess;  // no member carries a droplet
    const IbArgs<R>* a = (const IbArgs<R>*)args;
    hipLaunchKernelGGL(k_interp_batch<R>, dim3(npatch_total), dim3(IBT), dyn_lds(sizeof(R) == 8 ? IBM_LB_F64 : IBM_LB_F32),
                       s, a, map);
    hipLaunchKernelGGL(k_hc_fused_batch<R>, dim3(npatch_total), dim3(IBT), 0, s, a, map);
    hipLaunchKernelGGL(k_hc_finish_batch<R>, dim3(ndrop), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_fs_batch<R>, dim3(npatch_total), dim3(IBT), dyn_lds_spread(), s, a, map, 1);
    return hipGetLastError();
}

hipError_t launch_ib_step_batch(int storage, const void* args, const int2* map, int npatch_total, int ndrop,
                                hipStream_t s) {
    if (storage == IBM_LB_F64) return batch_step_t<double>(args, map, npatch_total, ndrop, s);
    return batch_step_t<float>(args, map, npatch_total, ndrop, s);
}

hipError_t launch_ib_pre_batch(int storage, const void* args, const int2* map, int npatch_total, hipStream_t s) {
    if (npatch_total == 0) return hipSuccess;
    if (storage == IBM_LB_F64)
        hipLaunchKernelGGL(k_fs_batch<double>, dim3(npatch_total), dim3(IBT), dyn_lds_spread(), s,
                           (const IbArgs<double>*)args, map, 0);
    else
        hipLaunchKernelGGL(k_fs_batch<float>, dim3(npatch_total), dim3(IBT), dyn_lds_spread(), s,
                           (const IbArgs<float>*)args, map, 0);
    return hipGetLastError();
}

hipError_t launch_ib_pre(int storage, const Geom& g, const DevPtrs& d, int nv, double sigma,
                         const SmoothParams& sp, hipStream_t s) {
    const unsigned npatch = (nv + PATCH - 1) / PATCH;
    const size_t lds = dyn_lds_spread();
    if (storage == IBM_LB_F64) {
        IbArgs<double> a = make_args<double>(g, d, nv, sigma, sp);
        if (d.ind)
            hipLaunchKernelGGL(k_fs_patch_ind<double>, dim3(npatch), dim3(IBT), lds, s, a, (const V4<double>*)a.r, 0,
                               ind_args(g, d), 0, (int)npatch);
        else
            hipLaunchKernelGGL(k_fs_patch<double>, dim3(npatch), dim3(IBT), lds, s, a, (const V4<double>*)a.r, 0, 0,
                               (int)npatch);
        if (d.det)
            hipLaunchKernelGGL(k_spread_det<double>, dim3(g.TX * g.TY * g.TZ * DET_SLICES), dim3(64), 0, s, a,
                               (int)npatch);
    } else {
        IbArgs<float> a = make_args<float>(g, d, nv, sigma, sp);
        if (d.ind)
            hipLaunchKernelGGL(k_fs_patch_ind<float>, dim3(npatch), dim3(IBT), lds, s, a, (const V4<float>*)a.r, 0,
                               ind_args(g, d), 0, (int)npatch);
        else
            hipLaunchKernelGGL(k_fs_patch<float>, dim3(npatch), dim3(IBT), lds, s, a, (const V4<float>*)a.r, 0, 0,
                               (int)npatch);
        if (d.det)
            hipLaunchKernelGGL(k_spread_det<float>, dim3(g.TX * g.TY * g.TZ * DET_SLICES), dim3(64), 0, s, a,
                               (int)npatch);
    }
    return hipGetLastError();
}

hipError_t launch_ib_step(int storage, const Geom& g, const DevPtrs& d, int nv, double sigma,
                          const SmoothParams& sp, hipStream_t s, hipEvent_t done, bool hc_split) {
    const size_t lds = dyn_lds(storage);
    if (storage == IBM_LB_F64) return launch_step_t<double>(g, d, nv, sigma, sp, s, lds, done, hc_split);
    return launch_step_t<float>(g, d, nv, sigma, sp, s, lds, done, hc_split);
}

}  // namespace ibmlb
