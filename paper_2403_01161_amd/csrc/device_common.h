// Device helpers shared by the lattice and immersed-boundary kernels.
#pragma once

#include <math.h>

#include "ibmlb_internal.h"

namespace ibmlb {

__device__ inline int wrap(int j, int L) { return j < 0 ? j + L : (j >= L ? j - L : j); }

// Peskin 4-point weights of the four nodes floor(s)-1 .. floor(s)+2 for a
// coordinate with fractional part f in [0, 1). The four stencil arguments
// 1+f, f, 1-f, 2-f share the radicand 1 + 4f - 4f^2 of the two branches of
// phi(x) (Sec. 3.1), so one square root serves the whole axis.
template <class R>
__device__ inline void peskin4(R f, R w[4]) {
    R q = sqrt(R(1) + R(4) * f - R(4) * f * f);
    w[0] = (R(3) - R(2) * f - q) * R(0.125);
    w[1] = (R(3) - R(2) * f + q) * R(0.125);
    w[2] = (R(1) + R(2) * f + q) * R(0.125);
    w[3] = (R(1) + R(2) * f - q) * R(0.125);
}

// Stencil of one axis for a coordinate `rel` relative to the box centre:
// the unwrapped absolute index of the first stencil node (floor - 1) and the
// fractional part. False if the coordinate is not finite (or absurdly large)
// or the stencil leaves a wall axis.
template <class R>
__device__ inline bool stencil_base(R rel, int xci, double xcf, int L, int periodic, int* first,
                                    R* frac) {
    R s = rel + R(xcf);
    if (!(fabs(s) < R(1e7))) return false;
    R fl = floor(s);
    *frac = s - fl;
    int b = int(fl) + xci - 1;
    *first = b;
    return periodic || (b >= 0 && b + 3 <= L - 1);
}

// Wrap an unwrapped node index into 0..L-1 (any distance).
__device__ inline int wrap_any(int j, int L) {
    int m = j % L;
    return m < 0 ? m + L : m;
}

// Node index of unwrapped lattice coordinates (periodic images folded in).
__device__ inline long long node_index(const Geom& g, int x, int y, int z) {
    return wrap_any(x, g.Lx) + (long long)g.Lx * (wrap_any(y, g.Ly) + (long long)g.Ly * wrap_any(z, g.Lz));
}

constexpr int MAXV = 15;  // valence capacity of a fan

// ---------------------------------------------------------------- topology
// Valence and neighbours of vertex k (unused slots are -1).
// Whole four-component record load and store through a generic or a
// global-address-space pointer (records in the global space cannot use the
// class's generic copy operations).
template <class T, class P>
__device__ __forceinline__ T ld4(P p) {
    return T{p->x, p->y, p->z, p->w};
}
template <class P, class T>
__device__ __forceinline__ void st4(P p, const T& v) {
    p->x = v.x;
    p->y = v.y;
    p->z = v.z;
    p->w = v.w;
}

template <class P>
__device__ inline int load_fan(P fan, int k, int nb[MAXV]) {
    const int4 a = ld4<int4>(fan + 4 * k), b = ld4<int4>(fan + 4 * k + 1);
    nb[0] = a.y; nb[1] = a.z; nb[2] = a.w;
    nb[3] = b.x; nb[4] = b.y; nb[5] = b.z; nb[6] = b.w;
    if (a.x > 7) {
        const int4 c = ld4<int4>(fan + 4 * k + 2), d = ld4<int4>(fan + 4 * k + 3);
        nb[7] = c.x; nb[8] = c.y; nb[9] = c.z; nb[10] = c.w;
        nb[11] = d.x; nb[12] = d.y; nb[13] = d.z; nb[14] = d.w;
    } else {
#pragma unroll
        for (int j = 7; j < MAXV; ++j) nb[j] = -1;
    }
    return a.x;
}

template <class T>
__device__ inline T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

}  // namespace ibmlb
