// Inside/outside indicator of the droplet on the lattice, for a viscosity
// ratio chi != 1 (Sec. 2: the droplet phase has viscosity chi mu, so by
// Eq. tau_to_nu the nodes inside the surface relax with
// tau_in = 1/2 + chi (tau - 1/2)).
//
// Built after every step from the committed mesh, by parity along x-rows:
//   k_ind_cross  one thread per triangle: for every lattice row (y, z) whose
//                point lies in the triangle's (y, z) projection, the crossing
//                x* of the row with the triangle toggles bit 1 of the byte of
//                the first node at or beyond x* (32-bit atomic XOR on the
//                containing word) and widens the row's [lo, hi] node range;
//   k_ind_scan   one thread per row: a running XOR of the toggles over
//                [lo, hi] leaves bit 0 = inside (an odd number of crossings at
//                or before the node) and clears the toggles and the range.
// The lattice kernel reads bit 0 and clears the byte, so between steps the
// array holds exactly the indicator of the current mesh.
//
// Robustness of the parity count: the point-in-projection test evaluates
// each edge function on the edge's endpoints taken in ascending vertex
// order, so the two triangles of an edge see exactly opposite values; an
// exact zero is decided by the sign the function takes on the row moved by
// (eps, eps^2), eps -> 0+ (symbolic perturbation, Edelsbrunner and Muecke
// 1990). Every row then crosses a closed surface an even number of times,
// also through edges and vertices, and a node's parity equals its winding
// number modulo 2.
#include <hip/hip_ext.h>
#include <limits.h>

#include "ibmlb_internal.h"

namespace ibmlb {

constexpr int IND_LINE_EMPTY = 0x7f7f7f7f;  // also the byte pattern 0x7f of a fresh range

// Sign of the edge function of the directed edge lo -> hi at the row point
// (Y, Z) moved by (eps, eps^2): e = dy (Z - lo.z) - dz (Y - lo.y), then the
// coefficients -dz of eps and dy of eps^2. No contraction: the products must
// round the same way for every triangle of the edge.
__device__ inline int edge_sign(double ly, double lz, double hy, double hz, double Y, double Z) {
#pragma clang fp contract(off)
    const double dy = hy - ly, dz = hz - lz;
    const double p1 = dy * (Z - lz);
    const double p2 = dz * (Y - ly);
    const double e = p1 - p2;
    if (e != 0.0) return e > 0.0 ? 1 : -1;
    if (dz != 0.0) return dz < 0.0 ? 1 : -1;
    return dy > 0.0 ? 1 : (dy < 0.0 ? -1 : 0);
}

__device__ inline double edge_value(double ly, double lz, double hy, double hz, double Y, double Z) {
#pragma clang fp contract(off)
    const double p1 = (hy - ly) * (Z - lz);
    const double p2 = (hz - lz) * (Y - ly);
    return p1 - p2;
}

// Oriented edge a -> b (ids ia, ib) through its canonical direction.
__device__ inline void oriented_edge(int ia, double ay, double az, int ib, double by, double bz, double Y, double Z,
                                     int* s, double* v) {
    if (ia < ib) {
        *s = edge_sign(ay, az, by, bz, Y, Z);
        *v = edge_value(ay, az, by, bz, Y, Z);
    } else {
        *s = -edge_sign(by, bz, ay, az, Y, Z);
        *v = -edge_value(by, bz, ay, az, Y, Z);
    }
}

__device__ inline int clamp_floor(double v, int lo, int hi) {
    const double f = floor(v);
    return f < lo ? lo : (f > hi ? hi : int(f));
}

__device__ inline int clamp_ceil(double v, int lo, int hi) {
    const double c = ceil(v);
    return c < lo ? lo : (c > hi ? hi : int(c));
}

template <class R>
__global__ __launch_bounds__(64) void k_ind_cross(Geom g, const V4<R>* __restrict__ r,
                                                   const int4* __restrict__ tris, int nt, unsigned* ind_words,
                                                   int* line_lo, int* line_hi) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int4 tv = tris[t];
    const int id[3] = {tv.x, tv.y, tv.z};
    double P[3][3];
    for (int k = 0; k < 3; ++k) {
        const V4<R> p = r[id[k]];
        P[k][0] = double(p.x) + (g.xci[0] + g.xcf[0]);
        P[k][1] = double(p.y) + (g.xci[1] + g.xcf[1]);
        P[k][2] = double(p.z) + (g.xci[2] + g.xcf[2]);
        for (int a = 0; a < 3; ++a)
            if (!(fabs(P[k][a]) < 1e9)) return;  // non-finite positions are reported by the IB kernels
    }
    const double ymin = fmin(P[0][1], fmin(P[1][1], P[2][1])), ymax = fmax(P[0][1], fmax(P[1][1], P[2][1]));
    const double zmin = fmin(P[0][2], fmin(P[1][2], P[2][2])), zmax = fmax(P[0][2], fmax(P[1][2], P[2][2]));
    // rows on the projection's boundary count too (the perturbation decides)
    const int y0 = clamp_ceil(ymin, 0, g.Ly), y1 = clamp_floor(ymax, -1, g.Ly - 1);
    const int z0 = clamp_ceil(zmin, 0, g.Lz), z1 = clamp_floor(zmax, -1, g.Lz - 1);
    for (int Zi = z0; Zi <= z1; ++Zi)
        for (int Yi = y0; Yi <= y1; ++Yi) {
            const double Y = Yi, Z = Zi;
            int s01, s12, s20;
            double e01, e12, e20;
            oriented_edge(id[0], P[0][1], P[0][2], id[1], P[1][1], P[1][2], Y, Z, &s01, &e01);
            oriented_edge(id[1], P[1][1], P[1][2], id[2], P[2][1], P[2][2], Y, Z, &s12, &e12);
            oriented_edge(id[2], P[2][1], P[2][2], id[0], P[0][1], P[0][2], Y, Z, &s20, &e20);
            if (s01 == 0 || s01 != s12 || s12 != s20) continue;
            const double sum = e01 + e12 + e20;
            if (sum == 0.0) continue;  // projection of zero area
            // barycentric weight of a vertex: the edge function of the opposite edge
            const double xs = (e12 * P[0][0] + e20 * P[1][0] + e01 * P[2][0]) / sum;
            if (!(fabs(xs) < 1e9)) continue;
            const double cx = ceil(xs);
            if (cx > g.Lx - 1) continue;  // no node at or beyond the crossing
            const int X0 = cx < 0.0 ? 0 : int(cx);
            const int line = Yi + g.Ly * Zi;
            const long long n = (long long)line * g.Lx + X0;
            atomicXor(ind_words + (n >> 2), 2u << (8 * int(n & 3)));
            atomicMin(line_lo + line, X0);
            atomicMax(line_hi + line, X0);
        }
}

__global__ __launch_bounds__(256) void k_ind_scan(Geom g, unsigned char* ind, int* line_lo, int* line_hi) {
    const int line = blockIdx.x * blockDim.x + threadIdx.x;
    if (line >= g.Ly * g.Lz) return;
    const int lo = line_lo[line], hi = line_hi[line];
    if (lo > hi) return;
    // The walk is latency-bound: the row's bytes are read as aligned 32-bit
    // words of the whole array, eight per round trip (a word may hold bytes of
    // a neighbouring row, which are read but never written here); the bytes of
    // this row are then rewritten one by one.
    const long long n0 = (long long)line * g.Lx + lo, n1 = (long long)line * g.Lx + hi;
    const unsigned* words = reinterpret_cast<const unsigned*>(ind);
    unsigned par = 0;
    for (long long w0 = n0 >> 2; w0 <= (n1 >> 2); w0 += 8) {
        unsigned wv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) wv[k] = w0 + k <= (n1 >> 2) ? words[w0 + k] : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const long long n = 4 * (w0 + k) + b;
                if (n >= n0 && n <= n1) {
                    par ^= (wv[k] >> (8 * b + 1)) & 1u;
                    ind[n] = (unsigned char)par;
                }
            }
    }
    line_lo[line] = IND_LINE_EMPTY;
    line_hi[line] = -1;
}

// One wave per work-group for the triangles: a 20k-triangle mesh spreads over
// 320 work-groups instead of 80, so that the latency-bound threads run on
// every compute unit.
constexpr int IND_TB = 64;

hipError_t launch_indicator(int storage, const Geom& g, const DevPtrs& d, int nt, hipStream_t s, hipEvent_t done) {
    const unsigned nb = unsigned((nt + IND_TB - 1) / IND_TB);
    int* lo = d.ind_lines;
    int* hi = d.ind_lines + (long long)g.Ly * g.Lz;
    if (storage == IBM_LB_F64)
        hipLaunchKernelGGL(k_ind_cross<double>, dim3(nb), dim3(IND_TB), 0, s, g, (const V4<double>*)d.r, d.tris, nt,
                           (unsigned*)d.ind, lo, hi);
    else
        hipLaunchKernelGGL(k_ind_cross<float>, dim3(nb), dim3(IND_TB), 0, s, g, (const V4<float>*)d.r, d.tris, nt,
                           (unsigned*)d.ind, lo, hi);
    const unsigned nl = unsigned(((long long)g.Ly * g.Lz + 255) / 256);
    hipExtLaunchKernelGGL(k_ind_scan, dim3(nl), dim3(256), 0, s, nullptr, done, 0, g, d.ind, lo, hi);
    return hipGetLastError();
}

hipError_t launch_indicator_clear(const Geom& g, const DevPtrs& d, hipStream_t s) {
    hipError_t e = hipMemsetAsync(d.ind, 0, ind_bytes(g), s);
    if (e == hipSuccess) e = hipMemsetAsync(d.ind_lines, 0x7f, sizeof(int) * (size_t)g.Ly * g.Lz, s);
    if (e == hipSuccess)
        e = hipMemsetAsync(d.ind_lines + (long long)g.Ly * g.Lz, 0xff, sizeof(int) * (size_t)g.Ly * g.Lz, s);
    return e;
}

}  // namespace ibmlb
