// Crossings of the lattice x-rows with the droplet's triangles, the first
// half of the inside indicator for a viscosity ratio chi != 1 (Sec. 2). The
// per-triangle pass runs inside the force kernel (which already holds the
// final positions); the running parity over each row is k_ind_scan.
//
// Robustness of the parity count: the point-in-projection test evaluates
// each edge function on the edge's endpoints taken in ascending vertex
// order, so the two triangles of an edge see exactly opposite values; an
// exact zero is decided by the sign the function takes on the row moved by
// (eps, eps^2), eps -> 0+ (symbolic perturbation, Edelsbrunner and Muecke
// 1990). Every row then crosses a closed surface an even number of times,
// also through edges and vertices, and a node's parity equals its winding
// number modulo 2.
#pragma once

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

// Crossings of triangle (ids id, absolute positions P) with the lattice
// x-rows: for every row (y, z) whose point lies in the triangle's (y, z)
// projection, the crossing x* toggles bit 1 of the byte of the first node at
// or beyond x* (32-bit atomic XOR on the containing word) and widens the
// row's [lo, hi] node range. Rows on the projection's boundary count too (the
// perturbation decides).
// The rows are those of the box itself: a mesh that reaches beyond the node
// range [0, L - 1] of an axis (a periodic image would be needed) raises the
// domain flag in *flags instead.
__device__ inline void triangle_row_crossings(const Geom& g, const int id[3], const double P[3][3],
                                              unsigned* ind_words, int* line_lo, int* line_hi, int* flags) {
    const int Lax[3] = {g.Lx, g.Ly, g.Lz};
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) {
            if (!(fabs(P[k][a]) < 1e9)) return;  // non-finite positions are reported by the IB kernels
            if (P[k][a] < 0.0 || P[k][a] > Lax[a] - 1) {
                atomicOr(flags, DFLAG_DOMAIN);
                return;
            }
        }
    const double ymin = fmin(P[0][1], fmin(P[1][1], P[2][1])), ymax = fmax(P[0][1], fmax(P[1][1], P[2][1]));
    const double zmin = fmin(P[0][2], fmin(P[1][2], P[2][2])), zmax = fmax(P[0][2], fmax(P[1][2], P[2][2]));
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

}  // namespace ibmlb
