// Inside/outside indicator of the droplet on the lattice, for a viscosity
// ratio chi != 1 (Sec. 2: the droplet phase has viscosity chi mu, so by
// Eq. tau_to_nu the nodes inside the surface relax with
// tau_in = 1/2 + chi (tau - 1/2)).
//
// Built after every step from the committed mesh, by parity along x-rows:
//   the force kernel (k_fs_patch) toggles, for every triangle, the byte of
//   the first node at or beyond each row crossing (indicator_common.h);
//   k_ind_scan   one thread per row: a running XOR of the toggles over the
//                row's [lo, hi] range leaves bit 0 = inside (an odd number of
//                crossings at or before the node) and clears the toggles and
//                the range.
// The lattice kernel reads bit 0 in the marked tiles (the scan marks every
// tile with an inside node) and clears the byte, so between steps the array
// holds exactly the indicator of the current mesh.
#include <hip/hip_ext.h>

#include "indicator_common.h"

namespace ibmlb {

// Every tile that holds an inside node is marked for the step (mark[tile] =
// epoch, as the spreading marks the tiles its stencils touch): the lattice
// kernel reads the indicator in marked tiles only.
__global__ __launch_bounds__(256) void k_ind_scan(Geom g, unsigned char* ind, int* line_lo, int* line_hi, int* mark,
                                                  const Ctl* ctl) {
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
    const int y = line % g.Ly, z = line / g.Ly;
    const int trow = g.TX * ((y >> TILE_SHIFT) + g.TY * (z >> TILE_SHIFT));
    int in0 = g.Lx, in1 = -1;  // first and last inside node of the row
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
                    const int x = int(n - (long long)line * g.Lx);
                    in0 = par ? min(in0, x) : in0;
                    in1 = par ? x : in1;
                }
            }
    }
    // the tiles from the first to the last inside node (a gap between two
    // inside runs of a row marks a tile more, which is harmless)
    if (in1 >= 0) {
        const int ep = ctl->epoch;
        for (int tx = in0 >> TILE_SHIFT; tx <= (in1 >> TILE_SHIFT); ++tx) mark[trow + tx] = ep;
    }
    line_lo[line] = IND_LINE_EMPTY;
    line_hi[line] = -1;
}

hipError_t launch_indicator_scan(const Geom& g, const DevPtrs& d, hipStream_t s, hipEvent_t done) {
    const unsigned nl = unsigned(((long long)g.Ly * g.Lz + 255) / 256);
    hipExtLaunchKernelGGL(k_ind_scan, dim3(nl), dim3(256), 0, s, nullptr, done, 0, g, d.ind, d.ind_lines,
                          d.ind_lines + (long long)g.Ly * g.Lz, d.mark, (const Ctl*)d.ctl);
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
