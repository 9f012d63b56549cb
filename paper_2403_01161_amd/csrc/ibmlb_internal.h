// Internal declarations shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ibm_lb.h"

namespace ibmlb {

// Device-side sticky flags (bit set by any thread that sees the condition).
enum : int {
    DFLAG_DOMAIN = 1,
    DFLAG_NONFINITE = 2,
};

// IB tiles: 8x8x8 lattice nodes. A tile is "marked" for a step when some
// vertex stencil touches it; only marked tiles carry force and velocity.
constexpr int TILE_SHIFT = 3;

// Positions on the GPU are stored relative to the box centre x_c so that
// FP32 keeps the resolution of the droplet scale, not of the box scale.
template <class R>
struct alignas(4 * sizeof(R)) V4 {
    R x, y, z, w;
};

// Geometry of one lattice as kernels see it.
struct Geom {
    int Lx, Ly, Lz;
    int px, py, pz;          // periodic flags
    int TX, TY, TZ;          // tile grid
    long long N;             // nodes
    int xci[3];              // floor(x_c)
    double xcf[3];           // x_c - floor(x_c), 0 or 0.5
};

struct LatticeParams {
    double omega;            // 1/tau
    double kguo;             // 1 - 1/(2 tau)
    double rho0;
    double tau;
    float scale, inv_scale;  // 16-bit deviation scaling
};

// Rates of the MRT collision, one per moment of the basis in lattice_common.h
// (the shear moments at 1/tau).
struct MrtRates {
    double s[19];
};

struct SmoothParams {
    double alpha, gamma, tol;
    int max_iter, sign;
};

// Control block in device memory.
struct Ctl {
    int epoch;               // step epoch used by tile marks
    int flags;               // DFLAG_*
    int iters;               // smoothing iterations of the last step
    int cap_hits;            // steps that hit the smoothing cap since last read
    int pad[60];
};

// Device pointers of one droplet system (types erased; real is double for
// IBM_LB_F64, float otherwise).
struct DevPtrs {
    void* f[2];              // populations [19][N] in the storage type
    void* F;                 // force density [3][N] (real)
    void* u;                 // velocity [3][N] (real), valid in marked tiles
    int* mark;               // [TX*TY*TZ]
    Ctl* ctl;
    void* r;                 // V4<real> [nv] current positions (relative to x_c)
    void* o;                 // V4 [nv] after the Euler move
    void* qa;                // V4 [nv] smoothing scratch
    void* qb;
    void* pp;
    void* bb;
    int4* tris;              // [nt]
    int4* fan;               // [nv][4]: valence, then the ordered one-ring (15 slots)
    int4* lfan;              // [nv][4]: the same fan in patch-local slots (own vertices, then the halo)
    int* hstart;             // [npatch + 1] halo offsets of each IB_PATCH-vertex patch
    int* hids;               // halo vertices (outside the patch, in some ring of it), per patch ascending
    double* obs_part;        // [OBS_BLOCKS][16]
    double* mass_part;       // [MASS_BLOCKS][4]
    double* obs_out;         // [48] final observables
    double* Abuf;            // [ACAP][9] gradient rows
    unsigned long long* red; // [RED_SLOTS + 1] grid-wide max |p - q| (spread over slots), arrival count
    unsigned char* ind;      // [N rounded up to 4] inside indicator (viscosity ratio only)
    int* ind_lines;          // [2][Ly Lz] node range of each x-row's crossings (viscosity ratio only)
    int4* ptris;             // [nt] triangles grouped by the patch of their lowest vertex (viscosity ratio only)
    int* ptstart;            // [npatch + 1] start of each patch's triangles (viscosity ratio only)
    int* perm;               // [nv] caller index of each internal vertex
    void* det;               // [nv] staged stencils of the deterministic spreading, or null
    int* pbox;               // [npatch][8] patch windows of the deterministic spreading
};

// Bytes of the indicator array (whole 32-bit words, for the atomic toggles).
inline size_t ind_bytes(const Geom& g) { return ((size_t)g.N + 3) / 4 * 4; }

// Relaxation inside the droplet for a viscosity ratio chi != 1:
// tau_in = 1/2 + chi (tau - 1/2).
struct ChiRates {
    double omega_in;         // 1/tau_in
    double kguo_in;          // 1 - 1/(2 tau_in)
};

// One ensemble member as the batched lattice kernel sees it. A points at the
// member's gradient rows; a launch reads the row at A + `step` (an offset in
// doubles that selects the staging half and the step).
struct LatDesc {
    Geom g;
    LatticeParams lp;
    void* f[2];
    void* F;
    void* u;
    int* mark;
    Ctl* ctl;
    const double* A;
    const double* mrt;       // [19] the member's MRT rates, or null (BGK)
};

// Vertices per surface patch: the set-up renumbering makes every run of
// IB_PATCH consecutive vertices spatially compact; the patch-organised IB
// kernels give one work-group to one patch.
constexpr int IB_PATCH = 64;

// Slots of the smoothing's grid-wide maximum: work-group p folds its value
// into slot p mod RED_SLOTS (device-scope atomics on one address serialise,
// and a step has up to thousands of work-groups); readers take the maximum of
// all slots. Slot RED_SLOTS counts arrivals.
constexpr int RED_SLOTS = 64;

constexpr int OBS_BLOCKS = 128;
constexpr int MASS_BLOCKS = 512;
constexpr int ACAP = 4096;
constexpr int OBS_OUT_N = 48;

// Kernel launchers (kernels.hip). All enqueue on `s` and return the
// hipError_t of the launch.
hipError_t launch_init(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d,
                       const double* A0, int rest, hipStream_t s);
// Lattice-kernel variant: bit 0 = non-temporal population loads; bits 1-2 =
// work-group size LAT_BS[(variant >> 1) & 3] (rows layout: the least number
// of whole x-rows, at least one, that fits in it); bit 4 (VAR_ROWS) = row
// layout; bit 3 (VAR_X) = XCD-grouped block order in the linear layout,
// non-temporal population stores in the row layout.
constexpr int LATTICE_VARIANTS = 32;
constexpr int LAT_BS[4] = {128, 256, 512, 64};
constexpr int VAR_X = 8;
constexpr int VAR_ROWS = 16;
// Step variant = lattice variant (bits 0-4) + bit 5 (VAR_HC_SPLIT): the
// smoothing's finish split from its first launch, folded into the force
// kernel (single droplets; with deterministic spreading, and always for
// ensembles, a launch of its own).
constexpr int VAR_HC_SPLIT = 32;
// Bit 6 (VAR_AA): one population copy updated in place, even and odd steps
// alternating (linear layout only).
constexpr int VAR_AA = 64;
constexpr int STEP_VARIANTS = 128;
// Rows per work-group of a row-layout variant for rows of Lx nodes; 0 when
// the variant is not a row layout or Lx exceeds the largest work-group.
int lattice_rows_per_block(int variant, int Lx);
// Whether the variant can run on this lattice.
int lattice_variant_ok(int variant, const Geom& g);
// e0/e1 (may be null): events stamped at the start and at the completion of
// the dispatch.
// parity: for an in-place variant, 0 for the even step, 1 for the odd one.
// mrt (may be null): MRT collision with these rates instead of BGK (any
// layout).
// chi (may be null): nodes whose indicator byte d.ind is set relax with
// these rates; the byte is cleared (BGK, two copies, linear or row layout).
hipError_t launch_lattice(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d,
                          int cur, bool ib, const double* A_row, int variant, int parity, hipStream_t s,
                          hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, const MrtRates* mrt = nullptr,
                          const ChiRates* chi = nullptr);
// Second half of the indicator: the running parity over each x-row of the
// toggles that the force kernel left (d.ind non-null makes the force kernel
// cross the mesh with the rows; d.ind must hold zeros and empty row ranges
// before it); done (may be null) is stamped at completion.
hipError_t launch_indicator_scan(const Geom& g, const DevPtrs& d, hipStream_t s, hipEvent_t done);
// Zero the indicator and empty every row range (not for graph capture).
hipError_t launch_indicator_clear(const Geom& g, const DevPtrs& d, hipStream_t s);
// After an even in-place step: f[cur] back to natural order, in place.
hipError_t launch_aa_settle(int storage, const Geom& g, const DevPtrs& d, int cur, hipStream_t s);
hipError_t launch_bump_epoch(const DevPtrs& d, hipStream_t s);
// Wet-node velocity walls on the streamed populations f[cur] (natural order)
// with the gradient row A_row.
hipError_t launch_wet_walls(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur,
                            const double* A_row, hipStream_t s);
// Face nodes of the non-periodic axes (the wet-node walls' work).
long long wall_node_count(const Geom& g);
// Ensemble form: map [nblocks] entries {member, block of 256 face nodes}, the
// members' lattice launch having read copy cur (the walls act on cur ^ 1)
// with gradient rows at desc[i].A + arow.
hipError_t launch_wet_walls_batch(int storage, const LatDesc* desc, const int2* map, int nblocks, int cur,
                                  long long arow, hipStream_t s);
// maps: eight block maps, concatenated (table q from entry moff[q],
// nblocks[q] entries; entry b = {member, block index within the member}).
// Tables 0-3: linear layout with LAT_BS[q]-node blocks; tables 4-7: row
// layout with work-groups of LAT_BS[q - 4] threads, each member taking
// floor(LAT_BS[q - 4] / Lx) whole rows per block (nblocks[q] = -1 when a
// member's rows exceed that size). The first nib[q] entries of table q
// belong to members with a droplet, the rest to members without: two
// launches, each compiled for one kind.
// mrt: every member runs the MRT collision with the rates desc[i].mrt.
hipError_t launch_lattice_batch(int storage, const LatDesc* desc, const int2* maps, const int moff[8],
                                const int nblocks[8], const int nib[8], int cur, long long step, int variant,
                                bool mrt, hipStream_t s);
// desc[i].A = base + i * stride for the n members (on the stream).
hipError_t launch_set_rows(LatDesc* desc, int n, const double* base, long long stride, hipStream_t s);
hipError_t launch_moments(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d,
                          int cur, bool ib, double* rho_out, double* u_out, hipStream_t s);
hipError_t launch_observables(int storage, const Geom& g, const LatticeParams& lp,
                              const DevPtrs& d, int cur, int nv, int nt, double radius,
                              const double* A_row, hipStream_t s);
hipError_t launch_positions_to_abs(int storage, const Geom& g, const DevPtrs& d, int nv,
                                   double* out, hipStream_t s);
hipError_t launch_positions_from_abs(int storage, const Geom& g, const DevPtrs& d, int nv,
                                     const double* in, hipStream_t s);

// Patch-organised IB kernels (ib_patch.hip). patch_setup raises the dynamic
// LDS limit of the patch kernels. launch_ib_pre spreads the forces of the
// current mesh; launch_ib_step runs the IB half of one step (interpolation,
// Euler move, smoothing, next forces and spreading); `done` (may be null) is
// stamped when its last kernel completes. hc_split: the smoothing's finish
// runs as a launch of its own instead of in the last work-group to arrive.
hipError_t patch_setup(int storage);
int patch_window_nodes(int storage);
// Bytes of one vertex's staged stencil for the deterministic spreading.
size_t det_rec_bytes(int storage);
hipError_t launch_ib_pre(int storage, const Geom& g, const DevPtrs& d, int nv, double sigma,
                         const SmoothParams& sp, hipStream_t s);
hipError_t launch_ib_step(int storage, const Geom& g, const DevPtrs& d, int nv, double sigma,
                          const SmoothParams& sp, hipStream_t s, hipEvent_t done = nullptr,
                          bool hc_split = false);
// Ensemble forms: args is a device array of per-member IB argument records
// (ib_args_bytes each, filled by fill_ib_args), map the patch map
// [npatch_total] (entry b = {member, patch index within the member}).
size_t ib_args_bytes(int storage);
void fill_ib_args(int storage, const Geom& g, const DevPtrs& d, int nv, double sigma, const SmoothParams& sp,
                  void* out);
hipError_t launch_ib_pre_batch(int storage, const void* args, const int2* map, int npatch_total, hipStream_t s);
hipError_t launch_ib_step_batch(int storage, const void* args, const int2* map, int npatch_total, int ndrop,
                                hipStream_t s);
hipError_t launch_clear_force(int storage, const Geom& g, const DevPtrs& d, hipStream_t s);

size_t storage_bytes(int storage);
size_t real_bytes(int storage);

// ---------------------------------------------------------------- adjoint (adjoint.hip)
// Forward quantities of one step recorded for the adjoint (FP64).
struct AdjStep {
    double* rho;             // [N]
    double* u;               // [3][N], with F/2
    double* F;               // [3][N]
    double4* pos;            // [nv] positions at the start of the step (relative to x_c)
};

// Per-vertex adjoint work arrays (FP64, [nv] each).
struct AdjVerts {
    double4* rb;             // adjoint of the positions (current step boundary)
    double4* P;              // HC transpose: incoming adjoint of the iterate
    double4* PS;             // P / valence
    double4* Pp;             // adjoint of p'
    double4* PpS;            // Pp / valence
    double4* Ob;             // adjoint of o (= of U)
    double4* Qp;             // partial adjoint of q
    double4* phib;           // adjoint of the nodal forces
    double4* rt;             // adjoint of the positions before the force term
};

hipError_t launch_adj_record(int storage, const Geom& g, const LatticeParams& lp, const DevPtrs& d, int cur,
                             int nv, const AdjStep& st, int* prev_iters, hipStream_t s);
hipError_t launch_adj_record_iters(const DevPtrs& d, int* slot, hipStream_t s);
// The transposed smoothing of a step with `iters` iterations, up to the last
// iteration's pass b, which launch_adj_ib_spread (given the same `iters`)
// runs ahead of the transposed interpolation; with iters = 0 it takes obar =
// rbar there.
hipError_t launch_adj_hc(int nv, const int4* fan, const SmoothParams& sp, int iters, const AdjVerts& v,
                         hipStream_t s);
hipError_t launch_adj_ib_spread(const Geom& g, int nv, const int4* fan, double alpha, int iters, const double4* pos,
                                const AdjVerts& v, double* ubar, hipStream_t s);
int adj_lattice_blocks(long long N);
int adj_vertex_blocks(int nv);
hipError_t launch_adj_lattice(const Geom& g, const LatticeParams& lp, const double* fbin, double* fbout,
                              const AdjStep& st, double* ubar, double* Fbar, double* Apart, hipStream_t s);
hipError_t launch_adj_ib_back(const Geom& g, int nv, const int4* fan, double sigma, const AdjStep& st,
                              const double* Fbar, const AdjVerts& v, double* spart, hipStream_t s);
hipError_t launch_adj_reduce(int nsteps, int nbl, const double* Apart, int nbv, const double* spart, double* dA,
                             double* dsigma, hipStream_t s);
// which: 0 J = D, 1 J = lambda_max, 2 J = beta (the mesh part; the direct
// dependence on the last gradient row is added on the host).
hipError_t launch_adj_seed(int storage, int nv, const DevPtrs& d, double* coef, double4* rb, hipStream_t s,
                           int which = 0);
hipError_t launch_adj_perm_in(int nv, const int* perm, const double* user, double4* out, hipStream_t s);
hipError_t launch_adj_perm_out(int nv, const int* perm, const double4* in, double* user, hipStream_t s);
// dJ/dA0 of the linear initial state from fbar0 [19][N]: per-block partial
// sums part[nblocks][9] (row-major a, b).
hipError_t launch_adj_init_A0(const Geom& g, const LatticeParams& lp, const double A0[9], const double* fbar,
                              double* part, int nblocks, hipStream_t s);

}  // namespace ibmlb
