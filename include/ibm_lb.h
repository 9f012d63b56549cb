/*
 * ibm_lb.h — C-ABI of the MI355X (gfx950) IB-LB droplet library.
 *
 * One call of ibm_lb_step advances the coupled immersed-boundary /
 * lattice-Boltzmann droplet of Taglienti, Guglietta & Sbragaglia,
 * "Droplet dynamics in homogeneous isotropic turbulence with the immersed
 * boundary-lattice Boltzmann method" (arXiv 2403.01161), by whole timesteps.
 * Each timestep runs, on the GPU, in this order:
 *   1. surface-tension nodal forces of the mesh (Sec. 3.1, Eq. pi_drop),
 *      taken as phi_k = -sigma dA_surface/dr_k;
 *   2. spreading of the forces onto the lattice with the Peskin 4-point
 *      stencil (Sec. 3.1, Eq. ibm_force_d first line, stencil phi(x));
 *   3. a fused D3Q19 BGK collide with Guo forcing and push-streaming
 *      (Sec. 3.1, Eqs. LBMEQ, collision, equilibriumLB, Guo source,
 *      density_velocity_LB), with moving-wall velocity bounce-back
 *      (Eq. standard BB) imposing u = A (x - x_c) on the box faces
 *      (Sec. 2 Eq. linearized velocity; Sec. 3.1 Eq. velo_facce_cubo_da_gradiente);
 *   4. interpolation of the half-force-corrected velocity onto the mesh and
 *      the forward-Euler move (Eq. ibm_force_d second line, Eq. fwd_euler);
 *   5. extended Laplacian (HC) smoothing of the mesh (Sec. 3.3, Eqs.
 *      extended laplacian smoothing, HC_algo_full, distanceregularization).
 * Observables (Sec. 2: morphological tensor S, lambda_max, v_max, Eq. beta)
 * are FP64 reductions over the mesh computed on request.
 *
 * Conventions
 *  - Lattice nodes sit at integer coordinates 0..L[a]-1; the walls are half a
 *    spacing outside the outermost nodes; the box centre is x_c = (L-1)/2.
 *  - Gradients are row-major 3x3 doubles, A[3a+b] = d u_a / d x_b, so the
 *    imposed wall velocity is u_w = A (x_w - x_c).
 *  - Vertex coordinates crossing the ABI are absolute lattice coordinates,
 *    double [nv][3]. Triangles are int32 [nt][3], counter-clockwise seen
 *    from outside (outward normals).
 *  - Fields crossing the ABI are double, x fastest: rho [Lz][Ly][Lx],
 *    u [3][Lz][Ly][Lx].
 *  - Every function returns IBM_LB_OK (0) or a negative error code and never
 *    aborts. Work is enqueued on cfg->stream (a hipStream_t, NULL for the
 *    null stream) and is asynchronous unless stated; errors raised on the
 *    GPU (stencil outside the box, non-finite state) are sticky on the handle
 *    and returned by the next synchronising call. ibm_lb_last_error() gives a
 *    thread-local message for the last failure.
 *  - A handle is used by one host thread at a time.
 */
#ifndef IBM_LB_H
#define IBM_LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define IBM_LB_OK 0
#define IBM_LB_EINVAL (-1)     /* invalid argument or configuration */
#define IBM_LB_ENOMEM (-2)     /* device or host allocation failed, or workspace too small */
#define IBM_LB_EDEVICE (-3)    /* a HIP runtime call failed */
#define IBM_LB_EDOMAIN (-4)    /* a vertex stencil left the box across a wall */
#define IBM_LB_ENONFINITE (-5) /* non-finite or non-positive density, velocity or position */

/* ---- population storage formats (populations are stored as deviations
 * f_i - w_i rho0 from the rest equilibrium; the collision runs in FP64 for
 * IBM_LB_F64 and in FP32 for the other formats) ---- */
#define IBM_LB_F64 0
#define IBM_LB_F32 1
#define IBM_LB_F16DEV 2  /* FP16 of deviation * f16_scale (a power of two) */
#define IBM_LB_BF16DEV 3 /* BF16 of deviation */

/* ---- initial state ---- */
#define IBM_LB_INIT_LINEAR 0 /* f_eq(rho0, A0 (x - x_c)) - 3 tau w_i rho0 (c_i c_i - I/3):A0 */
#define IBM_LB_INIT_REST 1   /* f_i = w_i rho0 */

/* ---- observable flags ---- */
#define IBM_LB_OBS_DEGENERATE 1 /* lambda_1 - lambda_2 < 1e-12 radius^2: v_max, beta, theta are NaN */
#define IBM_LB_OBS_E_ZERO 2     /* ||E||_F == 0: beta is NaN */
#define IBM_LB_OBS_REG_CAP 4    /* smoothing hit reg_max_iter in a step since the last observables call */

/* ---- field selectors for ibm_lb_read_field ---- */
#define IBM_LB_FIELD_RHO 0
#define IBM_LB_FIELD_U 1

typedef struct ibm_lb ibm_lb;
typedef struct ibm_lb_batch ibm_lb_batch;

enum { IBM_LB_BGK = 0, IBM_LB_MRT = 1 };
enum { IBM_LB_WALLS_LINK = 0, IBM_LB_WALLS_WET = 1 };

typedef struct ibm_lb_config {
    int32_t L[3];          /* nodes per axis, each >= 8; at most 2^31 - 1 nodes in all */
    int32_t periodic[3];   /* per axis: 0 = moving walls, 1 = periodic */
    double tau;            /* BGK relaxation time (Eq. collision), > 0.5; nu = (tau - 1/2)/3 */
    double sigma;          /* surface tension (Eq. pi_drop), >= 0 */
    double radius;         /* rest radius R (> 0): scale of the degeneracy threshold */
    double rho0;           /* reference density (> 0, normally 1) */
    int32_t n_vertices;    /* 0 runs the lattice without a droplet */
    int32_t n_triangles;
    const double* vertices;    /* host [n_vertices][3], absolute coordinates; copied */
    const int32_t* triangles;  /* host [n_triangles][3]; copied */
    double reg_alpha;      /* smoothing alpha (Sec. 3.3; 0.1) */
    double reg_gamma;      /* smoothing gamma (0.51) */
    double reg_tol;        /* exit when max_i |x_p - x_q| < reg_tol (0.01) */
    int32_t reg_max_iter;  /* iteration cap per step (50); 0 disables smoothing */
    int32_t reg_sign;      /* +1: correction adds the neighbour mean of b (default); -1: subtracts it */
    int32_t storage;       /* IBM_LB_F64 / F32 / F16DEV / BF16DEV */
    int32_t init;          /* IBM_LB_INIT_LINEAR or IBM_LB_INIT_REST */
    double A0[9];          /* gradient of the initial linear field */
    double f16_scale;      /* IBM_LB_F16DEV only: power of two >= 1; 0 selects 4096 */
    void* stream;          /* hipStream_t the library enqueues on; NULL = null stream */
    void* workspace;       /* device memory of >= ibm_lb_workspace_size bytes, caller-owned
                              and kept alive until ibm_lb_destroy; NULL: the library
                              allocates (and frees) its own */
    size_t workspace_bytes;
    int32_t populations;   /* population copies: 2 (0 also selects 2), or 1 for in-place
                              streaming only (step variants with bit 6; the populations take
                              half the memory, 19 s bytes per node instead of 38 s) */
    int32_t collision;     /* IBM_LB_BGK (0, the paper's single relaxation time) or IBM_LB_MRT:
                              multiple relaxation times (Sec. 3.1 mentions it as an option) on
                              the orthogonal moment basis of d'Humieres et al. (2002), the shear
                              moments at 1/tau; MRT runs every layout (two copies: linear or
                              rows; one copy: in place), in ensembles whose members all run
                              it (each with its own rates), without the adjoint */
    double mrt_s[5];       /* MRT rates in (0, 2) of the energy, energy-square, heat-flux,
                              third-order stress and third-order antisymmetric moments;
                              0 selects 1.19, 1.4, 1.2, 1.4, 1.98 */
    int32_t walls;         /* IBM_LB_WALLS_LINK (0): link-wise moving-wall bounce-back, walls
                              half a link outside the boundary nodes; IBM_LB_WALLS_WET: the
                              paper's wet-node velocity walls through the boundary nodes
                              (Sec. 3.1: Zou-He faces with the transverse correction of
                              Eq. ZH_bulk; edge and corner nodes rebuilt to hold their density,
                              the wall velocity and the linear field's populations, with the
                              along-edge correction of Eq. ZH_edges and the buried links and
                              rest population reset), two population copies (single droplets
                              and ensembles), without the adjoint */
    double chi;            /* viscosity ratio of droplet to carrier (Sec. 2), in [0, 1e6]; 0 or 1:
                              one fluid. Otherwise the nodes inside the mesh (parity of the mesh
                              crossings along x, i.e. the winding number modulo 2) relax with
                              tau_in = 1/2 + chi (tau - 1/2) (Eq. tau_to_nu at one density) in
                              the BGK rate and the Guo factor; the inside is rebuilt from the mesh
                              after every step. BGK (every lattice variant, one or two
                              population copies), single droplets, without the adjoint. The inside is
                              taken within the box's own node range: a vertex beyond [0, L - 1]
                              on any axis (a droplet across a periodic boundary) ends the run
                              with IBM_LB_EDOMAIN. The initial non-equilibrium part uses tau
                              everywhere */
    int32_t deterministic; /* spreading (Sec. 3.1, Eq. ibm_force_d, first line). 0: each surface
                              patch sums its vertices' contributions in an FP64 LDS window with
                              LDS atomics and adds it to F with device atomics, so the order of
                              the additions, and the last bits of F, may change from run to run.
                              1: every node of a tile touched by a stencil gathers its
                              contributions in increasing vertex order, in FP64, and F is stored
                              once per node: a run repeats bit for bit (and differs from mode 0
                              by the order of the additions only). Single droplets; the
                              workspace grows by 76 B (FP64: 136 B) per vertex and 32 B per
                              64-vertex patch */
} ibm_lb_config;

typedef struct ibm_lb_obs {
    int64_t step;          /* completed timesteps */
    double volume;         /* enclosed volume of the mesh */
    double centroid[3];    /* absolute coordinates */
    double S[9];           /* morphological tensor (5/V) int (x-xb)(x-xb)^T dV, row-major */
    double eigval[3];      /* eigenvalues of S, descending (lambda_max first) */
    double eigvec[9];      /* row k = unit eigenvector of eigval[k] */
    double D;              /* (sqrt(l1) - sqrt(l3)) / (sqrt(l1) + sqrt(l3)) */
    double beta;           /* Eq. beta with E = (A + A^T)/2 of the last step */
    double theta_deg;      /* atan2(v1_y, v1_x) folded into (-90, 90] degrees */
    double mass;           /* sum over nodes of sum_i f_i */
    double momentum[3];    /* sum over nodes of sum_i c_i f_i */
    int32_t reg_iters;     /* smoothing iterations of the last step */
    int32_t flags;         /* IBM_LB_OBS_* */
    double min_angle_deg;  /* mesh quality: smallest interior angle of any triangle (degrees) */
    double edge_min;       /* shortest mesh edge (lattice units) */
    double edge_max;       /* longest mesh edge */
} ibm_lb_obs;

/* Device bytes the configuration needs when cfg->workspace is supplied.
 * Errors: EINVAL (bad configuration). */
int ibm_lb_workspace_size(const ibm_lb_config* cfg, size_t* bytes);

/* Validate cfg, copy the mesh and build its adjacency, lay out device memory
 * and enqueue the initial state on cfg->stream. *out is owned by the library
 * until ibm_lb_destroy. Errors: EINVAL (L < 8, tau <= 0.5, sigma < 0,
 * radius <= 0, rho0 <= 0, bad storage/init, index out of range, open or
 * inward mesh, a vertex stencil outside a wall axis), ENOMEM, EDEVICE. */
int ibm_lb_init(const ibm_lb_config* cfg, ibm_lb** out);

/* Advance nsteps timesteps holding the gradient A fixed (the paper's
 * protocol holds each gradient sample for N steps, Sec. 3.2). A is a host
 * pointer, copied before return. Asynchronous. Errors: EINVAL, sticky. */
int ibm_lb_step(ibm_lb* h, const double A[9], int32_t nsteps);

/* Advance nsteps timesteps, step n using A + 9 n. on_device = 0: A is host
 * memory, copied before return. on_device = 1: A is device memory the
 * caller keeps unchanged until the next synchronising call. Asynchronous. */
int ibm_lb_step_table(ibm_lb* h, const double* A, int32_t nsteps, int32_t on_device);

/* Synchronise the stream and fill *out (FP64 reductions on the GPU).
 * Returns the sticky GPU error if one was raised. */
int ibm_lb_observables(ibm_lb* h, ibm_lb_obs* out);

/* Synchronising reads for tests and analysis. vertices: host double [nv][3]
 * absolute. read_field: which = IBM_LB_FIELD_RHO (rho^n, host double [N]) or
 * IBM_LB_FIELD_U (u^n including F^n/2 from the current mesh, host double
 * [3][N]). read_field allocates a temporary device buffer. */
int ibm_lb_read_vertices(ibm_lb* h, double* out);
int ibm_lb_read_field(ibm_lb* h, int32_t which, double* out);

/* ibm_lb_read_vertices without any allocation, for callers that cannot
 * allocate (code that must not call hipMalloc or hipFree, such as tight
 * serving or analysis loops and harnesses that forbid allocation): the same
 * output as ibm_lb_read_vertices (host double [nv][3], absolute coordinates,
 * caller vertex order; synchronising), staged through a fixed device array
 * that the library holds on each GPU it runs on until the process ends
 * (3 IBM_LB_NOALLOC_MAX_VERTICES doubles, 6 MiB). Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (other host
 * threads, other streams) race: serialise them. No device or host memory is
 * allocated, also on error. Errors: EINVAL (NULL handle, NULL out with a
 * mesh, more than IBM_LB_NOALLOC_MAX_VERTICES vertices: use
 * ibm_lb_read_vertices), EDEVICE, sticky. */
#define IBM_LB_NOALLOC_MAX_VERTICES 262144
int ibm_lb_read_vertices_noalloc(ibm_lb* h, double* out);

/* Inside indicator that the next step's collision uses (Sec. 2, viscosity
 * ratio chi), host uint8 [N] (x fastest): 1 for a node inside the current
 * mesh, else 0. Synchronising. EINVAL for a handle without a viscosity
 * ratio. */
int ibm_lb_read_indicator(ibm_lb* h, uint8_t* out);

/* Checkpoints: ibm_lb_state_bytes is the size of the state (populations,
 * vertices, step counter). save/load copy it to/from dst/src, which may be
 * host or device memory of at least that many bytes (caller-owned); both
 * synchronise the stream. Errors: EINVAL (size too small), EDEVICE. */
size_t ibm_lb_state_bytes(const ibm_lb* h);
int ibm_lb_save(ibm_lb* h, void* dst, size_t n);
int ibm_lb_load(ibm_lb* h, const void* src, size_t n);

/* Step variants, 0 <= variant < 128. Bits 0-4 select the lattice kernel's
 * variant (all compute the same per-node arithmetic; they differ only in how
 * nodes map to work-groups and how populations reach memory):
 *   bit 0     non-temporal population loads;
 *   bits 1-2  work-group size {128, 256, 512, 64}[(variant >> 1) & 3]; in the
 *             row layout, the least number of whole x-rows (at least one)
 *             that fits in it;
 *   bit 4     row layout: a work-group owns whole x-rows and hands the
 *             populations moving along x to their target thread through
 *             LDS, so every population store is row-aligned (needs
 *             Lx <= 512); otherwise the linear layout (consecutive nodes per
 *             work-group, each population stored straight at its target);
 *   bit 3     linear layout: work-groups ordered so that each XCD takes a
 *             contiguous eighth of the lattice; row layout: non-temporal
 *             population stores.
 * Bit 5 runs the end of the smoothing (convergence test, further
 * iterations, iteration count) at the start of the force kernel instead of
 * in the last of the smoothing's work-groups to finish (which needs a
 * device-scope release in every work-group): every force work-group reads
 * the first iteration's maximum; in the rare step that needs further
 * iterations, the first work-group runs them and then spreads every vertex
 * with direct atomics. With deterministic spreading the end runs as a
 * one-work-group launch of its own; ensembles always run it so and ignore
 * the bit.
 * Bit 6 (linear layout only; single droplets only) streams in place: one
 * population copy, read and written by the same thread at the same
 * locations, with even and odd steps in two index mappings (the AA pattern
 * of Bailey et al., 2009). After an odd number of such steps the copy holds
 * the populations in the odd mapping; every call that reads them (fields,
 * observables, save, objective gradient) or steps with another variant
 * first returns them to natural order in place (one pass of pairwise swaps).
 * A handle made with populations = 1 holds one copy and runs only variants
 * with bit 6 (default 96). The adjoint's recompute of a segment runs
 * without bit 6 on two copies; on one copy each recomputed step is followed
 * by the return to natural order.
 *
 * Autotuner: picks the variant for this configuration by timing `reps` whole
 * steps with each lattice variant that can run (bit 5 set; with and without
 * bit 6), in four
 * interleaved rounds, from a snapshot of the state that is restored
 * afterwards (the state after the call equals the state before; the force
 * field is spread again at the next step). Times within 1 % of the fastest
 * count as ties, which go to the default variant, else to the first
 * candidate (bit 6 clear before bit 6 set, then by index).
 * Synchronises the stream.
 * *variant (may be NULL) receives the choice. Errors: EINVAL, ENOMEM,
 * EDEVICE, sticky.
 *
 * ibm_lb_set_variant selects a variant directly (EINVAL if out of range,
 * bits 4 and 6 together, bit 6 clear on a one-copy handle, bit 6 with
 * wet-node walls, or the row layout cannot take this box). The default is 33 (linear layout,
 * 128-thread work-groups, non-temporal loads, bit 5), or 96 on a one-copy
 * handle (in place, 128-thread work-groups, bit 5). */
int ibm_lb_autotune(ibm_lb* h, int32_t reps, int32_t* variant);
int ibm_lb_set_variant(ibm_lb* h, int32_t variant);

/* Kernel timing of the fused lattice kernel: when enabled, each lattice
 * launch is timed on the handle's stream from the completion of the dispatch
 * before it to its own completion, both stamped by the dispatches themselves
 * (hipExtLaunchKernel stop events; the first launch of each call starts
 * from an event recorded just before it). Consecutive dispatches of one
 * stream start as the previous one completes, so this is the kernel's
 * duration without the cost of separate event packets around it.
 * ibm_lb_timing_read synchronises and returns the summed elapsed time (ms)
 * and launch count since the last read. */
int ibm_lb_timing_enable(ibm_lb* h, int32_t enable);
int ibm_lb_timing_read(ibm_lb* h, double* lattice_ms, int64_t* launches);

/* ---- ensembles of independent droplets (one set of launches per step) ----
 * The paper's statistics come from many independent trajectories, one
 * droplet each (Sec. 4); an ensemble advances n of them together. Members
 * may differ in box size, periodicity, tau, sigma, MRT rates, mesh and
 * gradient history but share one storage format and one collision (BGK or
 * MRT). Each step is one batched launch of the fused
 * lattice kernel over every member's nodes, then the batched IB kernels over
 * every member's surface patches; work-groups map to members by per-block
 * tables, so heterogeneous boxes balance by block count. Runs of steps are
 * replayed as captured HIP graphs (ibm_lb_batch_set_graph).
 *
 * ibm_lb_batch_init: cfgs[n] as for ibm_lb_init (each member's workspace
 *   rule applies; cfgs[i].stream is ignored); all work goes to `stream`.
 *   Errors: EINVAL (n < 1, mixed storage or collision, a member with one
 *   population copy, a viscosity ratio or deterministic spreading, any
 *   member invalid), ENOMEM, EDEVICE. Members may mix link and wet-node
 *   walls (the latter after each batched lattice launch, batched too).
 * ibm_lb_batch_step: A_tables is host memory [n][nsteps][9] (member-major),
 *   copied before return; member i's step j uses A_tables + 9 (i nsteps + j).
 * ibm_lb_batch_observables: out[n]; synchronising; returns the first member
 *   error. ibm_lb_batch_member gives member i's handle for synchronising
 *   reads (vertices, fields, observables, save); stepping a member on its
 *   own while it belongs to an ensemble is not supported.
 * ibm_lb_batch_autotune: as ibm_lb_autotune for the batched steps (gradient
 *   rows of the last upload); every member is restored afterwards. In the
 *   batched row layout a work-group of the selected size takes
 *   floor(size / Lx) whole rows of one member, so a row variant runs only
 *   when every member's Lx fits in the work-group.
 * ibm_lb_batch_set_variant: as ibm_lb_set_variant (EINVAL if the variant
 *   cannot run on every member, or has bit 6).
 * ibm_lb_batch_set_graph: runs of `steps` batched steps (even, at most 4096;
 *   default 32) go to the GPU as one captured HIP graph, replayed with the
 *   gradient rows of the run; 0 uses plain launches throughout. Graphs are
 *   captured on first use for each population parity and lattice variant
 *   (on a private stream; nothing runs during capture) and hold no memset
 *   nodes. Synchronises the ensemble's stream. Errors: EINVAL, EDEVICE.
 * ibm_lb_batch_destroy frees the ensemble and its members. */
int ibm_lb_batch_init(const ibm_lb_config* cfgs, int32_t n, void* stream, ibm_lb_batch** out);
int ibm_lb_batch_step(ibm_lb_batch* b, const double* A_tables, int32_t nsteps);
int ibm_lb_batch_observables(ibm_lb_batch* b, ibm_lb_obs* out);
int ibm_lb_batch_member(ibm_lb_batch* b, int32_t i, ibm_lb** out);
int ibm_lb_batch_autotune(ibm_lb_batch* b, int32_t reps, int32_t* variant);
int ibm_lb_batch_set_variant(ibm_lb_batch* b, int32_t variant);
int ibm_lb_batch_set_graph(ibm_lb_batch* b, int32_t steps);
void ibm_lb_batch_destroy(ibm_lb_batch* b);

/* ---- adjoint: reverse-mode derivatives of the droplet deformation ----
 * Objective J = D(r^T) = (sqrt(l1) - sqrt(l3)) / (sqrt(l1) + sqrt(l3)) of the
 * morphological tensor S of the final mesh (Sec. 2). The adjoint is the
 * exact transpose of the linearised timestep (forces, spreading, moments,
 * interpolation, BGK + Guo collision, streaming with moving-wall bounce-back,
 * Euler move, HC smoothing), with the smoothing iteration count of every step
 * held at the value the forward run took: the tolerance test is a discrete
 * decision and has no derivative. The adjoint computes in FP64 for every
 * storage format.
 *
 * ibm_lb_objective_grad: synchronises; *value = D of the current mesh and
 *   rbar (device double [nv][3], caller vertex order) = dD/dr. Errors:
 *   EINVAL (no mesh; l1 - l2 or l2 - l3 below 1e-12 radius^2, where D has no
 *   derivative), sticky.
 * ibm_lb_shape_objective_grad: the same for objective IBM_LB_OBJ_D (as
 *   above), IBM_LB_OBJ_LAMBDA_MAX (the largest eigenvalue of S; needs
 *   l1 - l2 >= 1e-12 radius^2) or IBM_LB_OBJ_BETA (Eq. beta with the strain
 *   E of the last gradient row; needs l1 - l2 >= 1e-12 radius^2 and E != 0).
 *   dA_last (host double[9], may be NULL) receives the objective's direct
 *   derivative with respect to the last gradient row (nonzero for beta
 *   only), to be added to the last row of the adjoint's dJ/dA. The adjoint
 *   sweep is the same for every objective: rbar seeds ibm_lb_adjoint_segment.
 *
 * ibm_lb_adjoint_segment: reverse one segment of nsteps >= 1 steps.
 *   ckpt (host or device, ckpt_bytes) is the checkpoint ibm_lb_save wrote at
 *   the segment's first step and A its gradient rows [nsteps][9] (host memory
 *   if A_on_device = 0, else device). The library reloads ckpt and recomputes
 *   the segment, recording rho, u and F on every node and the positions and
 *   smoothing iteration counts of every step (FP64, 56 N + 32 nv bytes per
 *   step, in device memory the library allocates and keeps until
 *   ibm_lb_destroy), then sweeps the steps backwards.
 *   fbar_end: device double [19][N] (x fastest), the adjoint of the
 *   population deviations after the segment, NULL for zero (the final time of
 *   J = D(r^T)). rbar_end: device double [nv][3], caller vertex order, the
 *   adjoint of the positions after the segment.
 *   Outputs, device memory: fbar_begin and rbar_begin, the same at the
 *   segment start (they may alias the _end arrays; fbar_begin may be NULL);
 *   dA [nsteps][9], dJ/dA of each step (overwritten); dsigma [1], dJ/dsigma
 *   of the segment added to *dsigma.
 *   On return the handle holds the segment's end state. Work is enqueued on
 *   the handle's stream; the call synchronises once, after the recompute.
 *   Errors: EINVAL (bad arguments or checkpoint), ENOMEM, EDEVICE, sticky. */
enum { IBM_LB_OBJ_D = 0, IBM_LB_OBJ_LAMBDA_MAX = 1, IBM_LB_OBJ_BETA = 2 };
int ibm_lb_objective_grad(ibm_lb* h, double* value, double* rbar);
int ibm_lb_shape_objective_grad(ibm_lb* h, int32_t objective, double* value, double* rbar, double* dA_last);
/* ibm_lb_adjoint_initial: dJ/dA0 through the initial state (IBM_LB_INIT_LINEAR:
 * f_eq(rho0, A0 (x - x_c)) and its Chapman-Enskog part; zero for
 * IBM_LB_INIT_REST). fbar0: device double [19][N] (x fastest), the adjoint of
 * the population deviations at step 0 (fbar_begin of the first segment).
 * dA0: host double [9], row-major. Synchronising; the handle's state is not
 * used (A0, tau, rho0 and the box come from the configuration). Errors:
 * EINVAL (bad arguments, MRT, wet walls or a viscosity ratio), EDEVICE. */
int ibm_lb_adjoint_initial(ibm_lb* h, const double* fbar0, double* dA0);
int ibm_lb_adjoint_segment(ibm_lb* h, const void* ckpt, size_t ckpt_bytes, const double* A, int32_t nsteps,
                           int32_t A_on_device, const double* fbar_end, const double* rbar_end, double* fbar_begin,
                           double* rbar_begin, double* dA, double* dsigma);

void ibm_lb_destroy(ibm_lb* h);
const char* ibm_lb_strerror(int code);
const char* ibm_lb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IBM_LB_H */
