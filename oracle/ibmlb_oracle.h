/*
 * ibmlb_oracle.h — plain FP64 CPU oracle of the IB-LB droplet timestep.
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the HIP path; it is
 * never on the product path. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it. It shares no code, header, table or
 * helper with the HIP library.
 *
 * Method: Taglienti, Guglietta & Sbragaglia, "Droplet dynamics in homogeneous
 * isotropic turbulence with the immersed boundary-lattice Boltzmann method"
 * (arXiv 2403.01161).
 *   - D3Q19 BGK with Guo forcing: Sec. 3.1, Eqs. (LBMEQ), (collision),
 *     (equilibriumLB), Guo source, (density_velocity_LB).
 *   - IB coupling with the Peskin 4-point stencil: Sec. 3.1, Eq. (ibm_force_d),
 *     stencil phi(x), Eq. (fwd_euler).
 *   - Surface tension Pi = sigma I_2: Sec. 3.1, Eq. (pi_drop).
 *   - Moving walls imposing u = A (x - x_c): Sec. 2 Eq. (linearized velocity),
 *     Sec. 3.1 Eqs. (velo_facce_cubo_da_gradiente), (standard BB).
 *   - Extended Laplacian (HC) mesh smoothing: Sec. 3.3, Eqs. (extended
 *     laplacian smoothing), (HC_algo_full), (distanceregularization).
 *   - Morphological tensor S, lambda_max, beta: Sec. 2, Eq. (beta).
 *
 * Conventions: nodes at integer coordinates 0..L-1 per axis, node index
 * n = x + Lx (y + Ly z). Box centre x_c = (L-1)/2. Gradient A row-major,
 * A[3a+b] = du_a/dx_b. Vector fields are node-major [N][3] in this header.
 * Vertex coordinates are absolute lattice coordinates [nv][3].
 */
#ifndef IBMLB_ORACLE_H
#define IBMLB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define IBO_OK 0
#define IBO_EINVAL (-1)
#define IBO_ENOMEM (-2)
#define IBO_EDOMAIN (-4)
#define IBO_ENONFINITE (-5)

/* observable flags */
#define IBO_FLAG_DEGENERATE 1 /* lambda_1 - lambda_2 below 1e-12 R^2: v_max, beta, theta undefined */
#define IBO_FLAG_E_ZERO 2     /* ||E||_F == 0: beta undefined */
#define IBO_FLAG_REG_CAP 4    /* smoothing hit its iteration cap since the last observables call */

/* Number of doubles written by ibo_observables / ibo_shape. Layout:
 *  0 step, 1 volume, 2..4 centroid (absolute), 5..13 S (row-major),
 *  14..16 eigenvalues (descending), 17..25 eigenvectors (row k = vector k),
 *  26 D, 27 beta, 28 theta (degrees), 29 mass, 30..32 momentum,
 *  33 smoothing iterations of the last step, 34 flags. */
#define IBO_OBS_N 38

typedef struct ibo_params {
    int L[3];          /* nodes per axis, each >= 4 */
    int periodic[3];   /* 1: periodic axis, 0: moving bounce-back walls */
    double tau;        /* BGK relaxation time, > 0.5 */
    double sigma;      /* surface tension, >= 0 */
    double radius;     /* rest radius R (degeneracy threshold scale) */
    double rho0;       /* reference density (1) */
    int nv, nt;        /* mesh size; nv = 0 runs the lattice alone */
    const double* verts; /* [nv][3] absolute coordinates */
    const int* tris;     /* [nt][3] outward counter-clockwise */
    double reg_alpha, reg_gamma, reg_tol;
    int reg_max_iter;  /* 0 disables smoothing */
    int reg_sign;      /* +1: correction adds the neighbour mean of b; -1: subtracts it */
    int init_rest;     /* 0: linear field u = A0 (x - x_c) with its non-equilibrium part; 1: rest */
    double A0[9];
    int wall_bc;       /* 0: link-wise moving-wall bounce-back, walls at -1/2 and L-1/2;
                          1: wet-node velocity walls through the boundary nodes (Sec. 3.1,
                          the Zou-He conditions in the 3D form of Hecht and Harting), edge
                          and corner nodes carrying the wall velocity; 2: the same with the
                          edge and corner rules as printed (no wall-velocity term) */
    int collision;     /* 0: BGK (the paper's single relaxation time); 1: MRT */
    double mrt_s[5];   /* MRT rates of the energy, energy-square, heat-flux, third-order
                          stress and third-order antisymmetric moments; 0 selects 1.19,
                          1.4, 1.2, 1.4, 1.98; the shear rate is 1/tau */
    double chi;        /* viscosity ratio inside/outside the droplet (Sec. 2); 0 or 1: one
                          fluid. Nodes inside the mesh relax with tau_in = 1/2 + chi (tau - 1/2)
                          (same density, Eq. tau_to_nu); BGK only */
} ibo_params;

typedef struct ibo_sim ibo_sim;

/* ---- building blocks (each follows one passage of the paper) ---- */
void ibo_lattice(int c[19 * 3], double w[19], int opp[19]);
double ibo_phi(double r);
void ibo_equilibrium(double rho, const double u[3], double feq[19]);
void ibo_guo_source(double tau, const double u[3], const double F[3], double S[19]);
/* Moment basis of the MRT collision: M[19][19] (row k = moment k over the
 * velocities) and the squared row norms. */
void ibo_mrt_basis(double M[19 * 19], double norm2[19]);
void ibo_forces(int nv, const double* r, int nt, const int* tris, double sigma, double* phi);
int ibo_spread(const int L[3], const int periodic[3], int nv, const double* r,
               const double* phi, double* F);
int ibo_interp(const int L[3], const int periodic[3], int nv, const double* r,
               const double* u, double* U);
int ibo_hc(int nv, int nt, const int* tris, double alpha, double gamma, double tol,
           int max_iter, int sign, double* r, int* capped);
void ibo_eig3(const double S[9], double evals[3], double evecs[9]);
int ibo_shape(int nv, const double* r, int nt, const int* tris, const double A[9],
              double radius, double out[IBO_OBS_N]);
/* Inside/outside indicator of the closed mesh on the lattice (x fastest):
 * out[n] = 1 where the winding number of the surface about node n exceeds
 * 1/2, else 0. Nodes outside the mesh's bounding box are outside. */
void ibo_indicator(const int L[3], int nv, const double* r, int nt, const int* tris, unsigned char* out);
/* Winding number of the closed mesh about the point p (solid angles summed
 * over the triangles, divided by 4 pi). */
double ibo_winding(int nv, const double* r, int nt, const int* tris, const double p[3]);

/* ---- the coupled simulation ---- */
int ibo_create(const ibo_params* p, ibo_sim** out);
void ibo_destroy(ibo_sim* s);
/* Advance nsteps; step n uses A + 9*n*stride (stride 0: one fixed A). */
int ibo_step(ibo_sim* s, const double* A, int nsteps, int stride);
int ibo_observables(ibo_sim* s, double out[IBO_OBS_N]);
int ibo_get_vertices(const ibo_sim* s, double* r);
int ibo_set_vertices(ibo_sim* s, const double* r);
/* rho [N], u [N][3] of the current state (u includes F/2 from the current mesh). */
int ibo_fields(ibo_sim* s, double* rho, double* u);
/* Freeze the smoothing: the next n steps run exactly counts[j] HC iterations
 * each (no convergence test), so that a perturbed run takes the same discrete
 * path as the nominal one (finite-difference checks of derivatives). n = 0
 * restores the tolerance test. */
int ibo_freeze_iters(ibo_sim* s, const int* counts, int n);
/* Smoothing iterations of the last step. */
int ibo_last_iters(const ibo_sim* s);
int ibo_get_populations(const ibo_sim* s, double* f); /* [N][19] */
/* Indicator of the current mesh, the one the next step's collision uses ([N]). */
int ibo_get_indicator(const ibo_sim* s, unsigned char* out);
int ibo_set_populations(ibo_sim* s, const double* f); /* [N][19] */
long ibo_nodes(const ibo_sim* s);

#ifdef __cplusplus
}
#endif
#endif
