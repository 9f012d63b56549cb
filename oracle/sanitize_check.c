/*
 * sanitize_check.c — drives the FP64 oracle through every configuration it
 * supports, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (test infrastructure only: tests/test_oracle_sanitize.py compiles it with
 * ibmlb_oracle.c and runs it on the CPU).
 *
 * Usage: sanitize_check MESHFILE, where MESHFILE holds "nv nt", then nv
 * lines of absolute vertex coordinates and nt lines of triangle indices (a
 * closed, outward mesh centred in a 12^3 box). Exit status 0 when every call
 * returned what it should; the sanitizers abort on any memory or undefined
 * behaviour error.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ibmlb_oracle.h"

static int failures = 0;

static void expect(int cond, const char* what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static void run(const char* name, ibo_params p, const double* A, int nsteps)
{
    ibo_sim* s = NULL;
    int rc = ibo_create(&p, &s);
    expect(rc == IBO_OK, name);
    if (rc != IBO_OK) return;
    rc = ibo_step(s, A, nsteps, 0);
    expect(rc == IBO_OK, name);
    double obs[IBO_OBS_N];
    expect(ibo_observables(s, obs) == IBO_OK, name);
    const long N = ibo_nodes(s);
    double* rho = malloc(sizeof(double) * (size_t)N);
    double* u = malloc(sizeof(double) * 3 * (size_t)N);
    double* f = malloc(sizeof(double) * 19 * (size_t)N);
    unsigned char* ind = malloc((size_t)N);
    expect(ibo_fields(s, rho, u) == IBO_OK, name);
    expect(ibo_get_populations(s, f) == IBO_OK, name);
    expect(ibo_set_populations(s, f) == IBO_OK, name);
    if (p.nv) {
        double* r = malloc(sizeof(double) * 3 * (size_t)p.nv);
        expect(ibo_get_vertices(s, r) == IBO_OK, name);
        expect(ibo_set_vertices(s, r) == IBO_OK, name);
        free(r);
        int counts[3] = {1, 2, 0};
        expect(ibo_freeze_iters(s, counts, 3) == IBO_OK, name);
        expect(ibo_step(s, A, 3, 0) == IBO_OK, name);
        expect(ibo_last_iters(s) == 0, name);
        if (p.chi != 0.0 && p.chi != 1.0) expect(ibo_get_indicator(s, ind) == IBO_OK, name);
    }
    double m = 0.0;
    for (long n = 0; n < N; ++n) m += rho[n];
    expect(isfinite(m) && fabs(m / (double)N - p.rho0) < 1e-3, name);
    free(rho);
    free(u);
    free(f);
    free(ind);
    ibo_destroy(s);
}

int main(int argc, char** argv)
{
    if (argc < 2) return 2;
    FILE* fp = fopen(argv[1], "r");
    if (!fp) return 2;
    int nv = 0, nt = 0;
    if (fscanf(fp, "%d %d", &nv, &nt) != 2 || nv <= 0 || nt <= 0) return 2;
    double* V = malloc(sizeof(double) * 3 * (size_t)nv);
    int* T = malloc(sizeof(int) * 3 * (size_t)nt);
    for (int k = 0; k < 3 * nv; ++k)
        if (fscanf(fp, "%lf", &V[k]) != 1) return 2;
    for (int k = 0; k < 3 * nt; ++k)
        if (fscanf(fp, "%d", &T[k]) != 1) return 2;
    fclose(fp);

    /* building blocks */
    int c[57], opp[19];
    double w[19], feq[19], S[19], M[361], nrm[19];
    ibo_lattice(c, w, opp);
    const double u0[3] = {1e-3, -2e-3, 5e-4}, F0[3] = {1e-4, 0.0, -1e-4};
    ibo_equilibrium(1.0, u0, feq);
    ibo_guo_source(0.8, u0, F0, S);
    ibo_mrt_basis(M, nrm);
    expect(fabs(ibo_phi(0.0) - 0.5) < 1e-15, "phi(0)");
    double* phi = malloc(sizeof(double) * 3 * (size_t)nv);
    ibo_forces(nv, V, nt, T, 0.02, phi);
    const int L[3] = {12, 12, 12}, per[3] = {0, 0, 0}, per1[3] = {1, 1, 1};
    double* Ff = calloc(3 * 12 * 12 * 12, sizeof(double));
    double* Uf = calloc(3 * 12 * 12 * 12, sizeof(double));
    double* U = malloc(sizeof(double) * 3 * (size_t)nv);
    expect(ibo_spread(L, per, nv, V, phi, Ff) == IBO_OK, "spread");
    expect(ibo_spread(L, per1, nv, V, phi, Ff) == IBO_OK, "spread periodic");
    expect(ibo_interp(L, per, nv, V, Uf, U) == IBO_OK, "interp");
    double* r = malloc(sizeof(double) * 3 * (size_t)nv);
    memcpy(r, V, sizeof(double) * 3 * (size_t)nv);
    int capped = 0;
    expect(ibo_hc(nv, nt, T, 0.1, 0.51, 0.01, 50, 1, r, &capped) >= 0, "hc");
    expect(ibo_hc(nv, nt, T, 0.1, 0.51, 0.01, 50, -1, r, &capped) >= 0, "hc printed sign");
    const double Sm[9] = {2.0, 0.1, 0.0, 0.1, 1.0, 0.2, 0.0, 0.2, 3.0};
    double ev[3], evec[9], obs[IBO_OBS_N];
    ibo_eig3(Sm, ev, evec);
    const double A[9] = {1e-4, 2e-3, 0.0, -5e-4, -3e-4, 1e-3, 0.0, 2e-4, 2e-4};
    expect(ibo_shape(nv, V, nt, T, A, 2.5, obs) == IBO_OK, "shape");
    const double centre[3] = {5.5, 5.5, 5.5};
    expect(fabs(ibo_winding(nv, V, nt, T, centre) - 1.0) < 1e-9, "winding");
    unsigned char* ind = malloc(12 * 12 * 12);
    ibo_indicator(L, nv, V, nt, T, ind);

    /* the coupled step in every configuration */
    ibo_params p;
    memset(&p, 0, sizeof(p));
    for (int a = 0; a < 3; ++a) p.L[a] = 12;
    p.tau = 0.9;
    p.sigma = 0.02;
    p.radius = 2.5;
    p.rho0 = 1.0;
    p.nv = nv;
    p.nt = nt;
    p.verts = V;
    p.tris = T;
    p.reg_alpha = 0.1;
    p.reg_gamma = 0.51;
    p.reg_tol = 0.01;
    p.reg_max_iter = 50;
    p.reg_sign = 1;
    memcpy(p.A0, A, sizeof(A));
    run("link walls", p, A, 6);
    p.wall_bc = 1;
    run("wet walls", p, A, 6);
    p.wall_bc = 2;
    run("wet walls as printed", p, A, 6);
    p.wall_bc = 0;
    p.collision = 1;
    run("MRT", p, A, 6);
    p.collision = 0;
    p.chi = 4.0;
    run("viscosity ratio", p, A, 6);
    p.chi = 0.0;
    p.periodic[0] = p.periodic[2] = 1;
    const double shear[9] = {0.0, 2e-3, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    memcpy(p.A0, shear, sizeof(shear));
    run("periodic x and z", p, shear, 6);
    p.periodic[1] = 1;
    const double zero[9] = {0};
    memcpy(p.A0, zero, sizeof(zero));
    run("fully periodic", p, zero, 6);
    p.init_rest = 1;
    p.nv = 0;
    p.nt = 0;
    run("lattice only, rest", p, zero, 6);

    /* invalid configurations are rejected */
    ibo_sim* s = NULL;
    p.tau = 0.4;
    expect(ibo_create(&p, &s) == IBO_EINVAL, "tau <= 1/2 rejected");
    p.tau = 0.9;
    p.wall_bc = 3;
    expect(ibo_create(&p, &s) == IBO_EINVAL, "unknown wall rule rejected");

    free(phi);
    free(Ff);
    free(Uf);
    free(U);
    free(r);
    free(ind);
    free(V);
    free(T);
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("sanitize_check: all configurations ran clean\n");
    return 0;
}
