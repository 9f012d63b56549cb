// Drives the library's host-side validation and set-up arithmetic, for a build
// of api.hip with AddressSanitizer and UndefinedBehaviorSanitizer on its host
// code (test infrastructure only: tests/test_abi_sanitize.py builds and runs
// it on the CPU). ibm_lb_workspace_size runs every host step of ibm_lb_init
// that comes before device memory: the configuration checks, the closed-mesh
// and orientation checks, the patch renumbering by bisection, the ordered
// one-ring fans, the patch halos and the workspace layout; none of it calls
// the HIP runtime.
//
// Usage: abi_sanitize_check MESHFILE, where MESHFILE holds "nv nt", then nv
// lines of absolute vertex coordinates and nt lines of triangle indices (a
// closed, outward mesh centred in a 16^3 box). Exit status 0 when every call
// returned what it should; the sanitizers abort on any memory or undefined
// behaviour error.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ibm_lb.h"

static int failures = 0;

static void expect(bool cond, const char* what) {
    if (!cond) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, ibm_lb_last_error());
        ++failures;
    }
}

static ibm_lb_config base(const std::vector<double>& V, const std::vector<int32_t>& T) {
    ibm_lb_config c;
    std::memset(&c, 0, sizeof(c));
    for (int a = 0; a < 3; ++a) c.L[a] = 16;
    c.tau = 0.9;
    c.sigma = 0.02;
    c.radius = 3.0;
    c.rho0 = 1.0;
    c.n_vertices = (int32_t)(V.size() / 3);
    c.n_triangles = (int32_t)(T.size() / 3);
    c.vertices = V.data();
    c.triangles = T.data();
    c.reg_alpha = 0.1;
    c.reg_gamma = 0.51;
    c.reg_tol = 0.01;
    c.reg_max_iter = 50;
    c.reg_sign = 1;
    c.storage = IBM_LB_F32;
    return c;
}

static int size_rc(const ibm_lb_config& c, size_t* n = nullptr) {
    size_t b = 0;
    const int rc = ibm_lb_workspace_size(&c, &b);
    if (n) *n = b;
    return rc;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* fp = std::fopen(argv[1], "r");
    if (!fp) return 2;
    int nv = 0, nt = 0;
    if (std::fscanf(fp, "%d %d", &nv, &nt) != 2 || nv <= 0 || nt <= 0) return 2;
    std::vector<double> V(3 * (size_t)nv);
    std::vector<int32_t> T(3 * (size_t)nt);
    for (auto& v : V)
        if (std::fscanf(fp, "%lf", &v) != 1) return 2;
    for (auto& t : T)
        if (std::fscanf(fp, "%d", &t) != 1) return 2;
    std::fclose(fp);

    // every valid configuration the set-up distinguishes
    size_t n0 = 0;
    expect(size_rc(base(V, T), &n0) == IBM_LB_OK && n0 > 0, "valid droplet");
    for (int st : {IBM_LB_F64, IBM_LB_F32, IBM_LB_F16DEV, IBM_LB_BF16DEV}) {
        ibm_lb_config c = base(V, T);
        c.storage = st;
        expect(size_rc(c) == IBM_LB_OK, "storage formats");
        c.deterministic = 1;
        expect(size_rc(c) == IBM_LB_OK, "deterministic spreading");
        c.populations = 1;
        expect(size_rc(c) == IBM_LB_OK, "one population copy");
    }
    {
        ibm_lb_config c = base(V, T);
        c.chi = 4.0;
        expect(size_rc(c) == IBM_LB_OK, "viscosity ratio");
        c.chi = 1.0;
        c.collision = IBM_LB_MRT;
        expect(size_rc(c) == IBM_LB_OK, "MRT");
        c.populations = 1;
        expect(size_rc(c) == IBM_LB_OK, "MRT in place");
        c.populations = 0;
        c.collision = IBM_LB_BGK;
        c.walls = IBM_LB_WALLS_WET;
        expect(size_rc(c) == IBM_LB_OK, "wet walls");
        c.walls = IBM_LB_WALLS_LINK;
        c.periodic[0] = c.periodic[1] = c.periodic[2] = 1;
        expect(size_rc(c) == IBM_LB_OK, "periodic");
        c.n_vertices = c.n_triangles = 0;
        c.vertices = nullptr;
        c.triangles = nullptr;
        expect(size_rc(c) == IBM_LB_OK, "lattice only");
        c.L[0] = 1000;
        c.L[1] = 1000;
        c.L[2] = 3000;
        expect(size_rc(c) == IBM_LB_EINVAL, "box above 2^31 nodes");
    }

    // invalid parameters
    {
        ibm_lb_config c = base(V, T);
        c.tau = 0.5;
        expect(size_rc(c) == IBM_LB_EINVAL, "tau");
        c = base(V, T);
        c.L[1] = 7;
        expect(size_rc(c) == IBM_LB_EINVAL, "small box");
        c = base(V, T);
        c.deterministic = 3;
        expect(size_rc(c) == IBM_LB_EINVAL, "deterministic flag");
        c = base(V, T);
        c.f16_scale = 3.0;
        c.storage = IBM_LB_F16DEV;
        expect(size_rc(c) == IBM_LB_EINVAL, "f16 scale");
        c = base(V, T);
        c.mrt_s[2] = 2.5;
        c.collision = IBM_LB_MRT;
        expect(size_rc(c) == IBM_LB_EINVAL, "MRT rate");
        c = base(V, T);
        c.reg_tol = std::nan("");
        expect(size_rc(c) == IBM_LB_EINVAL, "NaN tolerance");
    }

    // invalid meshes
    {
        std::vector<int32_t> Tb = T;
        Tb[4] = nv;  // index out of range
        expect(size_rc(base(V, Tb)) == IBM_LB_EINVAL, "index out of range");
        Tb = T;
        std::swap(Tb[0], Tb[1]);  // one triangle flipped
        expect(size_rc(base(V, Tb)) == IBM_LB_EINVAL, "flipped triangle");
        Tb.assign(T.begin(), T.end() - 3);  // one triangle missing
        expect(size_rc(base(V, Tb)) == IBM_LB_EINVAL, "open mesh");
        Tb = T;
        for (int t = 0; t < nt; ++t) std::swap(Tb[3 * t + 1], Tb[3 * t + 2]);  // all inward
        expect(size_rc(base(V, Tb)) == IBM_LB_EINVAL, "inward mesh");
        Tb = T;
        Tb[1] = Tb[0];  // degenerate triangle
        expect(size_rc(base(V, Tb)) == IBM_LB_EINVAL, "degenerate triangle");
        std::vector<double> Vb = V;
        Vb[7] = std::nan("");
        expect(size_rc(base(Vb, T)) == IBM_LB_EINVAL, "NaN vertex");
        Vb = V;
        Vb[0] = 0.5;  // a stencil through the x wall
        expect(size_rc(base(Vb, T)) == IBM_LB_EINVAL, "stencil through a wall");
        ibm_lb_config c = base(V, T);
        c.n_triangles = 3;
        expect(size_rc(c) == IBM_LB_EINVAL, "too few triangles");
    }

    // ensembles refuse members they cannot run, before any device work
    {
        ibm_lb_config m[2] = {base(V, T), base(V, T)};
        m[1].deterministic = 1;
        ibm_lb_batch* b = nullptr;
        expect(ibm_lb_batch_init(m, 2, nullptr, &b) == IBM_LB_EINVAL && !b, "ensemble refuses a member");
    }
    expect(std::strlen(ibm_lb_strerror(IBM_LB_EDOMAIN)) > 0, "strerror");

    if (failures) {
        std::fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    std::printf("abi_sanitize_check: host validation ran clean\n");
    return 0;
}
