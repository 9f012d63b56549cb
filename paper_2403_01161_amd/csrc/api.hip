// C-ABI of the IB-LB droplet library: validation, device memory layout,
// launch sequencing and synchronising reads. The per-timestep order is the
// one documented in include/ibm_lb.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ibmlb_internal.h"

using namespace ibmlb;

namespace {

// Message of the last failure on this thread (fixed storage: recording an
// error allocates nothing).
thread_local char g_last_error[256];

int fail(int code, const char* msg) {
    snprintf(g_last_error, sizeof(g_last_error), "%s", msg);
    return code;
}

int fail(int code, const std::string& msg) { return fail(code, msg.c_str()); }

int hip_fail(hipError_t e, const char* where) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s", where, hipGetErrorString(e));
    return IBM_LB_EDEVICE;
}

#define HIP_TRY(expr, where)                          \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Byte offsets of every device array inside one workspace.
struct Layout {
    size_t f[2], F, u, mark, ctl, r, o, qa, qb, pp, bb, tris, fan, lfan, hstart, hids, obs_part, mass_part,
        obs_out, Abuf, red, ind, ind_lines, ptris, ptstart, perm, det, pbox, total;
};

// Per vertex: valence m and the one-ring neighbours n_0 .. n_{m-1} in
// counter-clockwise order, so that (k, n_j, n_{j+1 mod m}) are exactly the
// triangles around k with their orientation. FAN ints per vertex.
constexpr int FAN = 16;
struct MeshCSR {
    std::vector<int> fan;
};

// ind_b, lines: bytes of the indicator and x-rows of the lattice when the
// droplet has a viscosity ratio, else 0.
Layout make_layout(int storage, long long N, int ntiles, int nv, int nt, size_t nhalo, int copies, size_t ind_b = 0,
                   size_t lines = 0, bool det = false) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes > 0 ? bytes : 1);
        return o;
    };
    const size_t sb = storage_bytes(storage), rb = real_bytes(storage);
    L.f[0] = take(19ull * N * sb);
    L.f[1] = copies == 2 ? take(19ull * N * sb) : L.f[0];
    L.F = take(3ull * N * rb);
    L.u = take(3ull * N * rb);
    L.mark = take(sizeof(int) * (size_t)ntiles);
    L.ctl = take(sizeof(Ctl));
    const size_t v4 = 4 * rb * (size_t)nv;
    L.r = take(v4);
    L.o = take(v4);
    L.qa = take(v4);
    L.qb = take(v4);
    L.pp = take(v4);
    L.bb = take(v4);
    L.tris = take(sizeof(int4) * (size_t)nt);
    L.fan = take(sizeof(int) * FAN * (size_t)nv);
    L.lfan = take(sizeof(int) * FAN * (size_t)nv);
    L.hstart = take(sizeof(int) * ((size_t)(nv + IB_PATCH - 1) / IB_PATCH + 1));
    L.hids = take(sizeof(int) * nhalo);
    L.obs_part = take(sizeof(double) * 16 * OBS_BLOCKS);
    L.mass_part = take(sizeof(double) * 4 * MASS_BLOCKS);
    L.obs_out = take(sizeof(double) * OBS_OUT_N);
    L.Abuf = take(sizeof(double) * 9 * (ACAP + 1));
    L.red = take(sizeof(unsigned long long) * (RED_SLOTS + 1));
    L.ind = take(ind_b);
    L.ind_lines = take(sizeof(int) * 2 * lines);
    L.ptris = take(ind_b ? sizeof(int4) * (size_t)nt : 0);
    L.ptstart = take(ind_b ? sizeof(int) * ((size_t)(nv + IB_PATCH - 1) / IB_PATCH + 1) : 0);
    L.perm = take(sizeof(int) * (size_t)nv);
    const size_t npatch = (size_t)(nv + IB_PATCH - 1) / IB_PATCH;
    L.det = take(det ? det_rec_bytes(storage) * (size_t)nv : 0);
    L.pbox = take(det ? sizeof(int) * 8 * npatch : 0);
    L.total = off;
    return L;
}

// A viscosity ratio other than 1 (0 selects 1) with a droplet to define the inside.
bool chi_active(const ibm_lb_config* c) { return c->chi != 0.0 && c->chi != 1.0 && c->n_vertices > 0; }

// Validate the configuration and build the mesh adjacency.
int validate(const ibm_lb_config* c) {
    if (!c) return fail(IBM_LB_EINVAL, "config is NULL");
    for (int a = 0; a < 3; ++a)
        if (c->L[a] < 8) return fail(IBM_LB_EINVAL, "every box side needs at least 8 nodes");
    // population and field offsets are 64-bit; node coordinates and tile
    // indices are 32-bit
    if ((long long)c->L[0] * c->L[1] * c->L[2] > 0x7fffffffll)
        return fail(IBM_LB_EINVAL, "box above 2^31 - 1 nodes");
    if (!(c->tau > 0.5)) return fail(IBM_LB_EINVAL, "tau must exceed 1/2");
    if (!(c->sigma >= 0.0)) return fail(IBM_LB_EINVAL, "sigma must be >= 0");
    if (!(c->radius > 0.0)) return fail(IBM_LB_EINVAL, "radius must be > 0");
    if (!(c->rho0 > 0.0)) return fail(IBM_LB_EINVAL, "rho0 must be > 0");
    if (c->storage < IBM_LB_F64 || c->storage > IBM_LB_BF16DEV)
        return fail(IBM_LB_EINVAL, "unknown storage format");
    if (c->init != IBM_LB_INIT_LINEAR && c->init != IBM_LB_INIT_REST)
        return fail(IBM_LB_EINVAL, "unknown init mode");
    for (int k = 0; k < 9; ++k)
        if (!isfinite(c->A0[k])) return fail(IBM_LB_EINVAL, "A0 is not finite");
    if (c->storage == IBM_LB_F16DEV && c->f16_scale != 0.0) {
        int ex;
        double m = frexp(c->f16_scale, &ex);
        if (!(c->f16_scale >= 1.0) || m != 0.5 || c->f16_scale > 65536.0)
            return fail(IBM_LB_EINVAL, "f16_scale must be a power of two in [1, 65536]");
    }
    if (c->populations < 0 || c->populations > 2) return fail(IBM_LB_EINVAL, "populations must be 0, 1 or 2");
    if (c->collision != IBM_LB_BGK && c->collision != IBM_LB_MRT) return fail(IBM_LB_EINVAL, "unknown collision");
    for (int k = 0; k < 5; ++k)
        if (!(c->mrt_s[k] >= 0.0 && c->mrt_s[k] < 2.0)) return fail(IBM_LB_EINVAL, "MRT rates must lie in (0, 2)");
    if (c->walls != IBM_LB_WALLS_LINK && c->walls != IBM_LB_WALLS_WET) return fail(IBM_LB_EINVAL, "unknown walls");
    if (c->walls == IBM_LB_WALLS_WET && c->populations == 1)
        return fail(IBM_LB_EINVAL, "wet-node walls run with two population copies");
    if (!(c->chi >= 0.0 && c->chi <= 1e6)) return fail(IBM_LB_EINVAL, "chi must lie in [0, 1e6]");
    if (chi_active(c) && c->collision != IBM_LB_BGK) return fail(IBM_LB_EINVAL, "a viscosity ratio runs BGK");
    if (c->deterministic != 0 && c->deterministic != 1) return fail(IBM_LB_EINVAL, "deterministic must be 0 or 1");
    const int nv = c->n_vertices, nt = c->n_triangles;
    if (nv < 0 || nt < 0) return fail(IBM_LB_EINVAL, "negative mesh size");
    if (nv == 0 && nt == 0) return IBM_LB_OK;
    if (nv < 4 || nt < 4 || !c->vertices || !c->triangles)
        return fail(IBM_LB_EINVAL, "a mesh needs >= 4 vertices, >= 4 triangles and both arrays");
    if (c->reg_max_iter < 0) return fail(IBM_LB_EINVAL, "reg_max_iter must be >= 0");
    if (c->reg_max_iter > 0) {
        if (!(c->reg_alpha >= 0.0 && c->reg_alpha <= 1.0) || !(c->reg_gamma >= 0.0 && c->reg_gamma <= 1.0))
            return fail(IBM_LB_EINVAL, "reg_alpha and reg_gamma must lie in [0, 1]");
        if (c->reg_sign != 1 && c->reg_sign != -1) return fail(IBM_LB_EINVAL, "reg_sign must be +1 or -1");
        if (!(c->reg_tol >= 0.0) && !(c->reg_tol < 0.0)) return fail(IBM_LB_EINVAL, "reg_tol is NaN");
    }
    for (int k = 0; k < 3 * nv; ++k)
        if (!isfinite(c->vertices[k])) return fail(IBM_LB_EINVAL, "vertex coordinate not finite");
    const int32_t* T = c->triangles;
    for (int k = 0; k < 3 * nt; ++k)
        if (T[k] < 0 || T[k] >= nv) return fail(IBM_LB_EINVAL, "triangle index out of range");
    // closed, consistently oriented: every directed edge once, with its reverse
    std::map<std::pair<int, int>, int> edges;
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j) {
            int a = T[3 * t + j], b = T[3 * t + (j + 1) % 3];
            if (a == b) return fail(IBM_LB_EINVAL, "degenerate triangle");
            if (++edges[{a, b}] > 1) return fail(IBM_LB_EINVAL, "mesh is not consistently oriented");
        }
    for (auto& e : edges)
        if (!edges.count({e.first.second, e.first.first}))
            return fail(IBM_LB_EINVAL, "mesh is not closed");
    // outward orientation: positive enclosed volume
    double vol = 0.0;
    for (int t = 0; t < nt; ++t) {
        const double* a = c->vertices + 3 * T[3 * t];
        const double* b = c->vertices + 3 * T[3 * t + 1];
        const double* d = c->vertices + 3 * T[3 * t + 2];
        vol += (a[0] * (b[1] * d[2] - b[2] * d[1]) + a[1] * (b[2] * d[0] - b[0] * d[2]) +
                a[2] * (b[0] * d[1] - b[1] * d[0])) / 6.0;
    }
    if (!(vol > 0.0)) return fail(IBM_LB_EINVAL, "mesh encloses a non-positive volume (inward?)");
    // stencils inside the wall axes
    for (int k = 0; k < nv; ++k)
        for (int a = 0; a < 3; ++a) {
            if (c->periodic[a]) continue;
            double fl = floor(c->vertices[3 * k + a]);
            if (fl - 1.0 < 0.0 || fl + 2.0 > c->L[a] - 1)
                return fail(IBM_LB_EINVAL, "a vertex stencil leaves the box across a wall");
        }
    return IBM_LB_OK;
}

// Recursive bisection of the vertex set along the longest axis of its
// bounding box, splitting at a multiple of IB_PATCH vertices: every run of
// IB_PATCH consecutive vertices in the resulting order (one work-group's
// patch) is spatially compact.
void bisect(const double* V, int* idx, int n, std::vector<int>* out) {
    if (n <= IB_PATCH) {
        out->insert(out->end(), idx, idx + n);
        return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < n; ++k)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], V[3 * idx[k] + a]);
            hi[a] = std::max(hi[a], V[3 * idx[k] + a]);
        }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
        if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    int nl = ((n / 2 + IB_PATCH - 1) / IB_PATCH) * IB_PATCH;
    if (nl >= n) nl = n - IB_PATCH;
    std::nth_element(idx, idx + nl, idx + n, [&](int p, int q) {
        const double vp = V[3 * p + ax], vq = V[3 * q + ax];
        return vp < vq || (vp == vq && p < q);
    });
    bisect(V, idx, nl, out);
    bisect(V, idx + nl, n - nl, out);
}

// Internal vertex order (perm[new] = old) from the bisection above.
// Triangles are renumbered and sorted by their lowest new corner index; each
// keeps its corner order (orientation).
void renumber(const ibm_lb_config* c, std::vector<int>* perm, std::vector<int>* tris) {
    const int nv = c->n_vertices, nt = c->n_triangles;
    std::vector<int> idx(nv);
    for (int k = 0; k < nv; ++k) idx[k] = k;
    perm->clear();
    perm->reserve(nv);
    bisect(c->vertices, idx.data(), nv, perm);
    std::vector<int> inv(nv);
    for (int k = 0; k < nv; ++k) inv[(*perm)[k]] = k;
    std::vector<std::pair<int, int>> order(nt);
    for (int t = 0; t < nt; ++t) {
        int a = inv[c->triangles[3 * t]], b = inv[c->triangles[3 * t + 1]], d = inv[c->triangles[3 * t + 2]];
        order[t] = {std::min(a, std::min(b, d)), t};
    }
    std::stable_sort(order.begin(), order.end());
    tris->resize(3 * (size_t)nt);
    for (int j = 0; j < nt; ++j) {
        const int t = order[j].second;
        for (int q = 0; q < 3; ++q) (*tris)[3 * j + q] = inv[c->triangles[3 * t + q]];
    }
}

// Ordered one-rings of the internal numbering (see FAN). A vertex whose
// incident triangles do not form a single fan (non-manifold) or whose
// valence exceeds FAN - 1 is rejected.
int build_adjacency(int nv, int nt, const int* T, MeshCSR* csr) {
    std::vector<std::vector<std::pair<int, int>>> inc(nv);
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j) inc[T[3 * t + j]].push_back({T[3 * t + (j + 1) % 3], T[3 * t + (j + 2) % 3]});
    csr->fan.assign((size_t)FAN * nv, -1);
    for (int v = 0; v < nv; ++v) {
        auto& e = inc[v];
        const int m = (int)e.size();
        if (m < 3) return fail(IBM_LB_EINVAL, "vertex with fewer than three incident triangles");
        if (m > FAN - 1) return fail(IBM_LB_EINVAL, "vertex valence above 15 is not supported");
        int* f = &csr->fan[(size_t)FAN * v];
        f[0] = m;
        int cur = 0;
        std::vector<char> used(m, 0);
        for (int j = 0; j < m; ++j) {
            used[cur] = 1;
            f[1 + j] = e[cur].first;
            const int want = e[cur].second;
            int nxt = -1;
            for (int q = 0; q < m; ++q)
                if (!used[q] && e[q].first == want) nxt = q;
            if (j + 1 < m) {
                if (nxt < 0) return fail(IBM_LB_EINVAL, "non-manifold vertex (incident triangles are not one fan)");
                cur = nxt;
            } else if (want != f[1]) {
                return fail(IBM_LB_EINVAL, "non-manifold vertex (fan does not close)");
            }
        }
    }
    return IBM_LB_OK;
}

// Halos of the surface patches: for patch p (internal vertices
// [IB_PATCH p, IB_PATCH (p+1))), the ring neighbours of its vertices that lie
// outside it, ascending, in hids[hstart[p] .. hstart[p+1]); and every vertex's
// fan in patch-local slots: slot j < IB_PATCH is vertex IB_PATCH p + j, slot
// IB_PATCH + h the h-th halo vertex of the patch.
struct Halos {
    std::vector<int> hstart, hids, lfan;
};

void build_halos(int nv, const MeshCSR& csr, Halos* hl) {
    const int np = (nv + IB_PATCH - 1) / IB_PATCH;
    hl->hstart.assign(np + 1, 0);
    hl->hids.clear();
    hl->lfan.assign((size_t)FAN * nv, -1);
    for (int p = 0; p < np; ++p) {
        const int lo = p * IB_PATCH, hi = std::min(nv, lo + IB_PATCH);
        std::vector<int> h;
        for (int k = lo; k < hi; ++k) {
            const int* f = &csr.fan[(size_t)FAN * k];
            for (int j = 0; j < f[0]; ++j)
                if (f[1 + j] < lo || f[1 + j] >= hi) h.push_back(f[1 + j]);
        }
        std::sort(h.begin(), h.end());
        h.erase(std::unique(h.begin(), h.end()), h.end());
        for (int k = lo; k < hi; ++k) {
            const int* f = &csr.fan[(size_t)FAN * k];
            int* g = &hl->lfan[(size_t)FAN * k];
            g[0] = f[0];
            for (int j = 0; j < f[0]; ++j) {
                const int v = f[1 + j];
                g[1 + j] = (v >= lo && v < hi) ? v - lo
                                                : IB_PATCH + int(std::lower_bound(h.begin(), h.end(), v) - h.begin());
            }
        }
        hl->hids.insert(hl->hids.end(), h.begin(), h.end());
        hl->hstart[p + 1] = (int)hl->hids.size();
    }
}

struct MeshData {
    std::vector<int> perm, tris;
    MeshCSR csr;
    Halos halos;
};

int prepare(const ibm_lb_config* c, MeshData* m) {
    int rc = validate(c);
    if (rc || c->n_vertices == 0) return rc;
    renumber(c, &m->perm, &m->tris);
    rc = build_adjacency(c->n_vertices, c->n_triangles, m->tris.data(), &m->csr);
    if (rc) return rc;
    build_halos(c->n_vertices, m->csr, &m->halos);
    return IBM_LB_OK;
}

Geom make_geom(const ibm_lb_config* c) {
    Geom g{};
    g.Lx = c->L[0];
    g.Ly = c->L[1];
    g.Lz = c->L[2];
    g.px = c->periodic[0] ? 1 : 0;
    g.py = c->periodic[1] ? 1 : 0;
    g.pz = c->periodic[2] ? 1 : 0;
    g.TX = (g.Lx + 7) >> 3;
    g.TY = (g.Ly + 7) >> 3;
    g.TZ = (g.Lz + 7) >> 3;
    g.N = (long long)g.Lx * g.Ly * g.Lz;
    for (int a = 0; a < 3; ++a) {
        double xc = (c->L[a] - 1) / 2.0;
        g.xci[a] = (int)floor(xc);
        g.xcf[a] = xc - g.xci[a];
    }
    return g;
}

}  // namespace

// ---------------------------------------------------------------- allocation-free staging
// Device memory of ibm_lb_read_vertices_noalloc: one file-scope array, a copy
// of it on every GPU the library runs on, held until the process ends. Host
// code never passes the array's name (a host-side stand-in) to a kernel or a
// copy: it uses the address hipGetSymbolAddress gives on each device,
// resolved once per device in ibm_lb_init with that device current.
static __device__ __align__(256) double scratch[3 * IBM_LB_NOALLOC_MAX_VERTICES];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_addr[SCRATCH_DEVICES] = {};

// This device's address of `scratch` (dev is the current device).
hipError_t resolve_scratch(int dev, double** out) {
    *out = nullptr;
    if (dev < 0 || dev >= SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_addr[dev] = (double*)p;
    }
    *out = scratch_addr[dev];
    return hipSuccess;
}

// Absolute vertex coordinates in the caller's vertex order:
// out[3 perm[k] + a] = r_k,a + x_c,a.
template <class R>
__global__ void k_vertices_caller_order(Geom g, int nv, const V4<R>* __restrict__ r, const int* __restrict__ perm,
                                        double* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    const V4<R> p = r[k];
    double* o = out + 3ll * perm[k];
    o[0] = double(p.x) + (g.xci[0] + g.xcf[0]);
    o[1] = double(p.y) + (g.xci[1] + g.xcf[1]);
    o[2] = double(p.z) + (g.xci[2] + g.xcf[2]);
}

}  // namespace

struct ibm_lb {
    ibm_lb_config cfg;
    int storage = 0, nv = 0, nt = 0, device = 0;
    Geom g{};
    LatticeParams lp{};
    SmoothParams sp{};
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    Layout lay{};
    DevPtrs d{};
    int cur = 0;
    int64_t step = 0;
    int sticky = IBM_LB_OK;
    bool f_ready = false;        // F and tile marks hold the spread of the current mesh
    std::vector<int> perm;       // internal vertex k is caller vertex perm[k]
    int lattice_variant = 1 | VAR_HC_SPLIT;  // non-temporal loads, 128-thread work-groups, split smoothing
    int aa_parity = 0;           // in-place variants: 1 after an even step (f[cur] not in natural order)
    bool single = false;         // one population copy (f[1] aliases f[0]; in-place variants only)
    bool wet = false;            // wet-node velocity walls after every lattice step
    bool mrt = false;            // MRT collision with the rates below
    MrtRates mrt_rates{};
    bool chi = false;            // viscosity ratio: inner rates on the nodes inside the mesh
    ChiRates chi_rates{};
    double* stage = nullptr;     // pinned host staging for gradient rows
    hipEvent_t stage_done = nullptr;
    bool timing = false;
    // lattice timing: an event pool and (start, stop) pool indices per launch;
    // a launch is timed from the completion of the dispatch before it to its
    // own completion, both stamped by the dispatches themselves
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    std::vector<std::pair<int, int>> iv;
    int ev_pending = -1;  // pool index stamped by the last dispatch, or -1
    double acc_ms = 0.0;
    int64_t launches = 0;
    // adjoint buffers (allocated on first use, grown with the segment length)
    char* adj = nullptr;
    int adj_cap = 0;             // steps the records hold
    double* adj_fb[2] = {nullptr, nullptr};
    double *adj_ubar = nullptr, *adj_Fbar = nullptr, *adj_Apart = nullptr, *adj_spart = nullptr,
           *adj_coef = nullptr, *adj_rec = nullptr;
    double4* adj_pos = nullptr;
    int* adj_iters = nullptr;
    int* adj_perm = nullptr;
    AdjVerts adj_v{};
    double* scratch = nullptr;   // this device's address of the allocation-free staging array
};

namespace {

int set_device(ibm_lb* h) {
    HIP_TRY(hipSetDevice(h->device), "hipSetDevice");
    return IBM_LB_OK;
}

// Read the device flags after a synchronisation; record a sticky error.
int check_flags(ibm_lb* h) {
    Ctl c;
    HIP_TRY(hipMemcpy(&c, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost), "read flags");
    if (c.flags & DFLAG_NONFINITE) {
        h->sticky = IBM_LB_ENONFINITE;
        return fail(IBM_LB_ENONFINITE, "non-finite or non-positive density, velocity or position");
    }
    if (c.flags & DFLAG_DOMAIN) {
        h->sticky = IBM_LB_EDOMAIN;
        return fail(IBM_LB_EDOMAIN, "a vertex stencil left the box across a wall");
    }
    return IBM_LB_OK;
}

int sync_and_check(ibm_lb* h) {
    HIP_TRY(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return check_flags(h);
}

int accumulate_timing(ibm_lb* h) {
    for (size_t k = 0; k < h->ev_used; ++k) HIP_TRY(hipEventSynchronize(h->ev[k]), "hipEventSynchronize");
    for (const auto& p : h->iv) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, h->ev[p.first], h->ev[p.second]), "hipEventElapsedTime");
        h->acc_ms += ms;
    }
    h->launches += (int64_t)h->iv.size();
    h->iv.clear();
    h->ev_used = 0;
    h->ev_pending = -1;
    return IBM_LB_OK;
}

// Next event of the timing pool. Timing-only events without the
// system-scope fence: their stamps do not wait for a write-back of the L2
// to memory (which untimed launches overlap with later work); no data is
// read through them.
int take_event(ibm_lb* h, int* idx) {
    if (h->ev_used == h->ev.size()) {
        hipEvent_t e;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "hipEventCreate");
        h->ev.push_back(e);
    }
    *idx = (int)h->ev_used++;
    return IBM_LB_OK;
}

// Forces and spreading of the current mesh into F (marks at the current
// epoch), needed before the first lattice kernel after set-up or a load.
// With a viscosity ratio, also the indicator of the current mesh.
int ensure_force(ibm_lb* h) {
    if (h->f_ready || h->nv == 0) return IBM_LB_OK;
    if (h->chi) HIP_TRY(launch_indicator_clear(h->g, h->d, h->stream), "indicator clear");
    HIP_TRY(launch_ib_pre(h->storage, h->g, h->d, h->nv, h->cfg.sigma, h->sp, h->stream), "ib_pre launch");
    if (h->chi) HIP_TRY(launch_indicator_scan(h->g, h->d, h->stream, nullptr), "indicator launch");
    h->f_ready = true;
    return IBM_LB_OK;
}

// Enqueue nsteps timesteps; step j reads the gradient row A + 9 j*stride.
// Per step: the fused lattice kernel (which consumes F^n and writes u^n in
// the marked tiles), then the IB half: interpolation + Euler, smoothing and
// the next step's forces + spreading.
// Populations of f[cur] in natural order (after an even in-place step, one
// in-place pass of pairwise swaps); every reader of the populations and
// every change of layout calls this first.
int ensure_natural(ibm_lb* h) {
    if (!h->aa_parity) return IBM_LB_OK;
    HIP_TRY(launch_aa_settle(h->storage, h->g, h->d, h->cur, h->stream), "settle launch");
    h->aa_parity = 0;
    return IBM_LB_OK;
}

// keep_last: copy the last row used into the gradient slot that later calls
// (observables, wet-node walls of the next step) read; a caller that issues a
// run one step at a time asks for it on the run's last step only.
int enqueue_steps(ibm_lb* h, const double* A, int nsteps, int stride, bool keep_last = true) {
    const bool ib = h->nv > 0;
    int rc = ensure_force(h);
    if (rc) return rc;
    const bool aa = (h->lattice_variant & VAR_AA) != 0;
    if (!aa && (rc = ensure_natural(h))) return rc;
    h->ev_pending = -1;  // other work may have been queued since the last stamp
    for (int j = 0; j < nsteps; ++j) {
        const double* Arow = A + 9ll * j * stride;
        hipEvent_t e1 = nullptr, done = nullptr;
        int k0 = -1, k1 = -1, kd = -1;
        if (h->timing) {
            if (h->iv.size() >= 4096) {
                rc = accumulate_timing(h);
                if (rc) return rc;
            }
            if (h->ev_pending >= 0) {
                k0 = h->ev_pending;
            } else {
                if ((rc = take_event(h, &k0))) return rc;
                HIP_TRY(hipEventRecord(h->ev[k0], h->stream), "hipEventRecord");
            }
            if ((rc = take_event(h, &k1))) return rc;
            if (ib && (rc = take_event(h, &kd))) return rc;
            e1 = h->ev[k1];
            done = ib ? h->ev[kd] : nullptr;
        }
        HIP_TRY(launch_lattice(h->storage, h->g, h->lp, h->d, h->cur, ib, Arow, h->lattice_variant, h->aa_parity,
                               h->stream, nullptr, e1, h->mrt ? &h->mrt_rates : nullptr,
                               h->chi ? &h->chi_rates : nullptr),
                "lattice launch");
        if (h->wet)
            HIP_TRY(launch_wet_walls(h->storage, h->g, h->lp, h->d, h->cur ^ 1, Arow, h->stream), "walls launch");
        if (ib)
            HIP_TRY(launch_ib_step(h->storage, h->g, h->d, h->nv, h->cfg.sigma, h->sp, h->stream,
                                   h->chi ? nullptr : done, (h->lattice_variant & VAR_HC_SPLIT) != 0),
                    "ib_step launch");
        if (h->chi) HIP_TRY(launch_indicator_scan(h->g, h->d, h->stream, done), "indicator launch");
        if (h->timing) {
            h->iv.push_back({k0, k1});
            h->ev_pending = ib ? kd : k1;
        }
        if (aa) h->aa_parity ^= 1;
        else h->cur ^= 1;
        h->step++;
    }
    if (nsteps > 0 && keep_last) {
        const double* last = A + 9ll * (nsteps - 1) * stride;
        double* slot = h->d.Abuf + 9ll * ACAP;
        if (last != slot)
            HIP_TRY(hipMemcpyAsync(slot, last, 9 * sizeof(double), hipMemcpyDeviceToDevice, h->stream),
                    "copy last gradient");
    }
    return IBM_LB_OK;
}

// Copy n host gradient rows into the device gradient buffer (through pinned
// staging, so the caller's array may change once this returns).
int upload_rows(ibm_lb* h, const double* A, int n) {
    HIP_TRY(hipEventSynchronize(h->stage_done), "staging wait");
    memcpy(h->stage, A, sizeof(double) * 9 * (size_t)n);
    HIP_TRY(hipMemcpyAsync(h->d.Abuf, h->stage, sizeof(double) * 9 * (size_t)n, hipMemcpyHostToDevice,
                           h->stream),
            "upload gradient rows");
    HIP_TRY(hipEventRecord(h->stage_done, h->stream), "hipEventRecord");
    return IBM_LB_OK;
}

}  // namespace

extern "C" {

const char* ibm_lb_strerror(int code) {
    switch (code) {
        case IBM_LB_OK: return "ok";
        case IBM_LB_EINVAL: return "invalid argument";
        case IBM_LB_ENOMEM: return "out of memory";
        case IBM_LB_EDEVICE: return "HIP runtime error";
        case IBM_LB_EDOMAIN: return "vertex stencil outside the box";
        case IBM_LB_ENONFINITE: return "non-finite state";
        default: return "unknown error";
    }
}

const char* ibm_lb_last_error(void) { return g_last_error; }

int ibm_lb_workspace_size(const ibm_lb_config* cfg, size_t* bytes) {
    MeshData m;
    int rc = prepare(cfg, &m);
    if (rc) return rc;
    if (!bytes) return fail(IBM_LB_EINVAL, "bytes is NULL");
    Geom g = make_geom(cfg);
    const bool chi = chi_active(cfg);
    *bytes = make_layout(cfg->storage, g.N, g.TX * g.TY * g.TZ, cfg->n_vertices, cfg->n_triangles,
                         m.halos.hids.size(), cfg->populations == 1 ? 1 : 2, chi ? ind_bytes(g) : 0,
                         chi ? (size_t)g.Ly * g.Lz : 0, cfg->deterministic == 1 && cfg->n_vertices > 0)
                 .total;
    return IBM_LB_OK;
}

int ibm_lb_init(const ibm_lb_config* cfg, ibm_lb** out) {
    if (!out) return fail(IBM_LB_EINVAL, "out is NULL");
    *out = nullptr;
    MeshData mesh;
    int rc = prepare(cfg, &mesh);
    if (rc) return rc;
    const MeshCSR& csr = mesh.csr;
    ibm_lb* h = new (std::nothrow) ibm_lb();
    if (!h) return fail(IBM_LB_ENOMEM, "host allocation");
    h->cfg = *cfg;
    h->cfg.vertices = nullptr;
    h->cfg.triangles = nullptr;
    h->storage = cfg->storage;
    h->nv = cfg->n_vertices;
    h->nt = cfg->n_triangles;
    h->stream = (hipStream_t)cfg->stream;
    h->g = make_geom(cfg);
    h->lp.omega = 1.0 / cfg->tau;
    h->lp.kguo = 1.0 - 1.0 / (2.0 * cfg->tau);
    h->lp.rho0 = cfg->rho0;
    h->lp.tau = cfg->tau;
    double sc = (cfg->storage == IBM_LB_F16DEV) ? (cfg->f16_scale == 0.0 ? 4096.0 : cfg->f16_scale) : 1.0;
    h->lp.scale = (float)sc;
    h->lp.inv_scale = (float)(1.0 / sc);
    h->sp.alpha = cfg->reg_alpha;
    h->sp.gamma = cfg->reg_gamma;
    h->sp.tol = cfg->reg_tol;
    h->sp.max_iter = cfg->reg_max_iter;
    h->sp.sign = cfg->reg_sign == -1 ? -1 : 1;
    auto bail = [&](int code) {
        ibm_lb_destroy(h);
        return code;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return bail(hip_fail(e, "hipGetDevice"));
    // the allocation-free read's staging array on this device (an unresolved
    // address only disables that entry point)
    if (resolve_scratch(h->device, &h->scratch) != hipSuccess) h->scratch = nullptr;
    const int ntiles = h->g.TX * h->g.TY * h->g.TZ;
    h->single = cfg->populations == 1;
    h->mrt = cfg->collision == IBM_LB_MRT;
    h->wet = cfg->walls == IBM_LB_WALLS_WET;
    h->chi = chi_active(cfg);
    if (h->chi) {
        const double tau_in = 0.5 + cfg->chi * (cfg->tau - 0.5);  // nu_in = chi nu
        h->chi_rates.omega_in = 1.0 / tau_in;
        h->chi_rates.kguo_in = 1.0 - 1.0 / (2.0 * tau_in);
    }
    if (h->mrt) {
        // per moment of the basis: conserved density and momentum and the five
        // shear moments at 1/tau, the others from the configuration
        static const double dflt[5] = {1.19, 1.4, 1.2, 1.4, 1.98};
        double r[5];
        for (int k = 0; k < 5; ++k) r[k] = cfg->mrt_s[k] > 0.0 ? cfg->mrt_s[k] : dflt[k];
        const double sv = 1.0 / cfg->tau;
        const double rate[19] = {sv, r[0], r[1], sv, r[2], sv, r[2], sv, r[2],
                                 sv, r[3], sv, r[3], sv, sv, sv, r[4], r[4], r[4]};
        for (int k = 0; k < 19; ++k) h->mrt_rates.s[k] = rate[k];
    }
    if (h->single) h->lattice_variant = VAR_AA | VAR_HC_SPLIT;
    const bool det = cfg->deterministic == 1 && h->nv > 0;
    h->lay = make_layout(h->storage, h->g.N, ntiles, h->nv, h->nt, mesh.halos.hids.size(), h->single ? 1 : 2,
                         h->chi ? ind_bytes(h->g) : 0, h->chi ? (size_t)h->g.Ly * h->g.Lz : 0, det);
    if (cfg->workspace) {
        if (cfg->workspace_bytes < h->lay.total)
            return bail(fail(IBM_LB_ENOMEM, "workspace smaller than ibm_lb_workspace_size"));
        if (((uintptr_t)cfg->workspace) % ALIGN)
            return bail(fail(IBM_LB_EINVAL, "workspace must be 256-byte aligned"));
        h->ws = (char*)cfg->workspace;
        h->ws_bytes = cfg->workspace_bytes;
    } else {
        e = hipMalloc((void**)&h->ws, h->lay.total);
        if (e != hipSuccess) return bail(fail(IBM_LB_ENOMEM, "hipMalloc of the workspace failed"));
        h->own_ws = true;
        h->ws_bytes = h->lay.total;
    }
    e = hipHostMalloc((void**)&h->stage, sizeof(double) * 9 * ACAP, hipHostMallocDefault);
    if (e != hipSuccess) return bail(fail(IBM_LB_ENOMEM, "pinned staging allocation"));
    e = hipEventCreateWithFlags(&h->stage_done, hipEventDisableTiming);
    if (e != hipSuccess) return bail(hip_fail(e, "hipEventCreate"));
    e = hipEventRecord(h->stage_done, h->stream);
    if (e != hipSuccess) return bail(hip_fail(e, "hipEventRecord"));

    char* b = h->ws;
    const Layout& L = h->lay;
    DevPtrs& d = h->d;
    d.f[0] = b + L.f[0];
    d.f[1] = b + L.f[1];
    d.F = b + L.F;
    d.u = b + L.u;
    d.mark = (int*)(b + L.mark);
    d.ctl = (Ctl*)(b + L.ctl);
    d.r = b + L.r;
    d.o = b + L.o;
    d.qa = b + L.qa;
    d.qb = b + L.qb;
    d.pp = b + L.pp;
    d.bb = b + L.bb;
    d.tris = (int4*)(b + L.tris);
    d.fan = (int4*)(b + L.fan);
    d.lfan = (int4*)(b + L.lfan);
    d.hstart = (int*)(b + L.hstart);
    d.hids = (int*)(b + L.hids);
    d.obs_part = (double*)(b + L.obs_part);
    d.mass_part = (double*)(b + L.mass_part);
    d.obs_out = (double*)(b + L.obs_out);
    d.Abuf = (double*)(b + L.Abuf);
    d.red = (unsigned long long*)(b + L.red);
    d.ind = h->chi ? (unsigned char*)(b + L.ind) : nullptr;
    d.ind_lines = h->chi ? (int*)(b + L.ind_lines) : nullptr;
    d.ptris = h->chi ? (int4*)(b + L.ptris) : nullptr;
    d.ptstart = h->chi ? (int*)(b + L.ptstart) : nullptr;
    d.perm = (int*)(b + L.perm);
    d.det = det ? (void*)(b + L.det) : nullptr;
    d.pbox = det ? (int*)(b + L.pbox) : nullptr;
    h->perm = mesh.perm;
    if (h->nv > 0) {
        e = patch_setup(h->storage);
        if (e != hipSuccess) return bail(hip_fail(e, "patch kernel set-up"));
    }

    // Zero the fields that must start at zero (force, velocity, marks, control).
    const size_t rb = real_bytes(h->storage);
#define INIT_TRY(expr, where)                        \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return bail(hip_fail(e_, where)); \
    } while (0)
    INIT_TRY(hipMemsetAsync(d.F, 0, 3 * rb * (size_t)h->g.N, h->stream), "zero F");
    INIT_TRY(hipMemsetAsync(d.u, 0, 3 * rb * (size_t)h->g.N, h->stream), "zero u");
    INIT_TRY(hipMemsetAsync(d.mark, 0, sizeof(int) * (size_t)ntiles, h->stream), "zero marks");
    INIT_TRY(hipMemsetAsync(d.red, 0, (RED_SLOTS + 1) * sizeof(unsigned long long), h->stream),
             "zero reduction slots");
    Ctl ctl0{};
    ctl0.epoch = 1;
    INIT_TRY(hipMemcpyAsync(d.ctl, &ctl0, sizeof(Ctl), hipMemcpyHostToDevice, h->stream), "ctl");
    INIT_TRY(hipStreamSynchronize(h->stream), "sync");  // ctl0 is a stack value
    // initial gradient in the last-gradient slot; the initial populations read it
    double* slot = d.Abuf + 9ll * ACAP;
    INIT_TRY(hipMemcpy(slot, cfg->A0, 9 * sizeof(double), hipMemcpyHostToDevice), "A0");
    if (h->nv > 0) {
        std::vector<int4> tris(h->nt);
        for (int t = 0; t < h->nt; ++t)
            tris[t] = int4{mesh.tris[3 * t], mesh.tris[3 * t + 1], mesh.tris[3 * t + 2], 0};
        INIT_TRY(hipMemcpy(d.tris, tris.data(), sizeof(int4) * h->nt, hipMemcpyHostToDevice), "tris");
        if (h->chi) {
            // each triangle goes to the patch of its lowest vertex id, patch by patch
            const int npatch = (h->nv + IB_PATCH - 1) / IB_PATCH;
            std::vector<int> start(npatch + 1, 0);
            auto owner = [&](const int4& t) { return std::min(t.x, std::min(t.y, t.z)) / IB_PATCH; };
            for (const int4& t : tris) start[owner(t) + 1]++;
            for (int q = 0; q < npatch; ++q) start[q + 1] += start[q];
            std::vector<int4> pt(h->nt);
            std::vector<int> fill(start.begin(), start.end() - 1);
            for (const int4& t : tris) pt[fill[owner(t)]++] = t;
            INIT_TRY(hipMemcpy(d.ptris, pt.data(), sizeof(int4) * h->nt, hipMemcpyHostToDevice), "patch triangles");
            INIT_TRY(hipMemcpy(d.ptstart, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice),
                     "patch triangle starts");
        }
        INIT_TRY(hipMemcpy(d.fan, csr.fan.data(), sizeof(int) * csr.fan.size(), hipMemcpyHostToDevice), "fan");
        INIT_TRY(hipMemcpy(d.perm, mesh.perm.data(), sizeof(int) * h->nv, hipMemcpyHostToDevice), "perm");
        const Halos& hl = mesh.halos;
        INIT_TRY(hipMemcpy(d.lfan, hl.lfan.data(), sizeof(int) * hl.lfan.size(), hipMemcpyHostToDevice), "lfan");
        INIT_TRY(hipMemcpy(d.hstart, hl.hstart.data(), sizeof(int) * hl.hstart.size(), hipMemcpyHostToDevice),
                 "hstart");
        if (!hl.hids.empty())
            INIT_TRY(hipMemcpy(d.hids, hl.hids.data(), sizeof(int) * hl.hids.size(), hipMemcpyHostToDevice), "hids");
        std::vector<double> vin(3 * (size_t)h->nv);
        for (int k = 0; k < h->nv; ++k)
            for (int a = 0; a < 3; ++a) vin[3 * k + a] = cfg->vertices[3 * mesh.perm[k] + a];
        double* tmp = nullptr;
        INIT_TRY(hipMalloc((void**)&tmp, sizeof(double) * 3 * h->nv), "vertex upload buffer");
        hipError_t e1 = hipMemcpy(tmp, vin.data(), sizeof(double) * 3 * h->nv, hipMemcpyHostToDevice);
        hipError_t e2 = e1 == hipSuccess
                            ? launch_positions_from_abs(h->storage, h->g, d, h->nv, tmp, h->stream)
                            : e1;
        hipError_t e3 = hipStreamSynchronize(h->stream);
        (void)hipFree(tmp);
        if (e2 != hipSuccess) return bail(hip_fail(e2, "vertex upload"));
        if (e3 != hipSuccess) return bail(hip_fail(e3, "vertex upload"));
    }
    INIT_TRY(launch_init(h->storage, h->g, h->lp, d, slot, cfg->init == IBM_LB_INIT_REST, h->stream),
             "init launch");
#undef INIT_TRY
    *out = h;
    return IBM_LB_OK;
}

int ibm_lb_step_table(ibm_lb* h, const double* A, int32_t nsteps, int32_t on_device) {
    if (!h || !A || nsteps < 0) return fail(IBM_LB_EINVAL, "bad step arguments");
    if (h->sticky) return fail(h->sticky, "earlier asynchronous error");
    int rc = set_device(h);
    if (rc) return rc;
    if (on_device) return enqueue_steps(h, A, nsteps, 1);
    for (int done = 0; done < nsteps;) {
        int n = std::min(nsteps - done, ACAP);
        rc = upload_rows(h, A + 9ll * done, n);
        if (rc) return rc;
        rc = enqueue_steps(h, h->d.Abuf, n, 1);
        if (rc) return rc;
        done += n;
    }
    return IBM_LB_OK;
}

int ibm_lb_step(ibm_lb* h, const double A[9], int32_t nsteps) {
    if (!h || !A || nsteps < 0) return fail(IBM_LB_EINVAL, "bad step arguments");
    if (h->sticky) return fail(h->sticky, "earlier asynchronous error");
    int rc = set_device(h);
    if (rc) return rc;
    for (int k = 0; k < 9; ++k)
        if (!isfinite(A[k])) return fail(IBM_LB_EINVAL, "gradient not finite");
    rc = upload_rows(h, A, 1);
    if (rc) return rc;
    return enqueue_steps(h, h->d.Abuf, nsteps, 0);
}

int ibm_lb_observables(ibm_lb* h, ibm_lb_obs* out) {
    if (!h || !out) return fail(IBM_LB_EINVAL, "bad observables arguments");
    int rc = set_device(h);
    if (rc) return rc;
    if ((rc = ensure_natural(h))) return rc;
    HIP_TRY(launch_observables(h->storage, h->g, h->lp, h->d, h->cur, h->nv, h->nt, h->cfg.radius,
                               h->d.Abuf + 9ll * ACAP, h->stream),
            "observables launch");
    double o[OBS_OUT_N];
    HIP_TRY(hipMemcpyAsync(o, h->d.obs_out, sizeof(o), hipMemcpyDeviceToHost, h->stream), "observables copy");
    rc = sync_and_check(h);
    if (rc) return rc;
    memset(out, 0, sizeof(*out));
    out->step = h->step;
    const double xc[3] = {h->g.xci[0] + h->g.xcf[0], h->g.xci[1] + h->g.xcf[1], h->g.xci[2] + h->g.xcf[2]};
    out->volume = o[0];
    for (int a = 0; a < 3; ++a) out->centroid[a] = h->nv ? o[1 + a] + xc[a] : 0.0;
    for (int k = 0; k < 9; ++k) out->S[k] = o[4 + k];
    for (int k = 0; k < 3; ++k) out->eigval[k] = o[13 + k];
    for (int k = 0; k < 9; ++k) out->eigvec[k] = o[16 + k];
    out->D = o[25];
    out->beta = o[26];
    out->theta_deg = o[27];
    out->flags = (int)o[28];
    out->mass = (double)h->g.N * h->cfg.rho0 + o[29];
    for (int a = 0; a < 3; ++a) out->momentum[a] = o[30 + a];
    out->reg_iters = (int)o[33];
    if (o[34] > 0) out->flags |= IBM_LB_OBS_REG_CAP;
    out->min_angle_deg = o[35];
    out->edge_min = o[36];
    out->edge_max = o[37];
    return IBM_LB_OK;
}

int ibm_lb_read_vertices(ibm_lb* h, double* out) {
    if (!h || (!out && h->nv)) return fail(IBM_LB_EINVAL, "bad read_vertices arguments");
    if (h->nv == 0) return IBM_LB_OK;
    int rc = set_device(h);
    if (rc) return rc;
    double* tmp = nullptr;
    HIP_TRY(hipMalloc((void**)&tmp, sizeof(double) * 3 * h->nv), "hipMalloc");
    std::vector<double> in(3 * (size_t)h->nv);
    hipError_t e = launch_positions_to_abs(h->storage, h->g, h->d, h->nv, tmp, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(in.data(), tmp, sizeof(double) * 3 * h->nv, hipMemcpyDeviceToHost, h->stream);
    hipError_t e2 = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "read vertices");
    if (e2 != hipSuccess) return hip_fail(e2, "read vertices");
    for (int k = 0; k < h->nv; ++k)
        for (int a = 0; a < 3; ++a) out[3 * h->perm[k] + a] = in[3 * k + a];
    return check_flags(h);
}

int ibm_lb_read_vertices_noalloc(ibm_lb* h, double* out) {
    if (!h || (!out && h->nv)) return fail(IBM_LB_EINVAL, "bad read_vertices_noalloc arguments");
    if (h->nv > IBM_LB_NOALLOC_MAX_VERTICES)
        return fail(IBM_LB_EINVAL, "mesh above IBM_LB_NOALLOC_MAX_VERTICES vertices (use ibm_lb_read_vertices)");
    if (h->nv == 0) return IBM_LB_OK;
    int rc = set_device(h);
    if (rc) return rc;
    if (!h->scratch) return fail(IBM_LB_EDEVICE, "device address of the staging array unresolved");
    const int blocks = (h->nv + 255) / 256;
    if (h->storage == IBM_LB_F64)
        hipLaunchKernelGGL(k_vertices_caller_order<double>, dim3(blocks), dim3(256), 0, h->stream, h->g, h->nv,
                           (const V4<double>*)h->d.r, h->d.perm, h->scratch);
    else
        hipLaunchKernelGGL(k_vertices_caller_order<float>, dim3(blocks), dim3(256), 0, h->stream, h->g, h->nv,
                           (const V4<float>*)h->d.r, h->d.perm, h->scratch);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, h->scratch, sizeof(double) * 3 * h->nv, hipMemcpyDeviceToHost, h->stream);
    const hipError_t e2 = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "read vertices (no allocation)");
    if (e2 != hipSuccess) return hip_fail(e2, "read vertices (no allocation)");
    return check_flags(h);
}

int ibm_lb_read_field(ibm_lb* h, int32_t which, double* out) {
    if (!h || !out || (which != IBM_LB_FIELD_RHO && which != IBM_LB_FIELD_U))
        return fail(IBM_LB_EINVAL, "bad read_field arguments");
    int rc = set_device(h);
    if (rc) return rc;
    if ((rc = ensure_natural(h))) return rc;
    const size_t N = (size_t)h->g.N;
    double* tmp = nullptr;
    HIP_TRY(hipMalloc((void**)&tmp, sizeof(double) * 4 * N), "hipMalloc");
    const bool ib = which == IBM_LB_FIELD_U && h->nv > 0;
    if (ib) {
        rc = ensure_force(h);
        if (rc) {
            (void)hipFree(tmp);
            return rc;
        }
    }
    hipError_t e = launch_moments(h->storage, h->g, h->lp, h->d, h->cur, ib, tmp, tmp + N, h->stream);
    if (e == hipSuccess) {
        const double* src = which == IBM_LB_FIELD_RHO ? tmp : tmp + N;
        size_t cnt = which == IBM_LB_FIELD_RHO ? N : 3 * N;
        e = hipMemcpyAsync(out, src, sizeof(double) * cnt, hipMemcpyDeviceToHost, h->stream);
    }
    hipError_t e2 = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(e, "read field");
    if (e2 != hipSuccess) return hip_fail(e2, "read field");
    return check_flags(h);
}

int ibm_lb_read_indicator(ibm_lb* h, uint8_t* out) {
    if (!h || !out) return fail(IBM_LB_EINVAL, "bad read_indicator arguments");
    if (!h->chi) return fail(IBM_LB_EINVAL, "the handle has no viscosity ratio (chi = 1 or no droplet)");
    if (h->sticky) return fail(h->sticky, "earlier asynchronous error");
    int rc = set_device(h);
    if (rc) return rc;
    if ((rc = ensure_force(h))) return rc;
    // bit 0: inside; the toggles (bit 1) are consumed within the build
    HIP_TRY(hipMemcpyAsync(out, h->d.ind, (size_t)h->g.N, hipMemcpyDeviceToHost, h->stream), "indicator copy");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    return check_flags(h);
}

namespace {
struct StateHeader {
    int64_t magic, storage, N, nv, step, pad[3];
};
constexpr int64_t STATE_MAGIC = 0x49424d4c42535431ll;
}  // namespace

size_t ibm_lb_state_bytes(const ibm_lb* h) {
    if (!h) return 0;
    return sizeof(StateHeader) + 19ull * h->g.N * storage_bytes(h->storage) +
           4ull * real_bytes(h->storage) * h->nv;
}

int ibm_lb_save(ibm_lb* h, void* dst, size_t n) {
    if (!h || !dst || n < ibm_lb_state_bytes(h)) return fail(IBM_LB_EINVAL, "bad save arguments");
    int rc = set_device(h);
    if (rc) return rc;
    if ((rc = ensure_natural(h))) return rc;
    rc = sync_and_check(h);
    if (rc) return rc;
    StateHeader hd{STATE_MAGIC, h->storage, h->g.N, h->nv, h->step, {0, 0, 0}};
    char* p = (char*)dst;
    HIP_TRY(hipMemcpy(p, &hd, sizeof(hd), hipMemcpyDefault), "save header");
    const size_t fb = 19ull * h->g.N * storage_bytes(h->storage);
    HIP_TRY(hipMemcpy(p + sizeof(hd), h->d.f[h->cur], fb, hipMemcpyDefault), "save populations");
    HIP_TRY(hipMemcpy(p + sizeof(hd) + fb, h->d.r, 4ull * real_bytes(h->storage) * h->nv, hipMemcpyDefault),
            "save vertices");
    return IBM_LB_OK;
}

int ibm_lb_load(ibm_lb* h, const void* src, size_t n) {
    if (!h || !src || n < ibm_lb_state_bytes(h)) return fail(IBM_LB_EINVAL, "bad load arguments");
    int rc = set_device(h);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    StateHeader hd;
    const char* p = (const char*)src;
    HIP_TRY(hipMemcpy(&hd, p, sizeof(hd), hipMemcpyDefault), "load header");
    if (hd.magic != STATE_MAGIC || hd.storage != h->storage || hd.N != h->g.N || hd.nv != h->nv)
        return fail(IBM_LB_EINVAL, "checkpoint does not match this configuration");
    const size_t fb = 19ull * h->g.N * storage_bytes(h->storage);
    HIP_TRY(hipMemcpy(h->d.f[h->cur], p + sizeof(hd), fb, hipMemcpyDefault), "load populations");
    h->aa_parity = 0;  // checkpoints hold natural order
    HIP_TRY(hipMemcpy(h->d.r, p + sizeof(hd) + fb, 4ull * real_bytes(h->storage) * h->nv, hipMemcpyDefault),
            "load vertices");
    h->step = hd.step;
    h->sticky = IBM_LB_OK;
    // the force field of the previous mesh is stale: clear it and retire its marks
    HIP_TRY(launch_clear_force(h->storage, h->g, h->d, h->stream), "clear force");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    Ctl c;
    HIP_TRY(hipMemcpy(&c, h->d.ctl, sizeof(Ctl), hipMemcpyDeviceToHost), "ctl");
    c.flags = 0;
    c.cap_hits = 0;
    c.epoch += 1;
    HIP_TRY(hipMemcpy(h->d.ctl, &c, sizeof(Ctl), hipMemcpyHostToDevice), "ctl");
    h->f_ready = false;
    return IBM_LB_OK;
}

namespace {
// Candidates within 1 % of the fastest count as ties (run-to-run noise of
// the timing); among them the default lattice variant wins, then the first
// in candidate order, so that repeated tuning of one configuration settles
// on one choice.
int pick_variant(const int* cand, const float* t, int nc) {
    float tmin = 1e30f;
    for (int k = 0; k < nc; ++k) tmin = std::min(tmin, t[k]);
    for (int k = 0; k < nc; ++k)
        if ((cand[k] & (VAR_HC_SPLIT - 1)) == 1 && !(cand[k] & VAR_AA) && t[k] <= 1.01f * tmin) return cand[k];
    for (int k = 0; k < nc; ++k)
        if (t[k] <= 1.01f * tmin) return cand[k];
    return cand[0];
}
}  // namespace

int ibm_lb_autotune(ibm_lb* h, int32_t reps, int32_t* variant) {
    if (!h || reps < 1) return fail(IBM_LB_EINVAL, "bad autotune arguments");
    if (h->sticky) return fail(h->sticky, "earlier asynchronous error");
    int rc = set_device(h);
    if (rc) return rc;
    // Each variant advances `reps` whole steps (lattice kernel and IB half,
    // populations alternating between the two copies as in a run) with the
    // last gradient row; the state is saved first and restored after, so the
    // call leaves it as it found it.
    const size_t nb = ibm_lb_state_bytes(h);
    void* snap = nullptr;
    if (hipMalloc(&snap, nb) != hipSuccess) {
        (void)hipGetLastError();
        return fail(IBM_LB_ENOMEM, "autotune snapshot allocation");
    }
    rc = ibm_lb_save(h, snap, nb);
    if (rc) {
        (void)hipFree(snap);
        return rc;
    }
    const bool timing = h->timing;
    const int before = h->lattice_variant;
    h->timing = false;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    const double* Arow = h->d.Abuf + 9ll * ACAP;
    // interleaved rounds over the candidates; each scores its fastest round
    auto tune = [&](const int* cand, int nc, float* best_of) {
        for (int k = 0; k < nc; ++k) best_of[k] = 1e30f;
        for (int round = 0; round < 4 && e == hipSuccess && rc == IBM_LB_OK; ++round)
            for (int k = 0; k < nc && e == hipSuccess && rc == IBM_LB_OK; ++k) {
                if (!lattice_variant_ok(cand[k], h->g)) continue;
                h->lattice_variant = cand[k];
                rc = enqueue_steps(h, Arow, 1, 0);  // untimed: first launch of this variant in the round
                if (rc) break;
                e = hipEventRecord(a, h->stream);
                if (e == hipSuccess) rc = enqueue_steps(h, Arow, reps, 0);
                if (rc) break;
                if (e == hipSuccess) e = hipEventRecord(b, h->stream);
                if (e == hipSuccess) e = hipEventSynchronize(b);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
                if (e == hipSuccess) best_of[k] = std::min(best_of[k], ms);
            }
    };
    // the lattice variants with two population copies, then the in-place
    // ones (linear layout), each with the smoothing's finish as its own
    // launch (measured faster than finishing in the last work-group, whose
    // arrival needs a device-scope release in every work-group)
    int cand[2 * LATTICE_VARIANTS];
    float best_of[2 * LATTICE_VARIANTS];
    int nc = 0;
    if (!h->single)
        for (int v = 0; v < LATTICE_VARIANTS; ++v)
            cand[nc++] = v | VAR_HC_SPLIT;
    if (!h->wet)
        for (int v = 0; v < LATTICE_VARIANTS; ++v)
            if (!(v & VAR_ROWS)) cand[nc++] = v | VAR_HC_SPLIT | VAR_AA;
    tune(cand, nc, best_of);
    int best_v = before;
    if (e == hipSuccess && rc == IBM_LB_OK) best_v = pick_variant(cand, best_of, nc);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    h->timing = timing;
    h->lattice_variant = best_v;
    const int rc_load = ibm_lb_load(h, snap, nb);
    (void)hipFree(snap);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    if (rc) return rc;
    if (rc_load) return rc_load;
    if (variant) *variant = best_v;
    return IBM_LB_OK;
}

int ibm_lb_set_variant(ibm_lb* h, int32_t variant) {
    if (!h) return fail(IBM_LB_EINVAL, "handle is NULL");
    if (!lattice_variant_ok(variant, h->g)) return fail(IBM_LB_EINVAL, "lattice variant cannot run on this box");
    if (h->single && !(variant & VAR_AA))
        return fail(IBM_LB_EINVAL, "a handle with one population copy runs in-place variants only");
    if (h->wet && (variant & VAR_AA)) return fail(IBM_LB_EINVAL, "wet-node walls run with two copies");
    h->lattice_variant = variant;
    return IBM_LB_OK;
}

int ibm_lb_timing_enable(ibm_lb* h, int32_t enable) {
    if (!h) return fail(IBM_LB_EINVAL, "handle is NULL");
    h->timing = enable != 0;
    return IBM_LB_OK;
}

int ibm_lb_timing_read(ibm_lb* h, double* lattice_ms, int64_t* launches) {
    if (!h || !lattice_ms || !launches) return fail(IBM_LB_EINVAL, "bad timing arguments");
    int rc = set_device(h);
    if (rc) return rc;
    rc = accumulate_timing(h);
    if (rc) return rc;
    *lattice_ms = h->acc_ms;
    *launches = h->launches;
    h->acc_ms = 0.0;
    h->launches = 0;
    return IBM_LB_OK;
}

// ---------------------------------------------------------------- adjoint
namespace {

// Device memory of the adjoint for segments of up to `steps` steps: per-step
// records (rho, u, F: 7 N doubles; positions: nv double4; iteration count),
// two adjoint population copies, the adjoint velocity and force fields,
// per-vertex work arrays and the per-step block partials of dJ/dA, dJ/dsigma.
int adj_reserve(ibm_lb* h, int steps) {
    if (h->adj && h->adj_cap >= steps) return IBM_LB_OK;
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    if (h->adj) (void)hipFree(h->adj);
    h->adj = nullptr;
    h->adj_cap = 0;
    const size_t N = (size_t)h->g.N, nv = (size_t)h->nv;
    const size_t nbl = (size_t)adj_lattice_blocks(h->g.N), nbv = (size_t)adj_vertex_blocks(h->nv);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes > 0 ? bytes : 1);
        return o;
    };
    const size_t o_rec = take(sizeof(double) * 7 * N * steps);
    const size_t o_pos = take(sizeof(double4) * nv * steps);
    const size_t o_it = take(sizeof(int) * (size_t)steps);
    const size_t o_fb0 = take(sizeof(double) * 19 * N);
    const size_t o_fb1 = take(sizeof(double) * 19 * N);
    const size_t o_ub = take(sizeof(double) * 3 * N);
    const size_t o_Fb = take(sizeof(double) * 3 * N);
    const size_t o_Ap = take(sizeof(double) * 9 * nbl * steps);
    const size_t o_sp = take(sizeof(double) * (nbv > 0 ? nbv : 1) * steps);
    const size_t o_coef = take(sizeof(double) * 16);
    const size_t o_perm = take(sizeof(int) * nv);
    size_t o_v[9];
    for (int k = 0; k < 9; ++k) o_v[k] = take(sizeof(double4) * nv);
    char* b = nullptr;
    if (hipMalloc((void**)&b, off) != hipSuccess) {
        (void)hipGetLastError();
        return fail(IBM_LB_ENOMEM, "hipMalloc of the adjoint records failed");
    }
    h->adj = b;
    h->adj_cap = steps;
    h->adj_rec = (double*)(b + o_rec);
    h->adj_pos = (double4*)(b + o_pos);
    h->adj_iters = (int*)(b + o_it);
    h->adj_fb[0] = (double*)(b + o_fb0);
    h->adj_fb[1] = (double*)(b + o_fb1);
    h->adj_ubar = (double*)(b + o_ub);
    h->adj_Fbar = (double*)(b + o_Fb);
    h->adj_Apart = (double*)(b + o_Ap);
    h->adj_spart = (double*)(b + o_sp);
    h->adj_coef = (double*)(b + o_coef);
    h->adj_perm = (int*)(b + o_perm);
    double4** vv[9] = {&h->adj_v.rb, &h->adj_v.P,  &h->adj_v.PS,   &h->adj_v.Pp, &h->adj_v.PpS,
                       &h->adj_v.Ob, &h->adj_v.Qp, &h->adj_v.phib, &h->adj_v.rt};
    for (int k = 0; k < 9; ++k) *vv[k] = (double4*)(b + o_v[k]);
    if (nv > 0)
        HIP_TRY(hipMemcpy(h->adj_perm, h->perm.data(), sizeof(int) * nv, hipMemcpyHostToDevice), "perm upload");
    return IBM_LB_OK;
}

AdjStep adj_step(ibm_lb* h, int j) {
    const size_t N = (size_t)h->g.N;
    double* base = h->adj_rec + 7 * N * (size_t)j;
    return AdjStep{base, base + N, base + 4 * N, h->adj_pos + (size_t)h->nv * j};
}

}  // namespace

extern "C" {

int ibm_lb_objective_grad(ibm_lb* h, double* value, double* rbar) {
    return ibm_lb_shape_objective_grad(h, IBM_LB_OBJ_D, value, rbar, nullptr);
}

int ibm_lb_shape_objective_grad(ibm_lb* h, int32_t objective, double* value, double* rbar, double* dA_last) {
    if (!h || !value || !rbar) return fail(IBM_LB_EINVAL, "bad objective_grad arguments");
    if (objective < IBM_LB_OBJ_D || objective > IBM_LB_OBJ_BETA) return fail(IBM_LB_EINVAL, "unknown objective");
    if (h->mrt || h->wet || h->chi)
        return fail(IBM_LB_EINVAL, "the adjoint covers the one-fluid BGK step with link walls");
    if (h->nv == 0) return fail(IBM_LB_EINVAL, "the objective needs a mesh");
    if (h->sticky) return fail(h->sticky, "earlier asynchronous error");
    int rc = set_device(h);
    if (rc) return rc;
    if ((rc = ensure_natural(h))) return rc;
    rc = adj_reserve(h, std::max(h->adj_cap, 1));
    if (rc) return rc;
    HIP_TRY(launch_observables(h->storage, h->g, h->lp, h->d, h->cur, h->nv, h->nt, h->cfg.radius,
                               h->d.Abuf + 9ll * ACAP, h->stream),
            "observables launch");
    double o[OBS_OUT_N];
    HIP_TRY(hipMemcpyAsync(o, h->d.obs_out, sizeof(o), hipMemcpyDeviceToHost, h->stream), "observables copy");
    rc = sync_and_check(h);
    if (rc) return rc;
    const double tie = 1e-12 * h->cfg.radius * h->cfg.radius;
    if (!(o[13] - o[14] >= tie) || (objective == IBM_LB_OBJ_D && !(o[14] - o[15] >= tie)))
        return fail(IBM_LB_EINVAL, "repeated eigenvalue of S: the objective has no derivative here");
    if (objective == IBM_LB_OBJ_BETA && (o[28] != o[28] || (int)o[28] & IBM_LB_OBS_E_ZERO))
        return fail(IBM_LB_EINVAL, "beta needs a nonzero strain E");
    *value = objective == IBM_LB_OBJ_D ? o[25] : (objective == IBM_LB_OBJ_LAMBDA_MAX ? o[13] : o[26]);
    if (dA_last) {
        // beta = v1^T E v1 / |E| also depends on the last gradient row through
        // E = (A + A^T)/2: dbeta/dA = v1 v1^T / |E| - beta E / |E|^2 (symmetric);
        // D and lambda_max do not
        for (int k = 0; k < 9; ++k) dA_last[k] = 0.0;
        if (objective == IBM_LB_OBJ_BETA) {
            double A[9], E[9], En = 0.0;
            HIP_TRY(hipMemcpy(A, h->d.Abuf + 9ll * ACAP, sizeof(A), hipMemcpyDeviceToHost), "gradient row");
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    E[3 * i + j] = 0.5 * (A[3 * i + j] + A[3 * j + i]);
                    En += E[3 * i + j] * E[3 * i + j];
                }
            En = sqrt(En);
            const double* v1 = o + 16;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) dA_last[3 * i + j] = v1[i] * v1[j] / En - o[26] * E[3 * i + j] / (En * En);
        }
    }
    HIP_TRY(launch_adj_seed(h->storage, h->nv, h->d, h->adj_coef, h->adj_v.rb, h->stream, objective),
            "seed launch");
    HIP_TRY(launch_adj_perm_out(h->nv, h->adj_perm, h->adj_v.rb, rbar, h->stream), "seed permute");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    return IBM_LB_OK;
}

int ibm_lb_adjoint_initial(ibm_lb* h, const double* fbar0, double* dA0) {
    if (!h || !fbar0 || !dA0) return fail(IBM_LB_EINVAL, "bad adjoint_initial arguments");
    if (h->mrt || h->wet || h->chi)
        return fail(IBM_LB_EINVAL, "the adjoint covers the one-fluid BGK step with link walls");
    if (h->sticky) return fail(h->sticky, "earlier asynchronous error");
    for (int c = 0; c < 9; ++c) dA0[c] = 0.0;
    if (h->cfg.init == IBM_LB_INIT_REST) return IBM_LB_OK;  // f^0 does not depend on A0
    int rc = set_device(h);
    if (rc) return rc;
    // the observables' partial-sum slots serve as the block partials (OBS_BLOCKS x 16 doubles)
    const int nb = OBS_BLOCKS;
    HIP_TRY(launch_adj_init_A0(h->g, h->lp, h->cfg.A0, fbar0, h->d.obs_part, nb, h->stream), "adjoint A0 launch");
    std::vector<double> part(9 * (size_t)nb);
    HIP_TRY(hipMemcpyAsync(part.data(), h->d.obs_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost,
                           h->stream),
            "adjoint A0 copy");
    HIP_TRY(hipStreamSynchronize(h->stream), "sync");
    for (int b = 0; b < nb; ++b)
        for (int c = 0; c < 9; ++c) dA0[c] += part[9 * (size_t)b + c];
    return IBM_LB_OK;
}

int ibm_lb_adjoint_segment(ibm_lb* h, const void* ckpt, size_t ckpt_bytes, const double* A, int32_t nsteps,
                           int32_t A_on_device, const double* fbar_end, const double* rbar_end, double* fbar_begin,
                           double* rbar_begin, double* dA, double* dsigma) {
    if (!h || !ckpt || !A || nsteps < 1 || !dA || !dsigma)
        return fail(IBM_LB_EINVAL, "bad adjoint_segment arguments");
    if (h->nv > 0 && (!rbar_end || !rbar_begin))
        return fail(IBM_LB_EINVAL, "rbar_end and rbar_begin are required with a mesh");
    if (h->mrt || h->wet || h->chi)
        return fail(IBM_LB_EINVAL, "the adjoint covers the one-fluid BGK step with link walls");
    int rc = set_device(h);
    if (rc) return rc;
    rc = ibm_lb_load(h, ckpt, ckpt_bytes);
    if (rc) return rc;
    rc = adj_reserve(h, nsteps);
    if (rc) return rc;
    // the recompute records every step's populations in natural order: with
    // two copies it streams through both; with one, each step is an even
    // in-place step followed by the in-place return to natural order
    struct KeepVariant {
        ibm_lb* h;
        int v;
        ~KeepVariant() { h->lattice_variant = v; }
    } keep{h, h->lattice_variant};
    if (!h->single) h->lattice_variant &= ~VAR_AA;
    const long long N = h->g.N;
    const int nv = h->nv;
    hipStream_t s = h->stream;
    // 1. recompute the segment, recording what the transposed step needs
    for (int done = 0; done < nsteps;) {
        const int n = A_on_device ? nsteps : std::min(nsteps - done, ACAP);
        const double* rows = A + 9ll * done;
        if (!A_on_device) {
            rc = upload_rows(h, rows, n);
            if (rc) return rc;
            rows = h->d.Abuf;
        }
        for (int j = 0; j < n; ++j) {
            rc = ensure_force(h);
            if (rc) return rc;
            if ((rc = ensure_natural(h))) return rc;
            // the record of step done + j also takes step done + j - 1's iteration count
            HIP_TRY(launch_adj_record(h->storage, h->g, h->lp, h->d, h->cur, nv, adj_step(h, done + j),
                                      done + j > 0 ? h->adj_iters + done + j - 1 : nullptr, s),
                    "record launch");
            rc = enqueue_steps(h, rows + 9ll * j, 1, 1, done + j == nsteps - 1);
            if (rc) return rc;
        }
        done += n;
    }
    HIP_TRY(launch_adj_record_iters(h->d, h->adj_iters + nsteps - 1, s), "record iterations");
    std::vector<int> iters(nsteps);
    HIP_TRY(hipMemcpyAsync(iters.data(), h->adj_iters, sizeof(int) * nsteps, hipMemcpyDeviceToHost, s),
            "read iteration counts");
    rc = sync_and_check(h);
    if (rc) return rc;
    // 2. adjoint state at the segment end
    int c = 0;
    if (fbar_end)
        HIP_TRY(hipMemcpyAsync(h->adj_fb[0], fbar_end, sizeof(double) * 19 * N, hipMemcpyDeviceToDevice, s),
                "fbar_end copy");
    else
        HIP_TRY(hipMemsetAsync(h->adj_fb[0], 0, sizeof(double) * 19 * N, s), "fbar zero");
    HIP_TRY(hipMemsetAsync(h->adj_ubar, 0, sizeof(double) * 3 * N, s), "ubar zero");
    if (nv > 0) HIP_TRY(launch_adj_perm_in(nv, h->adj_perm, rbar_end, h->adj_v.rb, s), "rbar_end permute");
    // 3. backward sweep
    const int nbl = adj_lattice_blocks(N), nbv = nv > 0 ? adj_vertex_blocks(nv) : 0;
    for (int j = nsteps - 1; j >= 0; --j) {
        const AdjStep st = adj_step(h, j);
        if (nv > 0) {
            const int it = h->sp.max_iter > 0 ? iters[j] : 0;
            HIP_TRY(launch_adj_hc(nv, h->d.fan, h->sp, it, h->adj_v, s), "HC transpose");
            HIP_TRY(launch_adj_ib_spread(h->g, nv, h->d.fan, h->sp.alpha, it, st.pos, h->adj_v, h->adj_ubar, s),
                    "interp transpose");
        }
        HIP_TRY(launch_adj_lattice(h->g, h->lp, h->adj_fb[c], h->adj_fb[c ^ 1], st, h->adj_ubar, h->adj_Fbar,
                                   h->adj_Apart + 9ll * nbl * j, s),
                "lattice adjoint");
        if (nv > 0)
            HIP_TRY(launch_adj_ib_back(h->g, nv, h->d.fan, h->cfg.sigma, st, h->adj_Fbar, h->adj_v,
                                       h->adj_spart + (long long)nbv * j, s),
                    "vertex adjoint");
        c ^= 1;
    }
    HIP_TRY(launch_adj_reduce(nsteps, nbl, h->adj_Apart, nbv, h->adj_spart, dA, dsigma, s), "adjoint reduce");
    if (fbar_begin)
        HIP_TRY(hipMemcpyAsync(fbar_begin, h->adj_fb[c], sizeof(double) * 19 * N, hipMemcpyDeviceToDevice, s),
                "fbar_begin copy");
    if (nv > 0) HIP_TRY(launch_adj_perm_out(nv, h->adj_perm, h->adj_v.rb, rbar_begin, s), "rbar_begin permute");
    return IBM_LB_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- ensembles
struct ibm_lb_batch {
    std::vector<ibm_lb*> m;
    int storage = 0, device = 0, n = 0;
    hipStream_t stream = nullptr;
    LatDesc* lat_desc = nullptr;  // device [n]
    int2* lat_map = nullptr;      // device block maps of the eight layouts, concatenated
    int lat_moff[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int nblk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int nblk_ib[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // leading entries of each map: members with a droplet
    void* ib_args = nullptr;      // device [n] records
    int2* patch_map = nullptr;    // device [npatch_total] {member, patch}
    int npatch_total = 0;
    double* Atab = nullptr;       // device [2 halves][n][ACAP][9]
    double* stage = nullptr;      // pinned [2 halves][n][ACAP][9]
    hipEvent_t stage_done[2] = {nullptr, nullptr};
    int half = 0;
    int cur = 0;
    int64_t step = 0;
    bool f_ready = false;
    int variant = 1;
    bool mrt = false;             // every member runs MRT (rates per member in mrt_rates)
    double* mrt_rates = nullptr;  // device [n][19]
    int2* wall_map = nullptr;     // device [nwall] {member, block of 256 face nodes}: wet-node walls
    int nwall = 0;
    // HIP graphs of `graph_steps` batched steps (even; 0 = plain launches),
    // one per population parity, recaptured when the variant changes
    int graph_steps = 32;
    LatDesc* lat_desc_g = nullptr;  // descriptors whose gradient rows move with each replay
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int gvariant[2] = {-1, -1};
};

namespace {
bool batch_variant_ok(const ibm_lb_batch* b, int v) {
    if (v < 0 || v >= STEP_VARIANTS || (v & VAR_AA)) return false;
    return !(v & VAR_ROWS) || b->nblk[4 + ((v >> 1) & 3)] >= 0;
}

int batch_fail_cleanup(ibm_lb_batch* b, int code) {
    ibm_lb_batch_destroy(b);
    return code;
}
}  // namespace

int ibm_lb_batch_init(const ibm_lb_config* cfgs, int32_t n, void* stream, ibm_lb_batch** out) {
    if (!out || !cfgs || n < 1) return fail(IBM_LB_EINVAL, "bad batch_init arguments");
    *out = nullptr;
    for (int i = 1; i < n; ++i)
        if (cfgs[i].storage != cfgs[0].storage) return fail(IBM_LB_EINVAL, "ensemble members need one storage format");
    for (int i = 0; i < n; ++i) {
        if (cfgs[i].populations == 1) return fail(IBM_LB_EINVAL, "ensemble members keep two population copies");
        if (cfgs[i].collision != cfgs[0].collision)
            return fail(IBM_LB_EINVAL, "ensemble members share one collision (BGK or MRT)");
        if (chi_active(&cfgs[i])) return fail(IBM_LB_EINVAL, "ensemble members run one fluid");
        if (cfgs[i].deterministic) return fail(IBM_LB_EINVAL, "ensemble members spread with atomics");
    }
    ibm_lb_batch* b = new (std::nothrow) ibm_lb_batch();
    if (!b) return fail(IBM_LB_ENOMEM, "host allocation");
    b->n = n;
    b->storage = cfgs[0].storage;
    b->stream = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
        ibm_lb_config c = cfgs[i];
        c.stream = stream;
        ibm_lb* h = nullptr;
        int rc = ibm_lb_init(&c, &h);
        if (rc) {
            std::string msg = "member " + std::to_string(i) + ": " + g_last_error;
            batch_fail_cleanup(b, rc);
            return fail(rc, msg);
        }
        b->m.push_back(h);
    }
    b->device = b->m[0]->device;
    auto bail = [&](hipError_t e, const char* where) { return batch_fail_cleanup(b, hip_fail(e, where)); };
    hipError_t e;
    b->mrt = cfgs[0].collision == IBM_LB_MRT;
    if (b->mrt) {
        std::vector<double> rates(19 * (size_t)n);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < 19; ++k) rates[19 * (size_t)i + k] = b->m[i]->mrt_rates.s[k];
        if ((e = hipMalloc((void**)&b->mrt_rates, sizeof(double) * rates.size())) != hipSuccess)
            return bail(e, "MRT rates");
        if ((e = hipMemcpy(b->mrt_rates, rates.data(), sizeof(double) * rates.size(), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return bail(e, "MRT rates");
    }
    std::vector<LatDesc> ld(n);
    std::vector<int2> lm[8], lm_plain[8], pm, wm;
    bool rows_ok[4] = {true, true, true, true};
    const size_t rec = ib_args_bytes(b->storage);
    std::vector<char> args(rec * n);
    for (int i = 0; i < n; ++i) {
        ibm_lb* h = b->m[i];
        LatDesc& L = ld[i];
        L.g = h->g;
        L.lp = h->lp;
        L.f[0] = h->d.f[0];
        L.f[1] = h->d.f[1];
        L.F = h->d.F;
        L.u = h->d.u;
        L.mark = h->d.mark;
        L.ctl = h->d.ctl;
        L.A = nullptr;  // set below, once the table is allocated
        L.mrt = b->mrt ? b->mrt_rates + 19 * (size_t)i : nullptr;
        // members with a droplet first in every map, then the others (two
        // launches, each compiled for one kind)
        std::vector<int2>* dst = h->nv > 0 ? lm : lm_plain;
        for (int q = 0; q < 4; ++q) {
            for (int k = 0; k < (int)((h->g.N + LAT_BS[q] - 1) / LAT_BS[q]); ++k) dst[q].push_back(int2{i, k});
            const int rows = LAT_BS[q] / h->g.Lx;
            if (rows < 1) {
                rows_ok[q] = false;
                continue;
            }
            const long long nrows = (long long)h->g.Ly * h->g.Lz;
            for (int k = 0; k < (int)((nrows + rows - 1) / rows); ++k) dst[4 + q].push_back(int2{i, k});
        }
        for (int k = 0; k < (h->nv + IB_PATCH - 1) / IB_PATCH; ++k) pm.push_back(int2{i, k});
        if (h->wet)
            for (long long k = 0; k < (wall_node_count(h->g) + 255) / 256; ++k) wm.push_back(int2{i, (int)k});
        fill_ib_args(b->storage, h->g, h->d, h->nv, h->cfg.sigma, h->sp, args.data() + rec * i);
    }
    std::vector<int2> lall;
    for (int q = 0; q < 8; ++q) {
        if (q >= 4 && !rows_ok[q - 4]) {
            lm[q].clear();
            lm_plain[q].clear();
        }
        b->nblk_ib[q] = (int)lm[q].size();
        b->nblk[q] = q >= 4 && !rows_ok[q - 4] ? -1 : (int)(lm[q].size() + lm_plain[q].size());
        b->lat_moff[q] = (int)lall.size();
        lall.insert(lall.end(), lm[q].begin(), lm[q].end());
        lall.insert(lall.end(), lm_plain[q].begin(), lm_plain[q].end());
    }
    b->npatch_total = (int)pm.size();
    if (pm.empty()) pm.push_back(int2{0, 0});
    const size_t tab = (size_t)n * ACAP * 9;
    if ((e = hipMalloc((void**)&b->Atab, 2 * tab * sizeof(double))) != hipSuccess) return bail(e, "gradient tables");
    if ((e = hipHostMalloc((void**)&b->stage, 2 * tab * sizeof(double), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "pinned staging");
    if ((e = hipMemset(b->Atab, 0, 2 * tab * sizeof(double))) != hipSuccess) return bail(e, "gradient tables");
    for (int i = 0; i < n; ++i) ld[i].A = b->Atab + (size_t)i * ACAP * 9;
    if ((e = hipMalloc((void**)&b->lat_desc, sizeof(LatDesc) * n)) != hipSuccess) return bail(e, "descriptors");
    if ((e = hipMalloc((void**)&b->lat_map, sizeof(int2) * lall.size())) != hipSuccess) return bail(e, "maps");
    if ((e = hipMalloc(&b->ib_args, rec * n)) != hipSuccess) return bail(e, "ib records");
    if ((e = hipMalloc((void**)&b->patch_map, sizeof(int2) * pm.size())) != hipSuccess) return bail(e, "maps");
    b->nwall = (int)wm.size();
    if (b->nwall > 0) {
        if ((e = hipMalloc((void**)&b->wall_map, sizeof(int2) * wm.size())) != hipSuccess) return bail(e, "maps");
        if ((e = hipMemcpy(b->wall_map, wm.data(), sizeof(int2) * wm.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return bail(e, "maps");
    }
    if ((e = hipMemcpy(b->lat_desc, ld.data(), sizeof(LatDesc) * n, hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "descriptors");
    if ((e = hipMalloc((void**)&b->lat_desc_g, sizeof(LatDesc) * n)) != hipSuccess) return bail(e, "descriptors");
    if ((e = hipMemcpy(b->lat_desc_g, ld.data(), sizeof(LatDesc) * n, hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "descriptors");
    if ((e = hipMemcpy(b->lat_map, lall.data(), sizeof(int2) * lall.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "maps");
    if ((e = hipMemcpy(b->ib_args, args.data(), rec * n, hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "ib records");
    if ((e = hipMemcpy(b->patch_map, pm.data(), sizeof(int2) * pm.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return bail(e, "maps");
    for (int k = 0; k < 2; ++k) {
        if ((e = hipEventCreateWithFlags(&b->stage_done[k], hipEventDisableTiming)) != hipSuccess)
            return bail(e, "hipEventCreate");
        if ((e = hipEventRecord(b->stage_done[k], b->stream)) != hipSuccess) return bail(e, "hipEventRecord");
    }
    if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return bail(e, "sync");
    *out = b;
    return IBM_LB_OK;
}

namespace {
void drop_graphs(ibm_lb_batch* b) {
    for (int k = 0; k < 2; ++k) {
        if (b->gexec[k]) (void)hipGraphExecDestroy(b->gexec[k]);
        b->gexec[k] = nullptr;
        b->gvariant[k] = -1;
    }
}

// Capture graph_steps batched steps starting from population copy `cur`
// (on a private stream; nothing runs), reading gradient rows 0, 1, ... of
// the graph descriptors.
hipError_t capture_steps(ibm_lb_batch* b, int cur, hipGraphExec_t* out) {
    hipError_t e = hipSuccess;
    if (!b->cap_stream && (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int k = 0; k < b->graph_steps && le == hipSuccess; ++k) {
        le = launch_lattice_batch(b->storage, b->lat_desc_g, b->lat_map, b->lat_moff, b->nblk, b->nblk_ib,
                                  cur ^ (k & 1), 9ll * k, b->variant, b->mrt, b->cap_stream);
        if (le == hipSuccess)
            le = launch_wet_walls_batch(b->storage, b->lat_desc_g, b->wall_map, b->nwall, cur ^ (k & 1), 9ll * k,
                                        b->cap_stream);
        if (le == hipSuccess)
            le = launch_ib_step_batch(b->storage, b->ib_args, b->patch_map, b->npatch_total, b->n, b->cap_stream);
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap_stream, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le != hipSuccess ? le : e;
    }
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}
}  // namespace

int ibm_lb_batch_set_graph(ibm_lb_batch* b, int32_t steps) {
    if (!b) return fail(IBM_LB_EINVAL, "batch handle is NULL");
    if (steps < 0 || steps > ACAP || (steps & 1)) return fail(IBM_LB_EINVAL, "graph steps must be even, 0..4096");
    HIP_TRY(hipSetDevice(b->device), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    drop_graphs(b);
    b->graph_steps = steps;
    return IBM_LB_OK;
}

int ibm_lb_batch_step(ibm_lb_batch* b, const double* A_tables, int32_t nsteps) {
    if (!b || !A_tables || nsteps < 0) return fail(IBM_LB_EINVAL, "bad batch_step arguments");
    for (ibm_lb* h : b->m)
        if (h->sticky) return fail(h->sticky, "earlier asynchronous error in a member");
    HIP_TRY(hipSetDevice(b->device), "hipSetDevice");
    const int n = b->n;
    const size_t tab = (size_t)n * ACAP * 9;
    if (!b->f_ready) {
        HIP_TRY(launch_ib_pre_batch(b->storage, b->ib_args, b->patch_map, b->npatch_total, b->stream),
                "ib_pre launch");
        b->f_ready = true;
    }
    for (int done = 0; done < nsteps;) {
        const int len = std::min(nsteps - done, ACAP);
        const int hf = b->half;
        // wait until the staging half is free, then fill it member by member
        HIP_TRY(hipEventSynchronize(b->stage_done[hf]), "staging wait");
        double* sg = b->stage + hf * tab;
        for (int i = 0; i < n; ++i)
            memcpy(sg + (size_t)i * ACAP * 9, A_tables + ((size_t)i * nsteps + done) * 9, sizeof(double) * 9 * len);
        double* dst = b->Atab + hf * tab;
        HIP_TRY(hipMemcpyAsync(dst, sg, sizeof(double) * tab, hipMemcpyHostToDevice, b->stream), "upload tables");
        HIP_TRY(hipEventRecord(b->stage_done[hf], b->stream), "hipEventRecord");
        int j = 0;
        // whole graphs first (an even number of steps leaves the parity as it was)
        for (const int G = b->graph_steps; G > 0 && len - j >= G; j += G) {
            const int c = b->cur;
            if (!b->gexec[c] || b->gvariant[c] != b->variant) {
                if (b->gexec[c]) (void)hipGraphExecDestroy(b->gexec[c]);
                b->gexec[c] = nullptr;
                HIP_TRY(capture_steps(b, c, &b->gexec[c]), "graph capture");
                b->gvariant[c] = b->variant;
            }
            HIP_TRY(launch_set_rows(b->lat_desc_g, n, dst + 9ll * j, 9ll * ACAP, b->stream), "set rows");
            HIP_TRY(hipGraphLaunch(b->gexec[c], b->stream), "hipGraphLaunch");
        }
        for (; j < len; ++j) {
            HIP_TRY(launch_lattice_batch(b->storage, b->lat_desc, b->lat_map, b->lat_moff, b->nblk, b->nblk_ib, b->cur,
                                         (long long)hf * tab + 9ll * j, b->variant, b->mrt, b->stream),
                    "lattice batch launch");
            HIP_TRY(launch_wet_walls_batch(b->storage, b->lat_desc, b->wall_map, b->nwall, b->cur,
                                           (long long)hf * tab + 9ll * j, b->stream),
                    "walls batch launch");
            HIP_TRY(launch_ib_step_batch(b->storage, b->ib_args, b->patch_map, b->npatch_total, n, b->stream),
                    "ib batch launch");
            b->cur ^= 1;
        }
        // each member keeps its last gradient for the orientation observable
        for (int i = 0; i < n; ++i)
            HIP_TRY(hipMemcpyAsync(b->m[i]->d.Abuf + 9ll * ACAP, dst + (size_t)i * ACAP * 9 + 9ll * (len - 1),
                                   9 * sizeof(double), hipMemcpyDeviceToDevice, b->stream),
                    "copy last gradient");
        b->half ^= 1;
        done += len;
    }
    b->step += nsteps;
    for (ibm_lb* h : b->m) {
        h->cur = b->cur;
        h->step = b->step;
        h->f_ready = true;
    }
    return IBM_LB_OK;
}

int ibm_lb_batch_observables(ibm_lb_batch* b, ibm_lb_obs* out) {
    if (!b || !out) return fail(IBM_LB_EINVAL, "bad batch_observables arguments");
    int first_rc = IBM_LB_OK;
    for (int i = 0; i < b->n; ++i) {
        int rc = ibm_lb_observables(b->m[i], &out[i]);
        if (rc && !first_rc) first_rc = rc;
    }
    return first_rc;
}

int ibm_lb_batch_member(ibm_lb_batch* b, int32_t i, ibm_lb** out) {
    if (!b || !out || i < 0 || i >= b->n) return fail(IBM_LB_EINVAL, "bad batch_member arguments");
    *out = b->m[i];
    return IBM_LB_OK;
}

int ibm_lb_batch_autotune(ibm_lb_batch* b, int32_t reps, int32_t* variant) {
    if (!b || reps < 1) return fail(IBM_LB_EINVAL, "bad batch_autotune arguments");
    for (ibm_lb* h : b->m)
        if (h->sticky) return fail(h->sticky, "earlier asynchronous error in a member");
    HIP_TRY(hipSetDevice(b->device), "hipSetDevice");
    // Whole batched steps per variant (with the gradient rows already in the
    // first table half), members saved before and restored after.
    const int n = b->n;
    std::vector<size_t> nbytes(n);
    std::vector<void*> snap(n, nullptr);
    int rc = IBM_LB_OK;
    for (int i = 0; i < n && rc == IBM_LB_OK; ++i) {
        nbytes[i] = ibm_lb_state_bytes(b->m[i]);
        if (hipMalloc(&snap[i], nbytes[i]) != hipSuccess) {
            (void)hipGetLastError();
            snap[i] = nullptr;
            rc = fail(IBM_LB_ENOMEM, "batch autotune snapshot allocation");
        } else {
            rc = ibm_lb_save(b->m[i], snap[i], nbytes[i]);
        }
    }
    const int64_t step0 = b->step;
    const int before = b->variant;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipSuccess;
    if (rc == IBM_LB_OK) e = hipEventCreate(&e0);
    if (rc == IBM_LB_OK && e == hipSuccess) e = hipEventCreate(&e1);
    if (rc == IBM_LB_OK && e == hipSuccess && !b->f_ready) {
        e = launch_ib_pre_batch(b->storage, b->ib_args, b->patch_map, b->npatch_total, b->stream);
        b->f_ready = true;
    }
    float best_of[LATTICE_VARIANTS];
    for (int v = 0; v < LATTICE_VARIANTS; ++v) best_of[v] = 1e30f;
    auto batch_steps = [&](int v, int k) {
        hipError_t r = hipSuccess;
        for (int j = 0; j < k && r == hipSuccess; ++j) {
            r = launch_lattice_batch(b->storage, b->lat_desc, b->lat_map, b->lat_moff, b->nblk, b->nblk_ib, b->cur, 0, v,
                                     b->mrt, b->stream);
            if (r == hipSuccess)
                r = launch_wet_walls_batch(b->storage, b->lat_desc, b->wall_map, b->nwall, b->cur, 0, b->stream);
            if (r == hipSuccess)
                r = launch_ib_step_batch(b->storage, b->ib_args, b->patch_map, b->npatch_total, n, b->stream);
            b->cur ^= 1;
        }
        return r;
    };
    for (int round = 0; round < 4 && e == hipSuccess && rc == IBM_LB_OK; ++round)
        for (int v = 0; v < LATTICE_VARIANTS && e == hipSuccess; ++v) {
            if (!batch_variant_ok(b, v)) continue;
            e = batch_steps(v, 1);
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            if (e == hipSuccess) e = batch_steps(v, reps);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess) best_of[v] = std::min(best_of[v], ms);
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    int best_v = before;
    if (e == hipSuccess && rc == IBM_LB_OK) {
        int cand[LATTICE_VARIANTS];
        for (int v = 0; v < LATTICE_VARIANTS; ++v) cand[v] = v;
        best_v = pick_variant(cand, best_of, LATTICE_VARIANTS);
    }
    b->variant = best_v;
    // restore every member (each load clears its force field and retires its marks)
    for (int i = 0; i < n; ++i) {
        b->m[i]->cur = b->cur;
        if (snap[i]) {
            const int r = ibm_lb_load(b->m[i], snap[i], nbytes[i]);
            if (r && rc == IBM_LB_OK) rc = r;
            (void)hipFree(snap[i]);
        }
    }
    b->step = step0;
    b->f_ready = false;
    if (e != hipSuccess) return hip_fail(e, "batch autotune");
    if (rc) return rc;
    if (variant) *variant = best_v;
    return IBM_LB_OK;
}

int ibm_lb_batch_set_variant(ibm_lb_batch* b, int32_t variant) {
    if (!b) return fail(IBM_LB_EINVAL, "batch handle is NULL");
    if (!batch_variant_ok(b, variant)) return fail(IBM_LB_EINVAL, "lattice variant cannot run on every member");
    b->variant = variant;
    return IBM_LB_OK;
}

void ibm_lb_batch_destroy(ibm_lb_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream || !b->m.empty()) (void)hipStreamSynchronize(b->stream);
    for (auto& ev : b->stage_done)
        if (ev) (void)hipEventDestroy(ev);
    if (b->stage) (void)hipHostFree(b->stage);
    if (b->Atab) (void)hipFree(b->Atab);
    drop_graphs(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->lat_desc) (void)hipFree(b->lat_desc);
    if (b->lat_desc_g) (void)hipFree(b->lat_desc_g);
    if (b->lat_map) (void)hipFree(b->lat_map);
    if (b->ib_args) (void)hipFree(b->ib_args);
    if (b->patch_map) (void)hipFree(b->patch_map);
    if (b->mrt_rates) (void)hipFree(b->mrt_rates);
    if (b->wall_map) (void)hipFree(b->wall_map);
    for (ibm_lb* h : b->m) ibm_lb_destroy(h);
    delete b;
}

void ibm_lb_destroy(ibm_lb* h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    if (h->stage_done) (void)hipEventDestroy(h->stage_done);
    if (h->stage) (void)hipHostFree(h->stage);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
    if (h->adj) (void)hipFree(h->adj);
    delete h;
}

}  // extern "C"
