// sg_host.cpp -- mesh packer and C ABI of the straightest-geodesic library.
//
// The packer runs once per mesh on the host in float64 from the float32
// vertex positions: manifold validation (Sec. 4: every edge on one or two
// faces, each vertex fan connected), face adjacency (the only connectivity
// the walk uses, so non-orientable meshes are accepted), per-half-edge chart
// records and theta(x) = sum of corner angles at each vertex (Sec. 4), all
// rounded once to float32 or fixed-point angles and uploaded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "sg.h"
#include "sg_internal.h"
#include "sg_launch.h"

using sg::FaceRec;

struct sg_mesh_s {
    int device = 0;
    int cu_count = 0;
    int walk_blocks_per_cu = 0;
    int part_blocks_per_cu = 0;
    int64_t n_verts = 0, n_faces = 0;
    int32_t n_meshes = 1;
    double mean_edge = 0.0;
    FaceRec* d_face = nullptr;
    int32_t* d_F = nullptr;
    float* d_X = nullptr;
    int64_t* d_half = nullptr;
    int32_t* d_perm = nullptr;
    int32_t* d_order = nullptr;
    int32_t* d_twin = nullptr;
    float* d_geo = nullptr;
    int32_t* d_vc_off = nullptr;   // vertex -> corner lists (internal faces), for the vertex gradient
    int32_t* d_vc = nullptr;
    int32_t part_he[sg::kParts + 1] = {};
    int32_t has_flip = 0;
    size_t bytes = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timed, spare;   // walk-kernel event pairs
    sg::PackedMesh host;   // connectivity, links and face order, for sg_mesh_update_vertices
    std::vector<float> hX;  // vertex positions on the host (the projection grid is built from them)
    // projection-integration Exp: per-face data in user order and one grid per
    // mesh, built on the first call that needs them (and again after a vertex update)
    std::mutex pi_mu;
    bool pi_ready = false;
    sg::PiFace* d_piface = nullptr;
    sg::PiGrid* d_pigrid = nullptr;
    uint32_t* d_cell_start = nullptr;
    int32_t* d_cell_face = nullptr;
    size_t pi_bytes = 0;
    double pi_tie = 0.0, pi_slack = 0.0;
    sg::PiMesh pi() const {
        return sg::PiMesh{d_piface, d_pigrid, d_cell_start, d_cell_face, n_faces, n_meshes, pi_tie, pi_slack};
    }
    sg::DevMesh dev(int32_t hole_avoid = 0) const {
        sg::DevMesh d{d_face,  d_F,     d_X,     d_half, d_perm,     d_order,
                      n_faces, n_verts, has_flip, {},   d_twin, hole_avoid, reinterpret_cast<const float4*>(d_geo)};
        for (int p = 0; p <= sg::kParts; ++p) d.part_he[p] = part_he[p];
        return d;
    }
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SG_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

struct V3 {
    double x, y, z;
};
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double len(V3 a) { return std::sqrt(dot(a, a)); }

// angle between two vectors, robust for small angles
inline double angle_between(V3 a, V3 b) { return std::atan2(len(cross(a, b)), dot(a, b)); }

inline uint32_t to_fx(double rad) {
    const double u = std::nearbyint(rad * sg::kFxPerRad);
    return (uint32_t)(int64_t)u;
}

// union-find over face corners, used for the one-fan-per-vertex check
struct DSU {
    std::vector<int64_t> p;
    explicit DSU(int64_t n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int64_t find(int64_t x) {
        while (p[x] != x) {
            p[x] = p[p[x]];
            x = p[x];
        }
        return x;
    }
    void unite(int64_t a, int64_t b) {
        a = find(a);
        b = find(b);
        if (a != b) p[std::max(a, b)] = std::min(a, b);
    }
};

template <class T>
int upload(T** dptr, const std::vector<T>& h, size_t& bytes) {
    const size_t nb = h.size() * sizeof(T);
    hipError_t e = hipMalloc((void**)dptr, nb ? nb : sizeof(T));
    if (e != hipSuccess) return fail(SG_E_OOM, "hipMalloc(%zu): %s", nb, hipGetErrorString(e));
    bytes += nb;
    if (nb) {
        e = hipMemcpy(*dptr, h.data(), nb, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    }
    return SG_OK;
}

void free_pi(sg_mesh_s* m) {
    (void)hipFree(m->d_piface);
    (void)hipFree(m->d_pigrid);
    (void)hipFree(m->d_cell_start);
    (void)hipFree(m->d_cell_face);
    m->d_piface = nullptr;
    m->d_pigrid = nullptr;
    m->d_cell_start = nullptr;
    m->d_cell_face = nullptr;
    m->pi_bytes = 0;
    m->pi_ready = false;
}

void free_mesh(sg_mesh_s* m) {
    if (!m) return;
    for (auto& pr : m->timed) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (auto& pr : m->spare) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    (void)hipFree(m->d_face);
    (void)hipFree(m->d_F);
    (void)hipFree(m->d_X);
    (void)hipFree(m->d_half);
    (void)hipFree(m->d_perm);
    (void)hipFree(m->d_order);
    (void)hipFree(m->d_twin);
    (void)hipFree(m->d_geo);
    (void)hipFree(m->d_vc_off);
    (void)hipFree(m->d_vc);
    free_pi(m);
    delete m;
}

int check_opts(const sg_opts* in, sg_opts& o, const sg_mesh_s* m, int64_t n = -1) {
    sg_opts_default(&o);
    if (in) o = *in;
    if (o.max_steps <= 0) o.max_steps = 1 << 20;
    if (!(o.vertex_snap > 0.f)) o.vertex_snap = 1.0f / 2097152.0f;
    if (!(o.vertex_snap < 0.25f)) return fail(SG_E_ARG, "vertex_snap must be below 0.25");
    if (!(o.eps_v > 0.f)) o.eps_v = (float)(5e-3 * m->mean_edge);
    if (!(o.eps_p > 0.f)) o.eps_p = (float)(5e-3 * m->mean_edge);
    if (o.kernel < SG_KERNEL_AUTO || o.kernel > SG_KERNEL_PARTITIONED) return fail(SG_E_ARG, "unknown kernel %d", o.kernel);
    if (o.rays_per_lane <= 0) o.rays_per_lane = 1;
    if (o.rays_per_lane > 2) return fail(SG_E_ARG, "rays_per_lane must be 1 or 2");
    if (o.refill_min <= 0) o.refill_min = 48 * o.rays_per_lane;
    if (o.refill_min > 64 * o.rays_per_lane) return fail(SG_E_ARG, "refill_min must be at most 64 per ray slot");
    if (o.boundary_mode != SG_BOUNDARY_STOP && o.boundary_mode != SG_BOUNDARY_AVOID)
        return fail(SG_E_ARG, "unknown boundary_mode %d", o.boundary_mode);
    if (o.ray_queues <= 0) o.ray_queues = 8;
    if (o.gradx_records == 0) o.gradx_records = 256;
    if (o.ray_queues % 8 != 0 || o.ray_queues > sg::kMaxQueues)
        return fail(SG_E_ARG, "ray_queues must be a multiple of 8, at most %d", sg::kMaxQueues);
    // default schedule: three resident 256-lane blocks per CU, refill at 48 idle lanes (the
    // fastest in sweeps of 32-60 on 1M, 5.6M and 16.8M rays; the backward keeps 32)
    if (o.walk_blocks <= 0)
        o.walk_blocks = m->cu_count * std::min(3, o.kernel == SG_KERNEL_PARTITIONED ? m->part_blocks_per_cu
                                                                                   : m->walk_blocks_per_cu);
    // SG_KERNEL_AUTO: a forward batch (n >= 0) that fits the persistent walk's
    // resident lanes takes the plain kernel: every ray starts at once either way,
    // so the ordering passes and the queues only add time (65,536 rays on the
    // 327,680-face mesh: 0.255 against 0.326 ms); larger batches and every
    // other caller (n < 0) take the persistent walk
    if (o.kernel == SG_KERNEL_AUTO)
        o.kernel = n >= 0 && n <= (int64_t)o.walk_blocks * 256 * o.rays_per_lane ? SG_KERNEL_PLAIN
                                                                               : SG_KERNEL_PERSISTENT;
    return SG_OK;
}

sg::WalkSched sched(const sg_opts& o) { return sg::WalkSched{o.walk_blocks, o.refill_min, o.ray_queues}; }

// Workspace of a call: the caller's (checked) or a stream-ordered allocation.
struct Workspace {
    void* p = nullptr;
    bool own = false;
};

int take_workspace(const sg_opts& o, size_t need, hipStream_t st, Workspace& w) {
    w = Workspace{};
    if (need == 0) return SG_OK;
    if (o.workspace) {
        if (o.workspace_bytes < need)
            return fail(SG_E_ARG, "workspace too small: %llu bytes given, %llu needed",
                        (unsigned long long)o.workspace_bytes, (unsigned long long)need);
        if (reinterpret_cast<uintptr_t>(o.workspace) & 255u) return fail(SG_E_ARG, "workspace must be 256-byte aligned");
        w.p = o.workspace;
        return SG_OK;
    }
    hipError_t e = hipMallocAsync(&w.p, need, st);
    if (e != hipSuccess) return fail(SG_E_OOM, "workspace allocation: %s", hipGetErrorString(e));
    w.own = true;
    return SG_OK;
}

hipError_t give_workspace(Workspace& w, hipStream_t st) {
    hipError_t e = w.own ? hipFreeAsync(w.p, st) : hipSuccess;
    w = Workspace{};
    return e;
}

// The backward always runs the persistent walk: a partitioned choice of
// kernel takes the persistent walk's block count.  Its walks refill at 32 idle
// lanes by default (the forward's 48 made the finite-difference passes, whose
// queues interleave several walks per query, 3.3 -> 3.9 ms on 1M queries).
int check_bwd_opts(const sg_opts* in, sg_opts& o, sg_mesh m) {
    const int rc = check_opts(in, o, m);
    if (rc == SG_OK && o.kernel == SG_KERNEL_PARTITIONED) o.walk_blocks = m->cu_count * m->walk_blocks_per_cu;
    if (rc == SG_OK && !(in && in->refill_min > 0)) o.refill_min = 32 * o.rays_per_lane;
    return rc;
}

// have_*: which saved forward outputs the call is given (none: the size that covers every call)
size_t bwd_workspace_bytes(const sg_opts& o, sg_mesh m, int64_t n, int32_t mode, bool vjp, bool gradx,
                           bool have_f = false, bool have_b = false, bool have_v = false, bool have_status = false) {
    return sg::bwd_workspace(n, mode, m->has_flip != 0, vjp, gradx, m->n_faces, o.gradx_records, o.walk_blocks,
                             o.boundary_mode != SG_BOUNDARY_STOP, have_f, have_b, have_v, have_status);
}

size_t exp_workspace_bytes(const sg_opts& o, int64_t n, int32_t K) {
    if (o.kernel == SG_KERNEL_PLAIN || n <= 0) return 0;
    return o.kernel == SG_KERNEL_PARTITIONED ? sg::exp_partitioned_workspace(n, K, (o.debug & 2u) != 0u)
                                             : sg::exp_persistent_workspace(n, K);
}

// Builds the projection-integration data of a handle on the host (float64
// from the float32 positions, rounded once) and uploads it: per-face records
// in user order and one uniform grid per mesh whose cells list the faces
// whose bounding boxes, widened by a margin, meet them.  Cells are 1.5 mean
// edges wide (wider if a mesh would need more than 32 cells per face).
int ensure_pi(sg_mesh m) {
    std::lock_guard<std::mutex> lock(m->pi_mu);
    if (m->pi_ready) return SG_OK;
    try {
        const sg::PackedMesh& pm = m->host;
        const int64_t nf = m->n_faces;
        const std::vector<float>& X = m->hX;
        std::vector<int32_t> Fu(3 * nf);   // user order, global vertex ids
        for (int64_t u = 0; u < nf; ++u) {
            const int64_t fi = pm.perm[u];
            for (int k = 0; k < 3; ++k) Fu[3 * u + k] = pm.F[3 * fi + k];
        }
        auto P = [&](int64_t v) { return V3{X[3 * v], X[3 * v + 1], X[3 * v + 2]}; };
        double scale = 1.0;
        for (float x : X) scale = std::max(scale, (double)std::fabs(x));
        std::vector<sg::PiFace> face(nf);
        for (int64_t u = 0; u < nf; ++u) {
            const V3 x0 = P(Fu[3 * u]), x1 = P(Fu[3 * u + 1]), x2 = P(Fu[3 * u + 2]);
            const V3 c = cross(x1 - x0, x2 - x0);
            const double ic = 1.0 / len(c);
            sg::PiFace& F = face[u];
            const V3 xs[3] = {x0, x1, x2};
            float* dst[3] = {F.x0, F.x1, F.x2};
            for (int k = 0; k < 3; ++k) {
                dst[k][0] = (float)xs[k].x;
                dst[k][1] = (float)xs[k].y;
                dst[k][2] = (float)xs[k].z;
            }
            F.pad = 0.f;
            F.n[0] = c.x * ic;
            F.n[1] = c.y * ic;
            F.n[2] = c.z * ic;
        }
        const std::vector<int64_t>& fo = pm.face_off;
        const int nm = (int)fo.size() - 1;
        std::vector<sg::PiGrid> grid(nm);
        std::vector<double> lo(3 * (size_t)nm), hh(nm);
        uint64_t total = 0;
        for (int k = 0; k < nm; ++k) {
            sg::PiGrid& G = grid[k];
            G.face0 = (int32_t)fo[k];
            G.face1 = (int32_t)fo[k + 1];
            double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY}, el = 0.0;
            for (int64_t u = fo[k]; u < fo[k + 1]; ++u)
                for (int j = 0; j < 3; ++j) {
                    const V3 a = P(Fu[3 * u + j]), b = P(Fu[3 * u + (j + 1) % 3]);
                    el += len(b - a);
                    const double xa[3] = {a.x, a.y, a.z};
                    for (int c = 0; c < 3; ++c) {
                        mn[c] = std::min(mn[c], xa[c]);
                        mx[c] = std::max(mx[c], xa[c]);
                    }
                }
            const int64_t fm = fo[k + 1] - fo[k];
            if (fm == 0) {
                for (int c = 0; c < 3; ++c) mn[c] = mx[c] = 0.0;
                el = 1.0;
            }
            double h = 1.5 * el / (3.0 * (double)std::max<int64_t>(fm, 1));
            if (!(h > 0.0)) h = 1.0;
            const double cap = (double)std::max<int64_t>(32 * fm, 4096);
            int32_t n[3];
            double o[3];
            for (;;) {
                double cells = 1.0;
                for (int c = 0; c < 3; ++c) {
                    o[c] = mn[c] - 0.5 * h;
                    n[c] = (int32_t)std::max(1.0, std::ceil((mx[c] + 0.5 * h - o[c]) / h));
                    cells *= n[c];
                }
                if (cells <= cap) break;
                h *= 1.25;
            }
            G.ox = (float)o[0];
            G.oy = (float)o[1];
            G.oz = (float)o[2];
            G.h = (float)h;
            G.nx = n[0];
            G.ny = n[1];
            G.nz = n[2];
            G.cell0 = (uint32_t)total;
            total += (uint64_t)n[0] * n[1] * n[2];
            if (total >= ((uint64_t)1 << 31)) return fail(SG_E_OOM, "projection grid too large");
            lo[3 * k] = G.ox;
            lo[3 * k + 1] = G.oy;
            lo[3 * k + 2] = G.oz;
            hh[k] = G.h;
        }
        // cell ranges of each face's widened box (in the float32 origin and size the kernels use)
        auto range = [&](int64_t u, int k, int32_t* i0, int32_t* i1) {
            const sg::PiGrid& G = grid[k];
            const double h = hh[k], marg = 1e-3 * h + scale * std::ldexp(1.0, -20);
            const int32_t nn[3] = {G.nx, G.ny, G.nz};
            for (int c = 0; c < 3; ++c) {
                double a = INFINITY, b = -INFINITY;
                for (int j = 0; j < 3; ++j) {
                    const double x = X[3 * (int64_t)Fu[3 * u + j] + c];
                    a = std::min(a, x);
                    b = std::max(b, x);
                }
                const double t0 = std::floor((a - marg - lo[3 * k + c]) / h), t1 = std::floor((b + marg - lo[3 * k + c]) / h);
                i0[c] = (int32_t)std::min<double>(std::max(t0, 0.0), nn[c] - 1);
                i1[c] = (int32_t)std::min<double>(std::max(t1, 0.0), nn[c] - 1);
            }
        };
        std::vector<uint32_t> start(total + 1, 0u);
        std::vector<int32_t> cf;   // cell faces
        uint64_t entries = 0;
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<uint32_t> fill;
            if (pass == 1) {
                fill.assign(start.begin(), start.end() - 1);
                cf.assign(entries, 0);
            }
            for (int k = 0; k < nm; ++k) {
                const sg::PiGrid& G = grid[k];
                for (int64_t u = fo[k]; u < fo[k + 1]; ++u) {
                    int32_t i0[3], i1[3];
                    range(u, k, i0, i1);
                    for (int32_t iz = i0[2]; iz <= i1[2]; ++iz)
                        for (int32_t iy = i0[1]; iy <= i1[1]; ++iy)
                            for (int32_t ix = i0[0]; ix <= i1[0]; ++ix) {
                                const uint64_t cell = G.cell0 + ((uint64_t)iz * G.ny + iy) * G.nx + ix;
                                if (pass == 0) start[cell + 1]++;
                                else cf[fill[cell]++] = (int32_t)u;
                            }
                }
            }
            if (pass == 0) {
                for (uint64_t c = 0; c < total; ++c) start[c + 1] += start[c];
                entries = start[total];
                if (entries >= ((uint64_t)1 << 32) - 1) return fail(SG_E_OOM, "projection grid too large");
            } else {
                std::vector<sg::PiGrid> gcopy = grid;
                int rc = upload(&m->d_piface, face, m->pi_bytes);
                if (rc == SG_OK) rc = upload(&m->d_pigrid, gcopy, m->pi_bytes);
                if (rc == SG_OK) rc = upload(&m->d_cell_start, start, m->pi_bytes);
                if (rc == SG_OK) rc = upload(&m->d_cell_face, cf, m->pi_bytes);
                if (rc != SG_OK) {
                    free_pi(m);
                    return rc;
                }
            }
        }
        // distances within 1e-12 of the largest coordinate are one nearest point (float64 rounding);
        // the cell search reaches 1e-9 further, past any rounding of a box distance
        m->pi_tie = 1e-12 * scale;
        m->pi_slack = 1e-9 * scale;
        m->pi_ready = true;
        return SG_OK;
    } catch (const std::bad_alloc&) {
        free_pi(m);
        return fail(SG_E_OOM, "out of host memory");
    }
}

int check_pi_opts(const sg_pi_opts* in, sg_pi_opts& o) {
    sg_pi_opts_default(&o);
    if (in) o = *in;
    if (!(o.step > 0.f)) o.step = 0.01f;
    if (!(o.step <= 1.f)) return fail(SG_E_ARG, "PI step must be in (0, 1]");
    if (o.max_steps <= 0) o.max_steps = (int32_t)std::ceil(8.0 / (double)o.step);
    if (o.search != SG_PI_GRID && o.search != SG_PI_SCAN) return fail(SG_E_ARG, "unknown PI search %d", o.search);
    return SG_OK;
}

// Autotuner cache (per process): the schedule picked for a class of batches.
struct TuneKey {
    std::string arch;
    int cus, fclass, nclass, K, lclass, boundary;
    bool operator<(const TuneKey& o) const {
        return std::tie(arch, cus, fclass, nclass, K, lclass, boundary) <
               std::tie(o.arch, o.cus, o.fclass, o.nclass, o.K, o.lclass, o.boundary);
    }
};
struct TunePick {
    int32_t kernel, refill, blocks, rpl, queues;
    double ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TunePick> g_tune;

int ilog2(int64_t x) {
    int r = 0;
    while (x > 1) {
        x >>= 1;
        ++r;
    }
    return r;
}

// Checks the arguments of a forward call and fills its kernel arguments.
int exp_args(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v, int32_t K, const float* W,
             int32_t* f_out, float* b_out, float* p_out, float* v_out, float* W_out, int32_t* status,
             int32_t* n_cross, uint64_t* seq_hash, const sg_opts* opts, sg_opts& o, sg::ExpArgs& a) {
    if (!mesh) return fail(SG_E_ARG, "mesh is NULL");
    if (n < 0) return fail(SG_E_ARG, "n must be >= 0");
    if (K < 0 || K > 64) return fail(SG_E_ARG, "K must be in [0, 64]");
    int rc = check_opts(opts, o, mesh, n);
    if (rc != SG_OK) return rc;
    if (n == 0) return SG_OK;
    if (!f || !b || !v || !f_out || !b_out || !p_out || !v_out) return fail(SG_E_ARG, "a required array is NULL");
    if (K > 0 && (!W || !W_out)) return fail(SG_E_ARG, "W and W_out are required when K > 0");
    if ((o.debug & 2u) && !seq_hash) return fail(SG_E_ARG, "debug bit 1 needs seq_hash");
    if (o.kernel != SG_KERNEL_PLAIN && n >= ((int64_t)1 << 31))
        return fail(SG_E_ARG, "the persistent and partitioned walks take fewer than 2^31 rays per call");
    a = sg::ExpArgs{};
    a.n = n;
    a.f = f; a.b = b; a.v = v;
    a.K = K; a.W = W;
    a.f_out = f_out; a.b_out = b_out; a.p_out = p_out; a.v_out = v_out; a.W_out = W_out;
    a.status = status; a.n_cross = n_cross; a.seq_hash = seq_hash;
    a.max_steps = o.max_steps;
    a.snap = o.vertex_snap;
    a.debug = o.debug;
    a.rays_per_lane = o.rays_per_lane;
    return SG_OK;
}

}  // namespace

namespace sg {

int pack_mesh(const float* X_host, int64_t n_verts, const int32_t* F_host, int64_t n_faces,
              const int64_t* vert_offsets, const int64_t* face_offsets, int32_t n_meshes, PackedMesh& out) {
    try {
        if (!X_host || !F_host || n_verts <= 0 || n_faces <= 0) return fail(SG_E_ARG, "empty mesh");
        // face records are addressed with 32-bit byte offsets: n_faces * 32 < 2^32
        if (n_faces >= ((int64_t)1 << 27))
            return fail(SG_E_ARG, "mesh too large: %lld faces (at most 134,217,727)", (long long)n_faces);
        if (n_verts > ((int64_t)1 << 31) - 1) return fail(SG_E_ARG, "too many vertices");
        if (n_meshes < 1) return fail(SG_E_ARG, "n_meshes must be >= 1");
        if ((vert_offsets == nullptr) != (face_offsets == nullptr))
            return fail(SG_E_ARG, "vert_offsets and face_offsets must both be given or both be NULL");
        if (!vert_offsets && n_meshes != 1) return fail(SG_E_ARG, "offsets are required for several meshes");
        std::vector<int64_t> vo{0, n_verts}, fo{0, n_faces};
        if (vert_offsets) {
            vo.assign(vert_offsets, vert_offsets + n_meshes + 1);
            fo.assign(face_offsets, face_offsets + n_meshes + 1);
            if (vo[0] != 0 || fo[0] != 0 || vo[n_meshes] != n_verts || fo[n_meshes] != n_faces)
                return fail(SG_E_ARG, "offsets must start at 0 and end at the totals");
            for (int32_t m = 0; m < n_meshes; ++m)
                if (vo[m + 1] < vo[m] || fo[m + 1] < fo[m]) return fail(SG_E_ARG, "offsets must be non-decreasing");
        }
        // global vertex ids and float64 positions
        std::vector<int32_t> F(3 * n_faces);
        for (int32_t m = 0; m < n_meshes; ++m) {
            const int64_t nvm = vo[m + 1] - vo[m];
            for (int64_t f = fo[m]; f < fo[m + 1]; ++f)
                for (int k = 0; k < 3; ++k) {
                    const int64_t v = F_host[3 * f + k];
                    if (v < 0 || v >= nvm)
                        return fail(SG_E_ARG, "face %lld: vertex index %lld out of range", (long long)f, (long long)v);
                    F[3 * f + k] = (int32_t)(v + vo[m]);
                }
        }
        std::vector<V3> X(n_verts);
        for (int64_t v = 0; v < n_verts; ++v) {
            const float* p = X_host + 3 * v;
            if (!std::isfinite(p[0]) || !std::isfinite(p[1]) || !std::isfinite(p[2]))
                return fail(SG_E_ARG, "vertex %lld is not finite", (long long)v);
            X[v] = {(double)p[0], (double)p[1], (double)p[2]};
        }
        for (int64_t f = 0; f < n_faces; ++f) {
            const int32_t* t = &F[3 * f];
            if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2])
                return fail(SG_E_DEGENERATE, "face %lld repeats a vertex", (long long)f);
            if (!(len(cross(X[t[1]] - X[t[0]], X[t[2]] - X[t[0]])) > 0.0))
                return fail(SG_E_DEGENERATE, "face %lld has zero area", (long long)f);
        }
        // Spatial face order: recursive coordinate bisection of the face centroids
        // (median split along the longest box axis), within each mesh of a batch.
        // For one mesh the first three levels cut the faces into 8 contiguous parts
        // of equal count, one per XCD; deeper levels keep neighbouring faces close
        // in memory.  Everything below works
        // on internal ids; perm / order map user ids to internal ids and back.
        {
            std::vector<V3> cen(n_faces);
            for (int64_t f = 0; f < n_faces; ++f) {
                const V3 a = X[F[3 * f]], b = X[F[3 * f + 1]], c = X[F[3 * f + 2]];
                cen[f] = {(a.x + b.x + c.x) / 3.0, (a.y + b.y + c.y) / 3.0, (a.z + b.z + c.z) / 3.0};
            }
            std::vector<int64_t>& order = out.order;
            order.resize(n_faces);
            std::iota(order.begin(), order.end(), 0);
            struct Span { int64_t lo, hi; };
            // each mesh of a batch keeps its faces contiguous (meshes of one batch may overlap in space)
            std::vector<Span> stack;
            for (int32_t m = n_meshes - 1; m >= 0; --m)
                if (fo[m + 1] > fo[m]) stack.push_back({fo[m], fo[m + 1]});
            while (!stack.empty()) {
                const Span sp = stack.back();
                stack.pop_back();
                if (sp.hi - sp.lo <= 16) continue;
                V3 mn = cen[order[sp.lo]], mx = mn;
                for (int64_t i = sp.lo; i < sp.hi; ++i) {
                    const V3 c = cen[order[i]];
                    mn = {std::min(mn.x, c.x), std::min(mn.y, c.y), std::min(mn.z, c.z)};
                    mx = {std::max(mx.x, c.x), std::max(mx.y, c.y), std::max(mx.z, c.z)};
                }
                const double ex_ = mx.x - mn.x, ey_ = mx.y - mn.y, ez_ = mx.z - mn.z;
                const int ax = ex_ >= ey_ && ex_ >= ez_ ? 0 : (ey_ >= ez_ ? 1 : 2);
                const int64_t mid = sp.lo + (sp.hi - sp.lo) / 2;
                std::nth_element(order.begin() + sp.lo, order.begin() + mid, order.begin() + sp.hi,
                                 [&](int64_t u, int64_t w) {
                                     const double cu = ax == 0 ? cen[u].x : (ax == 1 ? cen[u].y : cen[u].z);
                                     const double cw = ax == 0 ? cen[w].x : (ax == 1 ? cen[w].y : cen[w].z);
                                     return cu < cw || (cu == cw && u < w);
                                 });
                stack.push_back({sp.lo, mid});
                stack.push_back({mid, sp.hi});
            }
            std::vector<int32_t> Fi(3 * n_faces);
            out.perm.resize(n_faces);
            for (int64_t i = 0; i < n_faces; ++i) {
                out.perm[order[i]] = (int32_t)i;
                for (int k = 0; k < 3; ++k) Fi[3 * i + k] = F[3 * order[i] + k];
            }
            F.swap(Fi);
            // the 8 parts: ranges [n_faces * p / 8, n_faces * (p + 1) / 8) of the bisection order
            for (int p = 0; p <= kParts; ++p) out.part_start[p] = n_faces * p / kParts;
        }
        // undirected edges: sort half-edges by (min, max) vertex key
        const int64_t nh = 3 * n_faces;
        std::vector<uint64_t> key(nh);
        std::vector<int64_t> order(nh);
        for (int64_t h = 0; h < nh; ++h) {
            const uint32_t a = (uint32_t)F[h], b = (uint32_t)F[(h / 3) * 3 + (h % 3 + 1) % 3];
            key[h] = ((uint64_t)std::min(a, b) << 32) | std::max(a, b);
            order[h] = h;
        }
        std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return key[x] < key[y] || (key[x] == key[y] && x < y); });
        std::vector<int64_t> twin(nh, -1);
        std::vector<uint8_t> vbnd(n_verts, 0);
        for (int64_t i = 0; i < nh;) {
            int64_t j = i + 1;
            while (j < nh && key[order[j]] == key[order[i]]) ++j;
            const int64_t h0 = order[i];
            const int32_t a = F[h0], b = F[(h0 / 3) * 3 + (h0 % 3 + 1) % 3];
            if (j - i > 2)
                return fail(SG_E_NONMANIFOLD, "edge (%d,%d) has %lld faces", std::min(a, b), std::max(a, b), (long long)(j - i));
            if (j - i == 2) {
                const int64_t h1 = order[i + 1];
                if (h0 / 3 == h1 / 3)
                    return fail(SG_E_DEGENERATE, "face %lld uses an edge twice", (long long)out.order[h0 / 3]);
                twin[h0] = h1;
                twin[h1] = h0;
            } else {
                vbnd[a] = vbnd[b] = 1;
            }
            i = j;
        }
        // one fan per vertex: corners at the same vertex are joined across shared edges
        {
            DSU dsu(nh);
            for (int64_t h = 0; h < nh; ++h) {
                const int64_t g = twin[h];
                if (g < h) continue;
                const int64_t f = h / 3, k = h % 3, fg = g / 3, kg = g % 3;
                const int32_t a = F[h], b = F[3 * f + (k + 1) % 3];
                // corner of f at a is h; corner of fg at a is whichever end of g equals a
                const int64_t ga = F[g] == a ? g : 3 * fg + (kg + 1) % 3;
                const int64_t gb = F[g] == b ? g : 3 * fg + (kg + 1) % 3;
                dsu.unite(h, ga);
                dsu.unite(3 * f + (k + 1) % 3, gb);
            }
            std::vector<int64_t> root(n_verts, -1);
            for (int64_t h = 0; h < nh; ++h) {
                const int32_t v = F[h];
                const int64_t r = dsu.find(h);
                if (root[v] < 0) root[v] = r;
                else if (root[v] != r) return fail(SG_E_NONMANIFOLD, "vertex %d: faces do not form one fan", v);
            }
        }
        // links across edges; the records' geometry comes from pack_geometry
        out.face.assign(n_faces, FaceRec{});
        for (int64_t h = 0; h < nh; ++h) {
            const int64_t g = twin[h];
            const uint32_t flip = g >= 0 && F[h] == F[g] ? 1u : 0u;   // same start vertex: orientations disagree
            out.face[h / 3].nb[h % 3] = g < 0 ? -1 : (int32_t)(((uint32_t)g << 1) | flip);
        }
        out.has_flip = 0;
        for (const FaceRec& q : out.face)
            for (int k = 0; k < 3; ++k)
                if (q.nb[k] >= 0 && (q.nb[k] & 1)) out.has_flip = 1;
        out.vbnd = std::move(vbnd);
        out.twin.assign(twin.begin(), twin.end());
        out.F = std::move(F);
        out.n_verts = n_verts;
        out.n_faces = n_faces;
        out.face_off = fo;
        return pack_geometry(X_host, out);

    } catch (const std::bad_alloc&) {
        return fail(SG_E_OOM, "out of host memory");
    } catch (...) {
        return fail(SG_E_ARG, "unexpected error while packing the mesh");
    }
}

int pack_geometry(const float* X_host, PackedMesh& pm) {
    try {
        const int64_t n_verts = pm.n_verts, n_faces = pm.n_faces;
        std::vector<V3> X(n_verts);
        for (int64_t v = 0; v < n_verts; ++v) {
            const float* p = X_host + 3 * v;
            if (!std::isfinite(p[0]) || !std::isfinite(p[1]) || !std::isfinite(p[2]))
                return fail(SG_E_ARG, "vertex %lld is not finite", (long long)v);
            X[v] = {(double)p[0], (double)p[1], (double)p[2]};
        }
        const std::vector<int32_t>& F = pm.F;
        // face records (float64 work, rounded once); vertex total angles from
        // the same fixed-point corners
        std::vector<int64_t> theta_fx(n_verts, 0);
        double esum = 0.0;
        int64_t ecount = 0;
        for (int64_t f = 0; f < n_faces; ++f) {
            const int32_t* t = &F[3 * f];
            if (!(len(cross(X[t[1]] - X[t[0]], X[t[2]] - X[t[0]])) > 0.0))
                return fail(SG_E_DEGENERATE, "face %lld has zero area", (long long)pm.order[f]);
            FaceRec& q = pm.face[f];
            uint32_t corner[3];
            for (int k = 0; k < 3; ++k) {
                const double l = len(X[t[(k + 1) % 3]] - X[t[k]]);
                q.l[k] = (float)l;
                const int64_t g = pm.twin[3 * f + k];
                if (g < 0 || g > 3 * f + k) {   // each undirected edge once
                    esum += l;
                    ++ecount;
                }
            }
            for (int k = 0; k < 2; ++k) {
                const V3 p = X[t[(k + 1) % 3]] - X[t[k]], r = X[t[(k + 2) % 3]] - X[t[k]];
                corner[k] = to_fx(angle_between(p, r));
            }
            corner[2] = sg::kPiFx - corner[0] - corner[1];
            q.c0 = corner[0];
            q.c1 = corner[1];
            for (int k = 0; k < 3; ++k) theta_fx[t[k]] += (int64_t)corner[k];
        }
        pm.half.assign(n_verts, 0);
        for (int64_t v = 0; v < n_verts; ++v) pm.half[v] = pm.vbnd[v] ? -1 : theta_fx[v] / 2;
        pm.X.assign(X_host, X_host + 3 * n_verts);
        pm.mean_edge = esum / (double)ecount;
        // 64-byte geometry records: the three vertices (w: the walk record's
        // edge lengths), its two corners and the user face id, so a start or
        // end frame takes one 64-byte segment
        pm.geo.assign(16 * (size_t)n_faces, 0.f);
        for (int64_t f = 0; f < n_faces; ++f) {
            float* g = &pm.geo[16 * (size_t)f];
            const FaceRec& q = pm.face[f];
            for (int k = 0; k < 3; ++k) {
                const int32_t v = F[3 * f + k];
                g[4 * k] = X_host[3 * (int64_t)v];
                g[4 * k + 1] = X_host[3 * (int64_t)v + 1];
                g[4 * k + 2] = X_host[3 * (int64_t)v + 2];
                g[4 * k + 3] = q.l[k];
            }
            const int32_t u = (int32_t)pm.order[f];
            std::memcpy(&g[12], &q.c0, sizeof q.c0);
            std::memcpy(&g[13], &q.c1, sizeof q.c1);
            std::memcpy(&g[14], &u, sizeof u);
        }
        return SG_OK;
    } catch (const std::bad_alloc&) {
        return fail(SG_E_OOM, "out of host memory");
    }
}

}  // namespace sg

extern "C" {

const char* sg_last_error(void) { return g_err.c_str(); }

void sg_opts_default(sg_opts* o) {
    if (!o) return;
    o->max_steps = 1 << 20;
    o->vertex_snap = 1.0f / 2097152.0f;
    o->eps_v = 0.f;
    o->eps_p = 0.f;
    o->kernel = SG_KERNEL_AUTO;
    o->debug = 0u;
    o->refill_min = 0;
    o->walk_blocks = 0;
    o->rays_per_lane = 0;
    o->ray_queues = 0;
    o->boundary_mode = SG_BOUNDARY_STOP;
    o->gradx_records = 0;
    o->workspace = nullptr;
    o->workspace_bytes = 0;
}

int sg_mesh_create(const float* X_host, int64_t n_verts, const int32_t* F_host, int64_t n_faces,
                   const int64_t* vert_offsets, const int64_t* face_offsets, int32_t n_meshes, sg_mesh* out) {
    if (!out) return fail(SG_E_ARG, "out is NULL");
    *out = nullptr;
    sg::PackedMesh pm;
    int rc = sg::pack_mesh(X_host, n_verts, F_host, n_faces, vert_offsets, face_offsets, n_meshes, pm);
    if (rc != SG_OK) return rc;
    auto* m = new (std::nothrow) sg_mesh_s();
    if (!m) return fail(SG_E_OOM, "out of host memory");
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) {
        delete m;
        return hip_fail(e, "hipGetDevice");
    }
    if (hipDeviceGetAttribute(&m->cu_count, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess ||
        m->cu_count <= 0)
        m->cu_count = 256;
    {   // the allocation-free forward's scratch address on this device (once per device)
        void* scr = nullptr;
        e = sg::noalloc_scratch(&scr);
        if (e != hipSuccess) {
            delete m;
            return hip_fail(e, "scratch address");
        }
    }
    m->walk_blocks_per_cu = sg::walk_blocks_per_cu();
    m->part_blocks_per_cu = sg::part_blocks_per_cu();
    m->n_verts = n_verts;
    m->n_faces = n_faces;
    m->n_meshes = n_meshes;
    m->mean_edge = pm.mean_edge;
    m->has_flip = pm.has_flip;
    for (int p = 0; p <= sg::kParts; ++p) m->part_he[p] = (int32_t)(3 * pm.part_start[p]);
    std::vector<int32_t> order32(pm.order.begin(), pm.order.end());
    // corners of each vertex (3 f + k over internal faces), grouped by vertex
    std::vector<int32_t> vc_off((size_t)n_verts + 1, 0), vc((size_t)3 * n_faces);
    for (int64_t c = 0; c < 3 * n_faces; ++c) ++vc_off[(size_t)pm.F[c] + 1];
    for (int64_t v = 0; v < n_verts; ++v) vc_off[(size_t)v + 1] += vc_off[(size_t)v];
    {
        std::vector<int32_t> at(vc_off.begin(), vc_off.end() - 1);
        for (int64_t c = 0; c < 3 * n_faces; ++c) vc[(size_t)at[(size_t)pm.F[c]]++] = (int32_t)c;
    }
    rc = upload(&m->d_face, pm.face, m->bytes);
    if (rc == SG_OK) rc = upload(&m->d_F, pm.F, m->bytes);
    if (rc == SG_OK) rc = upload(&m->d_X, pm.X, m->bytes);
    if (rc == SG_OK) rc = upload(&m->d_half, pm.half, m->bytes);
    if (rc == SG_OK) rc = upload(&m->d_perm, pm.perm, m->bytes);
    if (rc == SG_OK) rc = upload(&m->d_order, order32, m->bytes);
    if (rc == SG_OK) rc = upload(&m->d_twin, pm.twin, m->bytes);
    if (rc == SG_OK) rc = upload(&m->d_geo, pm.geo, m->bytes);
    if (rc == SG_OK) rc = upload(&m->d_vc_off, vc_off, m->bytes);
    if (rc == SG_OK) rc = upload(&m->d_vc, vc, m->bytes);
    if (rc != SG_OK) {
        free_mesh(m);
        return rc;
    }
    m->hX = std::move(pm.X);
    pm.X.clear();
    pm.geo.clear();
    pm.geo.shrink_to_fit();
    m->host = std::move(pm);
    *out = m;
    return SG_OK;
}

int sg_mesh_update_vertices(sg_mesh mesh, const float* X_host, int64_t n_verts) {
    if (!mesh) return fail(SG_E_ARG, "mesh is NULL");
    if (!X_host) return fail(SG_E_ARG, "X_host is NULL");
    if (n_verts != mesh->n_verts)
        return fail(SG_E_ARG, "n_verts %lld does not match the mesh's %lld", (long long)n_verts, (long long)mesh->n_verts);
    sg::PackedMesh& pm = mesh->host;
    // recompute on copies so that a rejected update leaves the mesh as it was
    const std::vector<FaceRec> face0 = pm.face;
    const std::vector<int64_t> half0 = pm.half;
    const double mean0 = pm.mean_edge;
    int rc = sg::pack_geometry(X_host, pm);
    if (rc != SG_OK) {
        pm.face = face0;
        pm.half = half0;
        pm.mean_edge = mean0;
        return rc;
    }
    hipError_t e = hipDeviceSynchronize();   // no walk may read the records while they change
    {
        std::lock_guard<std::mutex> lock(mesh->pi_mu);
        free_pi(mesh);   // the projection grid is rebuilt for the new positions on its next use
        mesh->hX.assign(X_host, X_host + 3 * n_verts);
    }
    if (e == hipSuccess) e = hipMemcpy(mesh->d_face, pm.face.data(), pm.face.size() * sizeof(FaceRec), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mesh->d_half, pm.half.data(), pm.half.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mesh->d_X, X_host, (size_t)n_verts * 3 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mesh->d_geo, pm.geo.data(), pm.geo.size() * sizeof(float), hipMemcpyHostToDevice);
    pm.X.clear();
    pm.geo.clear();
    if (e != hipSuccess) return hip_fail(e, "vertex update");
    mesh->mean_edge = pm.mean_edge;
    return SG_OK;
}

void sg_mesh_destroy(sg_mesh mesh) { free_mesh(mesh); }

int sg_mesh_info(sg_mesh mesh, double* mean_edge, int64_t* n_half_edges, size_t* device_bytes) {
    if (!mesh) return fail(SG_E_ARG, "mesh is NULL");
    if (mean_edge) *mean_edge = mesh->mean_edge;
    if (n_half_edges) *n_half_edges = 3 * mesh->n_faces;
    if (device_bytes) *device_bytes = mesh->bytes;
    return SG_OK;
}

int sg_mesh_walk_time(sg_mesh mesh, double* total_ms, int64_t* launches) {
    if (!mesh) return fail(SG_E_ARG, "mesh is NULL");
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto& pr : mesh->timed) {
        hipError_t e = hipEventSynchronize(pr.second);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess) return hip_fail(e, "walk timing");
        tot += ms;
        ++cnt;
        mesh->spare.push_back(pr);
    }
    mesh->timed.clear();
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    return SG_OK;
}

int sg_exp_transport(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v, int32_t K,
                     const float* W, int32_t* f_out, float* b_out, float* p_out, float* v_out, float* W_out,
                     int32_t* status, int32_t* n_cross, uint64_t* seq_hash, const sg_opts* opts, void* stream) {
    sg_opts o;
    sg::ExpArgs a{};
    int rc = exp_args(mesh, n, f, b, v, K, W, f_out, b_out, p_out, v_out, W_out, status, n_cross, seq_hash, opts, o,
                      a);
    if (rc != SG_OK || n == 0) return rc;
    const hipStream_t st = (hipStream_t)stream;
    if (o.kernel == SG_KERNEL_PLAIN) {
        hipError_t e = sg::launch_exp_plain(mesh->dev(o.boundary_mode), a, st);
        if (e != hipSuccess) return hip_fail(e, "forward launch");
        return SG_OK;
    }
    // persistent forms: per-ray chart states and queues live in a workspace
    const bool part = o.kernel == SG_KERNEL_PARTITIONED;
    Workspace ws;
    rc = take_workspace(o, exp_workspace_bytes(o, n, K), st, ws);
    if (rc != SG_OK) return rc;
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (o.debug & 4u) {
        if (!mesh->spare.empty()) {
            ev = mesh->spare.back();
            mesh->spare.pop_back();
        } else if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
            (void)give_workspace(ws, st);
            return fail(SG_E_HIP, "hipEventCreate failed");
        }
    }
    hipError_t e = part ? sg::launch_exp_partitioned(mesh->dev(o.boundary_mode), a, ws.p, o.walk_blocks, o.refill_min, st, ev.first,
                                                     ev.second)
                        : sg::launch_exp_persistent(mesh->dev(o.boundary_mode), a, ws.p, sched(o), st, ev.first,
                                                    ev.second);
    if (ev.first) mesh->timed.push_back(ev);
    const hipError_t e2 = give_workspace(ws, st);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    if (e2 != hipSuccess) return hip_fail(e2, "workspace release");
    return SG_OK;
}

static_assert(SG_NOALLOC_SCRATCH_BYTES == sg::kNoAllocScratchBytes, "scratch size in sg.h and the library agree");

int sg_exp_transport_noalloc(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v, int32_t K,
                             const float* W, int32_t* f_out, float* b_out, float* p_out, float* v_out, float* W_out,
                             int32_t* status, int32_t* n_cross, uint64_t* seq_hash, const sg_opts* opts,
                             void* stream) {
    sg_opts o;
    sg::ExpArgs a{};
    int rc = exp_args(mesh, n, f, b, v, K, W, f_out, b_out, p_out, v_out, W_out, status, n_cross, seq_hash, opts, o,
                      a);
    if (rc != SG_OK || n == 0) return rc;
    if (o.workspace) return fail(SG_E_ARG, "sg_exp_transport_noalloc uses the library's scratch: opts->workspace must be NULL");
    if (o.debug & 4u) return fail(SG_E_ARG, "sg_exp_transport_noalloc does not time the walk (debug bit 2)");
    if (o.kernel == SG_KERNEL_PARTITIONED)
        return fail(SG_E_ARG, "sg_exp_transport_noalloc runs the plain or the persistent kernel");
    const hipStream_t st = (hipStream_t)stream;
    if (o.kernel == SG_KERNEL_PLAIN) {   // one ray per lane: no scratch at all
        hipError_t e = sg::launch_exp_plain(mesh->dev(o.boundary_mode), a, st);
        if (e != hipSuccess) return hip_fail(e, "forward launch");
        return SG_OK;
    }
    const size_t need = sg::exp_persistent_workspace(n, K);
    if (need > sg::kNoAllocScratchBytes)
        return fail(SG_E_ARG, "%lld rays with K = %d need %llu bytes of scratch; the limit is %llu (SG_NOALLOC_SCRATCH_BYTES)",
                    (long long)n, (int)K, (unsigned long long)need, (unsigned long long)sg::kNoAllocScratchBytes);
    void* ws = nullptr;
    hipError_t e = sg::noalloc_scratch(&ws);
    if (e != hipSuccess) return hip_fail(e, "scratch address");
    e = sg::launch_exp_persistent(mesh->dev(o.boundary_mode), a, ws, sched(o), st, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return SG_OK;
}

int sg_exp_backward_transport(sg_mesh mesh, int32_t mode, int64_t n, const int32_t* f, const float* b,
                              const float* v, int32_t K, const int32_t* f_out, const float* b_out,
                              const float* v_out, const int32_t* status, const float* g_p, const float* g_b,
                              const float* g_v, const float* g_W, float* grad_v, float* grad_b, float* grad_W,
                              double* grad_X, const sg_opts* opts, void* stream) {
    if (!mesh) return fail(SG_E_ARG, "mesh is NULL");
    if (n < 0) return fail(SG_E_ARG, "n must be >= 0");
    if (mode != SG_BWD_EP && mode != SG_BWD_GFD) return fail(SG_E_ARG, "unknown backward mode %d", mode);
    if ((grad_v == nullptr) != (grad_b == nullptr)) return fail(SG_E_ARG, "grad_v and grad_b go together");
    if (K < 0 || K > 64) return fail(SG_E_ARG, "K must be in [0, 64]");
    if ((g_W == nullptr) != (grad_W == nullptr)) return fail(SG_E_ARG, "g_W and grad_W go together");
    if (g_W && K == 0) return fail(SG_E_ARG, "g_W needs K > 0");
    if ((g_v || g_W) && !grad_v) return fail(SG_E_ARG, "g_v and g_W need grad_v and grad_b");
    sg_opts o;
    int rc = check_bwd_opts(opts, o, mesh);
    if (rc != SG_OK) return rc;
    if (!(std::isfinite(o.eps_v) && std::isfinite(o.eps_p))) return fail(SG_E_ARG, "eps_v and eps_p must be finite");
    if (n == 0) return SG_OK;
    if (n >= ((int64_t)1 << 31)) return fail(SG_E_ARG, "the backward takes fewer than 2^31 queries per call");
    if (!f || !b || !v) return fail(SG_E_ARG, "a required array is NULL");
    if (!g_p && !g_b && !g_v && !g_W) return fail(SG_E_ARG, "no cotangent given (g_p, g_b, g_v and g_W are NULL)");
    const bool vjp = grad_v != nullptr;
    if (!vjp && !grad_X) return SG_OK;
    if (vjp && mode == SG_BWD_EP && !mesh->has_flip && (!f_out || !v_out))
        return fail(SG_E_ARG, "the extrinsic proxy needs the forward's f_out and v_out");
    sg::BwdArgs a{};
    a.n = n;
    a.mode = mode;
    a.f = f; a.b = b; a.v = v;
    a.f_out = f_out; a.b_out = b_out; a.v_out = v_out;
    a.status_in = status;
    a.g = g_p;
    a.g_bo = g_b;
    a.g_v = g_v;
    a.g_W = g_W;
    a.K = K;
    a.grad_v = grad_v; a.grad_b = grad_b;
    a.grad_W = grad_W;
    a.grad_X = (g_p || g_b) ? grad_X : nullptr;
    a.eps_v = o.eps_v; a.eps_p = o.eps_p;
    a.max_steps = o.max_steps;
    a.snap = o.vertex_snap;
    if (!vjp && !a.grad_X) return SG_OK;
    const hipStream_t st = (hipStream_t)stream;
    Workspace ws;
    a.gx_records = o.gradx_records;
    a.vc_off = mesh->d_vc_off;
    a.vc = mesh->d_vc;
    rc = take_workspace(o, bwd_workspace_bytes(o, mesh, n, mode, vjp, a.grad_X != nullptr, f_out != nullptr,
                                               b_out != nullptr, v_out != nullptr, status != nullptr),
                        st, ws);
    if (rc != SG_OK) return rc;
    hipError_t e = sg::launch_backward(mesh->dev(o.boundary_mode), a, ws.p, sched(o), st);
    const hipError_t e2 = give_workspace(ws, st);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    if (e2 != hipSuccess) return hip_fail(e2, "workspace release");
    return SG_OK;
}

int sg_exp_backward(sg_mesh mesh, int32_t mode, int64_t n, const int32_t* f, const float* b, const float* v,
                    const int32_t* f_out, const float* b_out, const float* v_out, const int32_t* status,
                    const float* g_p, float* grad_v, float* grad_b, double* grad_X, const sg_opts* opts,
                    void* stream) {
    if (n > 0 && !g_p) return fail(SG_E_ARG, "a required array is NULL");
    return sg_exp_backward_transport(mesh, mode, n, f, b, v, 0, f_out, b_out, v_out, status, g_p, nullptr, nullptr,
                                     nullptr, grad_v, grad_b, nullptr, grad_X, opts, stream);
}

int sg_exp_workspace_size(sg_mesh mesh, int64_t n, int32_t K, const sg_opts* opts, size_t* bytes) {
    if (!mesh || !bytes) return fail(SG_E_ARG, "mesh and bytes are required");
    if (n < 0) return fail(SG_E_ARG, "n must be >= 0");
    if (K < 0 || K > 64) return fail(SG_E_ARG, "K must be in [0, 64]");
    sg_opts o;
    int rc = check_opts(opts, o, mesh, n);
    if (rc != SG_OK) return rc;
    *bytes = exp_workspace_bytes(o, n, K);
    return SG_OK;
}

int sg_backward_workspace_size(sg_mesh mesh, int32_t mode, int64_t n, int32_t want_vjp, int32_t want_grad_X,
                               const sg_opts* opts, size_t* bytes) {
    if (!mesh || !bytes) return fail(SG_E_ARG, "mesh and bytes are required");
    if (n < 0) return fail(SG_E_ARG, "n must be >= 0");
    if (mode != SG_BWD_EP && mode != SG_BWD_GFD) return fail(SG_E_ARG, "unknown backward mode %d", mode);
    sg_opts o;
    int rc = check_bwd_opts(opts, o, mesh);
    if (rc != SG_OK) return rc;
    *bytes = (n == 0 || (!want_vjp && !want_grad_X)) ? 0
                                                     : bwd_workspace_bytes(o, mesh, n, mode, want_vjp != 0,
                                                                           want_grad_X != 0);
    return SG_OK;
}

int sg_autotune(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v, int32_t K, const float* W,
                sg_opts* opts, double* best_ms, void* stream) {
    if (!mesh || !opts) return fail(SG_E_ARG, "mesh and opts are required");
    if (n <= 0 || !f || !b || !v) return fail(SG_E_ARG, "autotuning needs a non-empty batch");
    if (K < 0 || K > 64 || (K > 0 && !W)) return fail(SG_E_ARG, "bad K or W");
    sg_opts base;
    int rc = check_opts(opts, base, mesh);
    if (rc != SG_OK) return rc;
    const bool retune = (opts->debug & 8u) != 0u;
    base.debug = 0u;
    base.workspace = nullptr;
    base.workspace_bytes = 0;
    const hipStream_t st = (hipStream_t)stream;
    // the cache key: device, mesh size, batch size, K, boundary rule and the batch's
    // length class (mean |v| over a strided sample of 256 rays, in mean edges)
    TuneKey key{};
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, mesh->device) != hipSuccess) return fail(SG_E_HIP, "hipGetDeviceProperties");
        key.arch = prop.gcnArchName;
        key.cus = mesh->cu_count;
        key.fclass = ilog2(mesh->n_faces);
        key.nclass = ilog2(n);
        key.K = K;
        key.boundary = base.boundary_mode;
        const int64_t ns = std::min<int64_t>(n, 256), stride = n / ns;
        std::vector<float> vs(3 * (size_t)ns);
        if (hipMemcpy2DAsync(vs.data(), 12, v, (size_t)stride * 12, 12, (size_t)ns, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return fail(SG_E_HIP, "copy of the length sample");
        double sum = 0.0;
        for (int64_t i = 0; i < ns; ++i)
            sum += std::sqrt((double)vs[3 * i] * vs[3 * i] + (double)vs[3 * i + 1] * vs[3 * i + 1] +
                             (double)vs[3 * i + 2] * vs[3 * i + 2]);
        const double rel = sum / (double)ns / std::max(mesh->mean_edge, 1e-30);
        key.lclass = std::isfinite(rel) ? (int)std::lround(2.0 * std::log2(std::max(rel, 1e-3))) : 0;
    }
    if (!retune) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            opts->kernel = it->second.kernel;
            opts->refill_min = it->second.refill;
            opts->walk_blocks = it->second.blocks;
            opts->rays_per_lane = it->second.rpl;
            opts->ray_queues = it->second.queues;
            if (best_ms) *best_ms = it->second.ms;
            return SG_OK;
        }
    }
    // scratch outputs and one workspace for every candidate, allocated before any timing
    void* buf = nullptr;
    const size_t per = 4 + 3 * 12 + (size_t)K * 12 + 4;
    const size_t ws_bytes = sg::exp_persistent_workspace(n, K);
    const size_t out_bytes = (per * (size_t)n + 1024 + 255) & ~(size_t)255;
    if (hipMalloc(&buf, out_bytes + ws_bytes) != hipSuccess) return fail(SG_E_OOM, "autotune scratch allocation");
    char* q = static_cast<char*>(buf);
    auto carve = [&](size_t bytes) { char* r = q; q += (bytes + 255) & ~(size_t)255; return r; };
    auto* fo = reinterpret_cast<int32_t*>(carve(4 * (size_t)n));
    auto* bo = reinterpret_cast<float*>(carve(12 * (size_t)n));
    auto* po = reinterpret_cast<float*>(carve(12 * (size_t)n));
    auto* vo = reinterpret_cast<float*>(carve(12 * (size_t)n));
    auto* Wo = K ? reinterpret_cast<float*>(carve(12 * (size_t)K * n)) : nullptr;
    void* ws = static_cast<char*>(buf) + out_bytes;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(buf);
        return fail(SG_E_HIP, "hipEventCreate failed");
    }
    // candidates: the plain kernel, and the persistent walk over rays per lane, resident
    // blocks per CU (waves per SIMD), refill thresholds (the compaction period) and ray queues
    std::vector<TunePick> cands;
    cands.push_back({SG_KERNEL_PLAIN, base.refill_min, base.walk_blocks, 1, base.ray_queues, 0.0});
    const int refills[] = {4, 8, 16, 24, 32, 48};
    for (int queues : {8, 16, 64})
        for (int rpl = 1; rpl <= 2; ++rpl)
            for (int bpc = 1; bpc <= mesh->walk_blocks_per_cu; ++bpc)
                for (int r : refills)
                    if (queues == 8 || rpl == 1)
                        cands.push_back({SG_KERNEL_PERSISTENT, r * rpl, bpc * mesh->cu_count, rpl, queues, 0.0});
    double best = 1e300;
    TunePick win = cands[1 < cands.size() ? 1 : 0];
    rc = SG_OK;
    for (const TunePick& c : cands) {
        sg_opts o = base;
        o.kernel = c.kernel;
        o.refill_min = c.refill;
        o.walk_blocks = c.blocks;
        o.rays_per_lane = c.rpl;
        o.ray_queues = c.queues;
        o.workspace = c.kernel == SG_KERNEL_PLAIN ? nullptr : ws;
        o.workspace_bytes = c.kernel == SG_KERNEL_PLAIN ? 0 : ws_bytes;
        double t = 1e300;
        for (int rep = 0; rep < 4 && rc == SG_OK; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(SG_E_HIP, "hipEventRecord failed"); break; }
            rc = sg_exp_transport(mesh, n, f, b, v, K, W, fo, bo, po, vo, Wo, nullptr, nullptr, nullptr, &o, stream);
            if (rc != SG_OK) break;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                rc = fail(SG_E_HIP, "event synchronization failed");
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) t = std::min(t, (double)ms);   // the first run warms caches
        }
        if (rc != SG_OK) break;
        if (t < best) { best = t; win = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (rc != SG_OK) return rc;
    win.ms = best;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[key] = win;
    }
    opts->kernel = win.kernel;
    opts->refill_min = win.refill;
    opts->walk_blocks = win.blocks;
    opts->rays_per_lane = win.rpl;
    opts->ray_queues = win.queues;
    if (best_ms) *best_ms = best;
    return SG_OK;
}

void sg_pi_opts_default(sg_pi_opts* o) {
    if (!o) return;
    o->step = 0.01f;
    o->max_steps = 0;
    o->search = SG_PI_GRID;
}

int sg_pi_exp(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v, int32_t K, const float* W,
              int32_t* f_out, float* b_out, float* p_out, float* v_out, float* W_out, int32_t* status,
              int32_t* n_steps, const sg_pi_opts* pi_opts, void* stream) {
    if (!mesh) return fail(SG_E_ARG, "mesh is NULL");
    if (n < 0) return fail(SG_E_ARG, "n must be >= 0");
    if (K < 0 || K > 64) return fail(SG_E_ARG, "K must be in [0, 64]");
    sg_pi_opts po;
    int rc = check_pi_opts(pi_opts, po);
    if (rc != SG_OK) return rc;
    if (n == 0) return SG_OK;
    if (!f || !b || !v || !f_out || !b_out || !p_out || !v_out) return fail(SG_E_ARG, "a required array is NULL");
    if (K > 0 && (!W || !W_out)) return fail(SG_E_ARG, "W and W_out are required when K > 0");
    rc = ensure_pi(mesh);
    if (rc != SG_OK) return rc;
    sg::PiArgs a{};
    a.n = n;
    a.f = f; a.b = b; a.v = v;
    a.K = K; a.W = W;
    a.f_out = f_out; a.b_out = b_out; a.p_out = p_out; a.v_out = v_out; a.W_out = W_out;
    a.status = status; a.n_steps = n_steps;
    a.step = po.step;
    a.max_steps = po.max_steps;
    a.scan = po.search == SG_PI_SCAN;
    hipError_t e = sg::launch_pi_exp(mesh->pi(), a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "PI launch");
    return SG_OK;
}

int sg_pi_backward_workspace_size(sg_mesh mesh, int32_t mode, int64_t n, size_t* bytes) {
    if (!mesh || !bytes) return fail(SG_E_ARG, "mesh and bytes are required");
    if (mode != SG_BWD_EP && mode != SG_BWD_GFD) return fail(SG_E_ARG, "unknown mode %d", mode);
    if (n < 0) return fail(SG_E_ARG, "n must be >= 0");
    *bytes = sg::pi_bwd_workspace(n, mode);
    return SG_OK;
}

int sg_pi_backward(sg_mesh mesh, int32_t mode, int64_t n, const int32_t* f, const float* b, const float* v,
                   const int32_t* f_out, const float* v_out, const float* g_p, float* grad_v, float* grad_b,
                   const sg_pi_opts* pi_opts, const sg_opts* opts, void* stream) {
    if (!mesh) return fail(SG_E_ARG, "mesh is NULL");
    if (mode != SG_BWD_EP && mode != SG_BWD_GFD) return fail(SG_E_ARG, "unknown mode %d", mode);
    if (n < 0) return fail(SG_E_ARG, "n must be >= 0");
    sg_opts o;
    int rc = check_opts(opts, o, mesh);
    if (rc != SG_OK) return rc;
    sg_pi_opts po;
    rc = check_pi_opts(pi_opts, po);
    if (rc != SG_OK) return rc;
    if (n == 0) return SG_OK;
    if (!f || !b || !v || !g_p || !grad_v || !grad_b) return fail(SG_E_ARG, "a required array is NULL");
    if (mode == SG_BWD_EP && (!f_out || !v_out)) return fail(SG_E_ARG, "EP needs the forward's f_out and v_out");
    if (n >= ((int64_t)1 << 29)) return fail(SG_E_ARG, "the PI backward takes fewer than 2^29 queries per call");
    rc = ensure_pi(mesh);
    if (rc != SG_OK) return rc;
    sg::BwdArgs a{};
    a.n = n;
    a.mode = mode;
    a.f = f; a.b = b; a.v = v;
    a.f_out = f_out; a.v_out = v_out;
    a.g = g_p;
    a.grad_v = grad_v; a.grad_b = grad_b;
    a.eps_v = o.eps_v; a.eps_p = o.eps_p;
    a.max_steps = o.max_steps;
    a.snap = o.vertex_snap;
    sg::PiArgs pa{};
    pa.step = po.step;
    pa.max_steps = po.max_steps;
    pa.scan = po.search == SG_PI_SCAN;
    const hipStream_t st = (hipStream_t)stream;
    Workspace ws;
    rc = take_workspace(o, sg::pi_bwd_workspace(n, mode), st, ws);
    if (rc != SG_OK) return rc;
    hipError_t e = sg::launch_pi_backward(mesh->pi(), mesh->dev(), a, pa, ws.p, st);
    const hipError_t e2 = give_workspace(ws, st);
    if (e != hipSuccess) return hip_fail(e, "PI backward launch");
    if (e2 != hipSuccess) return hip_fail(e2, "workspace release");
    return SG_OK;
}

int sg_exp(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v, int32_t* f_out, float* b_out,
           float* p_out, float* v_out, int32_t* status, int32_t* n_cross, uint64_t* seq_hash, const sg_opts* opts,
           void* stream) {
    return sg_exp_transport(mesh, n, f, b, v, 0, nullptr, f_out, b_out, p_out, v_out, nullptr, status, n_cross,
                            seq_hash, opts, stream);
}

}  // extern "C"
