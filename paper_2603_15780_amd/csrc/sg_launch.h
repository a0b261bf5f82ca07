// sg_launch.h -- launch interface between the C ABI (host) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "sg_internal.h"

namespace sg {

struct ExpArgs {
    int64_t n;
    const int32_t* f;
    const float* b;
    const float* v;
    int32_t K;
    const float* W;
    int32_t* f_out;
    float* b_out;
    float* p_out;
    float* v_out;
    float* W_out;
    int32_t* status;
    int32_t* n_cross;
    uint64_t* seq_hash;
    int32_t max_steps;
    float snap;
    uint32_t debug;
    int32_t rays_per_lane;   // persistent walk: 1 or 2 rays per lane
};

struct BwdArgs {
    int64_t n;
    int32_t mode;           // 0 extrinsic proxy, 1 geodesic finite differences
    const int32_t* f;
    const float* b;
    const float* v;
    const int32_t* f_out;   // saved forward outputs (extrinsic proxy; vertex gradient and GFD without a re-walk)
    const float* b_out;
    const float* v_out;
    const int32_t* status_in;   // the forward's saved per-ray status, or null
    const float* g;         // dL/dp', or null (zero)
    const float* g_bo;      // dL/db' [n,3] (end barycentrics), or null
    const float* g_v;       // dL/dv' [n,3], or null
    const float* g_W;       // dL/dW' [n,K,3], or null
    int32_t K;              // transported vectors per query (g_W, grad_W)
    float* grad_v;
    float* grad_b;
    float* grad_W;          // dL/dW [n,K,3] (with g_W)
    float eps_v, eps_p;
    int32_t max_steps;
    float snap;
    double* grad_X;         // [n_verts, 3] accumulated vertex-position gradient, or null
    const int32_t* slot;    // position of each query in the walk arrays (set by the launcher), or null
    int32_t gx_records;     // grad-X records reserved per query for binned accumulation (<= 0: atomics only)
    int32_t gfd_saved;      // (set by the launcher) GFD takes the base geodesic's end from f_out, b_out, v_out
    const int32_t* vc_off;  // [n_verts + 1] vertex -> corner list offsets (the vertex gradient's gather)
    const int32_t* vc;      // [3 n_faces] corners 3 f + k (internal face f, corner k) of each vertex
    // (set by the launcher) the vertex gradient's start terms: nine floats per query,
    // each query's rank among those of its start face, the faces' list offsets, the lists
    const float* sterm;
    const int32_t* srank;
    const uint32_t* fstart;
    int32_t* qlist;
};

// Host-side result of packing a mesh (float64 work, rounded once).
struct PackedMesh {
    std::vector<FaceRec> face;
    std::vector<int32_t> F;           // internal (bisection) face order
    std::vector<int64_t> order;       // internal face id -> user face id
    std::vector<int32_t> perm;        // user face id -> internal face id
    int64_t part_start[kParts + 1];   // internal face ranges of the XCD parts
    std::vector<float> X;
    std::vector<int64_t> half;
    std::vector<int32_t> twin;        // half-edge across each edge (internal ids), -1 on the boundary
    std::vector<uint8_t> vbnd;        // vertex lies on a boundary edge
    std::vector<float> geo;           // [n_faces, 16]: per-face positions, lengths, corners, user id (DevMesh::geo)
    std::vector<int64_t> face_off;    // [n_meshes + 1] user face offsets of the batched meshes
    int64_t n_verts = 0, n_faces = 0;
    double mean_edge = 0.0;
    int32_t has_flip = 0;
};

// Validates and packs a mesh on the host; returns SG_OK or an SG_E_* code.
int pack_mesh(const float* X_host, int64_t n_verts, const int32_t* F_host, int64_t n_faces,
              const int64_t* vert_offsets, const int64_t* face_offsets, int32_t n_meshes, PackedMesh& out);
// Recomputes the position-dependent parts of a packed mesh (face records'
// lengths and corners, half_theta, X, mean_edge) for new vertex positions,
// keeping its connectivity, links and face order.
int pack_geometry(const float* X_host, PackedMesh& pm);

// Plain forward: one ray per lane, run to completion (Alg. gpu_parallel).
hipError_t launch_exp_plain(const DevMesh& M, const ExpArgs& a, hipStream_t s);

// Schedule of a persistent walk launch.
constexpr int kMaxQueues = 64;
struct WalkSched {
    int blocks;       // 256-lane blocks launched
    int refill_min;   // idle lanes (of 64 per ray slot) that trigger a refill
    int queues;       // ray queues: a multiple of 8, at most kMaxQueues
};

// Persistent forward: init kernel, persistent work-queue walk, finish kernel.
// ws must hold exp_persistent_workspace(n, K) bytes of device memory.
size_t exp_persistent_workspace(int64_t n, int32_t K);
// Device scratch of the allocation-free forward (one copy per device, held
// until the process ends): its size, the devices it is looked up for, and the
// current device's address (looked up with hipGetSymbolAddress on the first
// request from each device).
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
constexpr int kNoAllocMaxDevices = 64;
hipError_t noalloc_scratch(void** out);
// ev0/ev1 (nullable) are recorded on s around the walk kernel.
hipError_t launch_exp_persistent(const DevMesh& M, const ExpArgs& a, void* ws, const WalkSched& w, hipStream_t s,
                                 hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
int walk_blocks_per_cu();
int part_blocks_per_cu();

// ---- projection integration (appendix "Projection Integration Exp Map")
// T: float for the ABI's arrays, double for the backward's internal stacks.
template <class T>
struct PiArgsT {
    int64_t n;
    const int32_t* f;   // user face ids
    const T* b;
    const T* v;
    int32_t K;
    const T* W;         // [n, K, 3] or null (K = 0)
    int32_t* f_out;
    T* b_out;
    T* p_out;
    T* v_out;
    T* W_out;
    int32_t* status;
    int32_t* n_steps;
    double step;        // s
    int32_t max_steps;
    int32_t scan;       // 1: scan every face of the mesh (the printed form), 0: grid search
};
using PiArgs = PiArgsT<float>;
hipError_t launch_pi_exp(const PiMesh& P, const PiArgs& a, hipStream_t s);
// EP (saved f', v') or GFD (seven PI walks per query, stacked in two launches).
size_t pi_bwd_workspace(int64_t n, int32_t mode);
hipError_t launch_pi_backward(const PiMesh& P, const DevMesh& M, const BwdArgs& a, const PiArgs& pa, void* ws,
                              hipStream_t s);
// The extrinsic proxy from saved outputs (shared by both Exp maps).
hipError_t launch_ep_saved(const DevMesh& M, const BwdArgs& a, hipStream_t s);

// Backward of the exponential map (extrinsic proxy or geodesic finite differences).
// have_*: which of the forward's saved outputs (f', b', v', status) the call is given.
size_t bwd_workspace(int64_t n, int32_t mode, bool has_flip, bool vjp, bool gradx, int64_t n_faces,
                     int32_t gx_records, int walk_blocks, bool hole, bool have_f, bool have_b, bool have_v,
                     bool have_status);
hipError_t launch_backward(const DevMesh& M, const BwdArgs& a, void* ws, const WalkSched& w, hipStream_t s);

// Partitioned forward: the walk runs on the XCD whose L2 holds the ray's
// current part of the mesh; rays crossing parts are handed over through queues.
size_t exp_partitioned_workspace(int64_t n, int32_t K, bool hashes);
hipError_t launch_exp_partitioned(const DevMesh& M, const ExpArgs& a, void* ws, int grid_blocks, int refill_min,
                                  hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

}  // namespace sg
