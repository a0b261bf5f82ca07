/*
 * sg.h -- C ABI of the MI355X straightest-geodesic library.
 *
 * Computes the discrete exponential map Exp_p(v) on triangle meshes by
 * straightest geodesics (Verninas et al., "Parallelised Differentiable
 * Straightest Geodesics for 3D Meshes": Sec. 3 eq. ivp for the definition,
 * Sec. 4 "Straightest geodesics" for the straightest rule, Alg. gpu_parallel
 * for one geodesic per GPU lane), the parallel transport of extra tangent
 * vectors along it (Sec. 4 "Parallel Transport"), and the backward schemes of
 * Sec. 4 (extrinsic proxy, eq. proxy_func; geodesic finite differences, eqs.
 * jv and jp), chained with an upstream gradient as in eq. chain.
 *
 * Conventions shared by every call:
 *  - Array arguments named in the comments as [n,3] are row-major float32 or
 *    int32 arrays in *device* memory (hipMalloc / torch CUDA tensors) unless
 *    the comment says host.  The caller owns them; the library never frees
 *    caller memory and keeps no pointer after the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every call except sg_mesh_create / sg_mesh_destroy / sg_mesh_info is
 *    asynchronous on that stream.
 *  - Return values: SG_OK or a negative SG_E_* code.  Argument and shape
 *    problems are found before anything is launched; a HIP failure maps to
 *    SG_E_HIP.  No C++ exception crosses this boundary.  sg_last_error()
 *    returns a message for the last failure on the calling thread.
 *  - Per-ray problems never fail a call: they go to the optional per-ray
 *    `status` array (SG_RAY_*).
 *  - A surface point is (face id, barycentric b) with p = sum_k b_k x_{F[f][k]}
 *    (Sec. 4); b is renormalised to sum 1 and must be non-negative.  Face ids
 *    are global over all meshes of a handle.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_mesh_s* sg_mesh;

enum {
    SG_OK = 0,
    SG_E_ARG = -1,          /* null pointer, bad size, bad option */
    SG_E_NONMANIFOLD = -2,  /* an edge with more than two faces, or a vertex whose faces form several fans (Sec. 4) */
    SG_E_DEGENERATE = -3,   /* a face repeating a vertex or with zero area */
    SG_E_HIP = -4,          /* a HIP runtime call failed */
    SG_E_OOM = -5           /* host or device allocation failed */
};

enum {
    SG_RAY_OK = 0,          /* traced the full length */
    SG_RAY_MAXSTEPS = 1,    /* stopped after max_steps crossings (Alg. gpu_parallel's MAX_STEPS) */
    SG_RAY_BOUNDARY = 2,    /* reached a boundary edge or boundary vertex and stopped there (Sec. 4) */
    SG_RAY_BADINPUT = 3     /* face id out of range, non-finite or negative input, or a vertex start whose
                               direction leaves the given face */
};

enum { SG_BWD_EP = 0, SG_BWD_GFD = 1 };
enum {
    SG_BOUNDARY_STOP = 0,   /* stop at a boundary edge or vertex, status SG_RAY_BOUNDARY (Sec. 4, the original rule) */
    SG_BOUNDARY_AVOID = 1   /* hole avoidance (Sec. 4; the hole branches of the appendix's transport_over_edge and
                               transport_over_vertex): a ray that reaches a boundary edge slides along it toward
                               the end its direction leans to; at a boundary vertex it resumes straight in the fan
                               face whose corner holds the projection of the direction recorded at the boundary,
                               choosing the face whose plane deviates least from that direction; when no face's
                               corner holds it, it slides on along the next boundary edge.  Each slide and
                               resumption counts as a step (n_cross, max_steps, seq_hash).  The reported end
                               direction is the recorded one projected onto the end face; extra vectors keep their
                               angle to it.  Such rays end with SG_RAY_OK when their length is used up. */
};
enum {
    SG_KERNEL_AUTO = 0,         /* forward: SG_KERNEL_PLAIN when n fits the persistent walk's resident lanes
                                   (walk_blocks x 256 x rays_per_lane, 196,608 by default on 256 CUs), else
                                   SG_KERNEL_PERSISTENT; the backward's walks are always persistent */
    SG_KERNEL_PLAIN = 1,        /* one ray per lane, run to completion (Alg. gpu_parallel) */
    SG_KERNEL_PERSISTENT = 2,   /* persistent waves refilled from ray queues (a share per XCD) */
    SG_KERNEL_PARTITIONED = 3   /* the mesh cut into 8 spatial parts, one per XCD: the walk runs in rounds (one
                                   launch each) in which the waves of XCD p walk the rays inside part p until
                                   they end or leave it, and rays that leave are queued for the next round;
                                   the last round walks every remaining ray to its end */
};

typedef struct {
    int32_t max_steps;     /* cap on crossings per ray (edge crossings + vertex passages); <= 0: 1 << 20 */
    float vertex_snap;     /* an exit point within this edge-parameter distance of an edge endpoint passes
                              through that vertex (straightest rule at vertices); <= 0: 2^-21 */
    float eps_v, eps_p;    /* GFD step sizes (absolute lengths); <= 0: 5e-3 * mean edge of the handle */
    int32_t kernel;        /* SG_KERNEL_*: which forward kernel runs the walk */
    uint32_t debug;        /* bit 0: fill n_cross; bit 1: fill seq_hash (FNV-1a 64 of the visited face ids);
                              bit 2: time the walk kernel with HIP events (read with sg_mesh_walk_time);
                              bit 3 (sg_autotune): tune again even for a cached class of batches */
    int32_t refill_min;    /* persistent kernel: a wave refetches rays once this many of its 64 lanes are
                              idle (of 128 ray slots with two rays per lane); <= 0: 48 per 64 slots in
                              the forward, 32 in the backward's walks */
    int32_t walk_blocks;   /* persistent kernel: 256-lane blocks launched; <= 0: three per CU */
    int32_t rays_per_lane; /* persistent kernel: rays each lane walks at once, 1 or 2; <= 0: tuned default */
    int32_t ray_queues;    /* persistent kernel: ray queues the walk claims rays from, a multiple of 8 (an
                              equal share of each XCD, which drains its queues one after another) up to 64;
                              <= 0: 8 */
    int32_t boundary_mode; /* SG_BOUNDARY_STOP (default) or SG_BOUNDARY_AVOID; honoured by every kernel and
                              the backward (the vertex gradient leaves out rays that slid) */
    int32_t gradx_records; /* vertex gradient: edge crossings per query for which the workspace holds records
                              (48 bytes each, at most 2^30 records per call) that are summed per half-edge in
                              LDS; crossings past them add their sums with float64 atomics (same result,
                              slower).  0: 256; < 0: none */
    void* workspace;       /* optional caller-owned device workspace, 256-byte aligned, at least the size
                              sg_exp_workspace_size / sg_backward_workspace_size report.  With it a call
                              allocates nothing, so it can be captured in a HIP graph (debug bit 2 aside).
                              Calls sharing one workspace must be ordered (same stream).  NULL: the call
                              takes a stream-ordered allocation (hipMallocAsync) and releases it. */
    uint64_t workspace_bytes;
} sg_opts;

/* Fills *o with the defaults above. */
void sg_opts_default(sg_opts* o);

/*
 * Builds a mesh handle from host arrays (Sec. 4: M = {X, F}; several meshes
 * may be batched by offsets, Sec. 4 "Parallelisation on the GPU").
 *   X_host [n_verts,3] float32 host, F_host [n_faces,3] int32 host.
 *   vert_offsets / face_offsets: host int64 arrays of n_meshes+1 entries
 *   (prefix sums), or both NULL with n_meshes = 1.  Vertex indices in F are
 *   local to their mesh; the library adds the vertex offset.  Rays name faces
 *   by global id (face_offsets[m] + local id).
 * Validates the manifold condition of Sec. 4, packs per-half-edge records in
 * float64 on the host (rounded once to float32 / fixed-point angles) and
 * uploads them.  Synchronous.  On success *out owns device memory until
 * sg_mesh_destroy.
 */
int sg_mesh_create(const float* X_host, int64_t n_verts, const int32_t* F_host, int64_t n_faces,
                   const int64_t* vert_offsets, const int64_t* face_offsets, int32_t n_meshes,
                   sg_mesh* out);
void sg_mesh_destroy(sg_mesh mesh);

/*
 * New vertex positions for an existing mesh handle (the same connectivity),
 * for optimisation loops over X (the vertex gradient of sg_exp_backward is
 * their gradient).  X_host [n_verts,3] float32 host, n_verts as at creation.
 * Re-packs the position-dependent parts in float64 on the host (edge lengths,
 * corner angles, vertex total angles, positions, mean edge) and uploads them;
 * adjacency, face order and the handle stay.  Synchronous: it waits for the
 * device to be idle first, since no call may read the mesh while it changes.
 * A zero-area face or a non-finite position returns SG_E_DEGENERATE /
 * SG_E_ARG and leaves the mesh unchanged.
 */
int sg_mesh_update_vertices(sg_mesh mesh, const float* X_host, int64_t n_verts);

/* Host outputs, each nullable: mean undirected edge length, number of
 * half-edge records, device bytes held by the handle. */
int sg_mesh_info(sg_mesh mesh, double* mean_edge, int64_t* n_half_edges, size_t* device_bytes);

/*
 * Exponential map (Sec. 3 eq. ivp; Alg. gpu_parallel).  For each ray i:
 *   in : f[n] int32, b[n,3] float32, v[n,3] float32 (projected onto the start
 *        face's plane; |v_t| is the length to trace).
 *   out: f_out[n] int32 end face, b_out[n,3] end barycentrics, p_out[n,3] end
 *        point, v_out[n,3] = |v_t| * end tangent (v transported to p').
 *   optional (NULL to skip): status[n] int32, n_cross[n] int32 (needs
 *        debug bit 0), seq_hash[n] uint64 (needs debug bit 1).
 * opts may be NULL (defaults).  n = 0 is a no-op.  The persistent and
 * partitioned kernels take n < 2^31 (SG_E_ARG otherwise); the plain kernel
 * any n.
 */
int sg_exp(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v,
           int32_t* f_out, float* b_out, float* p_out, float* v_out,
           int32_t* status, int32_t* n_cross, uint64_t* seq_hash,
           const sg_opts* opts, void* stream);

/*
 * sg_exp plus parallel transport (Sec. 4 "Parallel Transport") of K extra
 * vectors per ray: W[n,K,3] float32 in (projected onto the start face),
 * W_out[n,K,3] float32 out.  Each vector keeps its norm and its signed angle
 * to the geodesic's tangent.  K in [0, 64].
 */
int sg_exp_transport(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v,
                     int32_t K, const float* W,
                     int32_t* f_out, float* b_out, float* p_out, float* v_out, float* W_out,
                     int32_t* status, int32_t* n_cross, uint64_t* seq_hash,
                     const sg_opts* opts, void* stream);

/*
 * Allocation-free sg_exp_transport, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, and harnesses
 * that forbid hipMalloc.  Same arguments, outputs and per-ray semantics as
 * sg_exp_transport (the same kernels run).  The persistent walk's workspace
 * is a fixed device array inside the library, SG_NOALLOC_SCRATCH_BYTES
 * (128 MiB) per device, held by every device the library runs on until the
 * process ends; the call allocates nothing and calls no allocating routine.
 *   - n and K must fit it: sg_exp_workspace_size (persistent kernel) must
 *     report at most SG_NOALLOC_SCRATCH_BYTES, else SG_E_ARG before any
 *     launch (about 1.45M rays at K = 2, 1.76M at K = 0).
 *   - Every call on a device shares that device's array, so calls that
 *     overlap on one device race: order them on one stream or synchronize
 *     between them.  The kernels clear what must start at zero; the array
 *     keeps the last call's contents.
 *   - opts->kernel: SG_KERNEL_AUTO / SG_KERNEL_PERSISTENT, or SG_KERNEL_PLAIN
 *     (which needs no scratch, as SG_KERNEL_AUTO for a batch that fits the
 *     resident lanes); SG_KERNEL_PARTITIONED, opts->workspace != NULL
 *     and debug bit 2 (event timing) return SG_E_ARG.
 */
#define SG_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int sg_exp_transport_noalloc(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v,
                             int32_t K, const float* W,
                             int32_t* f_out, float* b_out, float* p_out, float* v_out, float* W_out,
                             int32_t* status, int32_t* n_cross, uint64_t* seq_hash,
                             const sg_opts* opts, void* stream);

/*
 * Backward of the exponential map (Sec. 4 "Differentiation").  Given
 * g_p[n,3] = dL/dp' (float32, device) for the queries (f, b, v) of an earlier
 * sg_exp call, and optionally that call's saved outputs f_out[n], b_out[n,3],
 * v_out[n,3] and status[n] (each nullable), returns
 *   grad_v[n,3] = dL/dv (tangent to the start face) and
 *   grad_b[n,3] = dL/db (component k = G . x_k, where G is the in-plane
 *                 gradient of L with respect to the start point),
 * both nullable together, and accumulates into grad_X[n_verts,3] (float64,
 * nullable; the caller zeroes it) dL/dX, the gradient with respect to the
 * vertex positions (global vertex ids).
 *   mode SG_BWD_EP  (eq. proxy_func): J^v = R = M_{p'} M_p^T with frames
 *        [e_par, e_perp, n] at both ends; grad_b = 0.  On meshes whose faces
 *        agree in orientation it reads the forward's f_out[n] and v_out[n,3]
 *        and walks nothing; otherwise (those two may be NULL) it re-walks the
 *        geodesic to find the end normal's orientation.
 *   mode SG_BWD_GFD (eqs. jv, jp and chain): geodesic finite differences with
 *        step sizes opts->eps_v, opts->eps_p.  Walks seven geodesics per
 *        query (the base, the e_perp-perturbed one, two short start-point
 *        steps, then the e_par step from p' and the two start-point-shifted
 *        geodesics): the four long ones in one persistent pass, the three
 *        short ones (length eps) one lane each.  With f_out, b_out and v_out
 *        given, on meshes whose faces agree in orientation, the base
 *        geodesic's end is taken from them (Appendix "Speed-up GFD and EP
 *        through batching": Exp(p, v) is the forward's) and six are walked.
 *        |v_t| = 0 takes e_par = e_u (the start face's x1 - x0 direction).
 *   grad_X (an extension; the paper has no vertex gradient): the exact
 *        derivative of p' = H_m o ... o H_1(p + v_t), the composition of the
 *        rigid unfoldings about the crossed edges, with the combinatorics
 *        frozen.  The geodesic is re-walked for the adjoint's per-edge
 *        terms (one record per crossing, summed per half-edge in float64
 *        after grouping by half-edge range); a pass over the faces maps each
 *        crossed edge's sums to its four hinge vertices, and a pass over the
 *        vertices adds each vertex's total to grad_X once (no atomics on
 *        grad_X: calls that accumulate into one grad_X must be ordered, for
 *        instance by running on one stream).  The
 *        adjoint starts from the end frame: taken from the forward's saved
 *        f_out, v_out and status when all three are given, the faces agree
 *        in orientation, hole avoidance is off and the mode is EP (or only
 *        grad_X is asked for); otherwise from one more walk (GFD walks it
 *        anyway).  Rays
 *        whose walk ends with a status other than SG_RAY_OK contribute
 *        nothing.  A vertex passage is not a hinge: such rays contribute their
 *        edge and start terms with the vertex rule held fixed, which is not
 *        the derivative of the map (give them g_p = 0 to exclude them).
 *        The order of the float64 sums depends on timing, so grad_X's last
 *        bits may differ between calls.
 * Queries the forward rejects (SG_RAY_BADINPUT) get NaN in grad_v, grad_b.
 * Uses a stream-ordered device workspace (GFD 224 bytes per query, 192 with
 * the forward's outputs; a re-walk 32; grad_X 96 per query plus 272 per face plus 48 per record, see
 * gradx_records).  opts: max_steps, vertex_snap, eps_v, eps_p, refill_min,
 * walk_blocks, ray_queues, gradx_records are honoured; kernel is ignored (the
 * persistent walk always runs).  n < 2^31 (SG_E_ARG otherwise).
 */
int sg_exp_backward(sg_mesh mesh, int32_t mode, int64_t n, const int32_t* f, const float* b, const float* v,
                    const int32_t* f_out, const float* b_out, const float* v_out, const int32_t* status,
                    const float* g_p, float* grad_v, float* grad_b, double* grad_X, const sg_opts* opts,
                    void* stream);

/*
 * sg_exp_backward with cotangents of every output of an earlier
 * sg_exp_transport call (an extension; the paper's backward takes dL/dp'
 * only), each float32 [n,3] device and nullable, at least one given:
 *   g_p = dL/dp';
 *   g_b = dL/db' (end barycentrics): inside the end face b'_k has the
 *         in-plane gradient n x (y_{k+2} - y_{k+1}) / (2 A), so it adds to
 *         dL/dp' and then follows EP or GFD like g_p (this is what chains
 *         steps of an iterated Exp through their start points);
 *   g_v = dL/dv' and g_W [n,K,3] = dL/dW': the walk carries the frame
 *         (d, n x d) from p to p', so W'_k = R W_k and v' = R v_t with R that
 *         frame map (Sec. 4 "Parallel Transport"), constant wherever the face
 *         sequence is; grad_v gains R^T g_v and grad_W [n,K,3] (with g_W)
 *         receives R^T g_W, both in the start face's plane, in either mode.
 * grad_X takes the g_p and g_b terms.  Other arguments as for sg_exp_backward.
 */
int sg_exp_backward_transport(sg_mesh mesh, int32_t mode, int64_t n, const int32_t* f, const float* b,
                              const float* v, int32_t K, const int32_t* f_out, const float* b_out,
                              const float* v_out, const int32_t* status, const float* g_p, const float* g_b,
                              const float* g_v,
                              const float* g_W, float* grad_v, float* grad_b, float* grad_W, double* grad_X,
                              const sg_opts* opts, void* stream);

/*
 * Device workspace (bytes, host output) that sg_exp / sg_exp_transport need
 * for n queries with K extra vectors (0 for sg_exp) under these options
 * (kernel and debug bits matter; SG_KERNEL_AUTO resolves with this n, so a
 * batch that fits the resident lanes needs none), and that
 * sg_exp_backward needs for n queries in `mode` with grad_v/grad_b
 * (want_vjp != 0) and/or grad_X (want_grad_X != 0).  0 means none.
 */
int sg_exp_workspace_size(sg_mesh mesh, int64_t n, int32_t K, const sg_opts* opts, size_t* bytes);
int sg_backward_workspace_size(sg_mesh mesh, int32_t mode, int64_t n, int32_t want_vjp, int32_t want_grad_X,
                               const sg_opts* opts, size_t* bytes);

/*
 * Projection-integration (PI) exponential map, the paper's comparison Exp
 * (appendix "Projection Integration Exp Map", Alg. projection-exp): repeat
 *   q = p + s v; (p', f') = nearest point of the mesh to q (project_to_mesh);
 *   v turned by the rotation taking f's normal to f''s (rotate_vector);
 *   l += |p' - p|
 * while l < |v_t|.  Readings: v (and W) are first projected onto the start
 * face's plane, as for sg_exp; the loop runs while the traced length is
 * short of |v_t| (the last step is not clamped, as printed); the nearest
 * point is the minimiser of the distance to each closed triangle over the
 * ray's own mesh, ties (distances within 2^-20 of the largest coordinate,
 * i.e. float32 rounding: a nearest point on an edge or vertex) going to the
 * face whose normal is most nearly parallel to q - p', then the smallest
 * face id; parallel normals leave v unchanged.
 *   search SG_PI_GRID (default): a uniform grid per mesh, cells visited in
 *     rings and skipped when farther than the best distance found, which
 *     selects what a scan of every face selects;
 *   search SG_PI_SCAN: the printed scan of every face of the mesh per step.
 * In/out arrays as for sg_exp_transport (K extra vectors keep their angle to
 * v); n_steps[n] int32 (nullable) receives the projection steps taken.
 * status: SG_RAY_OK, SG_RAY_MAXSTEPS (l still short after max_steps steps),
 * SG_RAY_BADINPUT.  The first PI call on a handle, and the first after
 * sg_mesh_update_vertices, builds the per-face records and grids on the host
 * and uploads them (synchronous; about 100 bytes per face plus 4 bytes per
 * cell).  Float32 arithmetic; the traced length is summed in float-float.
 */
enum { SG_PI_GRID = 0, SG_PI_SCAN = 1 };
typedef struct {
    float step;            /* s, in (0, 1]; <= 0: 0.01 */
    int32_t max_steps;     /* <= 0: ceil(8 / s) */
    int32_t search;        /* SG_PI_GRID or SG_PI_SCAN */
} sg_pi_opts;
void sg_pi_opts_default(sg_pi_opts* o);
int sg_pi_exp(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v, int32_t K,
              const float* W, int32_t* f_out, float* b_out, float* p_out, float* v_out, float* W_out,
              int32_t* status, int32_t* n_steps, const sg_pi_opts* pi_opts, void* stream);

/*
 * Backward of the PI map (the paper applies both of its schemes to PI).
 *   SG_BWD_EP: eq. proxy_func from the forward's saved f_out and v_out (the
 *     end frame takes the end face's own normal); no PI steps run.
 *   SG_BWD_GFD: eqs. jv, jp and chain with PI as the Exp: seven PI maps per
 *     query in two stacked launches (Appendix "Speed-up GFD and EP through
 *     batching"), step sizes opts->eps_v, opts->eps_p; f_out, v_out unused.
 * g_p[n,3] = dL/dp'; grad_v, grad_b [n,3] out as for sg_exp_backward (NaN for
 * rejected queries).  opts: eps_v, eps_p and workspace are honoured (GFD's
 * workspace: sg_pi_backward_workspace_size, about 600 bytes per query; NULL:
 * a stream-ordered allocation).  n < 2^29.
 */
int sg_pi_backward(sg_mesh mesh, int32_t mode, int64_t n, const int32_t* f, const float* b, const float* v,
                   const int32_t* f_out, const float* v_out, const float* g_p, float* grad_v, float* grad_b,
                   const sg_pi_opts* pi_opts, const sg_opts* opts, void* stream);
int sg_pi_backward_workspace_size(sg_mesh mesh, int32_t mode, int64_t n, size_t* bytes);

/*
 * Autotuner for the forward walk (Sec. 4 "Parallelisation on the GPU"
 * schedules one ray per thread; this picks the schedule that runs the
 * caller's batch fastest).  Times sg_exp_transport on the given queries
 * (device arrays as in sg_exp_transport; a representative sample is enough)
 * for the plain kernel and for the persistent kernel over rays per lane,
 * refill thresholds (the compaction period), resident blocks per CU (waves
 * per SIMD) and ray queues, then writes the fastest kernel, rays_per_lane,
 * refill_min,
 * walk_blocks, ray_queues into *opts (its other fields are kept and used).
 * Synchronizes `stream`; allocates and frees its own scratch outputs and
 * workspace (before any timing).  Not capturable.  *best_ms (nullable)
 * receives the winner's time per call.
 * The pick is cached per process, keyed by device (gfx arch, CU count), the
 * mesh's face-count class (power of two), the batch's size class, K, the
 * boundary rule and its length class (mean |v| of a 256-ray sample, in half
 * octaves of the mean edge); a batch of a cached class gets the cached pick
 * without timing.  opts->debug bit 3 forces a new tuning (and recaches).
 */
int sg_autotune(sg_mesh mesh, int64_t n, const int32_t* f, const float* b, const float* v, int32_t K,
                const float* W, sg_opts* opts, double* best_ms, void* stream);

/*
 * Walk-kernel timing (profiling aid).  Calls made with opts->debug bit 2
 * record a HIP event pair around their walk kernel on the call's stream.
 * This synchronizes those events, returns the summed elapsed milliseconds
 * and the number of timed launches (host outputs, nullable), and clears the
 * list.  Not thread-safe with concurrent timed calls on the same handle.
 */
int sg_mesh_walk_time(sg_mesh mesh, double* total_ms, int64_t* launches);

/* Message describing the last non-OK return on the calling thread. */
const char* sg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
