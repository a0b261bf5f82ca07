/*
 * sg_oracle.h -- float64 CPU oracle for the straightest-geodesic exponential
 * map on triangle meshes (Verninas et al., "Parallelised Differentiable
 * Straightest Geodesics for 3D Meshes", Sec. 4 and the appendix algorithms
 * geodesic_step / transport_over_edge / transport_over_vertex).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 */
#ifndef SG_ORACLE_H
#define SG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_E_ARG = -1, OR_E_NONMANIFOLD = -2, OR_E_DEGENERATE = -3, OR_E_OOM = -5 };
enum { OR_RAY_OK = 0, OR_RAY_MAXSTEPS = 1, OR_RAY_BOUNDARY = 2, OR_RAY_BADINPUT = 3 };

typedef struct or_mesh or_mesh;

typedef struct {
    int32_t max_steps;     /* cap on edge crossings + vertex passages */
    double vertex_snap;    /* exit point within this edge-parameter distance of an
                              edge endpoint counts as passing through that vertex */
    int32_t boundary_mode; /* 0: stop at the boundary (status BOUNDARY); 1: avoid
                              holes by tracing along the boundary (Sec. 4) */
} or_opts;

/* Builds adjacency, normals and vertex total angles from the canonical float32
 * mesh (upcast exactly).  Returns OR_OK or a negative error code. */
int or_mesh_build(const float* X, int64_t nv, const int32_t* F, int64_t nf, or_mesh** out);
/* The same from float64 positions (used to take central differences in X). */
int or_mesh_build64(const double* X, int64_t nv, const int32_t* F, int64_t nf, or_mesh** out);
void or_mesh_free(or_mesh* m);
double or_mesh_mean_edge(const or_mesh* m);
void or_mesh_theta(const or_mesh* m, double* theta /* [nv] */);
const char* or_last_error(void);

/* Batched exponential map with parallel transport of K extra vectors.
 * Inputs: f[n], b[n*3] (renormalised to sum 1), v[n*3] (projected onto the
 * start face), W[n*K*3].  Outputs (all caller-owned, float64 unless noted):
 * f_out, b_out, p_out, v_out = |v_t| * end tangent, W_out, status,
 * n_cross (edge crossings + vertex passages), seq_hash (FNV-1a 64 of the
 * visited face ids), min_vdist (closest approach of the path to a vertex of
 * the face it was in), traced (total traced length), sigma_end (+1/-1, the
 * end face's normal relative to the orientation carried along the path),
 * n_bnd (boundary slides, whole or partial, and resumptions under hole
 * avoidance), bnd_margin (the smallest margin of the decisions hole
 * avoidance took: |cos| of the angle between the recorded direction and an
 * edge it slid along, the sine margin of each corner test at a boundary
 * vertex, the gap between the smallest and the next transport error, and
 * the cosine gap of a slide's end choice; infinity if none).  min_vdist
 * counts the straight parts of the path only: slides run along boundary
 * edges, and a resumption starts at its boundary vertex by construction.
 * Any output pointer except f_out/b_out/p_out/v_out/status may be NULL.
 * nthreads <= 0 uses every online core. */
int or_exp_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b,
                 const double* v, int32_t K, const double* W, const or_opts* o,
                 int32_t* f_out, double* b_out, double* p_out, double* v_out,
                 double* W_out, int32_t* status, int32_t* n_cross, uint64_t* seq_hash,
                 double* min_vdist, double* traced, int8_t* sigma_end, int32_t* n_bnd,
                 double* bnd_margin, int32_t nthreads);

/* One ray with its event list: for each edge crossing or vertex passage,
 * kind (0 edge, 1 vertex, 2 boundary slide, 3 resumption after a slide), the
 * face entered and the 3D point of the event.
 * Returns the number of events written (at most cap). */
int32_t or_exp_trace(const or_mesh* m, int32_t f, const double* b, const double* v,
                     const or_opts* o, int32_t cap, int8_t* kind, int32_t* face,
                     int32_t* edge_v0, int32_t* edge_v1, double* point,
                     int32_t* f_out, double* p_out, int32_t* status);

/* Extrinsic-proxy backward (eq. proxy_func): grad_v = R^T g with
 * R = M_{p'} M_p^T, frames [e_par, e_perp, n]; the start-point gradient is zero. */
int or_ep_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b,
                const double* v, const or_opts* o, const double* g,
                double* grad_v, double* grad_b, int32_t nthreads);

/* Geodesic finite differences (eqs. jv, jp) at step sizes eps_v, eps_p, chained
 * with the upstream gradient g = dL/dp'.  Also returns the 2x2 Jacobians
 * (row-major, may be NULL) in the paper's local frames. */
int or_gfd_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b,
                 const double* v, const or_opts* o, double eps_v, double eps_p,
                 const double* g, double* grad_v, double* grad_b,
                 double* Jv, double* Jp, int32_t nthreads);

/* Cotangents of the transported outputs (an extension): W'_k = R W_k and
 * v' = R v_t with R the walk's frame map from (d0, n0 x d0) to
 * (d', sigma' n' x d'); returns grad_v [n*3] = P R^T g_v (zero if g_v is NULL)
 * and grad_W [n*K*3] = P R^T g_W, P the projection onto the start plane. */
int or_transport_vjp(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                     const or_opts* o, int32_t K, const double* g_v, const double* g_W, double* grad_v,
                     double* grad_W, int32_t nthreads);

/* Gradient of L = sum_i g_i . p'_i with respect to the vertex positions
 * (an extension: the paper differentiates only in v and p).  Away from
 * vertices p' = H_m o ... o H_1(p + v_t), a composition of the edge unfoldings
 * read as rigid hinge motions; the adjoint is taken through that chain in
 * float64, each hinge's local derivative by a central difference of its
 * closed form (step 1e-6 of the largest coordinate).  grad_X [nv*3] is
 * overwritten.  Rays that pass through a vertex, slide along a boundary, or
 * end with a status other than OK, contribute nothing; n_vertex [n]
 * (nullable) receives each ray's number of vertex passages, or -1 for a
 * status other than OK or a boundary slide. */
int or_gradx_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b,
                   const double* v, const or_opts* o, const double* g, double* grad_X,
                   int32_t* n_vertex, int32_t nthreads);

/* ---- projection integration (appendix "Projection Integration Exp Map",
 * Alg. projection-exp): the comparison Exp of the paper. */
typedef struct {
    double step;           /* s: each step moves the point by s v before projecting */
    int32_t max_steps;     /* cap on projection steps (status MAXSTEPS) */
} or_pi_opts;

/* Batched PI exponential map with K extra vectors rotated alongside v.
 * Inputs as for or_exp_batch.  Outputs: f_out, b_out, p_out, v_out (the
 * rotated v_t), W_out, status (OK or MAXSTEPS, BADINPUT), n_steps
 * (projection steps), traced (accumulated length), margin (the smallest
 * margin of a decision over the steps: the distance gap to the nearest face
 * outside a projection's tie, the alignment gap inside it, and the loop
 * test's gaps |v_t| - l before and l - |v_t| after the last step).  Any output pointer
 * except f_out/b_out/p_out/v_out/status may be NULL. */
int or_pi_exp_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                    int32_t K, const double* W, const or_pi_opts* o, int32_t* f_out, double* b_out,
                    double* p_out, double* v_out, double* W_out, int32_t* status, int32_t* n_steps,
                    double* traced, double* margin, int32_t nthreads);

/* project_to_mesh for n ambient points q[n*3]: the face holding the nearest
 * point of the mesh (ties as in or_pi_exp_batch), that point and its
 * barycentrics. */
int or_pi_project(const or_mesh* m, int64_t n, const double* q, int32_t* f_out, double* c_out, double* b_out,
                  double* margin);

/* The extrinsic proxy and geodesic finite differences with PI as the Exp
 * (the paper applies both schemes to PI, Fig. PIdiff-acc); arguments as for
 * or_ep_batch / or_gfd_batch.  The end frame takes the end face's own normal
 * (PI rotates from face normal to face normal). */
int or_pi_ep_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                   const or_pi_opts* o, const double* g, double* grad_v, double* grad_b, int32_t nthreads);
int or_pi_gfd_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                    const or_pi_opts* o, double eps_v, double eps_p, const double* g, double* grad_v,
                    double* grad_b, double* Jv, double* Jp, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
