// sg_pi.hip -- the projection-integration (PI) exponential map on gfx950
// (appendix "Projection Integration Exp Map", Alg. projection-exp) and the
// paper's two backward schemes over it (Sec. 4 "Differentiation": the
// extrinsic proxy, eq. proxy_func; geodesic finite differences, eqs. jv and
// jp), the comparison the paper draws against its straightest geodesics.
//
// A PI step moves the point by s v in the ambient space, projects the result
// onto the nearest point of the mesh, turns v (and the transported frame)
// from the old face's normal to the new one's, and adds the length actually
// moved, until that length reaches |v_t|.  The printed form finds the nearest
// point by scanning every face; that form is kept (one block-wide scan of
// LDS-staged face tiles per step).  The default finds the same point with a
// uniform grid per mesh: cells in rings around the query, each skipped when
// its box is farther than the best distance so far, so the choice is the one
// the scan makes, with the same distances and the same tie rule.
//
// Float64 arithmetic.  Which face is nearest is a discontinuous decision in
// the query point, taken about 1/s times per ray: a float32 point drifts by a
// few units of 1e-7 per step, enough to flip one of those decisions on a
// large share of rays (after which v turns about a different normal), so the
// map is evaluated in the precision of its definition.  MI355X runs float64
// vector arithmetic at half its float32 rate.
//
// One lane per ray.  Every ray takes about 1/s steps whatever its length, so
// rays in a launch are balanced and no persistent scheduling is needed.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sg_internal.h"
#include "sg_launch.h"

namespace sg {
namespace {

struct D3 {
    double x, y, z;
};
__device__ __forceinline__ D3 d3(double x, double y, double z) { return D3{x, y, z}; }
template <class T>
__device__ __forceinline__ D3 ld(const T* p) { return D3{(double)p[0], (double)p[1], (double)p[2]}; }
__device__ __forceinline__ D3 dsub(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 dscl(D3 a, double s) { return D3{a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ D3 daxpy(double s, D3 x, D3 y) {   // s x + y
    return D3{fma(s, x.x, y.x), fma(s, x.y, y.y), fma(s, x.z, y.z)};
}
__device__ __forceinline__ double ddot(D3 a, D3 b) { return fma(a.x, b.x, fma(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ D3 dcrs(D3 a, D3 b) {
    return D3{fma(a.y, b.z, -a.z * b.y), fma(a.z, b.x, -a.x * b.z), fma(a.x, b.y, -a.y * b.x)};
}
__device__ __forceinline__ double dlen(D3 a) { return sqrt(ddot(a, a)); }
// componentwise select (a conditional on whole objects can keep them in memory)
__device__ __forceinline__ D3 dsel(bool c, D3 a, D3 b) { return D3{c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z}; }
template <class T>
__device__ __forceinline__ void st3(T* p, D3 a) {
    p[0] = (T)a.x;
    p[1] = (T)a.y;
    p[2] = (T)a.z;
}

__device__ __forceinline__ D3 fnormal(const PiFace& F) { return D3{F.n[0], F.n[1], F.n[2]}; }

// Closest point of segment [a, b] to q: a + t (b - a) with t clamped to [0, 1].
__device__ __forceinline__ D3 edge_closest(D3 a, D3 b, D3 q, double& t) {
    const D3 ab = dsub(b, a);
    t = fmin(fmax(ddot(dsub(q, a), ab) / ddot(ab, ab), 0.0), 1.0);
    return daxpy(t, ab, a);
}

// The closest point c of face F to q, its barycentrics (face vertex order) and
// |q - c|.  Inside the triangle's prism c is the projection onto the plane
// (the barycentric solve of the Gram system); outside, the nearest point of a
// convex set lies on its boundary: the nearest of the three edges' clamped
// closest points (the first of equals in edge order 0, 1, 2).
__device__ __forceinline__ double face_closest(const PiFace& F, D3 q, D3& c, double& b0, double& b1, double& b2) {
    const D3 x0 = ld(F.x0), x1 = ld(F.x1), x2 = ld(F.x2);
    const D3 e1 = dsub(x1, x0), e2 = dsub(x2, x0), w = dsub(q, x0);
    const double g11 = ddot(e1, e1), g12 = ddot(e1, e2), g22 = ddot(e2, e2);
    const double r1 = ddot(w, e1), r2 = ddot(w, e2), det = fma(g11, g22, -g12 * g12);
    const double u = fma(g22, r1, -g12 * r2) / det, v = fma(g11, r2, -g12 * r1) / det;
    if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) {
        c = daxpy(v, e2, daxpy(u, e1, x0));
        b0 = 1.0 - u - v;
        b1 = u;
        b2 = v;
        return dlen(dsub(q, c));
    }
    double t0, t1, t2;
    const D3 p0 = edge_closest(x0, x1, q, t0), p1 = edge_closest(x1, x2, q, t1), p2 = edge_closest(x2, x0, q, t2);
    const double d0 = dlen(dsub(q, p0)), d1 = dlen(dsub(q, p1)), d2 = dlen(dsub(q, p2));
    double best = d0;
    c = p0;
    b0 = 1.0 - t0; b1 = t0; b2 = 0.0;
    if (d1 < best) {
        best = d1;
        c = p1;
        b0 = 0.0; b1 = 1.0 - t1; b2 = t1;
    }
    if (d2 < best) {
        best = d2;
        c = p2;
        b0 = t2; b1 = 0.0; b2 = 1.0 - t2;
    }
    return best;
}

// Distance from q to the closed box of grid cell (ix, iy, iz), squared.
__device__ __forceinline__ double box_dist2(const PiGrid& G, D3 q, int ix, int iy, int iz) {
    const double h = G.h;
    const double lx = fma((double)ix, h, (double)G.ox), ly = fma((double)iy, h, (double)G.oy),
                 lz = fma((double)iz, h, (double)G.oz);
    const double gx = fmax(fmax(lx - q.x, q.x - (lx + h)), 0.0);
    const double gy = fmax(fmax(ly - q.y, q.y - (ly + h)), 0.0);
    const double gz = fmax(fmax(lz - q.z, q.z - (lz + h)), 0.0);
    return fma(gx, gx, fma(gy, gy, gz * gz));
}

__device__ __forceinline__ int cell_of(double x, float o, float h, int n) {
    const double t = fmin(fmax((x - (double)o) / (double)h, -1.0), (double)n);
    return min(max((int)floor(t), 0), n - 1);
}

// Visits every face listed in a cell whose box lies within R of q, rings of
// cells outward from q's (clamped) cell.  `visit(face, R)` may shrink R.
// Every cell of ring r >= 2 is at least (r - 1) h from q, which ends the
// search once that exceeds R.
template <class Visit>
__device__ __forceinline__ void grid_visit(const PiMesh& P, const PiGrid& G, D3 q, double& R, Visit&& visit) {
    const int cx = cell_of(q.x, G.ox, G.h, G.nx), cy = cell_of(q.y, G.oy, G.h, G.ny), cz = cell_of(q.z, G.oz, G.h, G.nz);
    const int maxr = max(G.nx, max(G.ny, G.nz));
    for (int r = 0; r <= maxr; ++r) {
        if (r >= 2 && (double)(r - 1) * (double)G.h * 0.999 > R) break;
        for (int dz = -r; dz <= r; ++dz) {
            const int iz = cz + dz;
            if (iz < 0 || iz >= G.nz) continue;
            for (int dy = -r; dy <= r; ++dy) {
                const int iy = cy + dy;
                if (iy < 0 || iy >= G.ny) continue;
                const bool shell = dz == -r || dz == r || dy == -r || dy == r;
                const int stride = (shell || r == 0) ? 1 : 2 * r;   // inside the shell only dx = -r and r
                for (int dx = -r; dx <= r; dx += stride) {
                    const int ix = cx + dx;
                    if (ix < 0 || ix >= G.nx) continue;
                    if (box_dist2(G, q, ix, iy, iz) > R * R) continue;
                    const uint32_t cell = G.cell0 + (uint32_t)((iz * G.ny + iy) * G.nx + ix);
                    const uint32_t j1 = P.cell_start[cell + 1];
                    for (uint32_t j = P.cell_start[cell]; j < j1; ++j) visit(P.cell_face[j], R);
                }
            }
        }
    }
}

// The nearest point of the ray's mesh to q (project_to_mesh).  Faces within
// P.tie of the smallest distance are a tie (they share the nearest point, on
// an edge or a vertex); the tie goes to the face whose normal is most nearly
// parallel to q - c, then to the smallest face id.  Two visits: the smallest
// distance, then the choice among the tie.
struct PiHit {
    int32_t f;
    D3 c;
    double b0, b1, b2;
};

__device__ __forceinline__ double tie_alignment(const PiFace& F, D3 q, D3 c, double d) {
    return d > 0.0 ? fabs(ddot(fnormal(F), dsub(q, c))) / d : 0.0;
}

__device__ __forceinline__ PiHit project_grid(const PiMesh& P, const PiGrid& G, D3 q) {
    double dmin = __builtin_inf();
    double R = dmin;
    grid_visit(P, G, q, R, [&](int32_t fid, double& Rr) {
        D3 c;
        double b0, b1, b2;
        const double d = face_closest(P.face[fid], q, c, b0, b1, b2);
        if (d < dmin) {
            dmin = d;
            Rr = dmin + P.tie + P.slack;
        }
    });
    PiHit hit{-1, d3(0.0, 0.0, 0.0), 0.0, 0.0, 0.0};
    double best_al = -1.0;
    double R2 = dmin + P.tie + P.slack;
    const double dtie = dmin + P.tie;
    grid_visit(P, G, q, R2, [&](int32_t fid, double&) {
        const PiFace F = P.face[fid];
        D3 c;
        double b0, b1, b2;
        const double d = face_closest(F, q, c, b0, b1, b2);
        if (!(d <= dtie)) return;
        const double al = tie_alignment(F, q, c, d);
        if (al > best_al || (al == best_al && fid < hit.f)) {
            best_al = al;
            hit = PiHit{fid, c, b0, b1, b2};
        }
    });
    return hit;
}

// The mesh of a handle that holds user face f (meshes are user face ranges).
__device__ __forceinline__ int mesh_of(const PiMesh& P, int32_t f) {
    int lo = 0, hi = P.n_meshes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.grid[mid].face0 <= f) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One ray's state between steps.
struct PiRay {
    D3 p, v;            // point and vector (v stays in the current face's plane)
    D3 n, nc;           // current face normal; the start normal carried by the rotations
    D3 n0, d0;          // start normal and unit start tangent (extra vectors' frame)
    int32_t f;
    double b0, b1, b2;
    double L, l;        // |v_t| and the traced length
    int32_t steps;
    int32_t mesh;
};

__device__ __forceinline__ bool finite3(D3 a) {
    return __builtin_isfinite(a.x) && __builtin_isfinite(a.y) && __builtin_isfinite(a.z);
}

// initialise: the start point from (f, b), v and the extra vectors projected
// onto the start face's plane.  false: bad input.
template <class T>
__device__ __forceinline__ bool pi_init(const PiMesh& P, const PiArgsT<T>& a, int64_t i, PiRay& r) {
    const int32_t f0 = a.f[i];
    if (f0 < 0 || (int64_t)f0 >= P.n_faces) return false;
    const double b0 = a.b[3 * i], b1 = a.b[3 * i + 1], b2 = a.b[3 * i + 2];
    if (!(b0 >= 0.0 && b1 >= 0.0 && b2 >= 0.0)) return false;
    const double bs = b0 + b1 + b2;
    if (!(bs > 0.0) || !__builtin_isfinite(bs)) return false;
    const D3 v = ld(a.v + 3 * i);
    if (!finite3(v)) return false;
    for (int k = 0; k < a.K; ++k)
        if (!finite3(ld(a.W + 3 * (i * a.K + k)))) return false;
    const PiFace F = P.face[f0];
    r.b0 = b0 / bs;
    r.b1 = b1 / bs;
    r.b2 = b2 / bs;
    const D3 x0 = ld(F.x0), x1 = ld(F.x1), x2 = ld(F.x2);
    r.p = d3(r.b0 * x0.x + r.b1 * x1.x + r.b2 * x2.x, r.b0 * x0.y + r.b1 * x1.y + r.b2 * x2.y,
             r.b0 * x0.z + r.b1 * x1.z + r.b2 * x2.z);
    r.n0 = fnormal(F);
    r.n = r.n0;
    r.nc = r.n0;
    r.v = dsub(v, dscl(r.n0, ddot(v, r.n0)));
    r.L = dlen(r.v);
    r.d0 = dsel(r.L > 0.0, dscl(r.v, 1.0 / r.L), d3(0.0, 0.0, 0.0));
    r.f = f0;
    r.l = 0.0;
    r.steps = 0;
    r.mesh = mesh_of(P, f0);
    return true;
}

// rotate_vector: the rotation about n x n2 that takes unit normal n to n2,
// w c + u x w + u (u . w) / (1 + c) with u = n x n2, c = n . n2 (Rodrigues'
// formula with the angle's cosine and sine taken from c and |u|).  Parallel
// normals leave w unchanged.
__device__ __forceinline__ D3 turn(D3 n, D3 n2, D3 w, bool& turned) {
    const D3 u = dcrs(n, n2);
    turned = ddot(u, u) > 0.0;
    if (!turned) return w;
    const double c = ddot(n, n2);
    const double k = ddot(u, w) / (1.0 + c);
    const D3 uw = dcrs(u, w);
    return d3(fma(w.x, c, fma(u.x, k, uw.x)), fma(w.y, c, fma(u.y, k, uw.y)), fma(w.z, c, fma(u.z, k, uw.z)));
}

// One step after the projection of q = p + s v: the new face and point, v
// turned to the new face's normal, the length moved added.
__device__ __forceinline__ void pi_apply(const PiMesh& P, PiRay& r, const PiHit& h) {
    const D3 n2 = fnormal(P.face[h.f]);
    bool turned;
    r.v = turn(r.n, n2, r.v, turned);
    r.nc = dsel(turned, n2, r.nc);
    r.l += dlen(dsub(h.c, r.p));
    r.p = h.c;
    r.f = h.f;
    r.n = n2;
    r.b0 = h.b0;
    r.b1 = h.b1;
    r.b2 = h.b2;
    r.steps += 1;
}

template <class T>
__device__ __forceinline__ void pi_write_bad(const PiArgsT<T>& a, int64_t i) {
    const T nan = (T)__builtin_nan("");
    a.f_out[i] = a.f[i];
    for (int c = 0; c < 3; ++c) {
        a.b_out[3 * i + c] = a.b[3 * i + c];
        a.p_out[3 * i + c] = nan;
        a.v_out[3 * i + c] = nan;
    }
    for (int k = 0; k < 3 * a.K; ++k) a.W_out[3 * i * a.K + k] = nan;
    if (a.status) a.status[i] = kRayBadInput;
    if (a.n_steps) a.n_steps[i] = 0;
}

// Outputs: end face, barycentrics, point, turned v.  An extra vector keeps its
// components on the frame (tangent, carried normal x tangent), as it does
// under every rotation; |v_t| = 0 leaves the projected vectors.
template <class T>
__device__ __forceinline__ void pi_write(const PiArgsT<T>& a, int64_t i, const PiRay& r, int32_t status) {
    a.f_out[i] = r.f;
    st3(a.b_out + 3 * i, d3(r.b0, r.b1, r.b2));
    st3(a.p_out + 3 * i, r.p);
    st3(a.v_out + 3 * i, r.v);
    if (a.K > 0) {
        const double lv = dlen(r.v);
        const bool frame = r.L > 0.0 && lv > 0.0;
        const D3 d1 = dsel(frame, dscl(r.v, 1.0 / lv), d3(0.0, 0.0, 0.0));
        const D3 q0 = dcrs(r.n0, r.d0), q1 = dcrs(r.nc, d1);
        for (int k = 0; k < a.K; ++k) {
            const D3 w = ld(a.W + 3 * (i * a.K + k));
            const D3 wt = dsub(w, dscl(r.n0, ddot(w, r.n0)));
            st3(a.W_out + 3 * (i * a.K + k), dsel(frame, daxpy(ddot(wt, r.d0), d1, dscl(q1, ddot(wt, q0))), wt));
        }
    }
    if (a.status) a.status[i] = status;
    if (a.n_steps) a.n_steps[i] = r.steps;
}

// Grid search: each lane runs its ray to the end.
template <class T>
__global__ __launch_bounds__(256) void k_pi_exp_grid(PiMesh P, PiArgsT<T> a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    PiRay r;
    if (!pi_init(P, a, i, r)) {
        pi_write_bad(a, i);
        return;
    }
    const PiGrid G = P.grid[r.mesh];
    int32_t status = kRayOk;
    while (r.l < r.L) {
        if (r.steps >= a.max_steps) {
            status = kRayMaxSteps;
            break;
        }
        const PiHit h = project_grid(P, G, daxpy(a.step, r.v, r.p));
        if (h.f < 0) {   // no face within reach (not for a mesh with faces)
            status = kRayBadInput;
            break;
        }
        pi_apply(P, r, h);
    }
    pi_write(a, i, r, status);
}

// The printed form: every step scans every face of the mesh.  The block's
// rays step together; each face tile is staged in LDS once per pass and
// tested by every lane against its own query point.
constexpr int kPiTile = 256;

template <class T>
__global__ __launch_bounds__(256) void k_pi_exp_scan(PiMesh P, PiArgsT<T> a) {
    __shared__ PiFace tile[kPiTile];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    PiRay r;
    bool live = false, bad = false;
    int32_t status = kRayOk;
    int32_t f_lo = 0, f_hi = 0;
    if (i < a.n) {
        bad = !pi_init(P, a, i, r);
        live = !bad;
        if (live) {
            f_lo = P.grid[r.mesh].face0;
            f_hi = P.grid[r.mesh].face1;
        }
    }
    while (__syncthreads_or(live)) {
        bool stepping = false;
        D3 q = d3(0.0, 0.0, 0.0);
        if (live) {
            if (!(r.l < r.L)) {
                live = false;
            } else if (r.steps >= a.max_steps) {
                status = kRayMaxSteps;
                live = false;
            } else {
                stepping = true;
                q = daxpy(a.step, r.v, r.p);
            }
        }
        double dmin = __builtin_inf();
        for (int pass = 0; pass < 2; ++pass) {
            const double dtie = dmin + P.tie;
            double best_al = -1.0;
            PiHit hit{-1, d3(0.0, 0.0, 0.0), 0.0, 0.0, 0.0};
            for (int64_t t0 = 0; t0 < P.n_faces; t0 += kPiTile) {
                __syncthreads();
                if (t0 + threadIdx.x < P.n_faces) tile[threadIdx.x] = P.face[t0 + threadIdx.x];
                __syncthreads();
                if (!stepping) continue;
                const int cnt = (int)min((int64_t)kPiTile, P.n_faces - t0);
                for (int j = 0; j < cnt; ++j) {
                    const int32_t fid = (int32_t)(t0 + j);
                    if (fid < f_lo || fid >= f_hi) continue;
                    D3 c;
                    double b0, b1, b2;
                    const double d = face_closest(tile[j], q, c, b0, b1, b2);
                    if (pass == 0) {
                        dmin = fmin(dmin, d);
                    } else if (d <= dtie) {
                        const double al = tie_alignment(tile[j], q, c, d);
                        if (al > best_al) {   // faces come in id order: equal alignment keeps the smaller id
                            best_al = al;
                            hit = PiHit{fid, c, b0, b1, b2};
                        }
                    }
                }
            }
            if (pass == 1 && stepping) {
                if (hit.f < 0) {
                    status = kRayBadInput;
                    live = false;
                } else {
                    pi_apply(P, r, hit);
                }
            }
        }
    }
    if (i >= a.n) return;
    if (bad) pi_write_bad(a, i);
    else pi_write(a, i, r, status);
}

template <class T>
hipError_t launch_pi(const PiMesh& P, const PiArgsT<T>& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n + 255) / 256)), block(256);
    if (a.scan) hipLaunchKernelGGL(k_pi_exp_scan<T>, grid, block, 0, s, P, a);
    else hipLaunchKernelGGL(k_pi_exp_grid<T>, grid, block, 0, s, P, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- GFD over PI
// Eqs. jv and jp with PI as the Exp, batched as in the appendix "Speed-up GFD
// and EP through batching": launch 1 stacks Exp(p, v), Exp(p, v + eps_v
// e_perp), Exp(p, eps_p e_u) and Exp(p, eps_p e_v) (the last two carry v_t
// as an extra vector); launch 2 stacks Exp(p', eps_v d'), Exp(p_u, v_u) and
// Exp(p_v, v_v).  Rows are stacked by kind (kind k of query i at k n + i) in
// float64, so the differences of end points keep their digits.
struct PiStack {
    int32_t* f;
    double* b;
    double* v;
    double* W;
    int32_t* f_out;
    double* b_out;
    double* p_out;
    double* v_out;
    double* W_out;
    int32_t* status;
};

// The start frame of a backward query: unit e_u = x1 - x0, e_v = x2 - x0 of
// the start face, its normal, v_t, the tangent e_par (e_u when |v_t| = 0) and
// e_perp = n x e_par.
struct PiStart {
    D3 eu, ev, n, vt, epar, eperp;
    double L;
};

__device__ __forceinline__ bool pi_start(const PiMesh& P, const BwdArgs& a, int64_t i, PiStart& S) {
    const int32_t f = a.f[i];
    if (f < 0 || (int64_t)f >= P.n_faces) return false;
    const PiFace F = P.face[f];
    const D3 x0 = ld(F.x0);
    S.eu = dsub(ld(F.x1), x0);
    S.eu = dscl(S.eu, 1.0 / dlen(S.eu));
    S.ev = dsub(ld(F.x2), x0);
    S.ev = dscl(S.ev, 1.0 / dlen(S.ev));
    S.n = fnormal(F);
    const D3 v = ld(a.v + 3 * i);
    S.vt = dsub(v, dscl(S.n, ddot(v, S.n)));
    S.L = dlen(S.vt);
    S.epar = dsel(S.L > 0.0, dscl(S.vt, 1.0 / S.L), S.eu);
    S.eperp = dcrs(S.n, S.epar);
    return true;
}

__global__ __launch_bounds__(256) void k_pi_gfd_stage1(PiMesh P, BwdArgs a, PiStack s1) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int64_t n = a.n;
    PiStart S;
    const bool ok = pi_start(P, a, i, S);
    const D3 zero = d3(0.0, 0.0, 0.0);
    const D3 v = ld(a.v + 3 * i);
    const double ev = a.eps_v, ep = a.eps_p;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t row = k * n + i;
        s1.f[row] = a.f[i];
        for (int c = 0; c < 3; ++c) s1.b[3 * row + c] = a.b[3 * i + c];
        D3 w = v;
        if (ok && k == 1) w = daxpy(ev, S.eperp, S.vt);
        if (ok && k == 2) w = dscl(S.eu, ep);
        if (ok && k == 3) w = dscl(S.ev, ep);
        st3(s1.v + 3 * row, w);
        st3(s1.W + 3 * row, dsel(k >= 2 && ok, S.vt, zero));
    }
}

__global__ __launch_bounds__(256) void k_pi_gfd_stage2(PiMesh P, BwdArgs a, PiStack s1, PiStack s2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int64_t n = a.n;
    PiStart S;
    const bool ok = pi_start(P, a, i, S) && s1.status[i] != kRayBadInput;
    // Exp(p', eps_v d'): d' = v' / |v_t| (e_u when |v_t| = 0)
    const D3 vo = ld(s1.v_out + 3 * i);
    const D3 dend = dsel(S.L > 0.0, dscl(vo, 1.0 / S.L), S.eu);
    const int64_t src[3] = {i, 2 * n + i, 3 * n + i};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t row = k * n + i, sr = src[k];
        s2.f[row] = ok ? s1.f_out[sr] : -1;
        for (int c = 0; c < 3; ++c) s2.b[3 * row + c] = s1.b_out[3 * sr + c];
        st3(s2.v + 3 * row, k == 0 ? dscl(dend, (double)a.eps_v) : ld(s1.W_out + 3 * sr));
    }
}

// Columns (Exp(.) - p') / eps projected by M+_{p'} = (M^T M)^-1 M^T with
// M = [e_u', e_v'] of the end face, then the chain with g (eq. chain).
__device__ __forceinline__ void pinv2(D3 eu, D3 ev, D3 w, double& c0, double& c1) {
    const double a = ddot(eu, eu), bb = ddot(eu, ev), d = ddot(ev, ev);
    const double r1 = ddot(eu, w), r2 = ddot(ev, w), det = fma(a, d, -bb * bb);
    c0 = fma(d, r1, -bb * r2) / det;
    c1 = fma(a, r2, -bb * r1) / det;
}

__global__ __launch_bounds__(256) void k_pi_gfd_assemble(PiMesh P, BwdArgs a, PiStack s1, PiStack s2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int64_t n = a.n;
    PiStart S;
    if (!pi_start(P, a, i, S) || s1.status[i] == kRayBadInput) {
        const float nan = __builtin_nanf("");
        for (int c = 0; c < 3; ++c) a.grad_v[3 * i + c] = a.grad_b[3 * i + c] = nan;
        return;
    }
    const double ev = a.eps_v, ep = a.eps_p;
    const D3 p0 = ld(s1.p_out + 3 * i);
    const D3 col0 = dscl(dsub(ld(s2.p_out + 3 * i), p0), 1.0 / ev);
    const D3 col1 = dscl(dsub(ld(s1.p_out + 3 * (n + i)), p0), 1.0 / ev);
    const D3 col2 = dscl(dsub(ld(s2.p_out + 3 * (n + i)), p0), 1.0 / ep);
    const D3 col3 = dscl(dsub(ld(s2.p_out + 3 * (2 * n + i)), p0), 1.0 / ep);
    const PiFace E = P.face[s1.f_out[i]];
    D3 eu2 = dsub(ld(E.x1), ld(E.x0)), ev2 = dsub(ld(E.x2), ld(E.x0));
    eu2 = dscl(eu2, 1.0 / dlen(eu2));
    ev2 = dscl(ev2, 1.0 / dlen(ev2));
    double j00, j10, j01, j11, p00, p10, p01, p11;   // J^v and J^p: [row][col]
    pinv2(eu2, ev2, col0, j00, j10);
    pinv2(eu2, ev2, col1, j01, j11);
    pinv2(eu2, ev2, col2, p00, p10);
    pinv2(eu2, ev2, col3, p01, p11);
    const D3 g = a.g ? ld(a.g + 3 * i) : d3(0.0, 0.0, 0.0);
    const double h0 = ddot(eu2, g), h1 = ddot(ev2, g);
    // c = J^T M_{p'}^T g
    const double cv0 = fma(j00, h0, j10 * h1), cv1 = fma(j01, h0, j11 * h1);
    const double cp0 = fma(p00, h0, p10 * h1), cp1 = fma(p01, h0, p11 * h1);
    st3(a.grad_v + 3 * i, daxpy(cv0, S.epar, dscl(S.eperp, cv1)));
    // start-point gradient G in the face plane with M_p^T G = (cp0, cp1), M_p = [e_u e_v]
    const double aa = ddot(S.eu, S.eu), bb = ddot(S.eu, S.ev), dd = ddot(S.ev, S.ev);
    const double det = fma(aa, dd, -bb * bb);
    const double y0 = fma(dd, cp0, -bb * cp1) / det, y1 = fma(aa, cp1, -bb * cp0) / det;
    const D3 G = daxpy(y0, S.eu, dscl(S.ev, y1));
    const PiFace F = P.face[a.f[i]];
    a.grad_b[3 * i] = (float)ddot(G, ld(F.x0));
    a.grad_b[3 * i + 1] = (float)ddot(G, ld(F.x1));
    a.grad_b[3 * i + 2] = (float)ddot(G, ld(F.x2));
}

// Stack layout: per row f (4), b (24), v (24), W (24), f_out (4), b_out (24),
// p_out (24), v_out (24), W_out (24), status (4); launch 1 holds 4 n rows,
// launch 2 3 n rows (its W arrays unused).
struct PiStackLayout {
    size_t off[10];
    size_t bytes;
};

PiStackLayout stack_layout(int64_t rows) {
    const size_t sz[10] = {4, 24, 24, 24, 4, 24, 24, 24, 24, 4};
    PiStackLayout L{};
    size_t o = 0;
    for (int k = 0; k < 10; ++k) {
        L.off[k] = o;
        o = (o + (size_t)rows * sz[k] + 255) & ~(size_t)255;
    }
    L.bytes = o;
    return L;
}

PiStack carve(char* base, int64_t rows) {
    const PiStackLayout L = stack_layout(rows);
    PiStack s;
    s.f = reinterpret_cast<int32_t*>(base + L.off[0]);
    s.b = reinterpret_cast<double*>(base + L.off[1]);
    s.v = reinterpret_cast<double*>(base + L.off[2]);
    s.W = reinterpret_cast<double*>(base + L.off[3]);
    s.f_out = reinterpret_cast<int32_t*>(base + L.off[4]);
    s.b_out = reinterpret_cast<double*>(base + L.off[5]);
    s.p_out = reinterpret_cast<double*>(base + L.off[6]);
    s.v_out = reinterpret_cast<double*>(base + L.off[7]);
    s.W_out = reinterpret_cast<double*>(base + L.off[8]);
    s.status = reinterpret_cast<int32_t*>(base + L.off[9]);
    return s;
}

PiArgsT<double> stack_args(const PiArgs& base, const PiStack& s, int64_t rows, int32_t K) {
    PiArgsT<double> a{};
    a.n = rows;
    a.f = s.f; a.b = s.b; a.v = s.v;
    a.K = K; a.W = K ? s.W : nullptr;
    a.f_out = s.f_out; a.b_out = s.b_out; a.p_out = s.p_out; a.v_out = s.v_out; a.W_out = K ? s.W_out : nullptr;
    a.status = s.status;
    a.n_steps = nullptr;
    a.step = base.step;
    a.max_steps = base.max_steps;
    a.scan = base.scan;
    return a;
}

}  // namespace

hipError_t launch_pi_exp(const PiMesh& P, const PiArgs& a, hipStream_t s) { return launch_pi(P, a, s); }

size_t pi_bwd_workspace(int64_t n, int32_t mode) {
    if (mode != 1 || n <= 0) return 0;
    return stack_layout(4 * n).bytes + stack_layout(3 * n).bytes;
}

hipError_t launch_pi_backward(const PiMesh& P, const DevMesh& M, const BwdArgs& a, const PiArgs& pa, void* ws,
                              hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    if (a.mode == 0) return launch_ep_saved(M, a, s);   // end frame from the saved f', v' (end face's own normal)
    const int64_t n = a.n;
    char* base = reinterpret_cast<char*>(ws);
    const PiStack s1 = carve(base, 4 * n);
    const PiStack s2 = carve(base + stack_layout(4 * n).bytes, 3 * n);
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL(k_pi_gfd_stage1, grid, block, 0, s, P, a, s1);
    hipError_t e = launch_pi(P, stack_args(pa, s1, 4 * n, 1), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pi_gfd_stage2, grid, block, 0, s, P, a, s1, s2);
    e = launch_pi(P, stack_args(pa, s2, 3 * n, 0), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pi_gfd_assemble, grid, block, 0, s, P, a, s1, s2);
    return hipGetLastError();
}

}  // namespace sg
