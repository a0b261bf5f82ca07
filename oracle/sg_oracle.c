/*
 * sg_oracle.c -- float64 CPU oracle for straightest geodesics on triangle meshes.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library.  It shares no code
 * with the GPU path.
 *
 * What it follows (Verninas et al., "Parallelised Differentiable Straightest
 * Geodesics for 3D Meshes"):
 *   - Sec. 4 "Straightest geodesics": a point is (face, barycentric); the
 *     straightest rule keeps equal left/right angles, total angle 2 pi on faces
 *     and edges and theta(x) = sum of corner angles at a vertex.
 *   - Appendix, algorithm geodesic_step: barycentric rate of the direction,
 *     exit parameter lambda = min{-b_i / b^v_i > 0}, advance.
 *   - Appendix, algorithm transport_over_edge: rotate the direction about the
 *     shared edge so that the two faces are unfolded into one plane (written
 *     orientation-free, so meshes need not be orientable; Sec. "Main
 *     differences with SotA implementation").
 *   - Appendix, algorithm transport_over_vertex: walk the fan around the vertex
 *     accumulating corner angles from the reversed incoming direction until half
 *     of theta(x) is reached; leave along the fan edge rotated by the residual.
 *   - Sec. 4 "Parallel Transport": a transported vector keeps its angle to the
 *     geodesic tangent; across an edge it is rotated with the unfolding.
 *   - Alg. gpu_parallel: loop until the traced length reaches |v| or MAX_STEPS.
 *   - Eq. proxy_func (extrinsic proxy) and eqs. jv, jp (geodesic finite
 *     differences) for the backward.
 * Readings where the paper is silent or garbled:
 *   - the exact tests b_k = 1 / b_k = 0 of geodesic_step are replaced by
 *     classifying exits by the sign of the barycentric rate, and a vertex is
 *     passed when the exit point lies within `vertex_snap` (edge-parameter
 *     units) of an edge endpoint;
 *   - the last in-face step is clamped to the remaining length;
 *   - v is first projected onto the start face's plane (initialise_trace);
 *   - the outgoing direction at a vertex is the fan edge rotated inside its face
 *     by the residual angle (the vector rotation printed in
 *     transport_over_vertex is garbled);
 *   - extra vectors keep their signed angle to the tangent through a vertex;
 *   - the proxy's rotation is R = M_{p'} M_p^T (frame axes as columns), so that
 *     R^T carries the upstream gradient back from p' to p;
 *   - by default the tracer stops at a boundary edge or boundary vertex (Sec. 4,
 *     original behaviour).  With boundary_mode = 1 it avoids holes (Sec. 4 and
 *     the hole branches of transport_over_edge / transport_over_vertex): a ray
 *     that reaches a boundary edge slides along it to the end its direction
 *     leans toward (the paper leaves the choice open; exactly across the edge,
 *     the end with the smaller vertex id); at a boundary vertex it resumes
 *     straight in the fan face whose corner holds the projection of the
 *     direction recorded at the boundary and whose plane deviates least from
 *     it (the paper's transport_error, read as |d . n_face|), with the
 *     direction projected onto that face; when no face's corner holds it, the
 *     ray slides on along the next boundary edge of the hole (after a straight
 *     arrival, along the boundary edge that leans most toward the direction).
 *     Each slide and each resumption is one step; extra vectors keep their
 *     angle to the direction, which is the recorded one projected onto the
 *     current face.
 */
#define _GNU_SOURCE
#include "sg_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

struct or_mesh {
    int64_t nv, nf;
    double* X;      /* nv*3, exact upcast of the float32 mesh */
    int32_t* F;     /* nf*3 */
    double* N;      /* nf*3 unit face normals (x1-x0) x (x2-x0) */
    int64_t* nbr;   /* nf*3: face across local edge k = (F[k], F[k+1]), or -1 */
    int8_t* nbr_k;  /* nf*3: local index of that edge in the neighbour */
    double* theta;  /* nv: total angle */
    uint8_t* vbnd;  /* nv: vertex lies on a boundary edge */
    double mean_edge;
};

static __thread char g_err[256];
static void set_err(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}
const char* or_last_error(void) { return g_err; }

/* ---------------------------------------------------------------- vectors */
static inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void sub3(const double* a, const double* b, double* r) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }
static inline void cross3(const double* a, const double* b, double* r) {
    double x = a[1] * b[2] - a[2] * b[1], y = a[2] * b[0] - a[0] * b[2], z = a[0] * b[1] - a[1] * b[0];
    r[0] = x; r[1] = y; r[2] = z;
}
static inline double norm3(const double* a) { return sqrt(dot3(a, a)); }
static inline void scale3(double* a, double s) { a[0] *= s; a[1] *= s; a[2] *= s; }
static inline void unit3(double* a) { scale3(a, 1.0 / norm3(a)); }
/* component of a orthogonal to the unit vector u */
static inline void perp3(const double* a, const double* u, double* r) {
    double t = dot3(a, u);
    r[0] = a[0] - t * u[0]; r[1] = a[1] - t * u[1]; r[2] = a[2] - t * u[2];
}
static inline double angle3(const double* a, const double* c) {
    double x[3];
    cross3(a, c, x);
    return atan2(norm3(x), dot3(a, c));
}
static inline const double* VX(const or_mesh* m, int64_t v) { return m->X + 3 * v; }
static inline const double* FX(const or_mesh* m, int64_t f, int k) { return m->X + 3 * (int64_t)m->F[3 * f + k]; }

/* ------------------------------------------------------------ mesh build */
typedef struct { int32_t lo, hi; int64_t he; } edge_rec;
static int edge_cmp(const void* a, const void* b) {
    const edge_rec* x = a; const edge_rec* y = b;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    return x->he < y->he ? -1 : (x->he > y->he);
}

void or_mesh_free(or_mesh* m) {
    if (!m) return;
    free(m->X); free(m->F); free(m->N); free(m->nbr); free(m->nbr_k); free(m->theta); free(m->vbnd);
    free(m);
}

int or_mesh_build(const float* X, int64_t nv, const int32_t* F, int64_t nf, or_mesh** out) {
    *out = NULL;
    if (!X || nv <= 0) { set_err("empty mesh"); return OR_E_ARG; }
    double* X64 = malloc(sizeof(double) * 3 * nv);
    if (!X64) return OR_E_OOM;
    for (int64_t i = 0; i < 3 * nv; i++) X64[i] = (double)X[i];
    int rc = or_mesh_build64(X64, nv, F, nf, out);
    free(X64);
    return rc;
}

int or_mesh_build64(const double* X, int64_t nv, const int32_t* F, int64_t nf, or_mesh** out) {
    *out = NULL;
    if (!X || !F || nv <= 0 || nf <= 0) { set_err("empty mesh"); return OR_E_ARG; }
    or_mesh* m = calloc(1, sizeof *m);
    if (!m) return OR_E_OOM;
    m->nv = nv; m->nf = nf;
    m->X = malloc(sizeof(double) * 3 * nv);
    m->F = malloc(sizeof(int32_t) * 3 * nf);
    m->N = malloc(sizeof(double) * 3 * nf);
    m->nbr = malloc(sizeof(int64_t) * 3 * nf);
    m->nbr_k = malloc(sizeof(int8_t) * 3 * nf);
    m->theta = calloc(nv, sizeof(double));
    m->vbnd = calloc(nv, 1);
    edge_rec* E = malloc(sizeof(edge_rec) * 3 * nf);
    if (!m->X || !m->F || !m->N || !m->nbr || !m->nbr_k || !m->theta || !m->vbnd || !E) {
        free(E); or_mesh_free(m); return OR_E_OOM;
    }
    for (int64_t i = 0; i < 3 * nv; i++) {
        if (!isfinite(X[i])) { set_err("non-finite vertex coordinate"); free(E); or_mesh_free(m); return OR_E_ARG; }
        m->X[i] = X[i];
    }
    for (int64_t f = 0; f < nf; f++) {
        for (int k = 0; k < 3; k++) {
            int32_t v = F[3 * f + k];
            if (v < 0 || v >= nv) { set_err("face %lld: vertex index out of range", (long long)f); free(E); or_mesh_free(m); return OR_E_ARG; }
            m->F[3 * f + k] = v;
        }
        const int32_t* t = m->F + 3 * f;
        if (t[0] == t[1] || t[1] == t[2] || t[0] == t[2]) { set_err("face %lld repeats a vertex", (long long)f); free(E); or_mesh_free(m); return OR_E_DEGENERATE; }
        double e1[3], e2[3], n[3];
        sub3(FX(m, f, 1), FX(m, f, 0), e1);
        sub3(FX(m, f, 2), FX(m, f, 0), e2);
        cross3(e1, e2, n);
        double a = norm3(n);
        if (!(a > 0.0)) { set_err("face %lld has zero area", (long long)f); free(E); or_mesh_free(m); return OR_E_DEGENERATE; }
        scale3(n, 1.0 / a);
        memcpy(m->N + 3 * f, n, sizeof n);
        for (int k = 0; k < 3; k++) {
            int32_t a0 = t[k], a1 = t[(k + 1) % 3];
            E[3 * f + k].lo = a0 < a1 ? a0 : a1;
            E[3 * f + k].hi = a0 < a1 ? a1 : a0;
            E[3 * f + k].he = 3 * f + k;
            /* corner angle at t[k] */
            double p[3], q[3];
            sub3(FX(m, f, (k + 1) % 3), FX(m, f, k), p);
            sub3(FX(m, f, (k + 2) % 3), FX(m, f, k), q);
            m->theta[t[k]] += angle3(p, q);
        }
    }
    qsort(E, 3 * nf, sizeof(edge_rec), edge_cmp);
    double esum = 0.0;
    int64_t ecount = 0;
    for (int64_t s = 0; s < 3 * nf;) {
        int64_t e = s + 1;
        while (e < 3 * nf && E[e].lo == E[s].lo && E[e].hi == E[s].hi) e++;
        int64_t cnt = e - s;
        double d[3];
        sub3(VX(m, E[s].hi), VX(m, E[s].lo), d);
        esum += norm3(d);
        ecount++;
        if (cnt > 2) { set_err("edge (%d,%d) has %lld faces", E[s].lo, E[s].hi, (long long)cnt); free(E); or_mesh_free(m); return OR_E_NONMANIFOLD; }
        if (cnt == 1) {
            m->nbr[E[s].he] = -1; m->nbr_k[E[s].he] = -1;
            m->vbnd[E[s].lo] = 1; m->vbnd[E[s].hi] = 1;
        } else {
            int64_t h0 = E[s].he, h1 = E[s + 1].he;
            if (h0 / 3 == h1 / 3) { set_err("face %lld uses an edge twice", (long long)(h0 / 3)); free(E); or_mesh_free(m); return OR_E_DEGENERATE; }
            m->nbr[h0] = h1 / 3; m->nbr_k[h0] = (int8_t)(h1 % 3);
            m->nbr[h1] = h0 / 3; m->nbr_k[h1] = (int8_t)(h0 % 3);
        }
        s = e;
    }
    free(E);
    m->mean_edge = esum / (double)ecount;

    /* every vertex fan must be a single connected fan (manifold condition) */
    int64_t* start = calloc(nv + 1, sizeof(int64_t));
    int64_t* inc = malloc(sizeof(int64_t) * 3 * nf);
    uint8_t* seen = calloc(nf, 1);
    int64_t* stack = malloc(sizeof(int64_t) * 3 * nf);
    if (!start || !inc || !seen || !stack) { free(start); free(inc); free(seen); free(stack); or_mesh_free(m); return OR_E_OOM; }
    for (int64_t i = 0; i < 3 * nf; i++) start[m->F[i] + 1]++;
    for (int64_t v = 0; v < nv; v++) start[v + 1] += start[v];
    int64_t* fill = malloc(sizeof(int64_t) * (nv + 1));
    memcpy(fill, start, sizeof(int64_t) * (nv + 1));
    for (int64_t i = 0; i < 3 * nf; i++) inc[fill[m->F[i]]++] = i / 3;
    free(fill);
    int rc = OR_OK;
    for (int64_t v = 0; v < nv && rc == OR_OK; v++) {
        int64_t deg = start[v + 1] - start[v];
        if (deg == 0) continue;
        int64_t sp = 0, visited = 0;
        stack[sp++] = inc[start[v]];
        seen[inc[start[v]]] = 1;
        while (sp) {
            int64_t f = stack[--sp];
            visited++;
            for (int k = 0; k < 3; k++) {
                if (m->F[3 * f + k] != v && m->F[3 * f + (k + 1) % 3] != v) continue;
                int64_t g = m->nbr[3 * f + k];
                if (g >= 0 && !seen[g]) { seen[g] = 1; stack[sp++] = g; }
            }
        }
        if (visited != deg) { set_err("vertex %lld: faces do not form one fan", (long long)v); rc = OR_E_NONMANIFOLD; }
        for (int64_t i = start[v]; i < start[v + 1]; i++) seen[inc[i]] = 0;
    }
    free(start); free(inc); free(seen); free(stack);
    if (rc != OR_OK) { or_mesh_free(m); return rc; }
    *out = m;
    return OR_OK;
}

double or_mesh_mean_edge(const or_mesh* m) { return m->mean_edge; }
void or_mesh_theta(const or_mesh* m, double* theta) { memcpy(theta, m->theta, sizeof(double) * m->nv); }

/* ------------------------------------------------------------ tracing */
typedef struct {
    int32_t cap, n;
    int8_t* kind; int32_t* face; int32_t* ev0; int32_t* ev1; double* pt;
} trace_buf;

typedef struct {
    int32_t f, status, n_cross;
    double b[3], p[3], v[3];
    uint64_t hash;
    double min_vdist, traced;
    int8_t sigma;
    int32_t n_bnd;            /* boundary slides (whole or partial) and resumptions (hole avoidance) */
    double bnd_margin;        /* smallest margin of a hole-avoidance decision (see hole_chain) */
    double d0[3], L;          /* start tangent (unit) and length, for the backward */
    double pi_margin;         /* projection integration: smallest margin of a projection choice */
} ray_out;

static inline uint64_t fnv_face(uint64_t h, int32_t f) {
    uint32_t u = (uint32_t)f;
    for (int i = 0; i < 4; i++) { h ^= (u >> (8 * i)) & 0xffu; h *= 1099511628211ull; }
    return h;
}

static inline void bary_pos(const or_mesh* m, int64_t f, const double* b, double* p) {
    const double *x0 = FX(m, f, 0), *x1 = FX(m, f, 1), *x2 = FX(m, f, 2);
    for (int c = 0; c < 3; c++) p[c] = b[0] * x0[c] + b[1] * x1[c] + b[2] * x2[c];
}

/* barycentric representation of a tangent vector d in face f (rates sum to 0) */
static void bary_rate(const or_mesh* m, int64_t f, const double* d, double* bd) {
    double e1[3], e2[3];
    sub3(FX(m, f, 1), FX(m, f, 0), e1);
    sub3(FX(m, f, 2), FX(m, f, 0), e2);
    double g11 = dot3(e1, e1), g12 = dot3(e1, e2), g22 = dot3(e2, e2);
    double r1 = dot3(d, e1), r2 = dot3(d, e2);
    double det = g11 * g22 - g12 * g12;
    bd[1] = (g22 * r1 - g12 * r2) / det;
    bd[2] = (g11 * r2 - g12 * r1) / det;
    bd[0] = -bd[1] - bd[2];
}

static void clamp_renorm(double* b) {
    for (int k = 0; k < 3; k++) if (b[k] < 0.0) b[k] = 0.0;
    double s = b[0] + b[1] + b[2];
    b[0] /= s; b[1] /= s; b[2] /= s;
}

static double seg_point_dist(const double* a, const double* c, const double* x) {
    double ac[3], ax[3];
    sub3(c, a, ac);
    sub3(x, a, ax);
    double l2 = dot3(ac, ac);
    double t = l2 > 0 ? dot3(ax, ac) / l2 : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double q[3] = {a[0] + t * ac[0] - x[0], a[1] + t * ac[1] - x[1], a[2] + t * ac[2] - x[2]};
    return norm3(q);
}

/* Closest approach of segment a-c to the vertices of face f, except its
 * local vertex `skipv` (-1: none), the boundary vertex a resumed segment
 * starts from. */
static void seg_update(const or_mesh* m, int64_t f, const double* a, const double* c, double* best, int skipv) {
    for (int k = 0; k < 3; k++) {
        if (k == skipv) continue;
        double d = seg_point_dist(a, c, FX(m, f, k));
        if (d < *best) *best = d;
    }
}

static int local_index(const or_mesh* m, int64_t f, int32_t v) {
    for (int k = 0; k < 3; k++) if (m->F[3 * f + k] == v) return k;
    return -1;
}

static void trace_push(trace_buf* tb, int8_t kind, int32_t face, int32_t v0, int32_t v1, const double* p) {
    if (!tb || tb->n >= tb->cap) return;
    int i = tb->n++;
    tb->kind[i] = kind; tb->face[i] = face; tb->ev0[i] = v0; tb->ev1[i] = v1;
    memcpy(tb->pt + 3 * i, p, 3 * sizeof(double));
}

/* ------------------------------------------------------------ hole avoidance */
/* The fan of boundary vertex x0 through face f, as the chain of faces between
 * its two boundary edges: fan[0..n), rel[i] = orientation of fan[i] relative
 * to f (+1 / -1), y0 / y1 = the far vertex of the boundary edge at x0 of
 * fan[0] / fan[n-1].  Returns n (0 if x0 is not a boundary vertex). */
static int other_edge_at(const or_mesh* m, int64_t g, int32_t x0, int not_e) {
    int lx = local_index(m, g, x0);
    int ea = lx, eb = (lx + 2) % 3;   /* the two edges of g at x0 */
    return ea == not_e ? eb : ea;
}

static int fan_chain(const or_mesh* m, int64_t f, int32_t x0, int64_t* fan, int8_t* rel, int32_t* y0, int32_t* y1,
                     int cap) {
    /* walk one way from f to a boundary edge */
    int64_t cur = f;
    int e = local_index(m, f, x0);   /* edge x0 -> next */
    int sig = 1, guard = 0;
    for (;;) {
        int64_t g = m->nbr[3 * cur + e];
        if (g < 0) break;
        int ge = m->nbr_k[3 * cur + e];
        if (m->F[3 * g + ge] == m->F[3 * cur + e]) sig = -sig;
        cur = g;
        e = other_edge_at(m, g, x0, ge);
        if (++guard > cap || g == f) return 0;   /* closed fan: not a boundary vertex */
    }
    /* cur's edge e is a boundary edge at x0; enumerate back to the other end */
    int n = 0;
    int32_t a = m->F[3 * cur + e], bq = m->F[3 * cur + (e + 1) % 3];
    *y0 = a == x0 ? bq : a;
    int ein = e;
    for (;;) {
        if (n >= cap) return 0;
        fan[n] = cur;
        rel[n] = (int8_t)sig;
        n++;
        int eo = other_edge_at(m, cur, x0, ein);
        int64_t g = m->nbr[3 * cur + eo];
        if (g < 0) {
            int32_t c0 = m->F[3 * cur + eo], c1 = m->F[3 * cur + (eo + 1) % 3];
            *y1 = c0 == x0 ? c1 : c0;
            break;
        }
        int ge = m->nbr_k[3 * cur + eo];
        if (m->F[3 * g + ge] == m->F[3 * cur + eo]) sig = -sig;
        cur = g;
        ein = ge;
    }
    return n;
}

/* Is the projection w of d onto face g's plane inside g's corner at x0?
 * Returns the transport error |d . n_g| (the out-of-plane part), or -1.
 * *qual receives how far w is from the corner's nearer edge, as the sine of
 * the angle between them (the margin of the inside test). */
static double corner_fit(const or_mesh* m, int64_t g, int32_t x0, const double* d, double* w, double* qual) {
    const double* n = m->N + 3 * g;
    perp3(d, n, w);
    *qual = INFINITY;
    double wl = norm3(w);
    if (!(wl > 1e-300)) return -1.0;
    int lx = local_index(m, g, x0);
    double ea[3], eb[3], c[3];
    sub3(FX(m, g, (lx + 1) % 3), VX(m, x0), ea);
    sub3(FX(m, g, (lx + 2) % 3), VX(m, x0), eb);
    cross3(ea, eb, c);
    double sab = dot3(c, n);
    cross3(ea, w, c);
    double sa = dot3(c, n);
    cross3(w, eb, c);
    double sb = dot3(c, n);
    double qa = fabs(sa) / (norm3(ea) * wl), qb = fabs(sb) / (norm3(eb) * wl);
    *qual = qa < qb ? qa : qb;
    if (sa * sab < 0.0 || sb * sab < 0.0) return -1.0;
    return fabs(dot3(d, n));
}

#define FANCAP 4096

/* The hole-avoiding chain from a boundary event (see the header), run until
 * the ray resumes straight (returns 1: *f, b = the vertex, d = unit direction
 * in *f's plane, *sigma and *atv set), or its length is used up or the step
 * cap is reached (returns 0: *status, *f, b and the reported direction d set).
 * Entry: the ray is in face *f at point b with unit direction d (recorded as
 * the straightest direction); kind 0: b lies on the boundary edge (la, lb) of
 * *f; kind 1: the ray stands at boundary vertex x0 of *f.  The step that
 * reached the boundary is completed by the chain's first slide or
 * resumption; every further one is a step of its own. */
static int hole_chain(const or_mesh* m, int32_t max_steps, int64_t* f, double* b, double* d, int* sigma,
                      double* rem, double* traced, int32_t* steps, int* status, int* atv, ray_out* out,
                      trace_buf* tb, int kind, int la, int lb, int32_t x0) {
    static __thread int64_t fan[FANCAP];
    static __thread int8_t rel[FANCAP];
    double drec[3];
    memcpy(drec, d, sizeof drec);
    int64_t fc = *f;
    int32_t from = -1;   /* the vertex the last slide started from */
    int lt = -1, ls = -1, first = 1;
    if (kind == 0) {   /* slide along the exit edge toward the end the direction leans to */
        int32_t va = m->F[3 * fc + la], vb = m->F[3 * fc + lb];
        double e[3];
        sub3(VX(m, vb), VX(m, va), e);
        double dd = dot3(drec, e);
        int to_b = dd > 0.0 || (dd == 0.0 && vb < va);
        double q = fabs(dd) / norm3(e);   /* the slide's end: margin |cos(d, edge)| */
        if (q < out->bnd_margin) out->bnd_margin = q;
        lt = to_b ? lb : la;
        ls = to_b ? la : lb;
    }
    for (;;) {
        if (lt >= 0) {   /* sliding in fc from point b toward local vertex lt */
            out->n_bnd++;
            double p[3], q[3], e[3];
            bary_pos(m, fc, b, p);
            sub3(FX(m, fc, lt), p, q);
            sub3(FX(m, fc, lt), FX(m, fc, ls), e);
            double sl = norm3(q), elen = norm3(e);
            if (*rem <= sl) {
                double t = *rem / elen;
                b[lt] += t;
                b[ls] -= t;
                clamp_renorm(b);
                *traced += *rem;
                *rem = 0.0;
                perp3(drec, m->N + 3 * fc, d); unit3(d);
                *f = fc;
                *status = OR_RAY_OK;
                return 0;
            }
            if (!first) {
                if (*steps >= max_steps) {
                    perp3(drec, m->N + 3 * fc, d); unit3(d);
                    *f = fc;
                    *status = OR_RAY_MAXSTEPS;
                    return 0;
                }
                (*steps)++;
            }
            first = 0;
            *traced += sl;
            *rem -= sl;
            x0 = m->F[3 * fc + lt];
            from = m->F[3 * fc + ls];
            b[0] = b[1] = b[2] = 0.0;
            b[lt] = 1.0;
            out->n_cross++;
            out->hash = fnv_face(out->hash, (int32_t)fc);
            trace_push(tb, 2, (int32_t)fc, from, x0, VX(m, x0));
            lt = -1;
        }
        /* at boundary vertex x0 of face fc */
        int32_t y0 = -1, y1 = -1;
        int nfan = fan_chain(m, fc, x0, fan, rel, &y0, &y1, FANCAP);
        if (nfan == 0) {   /* not on a boundary (cannot happen on a checked mesh) */
            perp3(drec, m->N + 3 * fc, d); unit3(d);
            *f = fc;
            *status = OR_RAY_BOUNDARY;
            return 0;
        }
        double best = INFINITY, second = INFINITY, wb[3] = {0, 0, 0};
        int ib = -1;
        for (int i = 0; i < nfan; i++) {
            double w[3], qual;
            double err = corner_fit(m, fan[i], x0, drec, w, &qual);
            /* the face choice: margins of every inside test and best against runner-up */
            if (qual < out->bnd_margin) out->bnd_margin = qual;
            if (err >= 0.0 && err < best) { second = best; best = err; ib = i; memcpy(wb, w, sizeof w); }
            else if (err >= 0.0 && err < second) second = err;
        }
        if (second - best < out->bnd_margin) out->bnd_margin = second - best;
        if (!first && *steps >= max_steps) {
            perp3(drec, m->N + 3 * fc, d); unit3(d);
            *f = fc;
            *status = OR_RAY_MAXSTEPS;
            return 0;
        }
        if (ib >= 0) {   /* resume straight in fan[ib] */
            if (!first) (*steps)++;
            *f = fan[ib];
            *sigma *= rel[ib];
            memcpy(d, wb, sizeof wb);
            unit3(d);
            *atv = local_index(m, *f, x0);
            b[0] = b[1] = b[2] = 0.0;
            b[*atv] = 1.0;
            out->n_cross++;
            out->n_bnd++;
            out->hash = fnv_face(out->hash, (int32_t)*f);
            trace_push(tb, 3, (int32_t)*f, x0, -1, VX(m, x0));
            return 1;
        }
        /* no face holds the direction: slide on along a boundary edge of the hole */
        int end;
        if (from >= 0) end = (y0 == from) ? 1 : 0;
        else {
            double u0[3], u1[3];
            sub3(VX(m, y0), VX(m, x0), u0); unit3(u0);
            sub3(VX(m, y1), VX(m, x0), u1); unit3(u1);
            double c0 = dot3(drec, u0), c1 = dot3(drec, u1);
            end = (c1 > c0 || (c1 == c0 && y1 < y0)) ? 1 : 0;
            if (fabs(c1 - c0) < out->bnd_margin) out->bnd_margin = fabs(c1 - c0);
        }
        *sigma *= end ? rel[nfan - 1] : rel[0];
        fc = end ? fan[nfan - 1] : fan[0];
        int32_t y = end ? y1 : y0;
        ls = local_index(m, fc, x0);
        lt = local_index(m, fc, y);
        b[0] = b[1] = b[2] = 0.0;
        b[ls] = 1.0;
    }
}

/* Signed angles of the extra vectors to direction d about the oriented normal
 * sigma * n (a transported vector keeps its angle to the tangent). */
static void vec_angles(const double* n, int sigma, const double* d, int K, const double* W, double* psi) {
    double ns[3] = {sigma * n[0], sigma * n[1], sigma * n[2]};
    for (int k = 0; k < K; k++) {
        double c[3];
        cross3(d, W + 3 * k, c);
        psi[k] = atan2(dot3(c, ns), dot3(d, W + 3 * k));
    }
}

static void vec_rebuild(const double* n, int sigma, const double* d, int K, const double* psi, const double* wn,
                        double* W) {
    double ns[3] = {sigma * n[0], sigma * n[1], sigma * n[2]}, dp[3];
    cross3(ns, d, dp);
    for (int k = 0; k < K; k++)
        for (int c = 0; c < 3; c++) W[3 * k + c] = wn[k] * (cos(psi[k]) * d[c] + sin(psi[k]) * dp[c]);
}

/* One exponential map.  K extra vectors W (K*3) are transported into Wout. */
static void exp_one(const or_mesh* m, int32_t f0, const double* b0, const double* v0, int K,
                    const double* W0, const or_opts* o, ray_out* out, double* Wout, trace_buf* tb) {
    memset(out, 0, sizeof *out);
    out->f = f0;
    out->sigma = 1;
    out->min_vdist = INFINITY;
    out->bnd_margin = INFINITY;
    out->hash = 14695981039346656037ull;
    double wn[64];
    double snap = o ? o->vertex_snap : 1e-10;
    int32_t max_steps = o ? o->max_steps : (1 << 20);
    int hole = o ? o->boundary_mode == 1 : 0;

    int bad = (f0 < 0 || f0 >= m->nf);
    double b[3] = {0, 0, 0};
    if (!bad) {
        double s = 0.0;
        for (int k = 0; k < 3; k++) {
            b[k] = b0[k];
            if (!isfinite(b[k]) || b[k] < 0.0) bad = 1;
            s += b[k];
        }
        if (!(s > 0.0) || !isfinite(s)) bad = 1;
        else for (int k = 0; k < 3; k++) b[k] /= s;
        for (int c = 0; c < 3; c++) if (!isfinite(v0[c])) bad = 1;
        for (int i = 0; i < 3 * K; i++) if (!isfinite(W0[i])) bad = 1;
    }
    if (bad || K > 64) {
        out->status = OR_RAY_BADINPUT;
        for (int k = 0; k < 3; k++) { out->b[k] = b0[k]; out->p[k] = NAN; out->v[k] = NAN; }
        for (int i = 0; i < 3 * K; i++) Wout[i] = NAN;
        return;
    }
    int64_t f = f0;
    const double* n = m->N + 3 * f;
    double d[3];
    perp3(v0, n, d);
    double L = norm3(d);
    for (int k = 0; k < K; k++) {
        perp3(W0 + 3 * k, n, Wout + 3 * k);
        wn[k] = norm3(Wout + 3 * k);
    }
    out->hash = fnv_face(out->hash, (int32_t)f);
    if (!(L > 0.0)) {
        memcpy(out->b, b, sizeof b);
        bary_pos(m, f, b, out->p);
        out->L = 0.0;
        return;
    }
    scale3(d, 1.0 / L);
    memcpy(out->d0, d, sizeof d);
    out->L = L;

    int atv = -1, skip = -1, sigma = 1;
    int resume_v = -1;   /* local vertex a hole-avoidance resumption starts from (not a vertex passage) */
    int nz = (b[0] == 0.0) + (b[1] == 0.0) + (b[2] == 0.0);
    double bd[3];
    if (nz == 2) {
        atv = b[0] != 0.0 ? 0 : (b[1] != 0.0 ? 1 : 2);
        bary_rate(m, f, d, bd);
        for (int k = 0; k < 3; k++)
            if (k != atv && bd[k] < 0.0) {   /* direction leaves the given face's corner */
                out->status = OR_RAY_BADINPUT;
                memcpy(out->b, b, sizeof b);
                bary_pos(m, f, b, out->p);
                return;
            }
    }
    double rem = L, traced = 0.0;
    int32_t steps = 0;
    double p_prev[3], p_new[3];
    int status = OR_RAY_OK;
    for (;;) {
        bary_rate(m, f, d, bd);
        int ks = -1;
        double ts = INFINITY;
        if (atv >= 0) {
            if (bd[atv] < 0.0) { ks = atv; ts = b[atv] / -bd[atv]; }
        } else {
            for (int k = 0; k < 3; k++) {
                if (k == skip || !(bd[k] < 0.0)) continue;
                double t = b[k] / -bd[k];
                if (t < ts) { ts = t; ks = k; }
            }
        }
        bary_pos(m, f, b, p_prev);
        if (ks < 0) { status = OR_RAY_BADINPUT; break; }
        if (rem <= ts) {
            for (int k = 0; k < 3; k++) b[k] += rem * bd[k];
            clamp_renorm(b);
            traced += rem;
            bary_pos(m, f, b, p_new);
            seg_update(m, f, p_prev, p_new, &out->min_vdist, resume_v);
            rem = 0.0;
            break;
        }
        if (steps >= max_steps) { status = OR_RAY_MAXSTEPS; break; }
        for (int k = 0; k < 3; k++) b[k] += ts * bd[k];
        b[ks] = 0.0;
        clamp_renorm(b);
        rem -= ts;
        traced += ts;
        steps++;
        bary_pos(m, f, b, p_new);
        seg_update(m, f, p_prev, p_new, &out->min_vdist, resume_v);
        resume_v = -1;
        int e = (ks + 1) % 3, i = e, j = (e + 1) % 3;

        int vloc = -1;
        if (b[j] <= snap) vloc = i;
        else if (b[i] <= snap) vloc = j;

        if (vloc < 0) {
            /* ---- transport_over_edge: unfold f' into the plane of f about the shared edge */
            int64_t g = m->nbr[3 * f + e];
            if (g < 0 && hole) {
                double psi[64];
                vec_angles(m->N + 3 * f, sigma, d, K, Wout, psi);
                int resumed = hole_chain(m, max_steps, &f, b, d, &sigma, &rem, &traced, &steps, &status, &atv, out,
                                         tb, 0, i, j, -1);
                vec_rebuild(m->N + 3 * f, sigma, d, K, psi, wn, Wout);
                if (!resumed) break;
                resume_v = atv;
                skip = -1;
                continue;
            }
            if (g < 0) { status = OR_RAY_BOUNDARY; break; }
            int ge = m->nbr_k[3 * f + e];
            const double *xi = FX(m, f, i), *xj = FX(m, f, j), *xk = FX(m, f, ks), *z = FX(m, g, (ge + 2) % 3);
            double u[3], mf[3], mg[3], cf[3], cg[3], t1[3], t2[3];
            sub3(xj, xi, u); unit3(u);
            sub3(xk, xi, t1); perp3(t1, u, mf); unit3(mf);
            sub3(z, xi, t2); perp3(t2, u, mg); unit3(mg);
            cross3(u, mf, cf);
            cross3(u, mg, cg);
            /* rotation about u taking f's inward edge normal to g's outward one */
#define QROT(w, r) do { double a_ = dot3(w, u), b_ = dot3(w, mf), c_ = dot3(w, cf); \
            for (int q_ = 0; q_ < 3; q_++) (r)[q_] = a_ * u[q_] - b_ * mg[q_] - c_ * cg[q_]; } while (0)
            const double* ng = m->N + 3 * g;
            double r[3];
            QROT(d, r);
            perp3(r, ng, d); unit3(d);
            for (int k = 0; k < K; k++) {
                double* w = Wout + 3 * k;
                QROT(w, r);
                perp3(r, ng, w);
                double nw = norm3(w);
                if (nw > 0) scale3(w, wn[k] / nw);
            }
            QROT(m->N + 3 * f, r);
            if (dot3(r, ng) < 0) sigma = -sigma;
#undef QROT
            double bg[3];
            int32_t vi = m->F[3 * f + i];
            if (m->F[3 * g + ge] == vi) { bg[ge] = b[i]; bg[(ge + 1) % 3] = b[j]; }
            else { bg[ge] = b[j]; bg[(ge + 1) % 3] = b[i]; }
            bg[(ge + 2) % 3] = 0.0;
            trace_push(tb, 0, (int32_t)g, m->F[3 * f + i], m->F[3 * f + j], p_new);
            f = g;
            memcpy(b, bg, sizeof b);
            skip = (ge + 2) % 3;
            atv = -1;
        } else {
            /* ---- transport_over_vertex: fan walk to half the total angle */
            int32_t x0id = m->F[3 * f + vloc];
            const double* x0 = VX(m, x0id);
            out->min_vdist = 0.0;
            if (m->vbnd[x0id] && hole) {
                b[0] = b[1] = b[2] = 0.0; b[vloc] = 1.0;
                double psi[64];
                vec_angles(m->N + 3 * f, sigma, d, K, Wout, psi);
                int resumed = hole_chain(m, max_steps, &f, b, d, &sigma, &rem, &traced, &steps, &status, &atv, out,
                                         tb, 1, -1, -1, x0id);
                vec_rebuild(m->N + 3 * f, sigma, d, K, psi, wn, Wout);
                if (!resumed) break;
                resume_v = atv;
                skip = -1;
                continue;
            }
            if (m->vbnd[x0id]) {
                status = OR_RAY_BOUNDARY;
                b[0] = b[1] = b[2] = 0.0; b[vloc] = 1.0;
                break;
            }
            double nsig[3] = {sigma * m->N[3 * f], sigma * m->N[3 * f + 1], sigma * m->N[3 * f + 2]};
            double psi[64];
            for (int k = 0; k < K; k++) {
                double c[3];
                cross3(d, Wout + 3 * k, c);
                psi[k] = atan2(dot3(c, nsig), dot3(d, Wout + 3 * k));
            }
            double rdir[3] = {-d[0], -d[1], -d[2]};
            int32_t ynext = m->F[3 * f + (sigma > 0 ? (vloc + 2) % 3 : (vloc + 1) % 3)];
            double p1[3], p2[3], ydir[3];
            sub3(FX(m, f, (vloc + 1) % 3), x0, p1);
            sub3(FX(m, f, (vloc + 2) % 3), x0, p2);
            double corner = angle3(p1, p2);
            sub3(VX(m, ynext), x0, ydir);
            double acc = angle3(rdir, ydir);
            if (acc > corner) acc = corner;
            double half = 0.5 * m->theta[x0id];
            double outd[3];
            int64_t cur = f;
            int sig = sigma;
            if (acc >= half) {
                double w[3];
                perp3(ydir, rdir, w); unit3(w);
                for (int c = 0; c < 3; c++) outd[c] = cos(half) * rdir[c] + sin(half) * w[c];
            } else {
                int guard = 0;
                for (;;) {
                    int e2 = -1;
                    for (int k = 0; k < 3; k++) {
                        int32_t a0 = m->F[3 * cur + k], a1 = m->F[3 * cur + (k + 1) % 3];
                        if ((a0 == x0id && a1 == ynext) || (a1 == x0id && a0 == ynext)) { e2 = k; break; }
                    }
                    int64_t g = m->nbr[3 * cur + e2];
                    if (g < 0 || ++guard > 4096) { status = OR_RAY_BOUNDARY; break; }
                    int ge = m->nbr_k[3 * cur + e2];
                    if (m->F[3 * g + ge] == m->F[3 * cur + e2]) sig = -sig;   /* orientation flips */
                    int lx = local_index(m, g, x0id);
                    int lz = 3 - lx - local_index(m, g, ynext);
                    int32_t zid = m->F[3 * g + lz];
                    double u[3], zz[3];
                    sub3(VX(m, ynext), x0, u);
                    sub3(VX(m, zid), x0, zz);
                    double cg = angle3(u, zz);
                    if (acc + cg >= half) {
                        double beta = half - acc, w[3];
                        unit3(u);
                        perp3(zz, u, w); unit3(w);
                        for (int c = 0; c < 3; c++) outd[c] = cos(beta) * u[c] + sin(beta) * w[c];
                        cur = g;
                        break;
                    }
                    acc += cg;
                    ynext = zid;
                    cur = g;
                }
                if (status != OR_RAY_OK) {
                    b[0] = b[1] = b[2] = 0.0; b[vloc] = 1.0;
                    break;
                }
            }
            f = cur;
            sigma = sig;
            memcpy(d, outd, sizeof d);
            const double* nn = m->N + 3 * f;
            double nsig2[3] = {sigma * nn[0], sigma * nn[1], sigma * nn[2]}, dperp[3];
            cross3(nsig2, d, dperp);
            for (int k = 0; k < K; k++)
                for (int c = 0; c < 3; c++) Wout[3 * k + c] = wn[k] * (cos(psi[k]) * d[c] + sin(psi[k]) * dperp[c]);
            atv = local_index(m, f, x0id);
            b[0] = b[1] = b[2] = 0.0;
            b[atv] = 1.0;
            skip = -1;
            trace_push(tb, 1, (int32_t)f, x0id, -1, x0);
        }
        out->n_cross++;
        out->hash = fnv_face(out->hash, (int32_t)f);
    }
    out->f = (int32_t)f;
    out->status = status;
    memcpy(out->b, b, sizeof b);
    bary_pos(m, f, b, out->p);
    for (int c = 0; c < 3; c++) out->v[c] = L * d[c];
    out->traced = traced;
    out->sigma = (int8_t)sigma;
}

/* ------------------------------------------------------------ projection integration */
/* The projection-integration (PI) exponential map the paper compares against
 * (appendix "Projection Integration Exp Map", Alg. projection-exp): step the
 * point along the current vector in the ambient space, project it back onto
 * the mesh by scanning every face, rotate the vector from the old face's
 * normal to the new one's, and add the length actually moved, until that
 * length reaches |v|.
 * Readings where the paper is silent or garbled:
 *   - the step is p + s v with s a fraction of v (the printed formula), and
 *     the loop runs while the accumulated length is below |v_t| (no clamp of
 *     the last step, as printed); the algorithm's returned value is garbled
 *     and read as the final point, face and rotated vector;
 *   - v (and each extra vector) is first projected onto the start face's
 *     plane, as for the straightest map;
 *   - project_to_mesh returns the nearest point of the mesh: the minimiser of
 *     the distance to each closed triangle, minimised over all faces.  Where
 *     the nearest point lies inside a face this is the paper's rule (the
 *     containing face at the smallest distance); where it lies on an edge or a
 *     vertex, several faces attain it (ties within TIE_ABS of the smallest
 *     distance, in units of the mesh's largest coordinate), and the face whose
 *     normal is most nearly parallel to q - c is taken, then the smallest face
 *     id;
 *   - rotate_vector by alpha = acos(n . n') about n x n' is the rotation that
 *     takes n to n' (Rodrigues' formula); parallel normals leave the vectors
 *     unchanged, and so do opposite normals (the axis is undefined there);
 *   - a ray still short of |v_t| after max_steps steps ends with status
 *     MAXSTEPS.
 * The per-ray margin reports how close the ray came to a different result:
 * for each projection the gap between the smallest distance and the smallest
 * distance outside the tie, and the alignment gap inside a tie; for the loop
 * test, how far the traced length was from |v_t| before and after the last
 * step (on a plane with 1/s an integer the step count is decided by rounding). */
#define PI_TIE_ABS 1e-12

/* Closest point c of the closed triangle f to q, its barycentrics bc (face
 * vertex order) and the distance |q - c|.  Inside the triangle's prism c is
 * the projection onto the plane; outside, the nearest point of a convex set
 * lies on its boundary, so it is the nearest of the three edges' closest
 * points. */
static double tri_closest(const or_mesh* m, int64_t f, const double* q, double* c, double* bc) {
    const double *x0 = FX(m, f, 0), *x1 = FX(m, f, 1), *x2 = FX(m, f, 2);
    double e1[3], e2[3], w[3];
    sub3(x1, x0, e1);
    sub3(x2, x0, e2);
    sub3(q, x0, w);
    double g11 = dot3(e1, e1), g12 = dot3(e1, e2), g22 = dot3(e2, e2);
    double r1 = dot3(w, e1), r2 = dot3(w, e2), det = g11 * g22 - g12 * g12;
    double u = (g22 * r1 - g12 * r2) / det, v = (g11 * r2 - g12 * r1) / det;
    if (u >= 0.0 && v >= 0.0 && u + v <= 1.0) {
        bc[0] = 1.0 - u - v; bc[1] = u; bc[2] = v;
        for (int k = 0; k < 3; k++) c[k] = x0[k] + u * e1[k] + v * e2[k];
    } else {
        double best = INFINITY;
        for (int k = 0; k < 3; k++) {
            const double* a = FX(m, f, k);
            const double* b = FX(m, f, (k + 1) % 3);
            double ab[3], aq[3], pt[3];
            sub3(b, a, ab);
            sub3(q, a, aq);
            double t = dot3(aq, ab) / dot3(ab, ab);
            if (t < 0.0) t = 0.0;
            if (t > 1.0) t = 1.0;
            for (int j = 0; j < 3; j++) pt[j] = a[j] + t * ab[j];
            double dq[3];
            sub3(q, pt, dq);
            double d = norm3(dq);
            if (d < best) {
                best = d;
                memcpy(c, pt, sizeof pt);
                bc[k] = 1.0 - t; bc[(k + 1) % 3] = t; bc[(k + 2) % 3] = 0.0;
            }
        }
    }
    double dq[3];
    sub3(q, c, dq);
    return norm3(dq);
}

static double mesh_scale(const or_mesh* m) {
    double s = 1.0;
    for (int64_t i = 0; i < 3 * m->nv; i++) if (fabs(m->X[i]) > s) s = fabs(m->X[i]);
    return s;
}

/* project_to_mesh: the face holding the nearest point of the mesh to q (a
 * scan over every face), that point and its barycentrics.  *margin is lowered
 * to this choice's margin. */
static int64_t project_to_mesh(const or_mesh* m, double scale, const double* q, double* c, double* bc, double* margin) {
    double dmin = INFINITY;
    for (int64_t f = 0; f < m->nf; f++) {
        double cf[3], bf[3];
        double d = tri_closest(m, f, q, cf, bf);
        if (d < dmin) dmin = d;
    }
    const double tie = PI_TIE_ABS * scale;
    int64_t best = -1;
    double best_al = -1.0, second_al = -1.0, outside = INFINITY;
    for (int64_t f = 0; f < m->nf; f++) {
        double cf[3], bf[3];
        double d = tri_closest(m, f, q, cf, bf);
        if (d > dmin + tie) {
            if (d < outside) outside = d;
            continue;
        }
        double dq[3];
        sub3(q, cf, dq);
        double al = d > 0.0 ? fabs(dot3(m->N + 3 * f, dq)) / d : 0.0;
        if (al > best_al) {   /* ties in alignment keep the smaller face id */
            second_al = best_al;
            best_al = al; best = f;
            memcpy(c, cf, sizeof cf);
            memcpy(bc, bf, sizeof bf);
        } else if (al > second_al) {
            second_al = al;
        }
    }
    double mg = outside - dmin;
    if (second_al >= 0.0 && best_al - second_al < mg) mg = best_al - second_al;
    if (mg < *margin) *margin = mg;
    return best;
}

/* rotate_vector: the rotation taking unit normal n to unit normal n2, by the
 * angle alpha = acos(n . n2) about the axis n x n2 (Rodrigues' formula). */
static void rotate_normal_to_normal(const double* n, const double* n2, double* w) {
    double k[3];
    cross3(n, n2, k);
    double sk = norm3(k);
    if (!(sk > 0.0)) return;
    scale3(k, 1.0 / sk);
    double cs = dot3(n, n2);
    if (cs > 1.0) cs = 1.0;
    if (cs < -1.0) cs = -1.0;
    double alpha = acos(cs);
    double kw[3];
    cross3(k, w, kw);
    double kd = dot3(k, w), ca = cos(alpha), sa = sin(alpha);
    for (int j = 0; j < 3; j++) w[j] = w[j] * ca + kw[j] * sa + k[j] * kd * (1.0 - ca);
}

static void pi_one(const or_mesh* m, int32_t f0, const double* b0, const double* v0, int K, const double* W0,
                   const or_pi_opts* o, double scale, ray_out* out, double* Wout) {
    memset(out, 0, sizeof *out);
    out->f = f0;
    out->sigma = 1;
    out->min_vdist = INFINITY;
    out->bnd_margin = INFINITY;
    out->pi_margin = INFINITY;
    int bad = (f0 < 0 || f0 >= m->nf);
    double b[3] = {0, 0, 0};
    if (!bad) {
        double s = 0.0;
        for (int k = 0; k < 3; k++) {
            b[k] = b0[k];
            if (!isfinite(b[k]) || b[k] < 0.0) bad = 1;
            s += b[k];
        }
        if (!(s > 0.0) || !isfinite(s)) bad = 1;
        else for (int k = 0; k < 3; k++) b[k] /= s;
        for (int c = 0; c < 3; c++) if (!isfinite(v0[c])) bad = 1;
        for (int i = 0; i < 3 * K; i++) if (!isfinite(W0[i])) bad = 1;
    }
    if (bad || K > 64) {
        out->status = OR_RAY_BADINPUT;
        for (int k = 0; k < 3; k++) { out->b[k] = b0[k]; out->p[k] = NAN; out->v[k] = NAN; }
        for (int i = 0; i < 3 * K; i++) Wout[i] = NAN;
        return;
    }
    int64_t f = f0;
    const double* n = m->N + 3 * f;
    double p[3], v[3];
    bary_pos(m, f, b, p);
    perp3(v0, n, v);
    const double L = norm3(v);
    for (int k = 0; k < K; k++) perp3(W0 + 3 * k, n, Wout + 3 * k);
    out->L = L;
    if (L > 0.0) for (int c = 0; c < 3; c++) out->d0[c] = v[c] / L;
    double l = 0.0;
    int32_t steps = 0;
    int status = OR_RAY_OK;
    while (l < L) {
        /* the loop test's margin: how far short of |v_t| the traced length is */
        if (L - l < out->pi_margin) out->pi_margin = L - l;
        if (steps >= o->max_steps) { status = OR_RAY_MAXSTEPS; break; }
        double q[3], c[3], bc[3];
        for (int j = 0; j < 3; j++) q[j] = p[j] + o->step * v[j];
        int64_t f2 = project_to_mesh(m, scale, q, c, bc, &out->pi_margin);
        const double* n2 = m->N + 3 * f2;
        rotate_normal_to_normal(n, n2, v);
        for (int k = 0; k < K; k++) rotate_normal_to_normal(n, n2, Wout + 3 * k);
        double dp[3];
        sub3(c, p, dp);
        l += norm3(dp);
        memcpy(p, c, sizeof c);
        memcpy(b, bc, sizeof bc);
        f = f2;
        n = n2;
        steps++;
    }
    if (status == OR_RAY_OK && L > 0.0 && l - L < out->pi_margin) out->pi_margin = l - L;
    out->f = (int32_t)f;
    memcpy(out->b, b, sizeof b);
    memcpy(out->p, p, sizeof p);
    memcpy(out->v, v, sizeof v);
    out->status = status;
    out->n_cross = steps;
    out->traced = l;
}

/* ------------------------------------------------------------ batching */
typedef struct {
    const or_mesh* m;
    int64_t n;
    const int32_t* f; const double* b; const double* v; int32_t K; const double* W; const or_opts* o;
    int32_t* f_out; double* b_out; double* p_out; double* v_out; double* W_out;
    int32_t* status; int32_t* n_cross; uint64_t* seq_hash; double* min_vdist; double* traced; int8_t* sigma_end;
    int32_t* n_bnd; double* bnd_margin;
    /* backward */
    int mode;   /* 0 forward, 1 EP, 2 GFD */
    double eps_v, eps_p;
    const double* g; double* grad_v; double* grad_b; double* Jv; double* Jp;
    const double* g_vo; const double* g_W; double* grad_W;   /* transport cotangents (mode 3) */
    const or_pi_opts* pi;   /* non-NULL: projection integration is the Exp (modes 0, 1, 2) */
    double pi_scale;        /* largest coordinate magnitude, for the PI tie tolerance */
    double* pi_margin;
    int64_t next;
} job_t;

/* The Exp a job runs: the straightest walk, or projection integration. */
static void exp_any(const job_t* J, int32_t f0, const double* b0, const double* v0, int K, const double* W0,
                    ray_out* out, double* Wout) {
    if (J->pi) pi_one(J->m, f0, b0, v0, K, W0, J->pi, J->pi_scale, out, Wout);
    else exp_one(J->m, f0, b0, v0, K, W0, J->o, out, Wout, NULL);
}

static void ep_one(const job_t* J, int64_t i);
static void gfd_one(const job_t* J, int64_t i);
static void tvjp_one(const job_t* J, int64_t i);

static void fwd_one(const job_t* J, int64_t i) {
    ray_out r;
    double Wtmp[3 * 64];
    double* Wo = J->W_out ? J->W_out + 3 * J->K * i : Wtmp;
    exp_any(J, J->f[i], J->b + 3 * i, J->v + 3 * i, J->K, J->W ? J->W + 3 * J->K * i : NULL, &r, Wo);
    J->f_out[i] = r.f;
    memcpy(J->b_out + 3 * i, r.b, sizeof r.b);
    memcpy(J->p_out + 3 * i, r.p, sizeof r.p);
    memcpy(J->v_out + 3 * i, r.v, sizeof r.v);
    J->status[i] = r.status;
    if (J->n_cross) J->n_cross[i] = r.n_cross;
    if (J->seq_hash) J->seq_hash[i] = r.hash;
    if (J->min_vdist) J->min_vdist[i] = r.min_vdist;
    if (J->traced) J->traced[i] = r.traced;
    if (J->sigma_end) J->sigma_end[i] = r.sigma;
    if (J->n_bnd) J->n_bnd[i] = r.n_bnd;
    if (J->bnd_margin) J->bnd_margin[i] = r.bnd_margin;
    if (J->pi_margin) J->pi_margin[i] = r.pi_margin;
}

static void* worker(void* arg) {
    job_t* J = arg;
    const int64_t chunk = 4096;
    for (;;) {
        int64_t s = __atomic_fetch_add(&J->next, chunk, __ATOMIC_RELAXED);
        if (s >= J->n) break;
        int64_t e = s + chunk < J->n ? s + chunk : J->n;
        for (int64_t i = s; i < e; i++) {
            if (J->mode == 0) fwd_one(J, i);
            else if (J->mode == 1) ep_one(J, i);
            else if (J->mode == 2) gfd_one(J, i);
            else tvjp_one(J, i);
        }
    }
    return NULL;
}

static int run_job(job_t* J, int32_t nthreads) {
    if (nthreads <= 0) nthreads = (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    J->next = 0;
    if (nthreads == 1 || J->n < 4096) { worker(J); return OR_OK; }
    pthread_t th[256];
    int started = 0;
    for (int t = 0; t < nthreads; t++)
        if (pthread_create(&th[t], NULL, worker, J) == 0) started++;
        else break;
    if (!started) worker(J);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    return OR_OK;
}

int or_exp_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                 int32_t K, const double* W, const or_opts* o, int32_t* f_out, double* b_out,
                 double* p_out, double* v_out, double* W_out, int32_t* status, int32_t* n_cross,
                 uint64_t* seq_hash, double* min_vdist, double* traced, int8_t* sigma_end, int32_t* n_bnd,
                 double* bnd_margin, int32_t nthreads) {
    if (!m || n < 0 || K < 0 || K > 64 || (n > 0 && (!f || !b || !v || !f_out || !b_out || !p_out || !v_out || !status)) ||
        (K > 0 && n > 0 && (!W || !W_out))) {
        set_err("bad arguments");
        return OR_E_ARG;
    }
    job_t J = {0};
    J.m = m; J.n = n; J.f = f; J.b = b; J.v = v; J.K = K; J.W = W; J.o = o;
    J.f_out = f_out; J.b_out = b_out; J.p_out = p_out; J.v_out = v_out; J.W_out = W_out;
    J.status = status; J.n_cross = n_cross; J.seq_hash = seq_hash; J.min_vdist = min_vdist;
    J.traced = traced; J.sigma_end = sigma_end; J.n_bnd = n_bnd; J.bnd_margin = bnd_margin;
    return run_job(&J, nthreads);
}

int32_t or_exp_trace(const or_mesh* m, int32_t f, const double* b, const double* v, const or_opts* o,
                     int32_t cap, int8_t* kind, int32_t* face, int32_t* ev0, int32_t* ev1, double* point,
                     int32_t* f_out, double* p_out, int32_t* status) {
    trace_buf tb = {cap, 0, kind, face, ev0, ev1, point};
    ray_out r;
    exp_one(m, f, b, v, 0, NULL, o, &r, NULL, &tb);
    *f_out = r.f;
    memcpy(p_out, r.p, sizeof r.p);
    *status = r.status;
    return tb.n;
}

/* ------------------------------------------------------------ backward */
/* Extrinsic proxy (eq. proxy_func): J^v = R = M_{p'} M_p^T, J^p = 0. */
static void ep_one(const job_t* J, int64_t i) {
    const or_mesh* m = J->m;
    ray_out r;
    exp_any(J, J->f[i], J->b + 3 * i, J->v + 3 * i, 0, NULL, &r, NULL);
    const double* g = J->g + 3 * i;
    double* gv = J->grad_v + 3 * i;
    for (int c = 0; c < 3; c++) J->grad_b[3 * i + c] = 0.0;
    if (r.status == OR_RAY_BADINPUT) { for (int c = 0; c < 3; c++) gv[c] = NAN; return; }
    if (!(r.L > 0.0)) { memcpy(gv, g, 3 * sizeof(double)); return; }
    double Mp[3][3], Mq[3][3];   /* rows: e_par, e_perp, n */
    const double* n0 = m->N + 3 * (int64_t)J->f[i];
    memcpy(Mp[0], r.d0, sizeof r.d0);
    memcpy(Mp[2], n0, 3 * sizeof(double));
    cross3(Mp[2], Mp[0], Mp[1]);
    for (int c = 0; c < 3; c++) { Mq[0][c] = r.v[c] / r.L; Mq[2][c] = r.sigma * m->N[3 * (int64_t)r.f + c]; }
    unit3(Mq[0]);
    cross3(Mq[2], Mq[0], Mq[1]);
    /* R^T g = M_p (M_{p'}^T g) */
    double c3[3] = {dot3(Mq[0], g), dot3(Mq[1], g), dot3(Mq[2], g)};
    for (int c = 0; c < 3; c++) gv[c] = c3[0] * Mp[0][c] + c3[1] * Mp[1][c] + c3[2] * Mp[2][c];
}

/* projection of an ambient vector onto face f's non-orthogonal (e_u, e_v) frame */
static void pinv_face(const or_mesh* m, int64_t f, const double* w, double* c) {
    double eu[3], ev[3];
    sub3(FX(m, f, 1), FX(m, f, 0), eu); unit3(eu);
    sub3(FX(m, f, 2), FX(m, f, 0), ev); unit3(ev);
    double a = dot3(eu, eu), bb = dot3(eu, ev), d = dot3(ev, ev);
    double r1 = dot3(eu, w), r2 = dot3(ev, w), det = a * d - bb * bb;
    c[0] = (d * r1 - bb * r2) / det;
    c[1] = (a * r2 - bb * r1) / det;
}

/* Geodesic finite differences, eqs. jv and jp, chained with g (eq. chain). */
static void gfd_one(const job_t* J, int64_t i) {
    const or_mesh* m = J->m;
    const int32_t f = J->f[i];
    const double* b = J->b + 3 * i;
    const double* g = J->g + 3 * i;
    double ev = J->eps_v, ep = J->eps_p;
    ray_out r0, r1, r2, ru, rv, r3, r4;
    exp_any(J, f, b, J->v + 3 * i, 0, NULL, &r0, NULL);
    double* gv = J->grad_v + 3 * i;
    double* gb = J->grad_b + 3 * i;
    if (r0.status == OR_RAY_BADINPUT) {
        for (int c = 0; c < 3; c++) gv[c] = gb[c] = NAN;
        return;
    }
    double eu[3], evv[3];
    sub3(FX(m, f, 1), FX(m, f, 0), eu); unit3(eu);
    sub3(FX(m, f, 2), FX(m, f, 0), evv); unit3(evv);
    const double* n0 = m->N + 3 * (int64_t)f;
    double epar[3], eperp[3], dend[3];
    if (r0.L > 0.0) {
        memcpy(epar, r0.d0, sizeof epar);
        for (int c = 0; c < 3; c++) dend[c] = r0.v[c] / r0.L;
    } else {           /* |v| = 0: the tangent frame starts on e_u */
        memcpy(epar, eu, sizeof epar);
        memcpy(dend, eu, sizeof dend);
    }
    cross3(n0, epar, eperp);
    double vt[3];
    perp3(J->v + 3 * i, n0, vt);
    /* column e_par: short trace from p' along the transported tangent */
    double w[3];
    for (int c = 0; c < 3; c++) w[c] = ev * dend[c];
    exp_any(J, r0.f, r0.b, w, 0, NULL, &r1, NULL);
    /* column e_perp */
    for (int c = 0; c < 3; c++) w[c] = vt[c] + ev * eperp[c];
    exp_any(J, f, b, w, 0, NULL, &r2, NULL);
    /* start-point perturbations with v transported along them */
    double vu[3], vv[3];
    for (int c = 0; c < 3; c++) w[c] = ep * eu[c];
    exp_any(J, f, b, w, 1, vt, &ru, vu);
    for (int c = 0; c < 3; c++) w[c] = ep * evv[c];
    exp_any(J, f, b, w, 1, vt, &rv, vv);
    exp_any(J, ru.f, ru.b, vu, 0, NULL, &r3, NULL);
    exp_any(J, rv.f, rv.b, vv, 0, NULL, &r4, NULL);
    double col[4][3];
    for (int c = 0; c < 3; c++) {
        col[0][c] = (r1.p[c] - r0.p[c]) / ev;
        col[1][c] = (r2.p[c] - r0.p[c]) / ev;
        col[2][c] = (r3.p[c] - r0.p[c]) / ep;
        col[3][c] = (r4.p[c] - r0.p[c]) / ep;
    }
    double jv[2][2], jp[2][2], t[2];   /* jv[row][col] */
    pinv_face(m, r0.f, col[0], t); jv[0][0] = t[0]; jv[1][0] = t[1];
    pinv_face(m, r0.f, col[1], t); jv[0][1] = t[0]; jv[1][1] = t[1];
    pinv_face(m, r0.f, col[2], t); jp[0][0] = t[0]; jp[1][0] = t[1];
    pinv_face(m, r0.f, col[3], t); jp[0][1] = t[0]; jp[1][1] = t[1];
    if (J->Jv) { J->Jv[4 * i] = jv[0][0]; J->Jv[4 * i + 1] = jv[0][1]; J->Jv[4 * i + 2] = jv[1][0]; J->Jv[4 * i + 3] = jv[1][1]; }
    if (J->Jp) { J->Jp[4 * i] = jp[0][0]; J->Jp[4 * i + 1] = jp[0][1]; J->Jp[4 * i + 2] = jp[1][0]; J->Jp[4 * i + 3] = jp[1][1]; }
    /* M_{p'}^T g */
    double eu2[3], ev2[3];
    sub3(FX(m, r0.f, 1), FX(m, r0.f, 0), eu2); unit3(eu2);
    sub3(FX(m, r0.f, 2), FX(m, r0.f, 0), ev2); unit3(ev2);
    double h[2] = {dot3(eu2, g), dot3(ev2, g)};
    double cv[2] = {jv[0][0] * h[0] + jv[1][0] * h[1], jv[0][1] * h[0] + jv[1][1] * h[1]};
    double cp[2] = {jp[0][0] * h[0] + jp[1][0] * h[1], jp[0][1] * h[0] + jp[1][1] * h[1]};
    for (int c = 0; c < 3; c++) gv[c] = cv[0] * epar[c] + cv[1] * eperp[c];
    /* start-point gradient G in the face plane with M_p^T G = cp, M_p = [e_u e_v] */
    double a = dot3(eu, eu), bb = dot3(eu, evv), d = dot3(evv, evv), det = a * d - bb * bb;
    double y0 = (d * cp[0] - bb * cp[1]) / det, y1 = (a * cp[1] - bb * cp[0]) / det;
    double G[3];
    for (int c = 0; c < 3; c++) G[c] = y0 * eu[c] + y1 * evv[c];
    for (int k = 0; k < 3; k++) gb[k] = dot3(G, FX(m, f, k));
}

/* Cotangents of the transported outputs (an extension of the backward): the
 * walk carries the frame (d, sigma n x d) from (d0, n0 x d0) at p to
 * (d', sigma' n' x d') at p' (Sec. 4 "Parallel Transport": a transported
 * vector keeps its angle to the tangent), so W'_k = R W_k with R that frame
 * map, and v' = R v_t.  Hence dL/dv gains P R^T g_v and dL/dW_k = P R^T g_Wk,
 * P the projection onto the start face's plane (v and W are projected there
 * first).  |v_t| = 0 transports nothing: R = I. */
static void tvjp_one(const job_t* J, int64_t i) {
    const or_mesh* m = J->m;
    ray_out r;
    exp_one(m, J->f[i], J->b + 3 * i, J->v + 3 * i, 0, NULL, J->o, &r, NULL, NULL);
    double* gv = J->grad_v + 3 * i;
    if (r.status == OR_RAY_BADINPUT) {
        for (int c = 0; c < 3; c++) gv[c] = NAN;
        for (int k = 0; k < 3 * J->K; k++) J->grad_W[3 * J->K * i + k] = NAN;
        return;
    }
    const double* n0 = m->N + 3 * (int64_t)J->f[i];
    double d0[3], q0[3], d1[3], q1[3];
    int ident = !(r.L > 0.0);
    if (!ident) {
        memcpy(d0, r.d0, sizeof d0);
        cross3(n0, d0, q0);
        double ns[3];
        for (int c = 0; c < 3; c++) { d1[c] = r.v[c] / r.L; ns[c] = r.sigma * m->N[3 * (int64_t)r.f + c]; }
        unit3(d1);
        cross3(ns, d1, q1);
    }
#define TVJP(gin, gout) do {                                                                   \
        if (ident) { perp3(gin, n0, gout); }                                                    \
        else {                                                                                  \
            double a_ = dot3(gin, d1), b_ = dot3(gin, q1);                                      \
            for (int c = 0; c < 3; c++) (gout)[c] = a_ * d0[c] + b_ * q0[c];                    \
        }                                                                                       \
    } while (0)
    if (J->g_vo) TVJP(J->g_vo + 3 * i, gv);
    else for (int c = 0; c < 3; c++) gv[c] = 0.0;
    for (int k = 0; k < J->K; k++) TVJP(J->g_W + 3 * (J->K * i + k), J->grad_W + 3 * (J->K * i + k));
#undef TVJP
}

int or_transport_vjp(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                     const or_opts* o, int32_t K, const double* g_v, const double* g_W, double* grad_v,
                     double* grad_W, int32_t nthreads) {
    if (!m || n < 0 || K < 0 || (n > 0 && (!f || !b || !v || !grad_v)) || (K > 0 && n > 0 && (!g_W || !grad_W))) {
        set_err("bad arguments");
        return OR_E_ARG;
    }
    job_t J = {0};
    J.m = m; J.n = n; J.f = f; J.b = b; J.v = v; J.o = o; J.mode = 3; J.K = K;
    J.g_vo = g_v; J.g_W = g_W; J.grad_v = grad_v; J.grad_W = grad_W;
    return run_job(&J, nthreads);
}

int or_ep_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                const or_opts* o, const double* g, double* grad_v, double* grad_b, int32_t nthreads) {
    if (!m || n < 0 || (n > 0 && (!f || !b || !v || !g || !grad_v || !grad_b))) { set_err("bad arguments"); return OR_E_ARG; }
    job_t J = {0};
    J.m = m; J.n = n; J.f = f; J.b = b; J.v = v; J.o = o; J.mode = 1;
    J.g = g; J.grad_v = grad_v; J.grad_b = grad_b;
    return run_job(&J, nthreads);
}

int or_gfd_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                 const or_opts* o, double eps_v, double eps_p, const double* g, double* grad_v,
                 double* grad_b, double* Jv, double* Jp, int32_t nthreads) {
    if (!m || n < 0 || !(eps_v > 0) || !(eps_p > 0) || (n > 0 && (!f || !b || !v || !g || !grad_v || !grad_b))) {
        set_err("bad arguments");
        return OR_E_ARG;
    }
    job_t J = {0};
    J.m = m; J.n = n; J.f = f; J.b = b; J.v = v; J.o = o; J.mode = 2;
    J.eps_v = eps_v; J.eps_p = eps_p;
    J.g = g; J.grad_v = grad_v; J.grad_b = grad_b; J.Jv = Jv; J.Jp = Jp;
    return run_job(&J, nthreads);
}

/* ------------------------------------------------------------ vertex-position gradient */
/* Hinge map of an edge crossing (transport_over_edge read as a rigid motion):
 * H(y) = a + Q (y - a), Q the rotation about the line through a and b that
 * unfolds the plane of the face left (apex cp) onto the plane of the face
 * entered (apex cn): Q takes cp's side of the edge to the side opposite cn. */
static void hinge_apply(const double* a, const double* b, const double* cp, const double* cn, const double* y,
                        double* r) {
    double u[3], mf[3], mg[3], cf[3], cg[3], t[3], w[3];
    sub3(b, a, u); unit3(u);
    sub3(cp, a, t); perp3(t, u, mf); unit3(mf);
    sub3(cn, a, t); perp3(t, u, mg); unit3(mg);
    cross3(u, mf, cf);
    cross3(u, mg, cg);
    sub3(y, a, w);
    double pu = dot3(w, u), pm = dot3(w, mf), pc = dot3(w, cf);
    for (int c = 0; c < 3; c++) r[c] = a[c] + pu * u[c] - pm * mg[c] - pc * cg[c];
}

/* y_0 = p + v_t of the start face with vertices x[0..2] (barycentrics b, 3D v). */
static void start_point(const double* x, const double* b, const double* v, double* y) {
    double e1[3], e2[3], n[3], vt[3];
    sub3(x + 3, x, e1);
    sub3(x + 6, x, e2);
    cross3(e1, e2, n); unit3(n);
    perp3(v, n, vt);
    for (int c = 0; c < 3; c++) y[c] = b[0] * x[c] + b[1] * x[3 + c] + b[2] * x[6 + c] + vt[c];
}

typedef struct {
    const or_mesh* m;
    int64_t n;
    const int32_t* f; const double* b; const double* v; const double* g; const or_opts* o;
    double h;
    int32_t* n_vertex;
    int64_t next;
    pthread_mutex_t lock;
    double* grad;            /* nv*3, summed over threads at the end */
} gx_job;

/* One ray's contribution to dL/dX for L = g . p'.  Away from vertices
 * p' = H_m o ... o H_1(y_0) (hinge composition of the edge unfoldings), so
 * dL = lambda_0 . dy_0 + sum_j lambda_j . dH_j(y_{j-1}) with lambda_m = g and
 * lambda_{j-1} = Q_j^T lambda_j.  The local derivatives of y_0 and of each H_j
 * with respect to their (3 or 4) vertices are central differences of these
 * closed forms with step h.  Rays that pass through a vertex contribute
 * nothing (the vertex rule is not a hinge): the return value is their number
 * of vertex passages, or -1 for a ray that did not end with status OK. */
static int gradx_one(const or_mesh* m, int32_t f0, const double* b0, const double* v0, const double* g,
                     const or_opts* o, double h, double* grad) {
    int32_t cap = 1024;
    trace_buf tb;
    tb.cap = cap; tb.n = 0;
    tb.kind = malloc(cap); tb.face = malloc(sizeof(int32_t) * cap);
    tb.ev0 = malloc(sizeof(int32_t) * cap); tb.ev1 = malloc(sizeof(int32_t) * cap);
    tb.pt = malloc(sizeof(double) * 3 * cap);
    ray_out r;
    for (;;) {
        exp_one(m, f0, b0, v0, 0, NULL, o, &r, NULL, &tb);
        if (tb.n < tb.cap) break;
        cap *= 4;
        tb.cap = cap; tb.n = 0;
        tb.kind = realloc(tb.kind, cap); tb.face = realloc(tb.face, sizeof(int32_t) * cap);
        tb.ev0 = realloc(tb.ev0, sizeof(int32_t) * cap); tb.ev1 = realloc(tb.ev1, sizeof(int32_t) * cap);
        tb.pt = realloc(tb.pt, sizeof(double) * 3 * cap);
    }
    int nvert = 0;
    for (int32_t j = 0; j < tb.n; j++) nvert += tb.kind[j] == 1;
    if (r.status != OR_RAY_OK || r.n_bnd > 0 || nvert > 0) {
        free(tb.kind); free(tb.face); free(tb.ev0); free(tb.ev1); free(tb.pt);
        return (r.status != OR_RAY_OK || r.n_bnd > 0) ? -1 : nvert;
    }
    const int32_t nh = tb.n;
    /* hinge vertices: a, b on the edge, cp apex of the face left, cn apex of the face entered */
    int32_t* HV = malloc(sizeof(int32_t) * 4 * (nh > 0 ? nh : 1));
    double* Y = malloc(sizeof(double) * 3 * (nh + 1));
    double* LAM = malloc(sizeof(double) * 3 * (nh + 1));
    double bn[3] = {b0[0], b0[1], b0[2]};
    double bs = bn[0] + bn[1] + bn[2];
    for (int k = 0; k < 3; k++) bn[k] /= bs;
    double xs[9];
    for (int k = 0; k < 3; k++) memcpy(xs + 3 * k, FX(m, f0, k), 3 * sizeof(double));
    start_point(xs, bn, v0, Y);
    int64_t prev = f0;
    for (int32_t j = 0; j < nh; j++) {
        int32_t a = tb.ev0[j], bb = tb.ev1[j], g2 = tb.face[j];
        int32_t cp = -1, cn = -1;
        for (int k = 0; k < 3; k++) {
            int32_t q = m->F[3 * prev + k];
            if (q != a && q != bb) cp = q;
            q = m->F[3 * (int64_t)g2 + k];
            if (q != a && q != bb) cn = q;
        }
        HV[4 * j] = a; HV[4 * j + 1] = bb; HV[4 * j + 2] = cp; HV[4 * j + 3] = cn;
        hinge_apply(VX(m, a), VX(m, bb), VX(m, cp), VX(m, cn), Y + 3 * j, Y + 3 * (j + 1));
        prev = g2;
    }
    /* lambda_m = g; lambda_{j-1} = Q_j^T lambda_j, Q_j w = H_j(a + w) - a */
    memcpy(LAM + 3 * nh, g, 3 * sizeof(double));
    for (int32_t j = nh; j >= 1; j--) {
        const int32_t* hv = HV + 4 * (j - 1);
        const double *a = VX(m, hv[0]), *bb = VX(m, hv[1]), *cp = VX(m, hv[2]), *cn = VX(m, hv[3]);
        double Qt[3][3];   /* rows: Q e_c */
        for (int c = 0; c < 3; c++) {
            double y[3] = {a[0], a[1], a[2]}, r2[3];
            y[c] += 1.0;
            hinge_apply(a, bb, cp, cn, y, r2);
            for (int q = 0; q < 3; q++) Qt[c][q] = r2[q] - a[q];
        }
        for (int c = 0; c < 3; c++) LAM[3 * (j - 1) + c] = dot3(Qt[c], LAM + 3 * j);
    }
    /* start term */
    for (int k = 0; k < 3; k++)
        for (int c = 0; c < 3; c++) {
            double xp[9], xm[9], yp[3], ym[3];
            memcpy(xp, xs, sizeof xs); memcpy(xm, xs, sizeof xs);
            xp[3 * k + c] += h; xm[3 * k + c] -= h;
            start_point(xp, bn, v0, yp);
            start_point(xm, bn, v0, ym);
            double dy[3] = {(yp[0] - ym[0]) / (2 * h), (yp[1] - ym[1]) / (2 * h), (yp[2] - ym[2]) / (2 * h)};
            grad[3 * (int64_t)m->F[3 * (int64_t)f0 + k] + c] += dot3(LAM, dy);
        }
    /* hinge terms */
    for (int32_t j = 1; j <= nh; j++) {
        const int32_t* hv = HV + 4 * (j - 1);
        for (int w = 0; w < 4; w++)
            for (int c = 0; c < 3; c++) {
                double P[4][3], rp[3], rm[3];
                for (int q = 0; q < 4; q++) memcpy(P[q], VX(m, hv[q]), 3 * sizeof(double));
                P[w][c] += h;
                hinge_apply(P[0], P[1], P[2], P[3], Y + 3 * (j - 1), rp);
                P[w][c] -= 2 * h;
                hinge_apply(P[0], P[1], P[2], P[3], Y + 3 * (j - 1), rm);
                double dy[3] = {(rp[0] - rm[0]) / (2 * h), (rp[1] - rm[1]) / (2 * h), (rp[2] - rm[2]) / (2 * h)};
                grad[3 * (int64_t)hv[w] + c] += dot3(LAM + 3 * j, dy);
            }
    }
    free(HV); free(Y); free(LAM);
    free(tb.kind); free(tb.face); free(tb.ev0); free(tb.ev1); free(tb.pt);
    return 0;
}

static void* gx_worker(void* arg) {
    gx_job* J = arg;
    const or_mesh* m = J->m;
    double* g = calloc(3 * m->nv, sizeof(double));
    if (!g) return NULL;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t s = J->next;
        J->next += 256;
        pthread_mutex_unlock(&J->lock);
        if (s >= J->n) break;
        int64_t e = s + 256 < J->n ? s + 256 : J->n;
        for (int64_t i = s; i < e; i++) {
            int nvx = gradx_one(m, J->f[i], J->b + 3 * i, J->v + 3 * i, J->g + 3 * i, J->o, J->h, g);
            if (J->n_vertex) J->n_vertex[i] = nvx;
        }
    }
    pthread_mutex_lock(&J->lock);
    for (int64_t i = 0; i < 3 * m->nv; i++) J->grad[i] += g[i];
    pthread_mutex_unlock(&J->lock);
    free(g);
    return NULL;
}

int or_gradx_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                   const or_opts* o, const double* g, double* grad_X, int32_t* n_vertex, int32_t nthreads) {
    if (!m || n < 0 || !grad_X || (n > 0 && (!f || !b || !v || !g))) { set_err("bad arguments"); return OR_E_ARG; }
    memset(grad_X, 0, sizeof(double) * 3 * m->nv);
    double scale = 0.0;
    for (int64_t i = 0; i < 3 * m->nv; i++) scale = fmax(scale, fabs(m->X[i]));
    gx_job J;
    J.m = m; J.n = n; J.f = f; J.b = b; J.v = v; J.g = g; J.o = o;
    J.h = 1e-6 * (scale > 0 ? scale : 1.0);
    J.n_vertex = n_vertex; J.next = 0; J.grad = grad_X;
    pthread_mutex_init(&J.lock, NULL);
    if (nthreads <= 0) nthreads = (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 0; t < nthreads && n > 256 * t; t++)
        if (pthread_create(&th[t], NULL, gx_worker, &J) == 0) started++;
        else break;
    if (!started) gx_worker(&J);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&J.lock);
    return OR_OK;
}

int or_pi_exp_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                    int32_t K, const double* W, const or_pi_opts* o, int32_t* f_out, double* b_out,
                    double* p_out, double* v_out, double* W_out, int32_t* status, int32_t* n_steps,
                    double* traced, double* margin, int32_t nthreads) {
    if (!m || !o || !(o->step > 0.0) || o->max_steps < 0 || n < 0 || K < 0 || K > 64 ||
        (n > 0 && (!f || !b || !v || !f_out || !b_out || !p_out || !v_out || !status)) ||
        (K > 0 && n > 0 && (!W || !W_out))) {
        set_err("bad arguments");
        return OR_E_ARG;
    }
    job_t J;
    memset(&J, 0, sizeof J);
    J.m = m; J.n = n; J.f = f; J.b = b; J.v = v; J.K = K; J.W = W;
    J.f_out = f_out; J.b_out = b_out; J.p_out = p_out; J.v_out = v_out; J.W_out = W_out;
    J.status = status; J.n_cross = n_steps; J.traced = traced; J.pi_margin = margin;
    J.pi = o; J.pi_scale = mesh_scale(m);
    return run_job(&J, nthreads);
}

int or_pi_project(const or_mesh* m, int64_t n, const double* q, int32_t* f_out, double* c_out, double* b_out,
                  double* margin) {
    if (!m || n < 0 || (n > 0 && (!q || !f_out || !c_out || !b_out))) { set_err("bad arguments"); return OR_E_ARG; }
    const double scale = mesh_scale(m);
    for (int64_t i = 0; i < n; i++) {
        double mg = INFINITY;
        f_out[i] = (int32_t)project_to_mesh(m, scale, q + 3 * i, c_out + 3 * i, b_out + 3 * i, &mg);
        if (margin) margin[i] = mg;
    }
    return OR_OK;
}

int or_pi_ep_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                   const or_pi_opts* o, const double* g, double* grad_v, double* grad_b, int32_t nthreads) {
    if (!m || !o || !(o->step > 0.0) || n < 0 || (n > 0 && (!f || !b || !v || !g || !grad_v || !grad_b))) {
        set_err("bad arguments");
        return OR_E_ARG;
    }
    job_t J;
    memset(&J, 0, sizeof J);
    J.m = m; J.n = n; J.f = f; J.b = b; J.v = v; J.g = g; J.grad_v = grad_v; J.grad_b = grad_b; J.mode = 1;
    J.pi = o; J.pi_scale = mesh_scale(m);
    return run_job(&J, nthreads);
}

int or_pi_gfd_batch(const or_mesh* m, int64_t n, const int32_t* f, const double* b, const double* v,
                    const or_pi_opts* o, double eps_v, double eps_p, const double* g, double* grad_v,
                    double* grad_b, double* Jv, double* Jp, int32_t nthreads) {
    if (!m || !o || !(o->step > 0.0) || n < 0 || !(eps_v > 0.0) || !(eps_p > 0.0) ||
        (n > 0 && (!f || !b || !v || !g || !grad_v || !grad_b))) {
        set_err("bad arguments");
        return OR_E_ARG;
    }
    job_t J;
    memset(&J, 0, sizeof J);
    J.m = m; J.n = n; J.f = f; J.b = b; J.v = v; J.g = g; J.grad_v = grad_v; J.grad_b = grad_b; J.mode = 2;
    J.eps_v = eps_v; J.eps_p = eps_p; J.Jv = Jv; J.Jp = Jp;
    J.pi = o; J.pi_scale = mesh_scale(m);
    return run_job(&J, nthreads);
}
