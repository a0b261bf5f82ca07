// sg_kernels.hip -- gfx950 kernels of the straightest-geodesic exponential map.
//
// One ray per lane (Alg. gpu_parallel).  A ray is held in the chart of the
// half-edge it entered through (see sg_internal.h):
//   h        current half-edge record (face f = h / 3, entry edge k = h % 3)
//   s, t     distance of the entry point from the edge's start a and end b
//   phi      direction angle to the entry edge, fixed point, in [0, pi]
//   Lhi+Llo  remaining length, compensated sum
// Per crossing the lane gathers one 32-byte record, finds the exit edge
// (geodesic_step's lambda, restricted to the two non-entry edges), and
// changes chart.  Unfolding keeps the angle to the crossed edge, so the new
// direction is phi - A or phi + B (transport_over_edge), an exact integer add;
// only the position is rounded, once per crossing, in the local chart.
// Passing a vertex applies the straightest rule of Sec. 4 (equal angles
// theta(x)/2 on both sides, transport_over_vertex) by walking the fan with
// the same records.  Extra vectors keep their signed angle to the tangent
// (Sec. 4 "Parallel Transport"), so they are reconstructed at the end.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "sg_internal.h"
#include "sg_launch.h"

namespace sg {

#define SG_HD __host__ __device__

namespace {

// A ray that starts on a vertex must leave through the edge opposite it; the
// exit test (sign of `cross`) is biased to force that choice.
constexpr float kBig = 1.0e30f;
constexpr float kForceBC = kBig;    // vertex at a: leave through b-c
constexpr float kForceCA = -kBig;   // vertex at b: leave through c-a
constexpr uint32_t kForceBCBit = 2u, kForceCABit = 4u;   // the same, in a stored state record
constexpr uint32_t kParity = 1u;    // orientation flipped an odd number of times
constexpr uint32_t kSlidPar = 2u;   // (Ray::par) the walk slid along a boundary and resumed
constexpr uint32_t kSlidBit = 8u;   // the same, in a stored state record
constexpr uint32_t kDoneBit = 1u << 16;   // a Final record: the walk reached its end
constexpr uint32_t kBndBit = 1u << 17;    // a Final record: the walk slid along a boundary (hole avoidance)

// sin(x)/x and cos(x) as polynomials in u = x^2 on |x| <= pi/2 (least-squares
// minimax fits, max error about 1.4e-7 in float32).
SG_HD __forceinline__ float poly_sinc(float u) {
    float r = 2.579398596935789e-06f;
    r = fmaf(r, u, -1.9794619583990425e-04f);
    r = fmaf(r, u, 8.332779631018639e-03f);
    r = fmaf(r, u, -1.6666638851165771e-01f);
    return fmaf(r, u, 9.999999403953552e-01f);
}
SG_HD __forceinline__ float poly_cos(float u) {
    float r = -2.596159447421087e-07f;
    r = fmaf(r, u, 2.4754535843385383e-05f);
    r = fmaf(r, u, -1.3888237299397588e-03f);
    r = fmaf(r, u, 4.166662320494652e-02f);
    r = fmaf(r, u, -0.5f);
    return fmaf(r, u, 1.0f);
}

// sin and cos of a fixed-point angle in [0, pi] (evaluated about pi/2).
SG_HD __forceinline__ void sincos_fx(uint32_t phi, float& sn, float& cs) {
    const float x = (float)(int32_t)(phi - kHalfPiFx) * kRadPerFx;
    const float u = x * x;
    sn = poly_cos(u);
    cs = -x * poly_sinc(u);
}

SG_HD __forceinline__ uint64_t fnv_face(uint64_t h, uint32_t f) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        h ^= (f >> (8 * i)) & 0xffu;
        h *= 1099511628211ull;
    }
    return h;
}

struct Ray {
    int32_t h;
    float s, t;
    uint32_t phi;
    float Lhi, Llo;
    float bias;      // 0, or kForceBC / kForceCA right after a vertex
    uint32_t par;    // kParity if the orientation flipped an odd number of times; kSlidPar
    int32_t ncross;
    uint64_t hash;
};

// Chart of half-edge h = 3 f + k from face f's record: the edges and corners
// rotated by k, the apex from |ac| and the corner at a.
SG_HD __forceinline__ HalfEdgeRec rec_decode(const FaceRec q, uint32_t k) {
    // fields as scalars first, so the rotation by k stays selects on registers
    const float l0 = q.l[0], l1 = q.l[1], l2 = q.l[2];
    const int32_t n0 = q.nb[0], n1 = q.nb[1], n2 = q.nb[2];
    const uint32_t c0 = q.c0, c1 = q.c1, c2 = kPiFx - q.c0 - q.c1;
    HalfEdgeRec r;
    r.A = k == 0u ? c0 : (k == 1u ? c1 : c2);
    r.B = k == 0u ? c1 : (k == 1u ? c2 : c0);
    r.lab = k == 0u ? l0 : (k == 1u ? l1 : l2);
    r.lbc = k == 0u ? l1 : (k == 1u ? l2 : l0);
    r.lac = k == 0u ? l2 : (k == 1u ? l0 : l1);
    r.nbc = k == 0u ? n1 : (k == 1u ? n2 : n0);
    r.nca = k == 0u ? n2 : (k == 1u ? n0 : n1);
    float sn, cs;
    sincos_fx(r.A, sn, cs);
    r.cx = r.lac * cs;
    r.cy = r.lac * sn;
    return r;
}

// The walk's gather: one 32-byte record with a 32-bit byte offset (f < 2^27).
SG_HD __forceinline__ HalfEdgeRec rec_at(const DevMesh& M, int32_t h) {
    const uint32_t f = (uint32_t)h / 3u;
    const FaceRec q = *reinterpret_cast<const FaceRec*>(reinterpret_cast<const char*>(M.face) + (f << 5));
    return rec_decode(q, (uint32_t)h - 3u * f);
}

// The same chart from the 64-byte geometry record, which holds the walk
// record's lengths and corners (start and end frames read that record anyway;
// no caller of this form uses the neighbour links, which it leaves at -1).
SG_HD __forceinline__ HalfEdgeRec rec_geo(const DevMesh& M, int32_t h) {
    const uint32_t f = (uint32_t)h / 3u;
    const float4* g = M.geo + 4 * (int64_t)f;
    const float4 g0 = g[0], g1 = g[1], g2 = g[2], g3 = g[3];
    FaceRec q;
    q.l[0] = g0.w; q.l[1] = g1.w; q.l[2] = g2.w;
    q.c0 = __builtin_bit_cast(uint32_t, g3.x);
    q.c1 = __builtin_bit_cast(uint32_t, g3.y);
    q.nb[0] = q.nb[1] = q.nb[2] = -1;
    return rec_decode(q, (uint32_t)h - 3u * f);
}

// hardware reciprocal (about 1 ulp); the walk only needs local accuracy
SG_HD __forceinline__ float rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

SG_HD __forceinline__ float3 ld3(const float* p) { return make_float3(p[0], p[1], p[2]); }
SG_HD __forceinline__ float3 sub(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
// Position of vertex k (0..2, face order) of internal face f: one 64-byte
// record per face holds the three positions (w: the walk record's edge
// lengths), the walk record's two corners and the user face id, so an
// epilogue or a start frame takes one 64-byte segment.
SG_HD __forceinline__ float3 fvx(const DevMesh& M, int64_t f, int k) {
    const float4 q = M.geo[4 * f + k];
    return make_float3(q.x, q.y, q.z);
}
SG_HD __forceinline__ int32_t face_user(const DevMesh& M, int64_t f) { return __builtin_bit_cast(int32_t, M.geo[4 * f + 3].z); }
SG_HD __forceinline__ float dot(float3 a, float3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
SG_HD __forceinline__ float3 crs(float3 a, float3 b) {
    return make_float3(fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z), fmaf(a.x, b.y, -a.y * b.x));
}
SG_HD __forceinline__ float3 scl(float3 a, float s) { return make_float3(a.x * s, a.y * s, a.z * s); }
SG_HD __forceinline__ float3 nrm(float3 a) { return scl(a, 1.0f / sqrtf(dot(a, a))); }

enum InitResult { kInitOk = 0, kInitZero = 1, kInitBad = 2 };

// sin and cos of any fixed-point angle (full circle).
SG_HD __forceinline__ void sincos_full(uint32_t phi, float& sn, float& cs) {
    const bool upper = phi > kPiFx;
    sincos_fx(upper ? phi - kPiFx : phi, sn, cs);
    sn = upper ? -sn : sn;
    cs = upper ? -cs : cs;
}

// Rounds an angle in radians (|a| < pi) to fixed point with a split constant.
SG_HD __forceinline__ uint32_t rad_to_fx(float a) {
    const float khi = 683565248.0f, klo = 27.576432f;   // 2^32 / (2 pi) as a float pair
    const float p = a * khi;
    const float e = fmaf(a, khi, -p) + a * klo;
    const float pr = rintf(p);
    return (uint32_t)(int32_t)pr + (uint32_t)(int32_t)rintf((p - pr) + e);
}

// Starts a walk at a point of face f, given by its barycentrics (bA, bB, bC)
// in the order of the chart of half-edge h0 = 3 f + k0, moving at fixed-point
// angle phi0 to that chart's x-axis for length Lhi + Llo.  The ray is extended
// backwards to the edge it would have entered through, so the walk always
// starts on an entry edge with remaining length L + tau (initialise_trace).
// ell0 is the length of the chart's x-axis edge.  kGeo: the chart comes from
// the geometry record (a start frame has read that record), else from the
// compact walk record.
template <bool kGeo = true>
SG_HD int enter_face(const DevMesh& M, int32_t f, int k0, float ell0, float bA, float bB, float bC, uint32_t phi0,
                     float Lhi, float Llo, Ray& st) {
    const int32_t h0 = 3 * f + k0;
    const HalfEdgeRec r0 = kGeo ? rec_geo(M, h0) : rec_at(M, h0);
    float dy, dx;
    sincos_full(phi0, dy, dx);
    // barycentric rates of the direction in the chart
    const float icy = 1.0f / r0.cy, il0 = 1.0f / ell0;
    const float rc = dy * icy;
    const float rb = fmaf(dx, il0, -dy * r0.cx * icy * il0);
    const float ra = -(rb + rc);
    // a start on a vertex must point into this face's corner there
    if ((bA == 0.f) + (bB == 0.f) + (bC == 0.f) == 2) {
        if ((bA == 0.f && ra < 0.f) || (bB == 0.f && rb < 0.f) || (bC == 0.f && rc < 0.f)) return kInitBad;
    }
    // backward exit: the first barycentric that reaches 0 going along -d
    int ie = -1;
    float tau = 0.f;
    if (ra > 0.f) { tau = bA / ra; ie = 0; }
    if (rb > 0.f) { const float ti = bB / rb; if (ie < 0 || ti < tau) { tau = ti; ie = 1; } }
    if (rc > 0.f) { const float ti = bC / rc; if (ie < 0 || ti < tau) { tau = ti; ie = 2; } }
    if (ie < 0) return kInitBad;
    const int k = ie == 2 ? 0 : ie + 1;   // chart edge (a,b)=0, (b,c)=1, (c,a)=2 opposite vertex ie
    const float bk = k == 0 ? bA : (k == 1 ? bB : bC);
    const float rk = k == 0 ? ra : (k == 1 ? rb : rc);
    const float bk1 = k == 0 ? bB : (k == 1 ? bC : bA);
    const float rk1 = k == 0 ? rb : (k == 1 ? rc : ra);
    const float wk = fmaxf(fmaf(-tau, rk, bk), 0.f);
    const float wk1 = fmaxf(fmaf(-tau, rk1, bk1), 0.f);
    const float ell = k == 0 ? ell0 : (k == 1 ? r0.lbc : r0.lac);
    const float iw = 1.0f / (wk + wk1);
    st.s = wk1 * iw * ell;
    st.t = wk * iw * ell;
    const uint32_t th = k == 0 ? 0u : (k == 1 ? kPiFx - r0.B : kPiFx + r0.A);
    uint32_t phi = phi0 - th;
    if (st.s == 0.f || st.t == 0.f) {
        // start on a vertex: the direction must point into this face's corner there
        const uint32_t C0 = kPiFx - r0.A - r0.B;
        const uint32_t cA = k == 0 ? r0.A : (k == 1 ? r0.B : C0);   // corner at the entry edge's start
        const uint32_t cB = k == 0 ? r0.B : (k == 1 ? C0 : r0.A);   // corner at its end
        if (phi > kPiFx) return kInitBad;
        if (st.s == 0.f && phi > cA) return kInitBad;
        if (st.t == 0.f && phi < kPiFx - cB) return kInitBad;
    } else if (phi > kPiFx) {
        // a grazing interior start can round just outside [0, pi]
        phi = phi >= kPiFx + kHalfPiFx ? 0u : kPiFx;
    }
    st.phi = phi;
    st.h = 3 * f + (k0 + k) % 3;
    // remaining length (Lhi + tau) + Llo, compensated (TwoSum)
    const float sum = Lhi + tau;
    const float bv = sum - Lhi;
    st.Lhi = sum;
    st.Llo = ((Lhi - (sum - bv)) + (tau - bv)) + Llo;
    st.par = 0u;
    st.bias = st.s == 0.f ? kForceBC : (st.t == 0.f ? kForceCA : 0.f);
    st.ncross = 0;
    st.hash = fnv_face(14695981039346656037ull, (uint32_t)M.order[f]);
    return kInitOk;
}

// Start-face frame of a query: chart of half-edge 3 f (x-axis along x1 - x0).
struct StartFrame {
    int32_t f;              // internal face id
    float b0, b1, b2;       // normalised barycentrics
    float l0;               // |x1 - x0|
    float3 x0, ex, ey, n;   // origin and chart frame in 3D
};

// Internal face id of user face fu, or -1 when fu is out of range.
SG_HD __forceinline__ int32_t internal_face(const DevMesh& M, int32_t fu) {
    return (fu >= 0 && (int64_t)fu < M.n_faces) ? M.perm[fu] : -1;
}

// fi: the internal id of the query's face (-1: out of range).
SG_HD __forceinline__ int start_frame_int(const DevMesh& M, int32_t fi, const float* bp, StartFrame& S) {
    if (fi < 0) return kInitBad;
    S.f = fi;
    float b0 = bp[0], b1 = bp[1], b2 = bp[2];
    if (!(b0 >= 0.f && b1 >= 0.f && b2 >= 0.f)) return kInitBad;
    const float bs = b0 + b1 + b2;
    if (!(bs > 0.f) || !__builtin_isfinite(bs)) return kInitBad;
    S.b0 = b0 / bs; S.b1 = b1 / bs; S.b2 = b2 / bs;
    const int64_t f3 = 3 * (int64_t)S.f;
    S.x0 = fvx(M, f3 / 3, 0);
    const float3 x1 = fvx(M, f3 / 3, 1);
    const float3 x2 = fvx(M, f3 / 3, 2);
    const float3 e1 = sub(x1, S.x0), e2 = sub(x2, S.x0);
    S.l0 = sqrtf(dot(e1, e1));
    S.n = nrm(crs(e1, e2));
    S.ex = scl(e1, 1.0f / S.l0);
    S.ey = crs(S.n, S.ex);
    return kInitOk;
}

SG_HD __forceinline__ int start_frame(const DevMesh& M, int32_t fu, const float* bp, StartFrame& S) {
    return start_frame_int(M, internal_face(M, fu), bp, S);
}

// ---------------------------------------------------------------- float-float arithmetic
// A value is an unevaluated sum hi + lo of two floats (about 48 significant
// bits).  Built from the error-free transformations TwoSum (Knuth) and the
// FMA-based TwoProd (Ogita, Rump and Oishi, "Accurate sum and dot product",
// 2005), in the style of Dekker's and Bailey's double-length arithmetic.
// Used once per ray, where float32 alone would cost the walk 1e-7 of its
// start angle and length.
struct ff {
    float hi, lo;
};

SG_HD __forceinline__ ff two_sum(float a, float b) {
    const float s = a + b;
    const float bb = s - a;
    return ff{s, (a - (s - bb)) + (b - bb)};
}
SG_HD __forceinline__ ff fast_two_sum(float a, float b) {   // |a| >= |b|
    const float s = a + b;
    return ff{s, b - (s - a)};
}
SG_HD __forceinline__ ff two_prod(float a, float b) {
    const float p = a * b;
    return ff{p, fmaf(a, b, -p)};
}
SG_HD __forceinline__ ff ff_add(ff x, ff y) {
    const ff s = two_sum(x.hi, y.hi);
    return fast_two_sum(s.hi, s.lo + (x.lo + y.lo));
}
SG_HD __forceinline__ ff ff_neg(ff x) { return ff{-x.hi, -x.lo}; }
SG_HD __forceinline__ ff ff_sub(ff x, ff y) { return ff_add(x, ff_neg(y)); }
SG_HD __forceinline__ ff ff_mul(ff x, ff y) {
    const ff p = two_prod(x.hi, y.hi);
    return fast_two_sum(p.hi, fmaf(x.hi, y.lo, fmaf(x.lo, y.hi, p.lo)));
}
SG_HD __forceinline__ ff ff_mulf(ff x, float b) {
    const ff p = two_prod(x.hi, b);
    return fast_two_sum(p.hi, fmaf(x.lo, b, p.lo));
}
SG_HD __forceinline__ ff ff_div(ff x, ff y) {
    const float q1 = x.hi / y.hi;
    const ff r = ff_sub(x, ff_mulf(y, q1));
    return fast_two_sum(q1, r.hi / y.hi);
}
SG_HD __forceinline__ ff ff_sqrt(ff x) {   // x >= 0
    if (!(x.hi > 0.f)) return ff{0.f, 0.f};
    const float s = sqrtf(x.hi);
    const ff p = two_prod(s, s);
    return fast_two_sum(s, (((x.hi - p.hi) - p.lo) + x.lo) / (2.0f * s));
}
SG_HD __forceinline__ ff ff_abs(ff x) { return x.hi < 0.f ? ff_neg(x) : x; }
SG_HD __forceinline__ bool ff_gt(ff x, ff y) { return x.hi > y.hi || (x.hi == y.hi && x.lo > y.lo); }

// atan of t in [0, 1]: atan(t) = atan(c) + atan(r) with c = k / 8 nearest to t,
// r = (t - c) / (1 + t c) in [-1/16, 1/16], and atan(r) = r (1 - r^2/3 + ...)
// summed to r^11 (truncation below 3e-16).  atan(k / 8) as float pairs.
SG_HD __forceinline__ ff ff_atan01(ff t) {
    constexpr float kAtanHi[9] = {0.0f, 0x1.fd5baap-4f, 0x1.f5b760p-3f, 0x1.6f6194p-2f, 0x1.dac670p-2f,
                                  0x1.1e00bap-1f, 0x1.4978fap-1f, 0x1.700a7cp-1f, 0x1.921fb6p-1f};
    constexpr float kAtanLo[9] = {0.0f, -0x1.54f424p-30f, -0x1.b4dfc8p-29f, 0x1.e4def0p-30f, 0x1.586ed4p-28f,
                                  0x1.7bdfd6p-26f, 0x1.934f70p-28f, 0x1.5e118cp-27f, -0x1.777a5cp-26f};
    const int k = (int)rintf(t.hi * 8.0f);
    const float c = 0.125f * (float)k;
    const ff r = ff_div(ff_add(t, ff{-c, 0.f}), ff_add(ff{1.0f, 0.f}, ff_mulf(t, c)));
    const float r2 = r.hi * r.hi;
    float q = -1.0f / 11.0f;
    q = fmaf(q, r2, 1.0f / 9.0f);
    q = fmaf(q, r2, -1.0f / 7.0f);
    q = fmaf(q, r2, 1.0f / 5.0f);
    q = fmaf(q, r2, -1.0f / 3.0f);
    q *= r2;   // atan(r) = r + r q, |r q| <= 1.3e-3 |r|
    const ff at = ff_add(r, two_prod(r.hi, q));
    return ff_add(ff{kAtanHi[k], kAtanLo[k]}, at);
}

// atan2(y, x) in (-pi, pi] from octant reduction and ff_atan01.
SG_HD __forceinline__ ff ff_atan2(ff y, ff x) {
    const ff kPi{0x1.921fb6p+1f, -0x1.777a5cp-24f}, kHalfPi{0x1.921fb6p+0f, -0x1.777a5cp-25f};
    const ff ax = ff_abs(x), ay = ff_abs(y);
    const bool swap = ff_gt(ay, ax);
    if (!(ax.hi > 0.f) && !(ay.hi > 0.f)) return ff{0.f, 0.f};
    ff a = ff_atan01(swap ? ff_div(ax, ay) : ff_div(ay, ax));
    if (swap) a = ff_sub(kHalfPi, a);
    if (x.hi < 0.f) a = ff_sub(kPi, a);
    if (y.hi < 0.f) a = ff_neg(a);
    return a;
}

// initialise_trace (Alg. gpu_parallel): v is projected onto the start face;
// its angle to the chart's x-axis and its length start the walk.  With
// e1 = x1 - x0, e2 = x2 - x0, n = e1 x e2, D = |n| and w = n x e1, the
// components of v on the chart frame (e1 / |e1|, w / |w|) are B / |e1| and
// A / (|e1| D), where B = v.e1 and A = v.w.  They are evaluated in
// float-float from the float32 positions (the edge vectors exactly; D from
// the cross product, which keeps slim faces accurate), giving the length as a
// float pair Lhi + Llo and the angle atan2(A, B D) rounded once to fixed
// point.  In float32 the two would carry relative errors of about 1e-7, i.e.
// endpoint errors of 3e-7 at |v| = pi, along and across the ray; the walk
// itself keeps its errors near 1e-8.
SG_HD __forceinline__ void start_direction(const DevMesh& M, int32_t f, float3 vf, float& Lhi, float& Llo,
                                           uint32_t& phi0) {
    const int64_t f3 = 3 * (int64_t)f;
    const float3 q0 = fvx(M, f3 / 3, 0), q1 = fvx(M, f3 / 3, 1), q2 = fvx(M, f3 / 3, 2);
    const float p0[3] = {q0.x, q0.y, q0.z}, p1[3] = {q1.x, q1.y, q1.z}, p2[3] = {q2.x, q2.y, q2.z};
    const float v[3] = {vf.x, vf.y, vf.z};
    ff e1[3], e2[3];
    for (int c = 0; c < 3; ++c) {
        e1[c] = two_sum(p1[c], -p0[c]);
        e2[c] = two_sum(p2[c], -p0[c]);
    }
    ff n[3], w[3];
    for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        n[c] = ff_sub(ff_mul(e1[c1], e2[c2]), ff_mul(e1[c2], e2[c1]));
    }
    for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        w[c] = ff_sub(ff_mul(n[c1], e1[c2]), ff_mul(n[c2], e1[c1]));
    }
    ff A{0.f, 0.f}, B{0.f, 0.f}, g11{0.f, 0.f}, D2{0.f, 0.f};
    for (int c = 0; c < 3; ++c) {
        A = ff_add(A, ff_mulf(w[c], v[c]));
        B = ff_add(B, ff_mulf(e1[c], v[c]));
        g11 = ff_add(g11, ff_mul(e1[c], e1[c]));
        D2 = ff_add(D2, ff_mul(n[c], n[c]));
    }
    const ff D = ff_sqrt(D2);
    const ff X = ff_mul(B, D);
    // |v_t|^2 = (B^2 D^2 + A^2) / (|e1|^2 D^2)
    const ff L = ff_sqrt(ff_div(ff_add(ff_mul(X, X), ff_mul(A, A)), ff_mul(g11, D2)));
    Lhi = L.hi;
    Llo = L.lo;
    phi0 = 0u;
    if (L.hi > 0.f) {
        const ff kFxPerRadFF{0x1.45f306p+29f, 0x1.b93910p+4f};   // 2^32 / (2 pi)
        const ff q = ff_mul(ff_atan2(A, X), kFxPerRadFF);       // in (-2^31, 2^31]
        const int64_t base = (int64_t)q.hi;                      // q.hi is integral once |q.hi| >= 2^23
        phi0 = (uint32_t)(base + (int64_t)rintf((q.hi - (float)base) + q.lo));
    }
}

SG_HD int ray_init_int(const DevMesh& M, int32_t fi, const float* bp, const float* vp, Ray& st, float& L) {
    StartFrame S;
    if (start_frame_int(M, fi, bp, S) != kInitOk) return kInitBad;
    const float3 v = ld3(vp);
    if (!__builtin_isfinite(v.x) || !__builtin_isfinite(v.y) || !__builtin_isfinite(v.z)) return kInitBad;
    float Llo;
    uint32_t phi0;
    start_direction(M, S.f, v, L, Llo, phi0);
    if (!(L > 0.f)) return kInitZero;
    return enter_face(M, S.f, 0, S.l0, S.b0, S.b1, S.b2, phi0, L, Llo, st);
}

SG_HD int ray_init(const DevMesh& M, int32_t fu, const float* bp, const float* vp, Ray& st, float& L) {
    return ray_init_int(M, internal_face(M, fu), bp, vp, st, L);
}

// Starts a walk at chart point (ex, ey) of half-edge h (an end point of an
// earlier walk), direction phi to that chart's x-axis, length Lhi + Llo.
SG_HD int enter_chart(const DevMesh& M, int32_t h, float ex, float ey, uint32_t phi, float Lhi, float Llo, Ray& st) {
    const int32_t f = h / 3;
    const int k0 = h - 3 * f;
    const HalfEdgeRec r = rec_at(M, h);
    const float ell = r.lab;   // |ab| of this chart
    float bc = ey / r.cy;
    float bb = (ex - bc * r.cx) / ell;
    float ba = 1.0f - bb - bc;
    ba = fmaxf(ba, 0.f); bb = fmaxf(bb, 0.f); bc = fmaxf(bc, 0.f);
    const float is = 1.0f / (ba + bb + bc);
    return enter_face<false>(M, f, k0, ell, ba * is, bb * is, bc * is, phi, Lhi, Llo, st);
}

enum VertexResult { kVertexDone = 0, kVertexNoSnap = 1, kVertexBoundary = 2 };

// transport_over_vertex: the ray reached vertex x0 of face h/3.  Walk the fan
// from the reversed incoming direction, adding corner angles, until half the
// vertex's total angle is reached; leave along the fan edge of that face
// rotated by the residual.  `at_apex` says x0 is the apex c of the current
// chart (else x0 is a for a c-a exit, b for a b-c exit).
SG_HD __forceinline__ int vertex_rule(const DevMesh& M, Ray& st, const HalfEdgeRec& r, bool via_ca,
                                         bool at_apex, int32_t& x0_out) {
    const int32_t f = st.h / 3, k = st.h - 3 * (st.h / 3);
    int xl, hv, roleA;
    int64_t acc;
    float ell;
    if (at_apex) {
        xl = (k + 2) % 3;
        if (via_ca) {   // walk from -d towards c->a; virtual entry across b-c, x0 is that chart's b
            hv = 3 * f + (k + 1) % 3; roleA = 0;
            acc = (int64_t)(int32_t)(st.phi + r.B - kPiFx);
            ell = r.lbc;
        } else {        // walk from -d towards c->b; virtual entry across c-a, x0 is that chart's a
            hv = 3 * f + (k + 2) % 3; roleA = 1;
            acc = (int64_t)(int32_t)(r.A - st.phi);
            ell = r.lac;
        }
    } else if (via_ca) {   // passing vertex a: -d points back across a-b
        xl = k; hv = st.h; roleA = 1;
        acc = (int64_t)(kPiFx - st.phi);
        ell = st.s + st.t;
    } else {               // passing vertex b
        xl = (k + 1) % 3; hv = st.h; roleA = 0;
        acc = (int64_t)st.phi;
        ell = st.s + st.t;
    }
    const int32_t x0 = M.F[3 * (int64_t)f + xl];
    x0_out = x0;
    const int64_t half = M.half_theta[x0];
    if (half < 0) return kVertexBoundary;
    if (!at_apex && acc >= half) return kVertexNoSnap;
    uint32_t par = st.par;
    for (int guard = 0; guard < 4096; ++guard) {
        const HalfEdgeRec q = rec_at(M, hv);
        const uint32_t corner = roleA ? q.A : q.B;
        if (acc + (int64_t)corner >= half) {
            const uint32_t beta = (uint32_t)(half - acc);
            st.h = hv;
            st.phi = roleA ? beta : kPiFx - beta;
            st.s = roleA ? 0.f : ell;
            st.t = roleA ? ell : 0.f;
            st.par = par;
            st.bias = roleA ? kForceBC : kForceCA;
            return kVertexDone;
        }
        acc += corner;
        const int32_t nx = roleA ? q.nca : q.nbc;
        ell = roleA ? q.lac : q.lbc;
        if (nx < 0) return kVertexBoundary;
        hv = nx >> 1;
        const uint32_t flip = (uint32_t)nx & 1u;
        roleA ^= (int)flip;
        par ^= flip;
    }
    return kVertexBoundary;
}

// Barycentric coordinates of chart point (ex, ey) in face h/3, rotated from
// chart order (a, b, c) into face vertex order by the entry edge index k.
SG_HD __forceinline__ void chart_bary(const HalfEdgeRec& r, float ell, float ex, float ey, int k, float& o0,
                                           float& o1, float& o2) {
    float bc = ey / r.cy;
    float bb = (ex - bc * r.cx) / ell;
    float ba = 1.0f - bb - bc;
    ba = fmaxf(ba, 0.f); bb = fmaxf(bb, 0.f); bc = fmaxf(bc, 0.f);
    const float is = 1.0f / (ba + bb + bc);
    ba *= is; bb *= is; bc *= is;
    o0 = k == 0 ? ba : (k == 1 ? bc : bb);
    o1 = k == 0 ? bb : (k == 1 ? ba : bc);
    o2 = k == 0 ? bc : (k == 1 ? bb : ba);
}


// Stop point of a finished walk, in the chart of the last half-edge.
struct Final {
    int32_t h;
    float ex, ey;
    uint32_t phi;
    uint32_t flags;   // bit 0 parity, bits 8..15 status, bit 16 done
    int32_t ncross;
    uint64_t hash;
};
static_assert(sizeof(Final) == 32, "final state is one 32-byte sector");

enum StepEvent { kStepContinue = 0, kStepDone = 1 };

SG_HD __forceinline__ void set_final(Final& fin, const Ray& st, float ex, float ey, int32_t status) {
    fin.h = st.h;
    fin.ex = ex;
    fin.ey = ey;
    fin.phi = st.phi;
    fin.flags = (st.par & kParity) | ((uint32_t)status << 8) | kDoneBit | ((st.par & kSlidPar) ? kBndBit : 0u);
    fin.ncross = st.ncross;
    fin.hash = st.hash;
}

// ---------------------------------------------------------------- hole avoidance
// Sec. 4 and the hole branches of the appendix's transport_over_edge and
// transport_over_vertex.  A ray that reaches a boundary edge slides along it
// toward the end its direction leans to (exactly across it: the end with the
// smaller vertex id); at a boundary vertex it resumes straight in the fan face
// whose corner holds the projection of the direction recorded at the
// boundary, taking the face whose plane deviates least from it (|d . n|);
// when no face's corner holds it, it slides on along the next boundary edge of
// the hole (after a straight arrival, the boundary edge that leans most toward
// the direction).  The step that reached the boundary is completed by the
// first slide or resumption; each further one is a step of its own.  These
// moves are rare and run in 3D from the vertex positions.

// 3D frame of the chart of half-edge h: origin a, x-axis eu along a->b, ev
// toward c, and the face normal (b - a) x (c - a), normalised.
SG_HD __forceinline__ void chart_frame3(const DevMesh& M, int32_t h, float3& xa, float3& eu, float3& ev, float3& n) {
    const int32_t f = h / 3, k = h - 3 * (h / 3);
    const int64_t f3 = 3 * (int64_t)f;
    xa = fvx(M, f3 / 3, k);
    const float3 xb = fvx(M, f3 / 3, (k + 1) % 3);
    const float3 xc = fvx(M, f3 / 3, (k + 2) % 3);
    const float3 ab = sub(xb, xa);
    eu = nrm(ab);
    n = nrm(crs(ab, sub(xc, xa)));
    ev = crs(n, eu);
}

SG_HD __forceinline__ int32_t chart_vertex(const DevMesh& M, int32_t h, int which) {   // 0 a, 1 b, 2 c
    const int32_t f = h / 3, k = h - 3 * (h / 3);
    return M.F[3 * (int64_t)f + (k + which) % 3];
}

SG_HD __forceinline__ float3 proj_unit(float3 d, float3 n) { return nrm(sub(d, scl(n, dot(d, n)))); }

// Ends the walk at 3D point P of face f, direction d projected onto f: the
// chart of f in which the direction's angle lies in [0, pi].
SG_HD __forceinline__ void hole_final(const DevMesh& M, int32_t f, float3 P, float3 d, uint32_t par, int32_t ncross,
                                      uint64_t hash, int32_t status, Final& fin) {
    int32_t hb = 3 * f;
    float best = -2.f;
    float3 xa, eu, ev, n, bxa, beu, bev;
    for (int k = 0; k < 3; ++k) {
        chart_frame3(M, 3 * f + k, xa, eu, ev, n);
        const float dv = dot(d, ev);
        if (dv > best) { best = dv; hb = 3 * f + k; bxa = xa; beu = eu; bev = ev; }
    }
    chart_frame3(M, hb, xa, eu, ev, n);
    const float3 w = proj_unit(d, n);
    const float3 q = sub(P, bxa);
    const float ang = atan2f(fmaxf(dot(w, bev), 0.f), dot(w, beu));
    fin.h = hb;
    fin.ex = dot(q, beu);
    fin.ey = dot(q, bev);
    fin.phi = rad_to_fx(ang);
    fin.flags = (par & kParity) | ((uint32_t)status << 8) | kDoneBit | kBndBit;
    fin.ncross = ncross;
    fin.hash = hash;
}

// Does the projection of d onto the face of chart hv (x0 is its vertex a if
// roleA, else b) point into the face's corner at x0?  Returns |d . n| (the
// transport error) or -1, and the projection w.
SG_HD __forceinline__ float corner_fit(const DevMesh& M, int32_t hv, int roleA, float3 d, float3& w) {
    const int32_t f = hv / 3, k = hv - 3 * (hv / 3);
    const int64_t f3 = 3 * (int64_t)f;
    const int k0 = roleA ? k : (k + 1) % 3;   // x0's local index
    const float3 x0 = fvx(M, f3 / 3, k0);
    const float3 ea = sub(fvx(M, f3 / 3, (k0 + 1) % 3), x0);
    const float3 eb = sub(fvx(M, f3 / 3, (k0 + 2) % 3), x0);
    const float3 n = nrm(crs(ea, eb));   // here (ea x eb) . n > 0
    const float dn = dot(d, n);
    w = sub(d, scl(n, dn));
    if (!(dot(w, w) > 1e-30f)) return -1.f;
    if (dot(crs(ea, w), n) < 0.f || dot(crs(w, eb), n) < 0.f) return -1.f;
    return fabsf(dn);
}

// Compensated remaining length minus a segment.
SG_HD __forceinline__ void rem_sub(float& hi, float& lo, float seg) {
    const float nh = hi - seg;
    lo = lo + ((hi - nh) - seg);
    hi = nh;
}

// The chain from a boundary event: the ray stands at boundary vertex x0 of
// face fc (from: the vertex the last slide started from, or -1), with the
// recorded direction d.  Returns kStepContinue with st resumed at a vertex, or
// kStepDone with fin set.
SG_HD int hole_vertex_chain(const DevMesh& M, int32_t fc, int32_t x0, int32_t from, float3 d, float Lhi, float Llo,
                            uint32_t par, int32_t ncross, uint64_t hash, bool first, int32_t max_steps, Ray& st,
                            Final& fin) {
    for (int guard = 0; guard < (1 << 20); ++guard) {
        // the fan of x0 between its two boundary edges: first to one end ...
        int32_t hv = 3 * fc + (M.F[3 * (int64_t)fc] == x0 ? 0 : (M.F[3 * (int64_t)fc + 1] == x0 ? 1 : 2));
        int roleA = 1;
        uint32_t p = 0u;
        int g = 0;
        for (; g < 4096; ++g) {
            const HalfEdgeRec q = rec_at(M, hv);
            const int32_t nx = roleA ? q.nca : q.nbc;
            if (nx < 0) break;
            hv = nx >> 1;
            roleA ^= nx & 1;
            p ^= (uint32_t)nx & 1u;
        }
        const int32_t he0 = hv, y0 = chart_vertex(M, hv, 2);
        const uint32_t pe0 = p;
        // ... then back across the fan to the other end, testing each face
        {
            const int32_t f = hv / 3, k = hv - 3 * (hv / 3);
            hv = roleA ? 3 * f + (k + 2) % 3 : 3 * f + (k + 1) % 3;
            roleA ^= 1;
        }
        float best = 3.0e38f;
        int32_t hb = -1;
        int rb = 0;
        uint32_t pb = 0u;
        float3 wb = make_float3(0.f, 0.f, 0.f);
        int32_t he1 = hv, y1 = -1;
        uint32_t pe1 = p;
        for (g = 0; g < 4096; ++g) {
            float3 w;
            const float err = corner_fit(M, hv, roleA, d, w);
            if (err >= 0.f && err < best) { best = err; hb = hv; rb = roleA; pb = p; wb = w; }
            const HalfEdgeRec q = rec_at(M, hv);
            const int32_t nx = roleA ? q.nca : q.nbc;
            if (nx < 0) { he1 = hv; y1 = chart_vertex(M, hv, 2); pe1 = p; break; }
            hv = nx >> 1;
            roleA ^= nx & 1;
            p ^= (uint32_t)nx & 1u;
        }
        const float3 X0 = ld3(M.X + 3 * (int64_t)x0);
        if (!first && ncross >= max_steps) {
            float3 xa, eu, ev, n;
            chart_frame3(M, 3 * fc, xa, eu, ev, n);
            hole_final(M, fc, X0, proj_unit(d, n), par, ncross, hash, kRayMaxSteps, fin);
            return kStepDone;
        }
        if (hb >= 0) {   // resume straight in that face, from x0 (its chart with a = x0)
            const int32_t fb = hb / 3, kb = hb - 3 * (hb / 3);
            const int32_t hr = rb ? hb : 3 * fb + (kb + 1) % 3;
            const HalfEdgeRec r = rec_at(M, hr);
            float3 xa, eu, ev, n;
            chart_frame3(M, hr, xa, eu, ev, n);
            float ang = atan2f(dot(wb, ev), dot(wb, eu));
            uint32_t ph = rad_to_fx(fmaxf(ang, 0.f));
            ph = ph > r.A ? r.A : ph;
            st.h = hr;
            st.s = 0.f;
            st.t = r.lab;
            st.phi = ph;
            st.Lhi = Lhi;
            st.Llo = Llo;
            st.bias = kForceBC;
            st.par = (par ^ pb) | kSlidPar;
            st.ncross = ncross + 1;
            st.hash = fnv_face(hash, (uint32_t)M.order[fb]);
            return kStepContinue;
        }
        // no face holds the direction: slide on along a boundary edge of the hole
        int end;
        if (from >= 0) {
            end = y0 == from ? 1 : 0;
        } else {
            const float c0 = dot(d, nrm(sub(ld3(M.X + 3 * (int64_t)y0), X0)));
            const float c1 = dot(d, nrm(sub(ld3(M.X + 3 * (int64_t)y1), X0)));
            end = (c1 > c0 || (c1 == c0 && y1 < y0)) ? 1 : 0;
        }
        const int32_t fe = (end ? he1 : he0) / 3;
        const int32_t y = end ? y1 : y0;
        par ^= end ? pe1 : pe0;
        const float3 Y = ld3(M.X + 3 * (int64_t)y);
        const float3 e = sub(Y, X0);
        const float len = sqrtf(dot(e, e));
        float3 xa, eu, ev, n;
        chart_frame3(M, 3 * fe, xa, eu, ev, n);
        if (Lhi + Llo <= len) {   // the length ends on this boundary edge
            const float3 P = make_float3(fmaf(e.x, (Lhi + Llo) / len, X0.x), fmaf(e.y, (Lhi + Llo) / len, X0.y),
                                         fmaf(e.z, (Lhi + Llo) / len, X0.z));
            hole_final(M, fe, P, proj_unit(d, n), par, ncross, hash, kRayOk, fin);
            return kStepDone;
        }
        if (!first && ncross >= max_steps) {
            hole_final(M, fe, X0, proj_unit(d, n), par, ncross, hash, kRayMaxSteps, fin);
            return kStepDone;
        }
        rem_sub(Lhi, Llo, len);
        ++ncross;
        hash = fnv_face(hash, (uint32_t)M.order[fe]);
        first = false;
        from = x0;
        x0 = y;
        fc = fe;
    }
    st.ncross = max_steps;
    set_final(fin, st, 0.f, 0.f, kRayMaxSteps);
    return kStepDone;
}

// The ray in chart `old` (record r) reached the boundary edge it exits
// through (c-a if via_ca, else b-c) at edge fraction mu from the edge's
// non-apex end, with remaining length Lhi + Llo.  Slide along it.
SG_HD int hole_edge(const DevMesh& M, const Ray& old, const HalfEdgeRec& r, bool via_ca, float mu, float omu,
                    float Lhi, float Llo, int32_t max_steps, Ray& st, Final& fin) {
    const int32_t f = old.h / 3;
    // the exit point and the edge's two ends in the chart
    const float ax = via_ca ? 0.f : old.s + old.t;   // non-apex end (a or b)
    const float px = fmaf(mu, r.cx - ax, ax), py = mu * r.cy;
    float sn, cs;
    sincos_fx(old.phi, sn, cs);
    const float lean = fmaf(cs, r.cx - ax, sn * r.cy);   // direction . (apex - non-apex end)
    const int32_t vn = chart_vertex(M, old.h, via_ca ? 0 : 1), vc = chart_vertex(M, old.h, 2);
    const bool to_c = lean > 0.f || (lean == 0.f && vc < vn);
    const float len = via_ca ? r.lac : r.lbc;
    const float sl = (to_c ? omu : mu) * len;
    const float tx = to_c ? r.cx : ax, ty = to_c ? r.cy : 0.f;
    if (Lhi + Llo <= sl) {   // the length ends on the edge: the recorded direction is the chart's
        const float u = (Lhi + Llo) / sl;
        fin.h = old.h;
        fin.ex = fmaf(u, tx - px, px);
        fin.ey = fmaf(u, ty - py, py);
        fin.phi = old.phi;
        fin.flags = (old.par & kParity) | ((uint32_t)kRayOk << 8) | kDoneBit | kBndBit;
        fin.ncross = old.ncross;
        fin.hash = old.hash;
        return kStepDone;
    }
    rem_sub(Lhi, Llo, sl);
    float3 xa, eu, ev, n;
    chart_frame3(M, old.h, xa, eu, ev, n);
    const float3 d = make_float3(fmaf(cs, eu.x, sn * ev.x), fmaf(cs, eu.y, sn * ev.y), fmaf(cs, eu.z, sn * ev.z));
    return hole_vertex_chain(M, f, to_c ? vc : vn, to_c ? vn : vc, d, Lhi, Llo, old.par, old.ncross + 1,
                             fnv_face(old.hash, (uint32_t)M.order[f]), false, max_steps, st, fin);
}

// One geodesic_step: find the exit of the current face (the smallest positive
// barycentric exit parameter over the two non-entry edges), then cross the
// edge into the next chart (transport_over_edge).  The crossing is computed
// for every lane and committed with selects; stopping in the face, at the
// step cap, at a vertex or on the boundary is one rarely taken branch.
// kPre: the caller passes sin and cos of st.phi (psn, pcs), already computed.
template <bool kHash, bool kFlip, bool kHole, bool kPre = false>
SG_HD __forceinline__ int walk_step(const DevMesh& M, Ray& st, int32_t max_steps, float snap, Final& fin,
                                   bool alive = true, float psn = 0.f, float pcs = 0.f) {
    const HalfEdgeRec r = rec_at(M, st.h);
    float sn, cs;
    if constexpr (kPre) {
        sn = psn;
        cs = pcs;
    } else {
        sincos_fx(st.phi, sn, cs);
    }
    const float cross = fmaf(cs, r.cy, -sn * (r.cx - st.s));   // > 0: apex left of the ray
    const bool via_ca = (cross + st.bias) < 0.f;
    const float w = via_ca ? st.s : st.t;
    const float acr = fabsf(cross);
    const float rD = rcp(fmaf(w, sn, acr));
    const float lam = w * r.cy * rD;   // distance to the exit point
    const float Lr = st.Lhi + st.Llo;
    const float mu = w * sn * rD;      // exit point: fraction from the edge's non-apex end
    const float omu = acr * rD;        // 1 - mu: fraction from the apex
    const int32_t nx = via_ca ? r.nca : r.nbc;
    // the next chart: the crossed edge keeps its points and angles
    const float len = via_ca ? r.lac : r.lbc;
    const float dm = mu * len, dom = omu * len;
    float s2 = via_ca ? dm : dom;
    float t2 = via_ca ? dom : dm;
    uint32_t ph = via_ca ? st.phi - r.A : st.phi + r.B;
    uint32_t par = st.par;
    if (kFlip) {   // neighbour traverses the edge the same way: mirror the chart
        const uint32_t flip = (uint32_t)nx & 1u;
        const float tmp = s2;
        s2 = flip ? t2 : s2;
        t2 = flip ? tmp : t2;
        ph = flip ? kPiFx - ph : ph;
        par ^= flip;
    }
    const int32_t phs = (int32_t)ph;   // keep [0, pi] against rounding of grazing exits
    ph = (uint32_t)(phs < 0 ? 0 : phs);
    const float nh = st.Lhi - lam;                    // compensated remaining length
    const float lo = st.Llo + ((st.Lhi - nh) - lam);
    // (a lane slot without a ray steps a dummy state and never takes the rare branch)
    const bool rare = alive && (!(lam < Lr) || (st.ncross >= max_steps) || (mu < snap) || (omu < snap) || (nx < 0));
    // a lane that takes the rare branch keeps its state unchanged here, so the
    // branch reads the step's starting state from st itself (no second copy
    // of the state stays live across the update)
    st.s = rare ? st.s : s2;
    st.t = rare ? st.t : t2;
    st.phi = rare ? st.phi : ph;
    st.Lhi = rare ? st.Lhi : nh;
    st.Llo = rare ? st.Llo : lo;
    st.h = (rare || nx < 0) ? st.h : (nx >> 1);
    st.par = rare ? st.par : par;
    st.bias = rare ? st.bias : 0.f;
    st.ncross += rare ? 0 : 1;
    if (kHash && !rare) st.hash = fnv_face(st.hash, (uint32_t)M.order[st.h / 3]);
    if (!rare) return kStepContinue;

    // ---- rare events, in priority order (st is the step's starting state)
    if (!(lam < Lr)) {   // the ray ends inside this face (ties stay in the face)
        set_final(fin, st, fmaf(Lr, cs, st.s), Lr * sn, kRayOk);
        return kStepDone;
    }
    if (st.ncross >= max_steps) {
        set_final(fin, st, st.s, 0.f, kRayMaxSteps);
        return kStepDone;
    }
    if (mu < snap || omu < snap) {   // passing a vertex (transport_over_vertex)
        int32_t x0;
        Ray cand = st;
        const bool at_apex = omu < snap;
        const int vr = vertex_rule(M, cand, r, via_ca, at_apex, x0);
        if (vr == kVertexBoundary) {
            if constexpr (kHole) {   // the vertex lies lam along the ray, like a crossing
                float3 xa, eu, ev, n;
                chart_frame3(M, st.h, xa, eu, ev, n);
                const float3 d = make_float3(fmaf(cs, eu.x, sn * ev.x), fmaf(cs, eu.y, sn * ev.y),
                                             fmaf(cs, eu.z, sn * ev.z));
                const Ray o = st;
                return hole_vertex_chain(M, o.h / 3, x0, -1, d, nh, lo, o.par, o.ncross, o.hash, true, max_steps, st,
                                         fin);
            }
            set_final(fin, st, at_apex ? r.cx : (via_ca ? 0.f : st.s + st.t), at_apex ? r.cy : 0.f, kRayBoundary);
            return kStepDone;
        }
        if (vr == kVertexDone) {   // the vertex lies lam along the ray: consume it like a crossing
            cand.Lhi = nh;
            cand.Llo = lo;
            cand.ncross = st.ncross + 1;
            cand.hash = kHash ? fnv_face(st.hash, (uint32_t)M.order[cand.h / 3]) : 0ull;
            st = cand;
            return kStepContinue;
        }
    }
    if (nx < 0) {   // boundary edge: stop on it (Sec. 4, original behaviour), or slide along it
        if constexpr (kHole) {
            const Ray o = st;
            return hole_edge(M, o, r, via_ca, mu, omu, nh, lo, max_steps, st, fin);
        }
        set_final(fin, st, fmaf(lam, cs, st.s), lam * sn, kRayBoundary);
        return kStepDone;
    }
    // a vertex passed too far away to snap: an ordinary crossing
    st.s = s2;
    st.t = t2;
    st.phi = ph;
    st.Lhi = nh;
    st.Llo = lo;
    st.h = nx >> 1;
    st.par = par;
    st.bias = 0.f;
    if (kHash) st.hash = fnv_face(st.hash, (uint32_t)M.order[st.h / 3]);
    st.ncross = st.ncross + 1;
    return kStepContinue;
}

template <bool kHash, bool kFlip, bool kHole>
SG_HD __forceinline__ void walk_to_end(const DevMesh& M, Ray& st, int32_t max_steps, float snap, Final& fin) {
    while (walk_step<kHash, kFlip, kHole>(M, st, max_steps, snap, fin) == kStepContinue) {
    }
}

// Outputs of a ray that never walked: bad input (NaN outputs) or |v_t| = 0
// (the identity: start point, zero vector, projected extra vectors).
SG_HD void write_unwalked(const DevMesh& M, const ExpArgs& a, int64_t i, bool bad) {
    const int32_t f0 = a.f[i];
    a.f_out[i] = f0;
    float bo[3] = {a.b[3 * i], a.b[3 * i + 1], a.b[3 * i + 2]};
    const float nan = __builtin_nanf("");
    float3 p = make_float3(nan, nan, nan);
    float3 n = make_float3(0.f, 0.f, 0.f);
    if (!bad) {
        const float s = bo[0] + bo[1] + bo[2];
        bo[0] /= s; bo[1] /= s; bo[2] /= s;
        const int64_t f3 = 3 * (int64_t)M.perm[f0];
        const float3 x0 = fvx(M, f3 / 3, 0);
        const float3 x1 = fvx(M, f3 / 3, 1);
        const float3 x2 = fvx(M, f3 / 3, 2);
        p = make_float3(bo[0] * x0.x + bo[1] * x1.x + bo[2] * x2.x, bo[0] * x0.y + bo[1] * x1.y + bo[2] * x2.y,
                        bo[0] * x0.z + bo[1] * x1.z + bo[2] * x2.z);
        n = nrm(crs(sub(x1, x0), sub(x2, x0)));
    }
    a.b_out[3 * i] = bo[0]; a.b_out[3 * i + 1] = bo[1]; a.b_out[3 * i + 2] = bo[2];
    a.p_out[3 * i] = p.x; a.p_out[3 * i + 1] = p.y; a.p_out[3 * i + 2] = p.z;
    const float vz = bad ? nan : 0.f;
    a.v_out[3 * i] = vz; a.v_out[3 * i + 1] = vz; a.v_out[3 * i + 2] = vz;
    for (int kk = 0; kk < a.K; ++kk) {
        const float3 w = ld3(a.W + 3 * (i * a.K + kk));
        const float3 wt = bad ? make_float3(nan, nan, nan) : sub(w, scl(n, dot(w, n)));
        float* o = a.W_out + 3 * (i * a.K + kk);
        o[0] = wt.x; o[1] = wt.y; o[2] = wt.z;
    }
    if (a.status) a.status[i] = bad ? kRayBadInput : kRayOk;
    if (a.n_cross) a.n_cross[i] = 0;
    if (a.seq_hash) a.seq_hash[i] = bad ? 0ull : fnv_face(14695981039346656037ull, (uint32_t)f0);
}

// Unit tangent d0 of ray i's projected v on its start face and n0 x d0.
// fi: the internal id of query i's start face.
SG_HD __forceinline__ void start_tangent_frame_int(const DevMesh& M, const ExpArgs& a, int64_t i, int32_t fi,
                                                   float3& d0, float3& q0) {
    const int64_t g3 = 3 * (int64_t)fi;
    const float3 x0 = fvx(M, g3 / 3, 0);
    const float3 x1 = fvx(M, g3 / 3, 1);
    const float3 x2 = fvx(M, g3 / 3, 2);
    const float3 n0 = nrm(crs(sub(x1, x0), sub(x2, x0)));
    const float3 v = ld3(a.v + 3 * i);
    d0 = nrm(sub(v, scl(n0, dot(v, n0))));
    q0 = crs(n0, d0);
}

SG_HD __forceinline__ void start_tangent_frame(const DevMesh& M, const ExpArgs& a, int64_t i, float3& d0, float3& q0) {
    start_tangent_frame_int(M, a, i, M.perm[a.f[i]], d0, q0);
}

// Epilogue: end face, barycentrics, 3D point, transported tangent and vectors.
// aux (nullable): the start-side terms saved at init, [L, (w . d0, w . q0) x K].
SG_HD void write_final(const DevMesh& M, const ExpArgs& a, int64_t i, const Final& fin, float L,
                       const float* aux = nullptr) {
    const int32_t fe = fin.h / 3;
    const int ke = fin.h - 3 * fe;
    const HalfEdgeRec r = rec_geo(M, fin.h);
    const int64_t f3 = 3 * (int64_t)fe;
    const float3 y0 = fvx(M, f3 / 3, 0);
    const float3 y1 = fvx(M, f3 / 3, 1);
    const float3 y2 = fvx(M, f3 / 3, 2);
    const float3 ya = ke == 0 ? y0 : (ke == 1 ? y1 : y2);
    const float3 yb = ke == 0 ? y1 : (ke == 1 ? y2 : y0);
    const float3 yc = ke == 0 ? y2 : (ke == 1 ? y0 : y1);
    const float3 eab = sub(yb, ya);
    const float ell = sqrtf(dot(eab, eab));
    float bo[3];
    chart_bary(r, ell, fin.ex, fin.ey, ke, bo[0], bo[1], bo[2]);
    a.f_out[i] = face_user(M, fe);
    a.b_out[3 * i] = bo[0]; a.b_out[3 * i + 1] = bo[1]; a.b_out[3 * i + 2] = bo[2];
    a.p_out[3 * i] = fmaf(bo[0], y0.x, fmaf(bo[1], y1.x, bo[2] * y2.x));
    a.p_out[3 * i + 1] = fmaf(bo[0], y0.y, fmaf(bo[1], y1.y, bo[2] * y2.y));
    a.p_out[3 * i + 2] = fmaf(bo[0], y0.z, fmaf(bo[1], y1.z, bo[2] * y2.z));
    const float3 ex3 = scl(eab, 1.0f / ell);
    const float3 n3 = nrm(crs(eab, sub(yc, ya)));
    const float3 ey3 = crs(n3, ex3);
    float sn, cs;
    sincos_fx(fin.phi, sn, cs);
    const float3 d3 = make_float3(fmaf(cs, ex3.x, sn * ey3.x), fmaf(cs, ex3.y, sn * ey3.y), fmaf(cs, ex3.z, sn * ey3.z));
    a.v_out[3 * i] = L * d3.x; a.v_out[3 * i + 1] = L * d3.y; a.v_out[3 * i + 2] = L * d3.z;
    if (a.K > 0) {
        // each extra vector keeps its components on the frame (tangent, normal x tangent)
        float3 d0, q0;
        if (!aux) start_tangent_frame(M, a, i, d0, q0);
        const float sg = (fin.flags & kParity) ? -1.0f : 1.0f;
        const float3 q3 = scl(crs(n3, d3), sg);
        for (int kk = 0; kk < a.K; ++kk) {
            float wx, wy;
            if (aux) {
                wx = aux[1 + 2 * kk];
                wy = aux[2 + 2 * kk];
            } else {
                const float3 w = ld3(a.W + 3 * (i * a.K + kk));
                wx = dot(w, d0);
                wy = dot(w, q0);
            }
            float* o = a.W_out + 3 * (i * a.K + kk);
            o[0] = fmaf(wx, d3.x, wy * q3.x);
            o[1] = fmaf(wx, d3.y, wy * q3.y);
            o[2] = fmaf(wx, d3.z, wy * q3.z);
        }
    }
    if (a.status) a.status[i] = (int32_t)((fin.flags >> 8) & 0xffu);
    if (a.n_cross) a.n_cross[i] = fin.ncross;
    if (a.seq_hash) a.seq_hash[i] = fin.hash;
}

// |v_t| of ray i (projection of v onto the start face), recomputed where the
// walk state did not keep it.
SG_HD __forceinline__ float tangent_length(const DevMesh& M, const ExpArgs& a, int64_t i) {
    const int64_t f3 = 3 * (int64_t)M.perm[a.f[i]];
    const float3 x0 = fvx(M, f3 / 3, 0);
    const float3 x1 = fvx(M, f3 / 3, 1);
    const float3 x2 = fvx(M, f3 / 3, 2);
    const float3 e1 = sub(x1, x0), e2 = sub(x2, x0);
    const float l0 = sqrtf(dot(e1, e1));   // same arithmetic as ray_init
    const float3 n = nrm(crs(e1, e2));
    const float3 ex = scl(e1, 1.0f / l0);
    const float3 ey = crs(n, ex);
    const float3 v = ld3(a.v + 3 * i);
    const float vx = dot(v, ex), vy = dot(v, ey);
    return sqrtf(fmaf(vx, vx, vy * vy));
}

template <bool kHash, bool kFlip, bool kHole>
SG_HD void exp_ray(const DevMesh& M, const ExpArgs& a, int64_t i) {
    Ray st;
    float L = 0.f;
    const int ir = ray_init(M, a.f[i], a.b + 3 * i, a.v + 3 * i, st, L);
    if (ir != kInitOk) {
        write_unwalked(M, a, i, ir == kInitBad);
        return;
    }
    Final fin;
    walk_to_end<kHash, kFlip, kHole>(M, st, a.max_steps, a.snap, fin);
    write_final(M, a, i, fin, L);
}

template <bool kHash, bool kFlip, bool kHole>
__global__ __launch_bounds__(256) void k_exp_plain(DevMesh M, ExpArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    exp_ray<kHash, kFlip, kHole>(M, a, i);
}

// ---------------------------------------------------------------- persistent form
// 32-byte walk state in the workspace: the initial chart state written by
// k_init, overwritten in place by the Final record when the walk ends.
struct alignas(32) StateRec {
    int32_t h;        // < 0: the ray needs no walk (its outputs are already written)
    float s, t;
    uint32_t phi;
    float Lhi, Llo;
    uint32_t flags;   // force-exit bits and parity
    int32_t ncross;
};

SG_HD __forceinline__ StateRec pack_state(const Ray& st) {
    StateRec r;
    r.h = st.h; r.s = st.s; r.t = st.t; r.phi = st.phi; r.Lhi = st.Lhi; r.Llo = st.Llo;
    r.flags = (st.par & kParity) | (st.bias > 0.f ? kForceBCBit : (st.bias < 0.f ? kForceCABit : 0u)) |
              ((st.par & kSlidPar) ? kSlidBit : 0u);
    r.ncross = st.ncross;
    return r;
}

SG_HD __forceinline__ void unpack_state(const StateRec& r, Ray& st) {
    st.h = r.h; st.s = r.s; st.t = r.t; st.phi = r.phi; st.Lhi = r.Lhi; st.Llo = r.Llo;
    st.bias = (r.flags & kForceBCBit) ? kForceBC : ((r.flags & kForceCABit) ? kForceCA : 0.f);
    st.par = (r.flags & kParity) | ((r.flags & kSlidBit) ? kSlidPar : 0u);
    st.ncross = r.ncross;
}
static_assert(sizeof(StateRec) == 32, "state record is one 32-byte sector");

// ---------------------------------------------------------------- spatial ray order
// The persistent walk takes rays in the order of their start faces (the
// internal face order is a spatial bisection order), so the rays in flight at
// any moment start close together and share the records they fetch.  A
// counting sort by start-face bucket: one atomic per ray on its bucket's
// counter gives its rank inside the bucket, one block scans the counts, and
// the ray's walk slot is the bucket's start plus that rank.  Rays with a face
// id out of range go to a last bucket.
constexpr int kMaxBuckets = 8192;

// Ray queues of the persistent walk (their use is described at queue_claim).
constexpr int kQueueStride = 32;   // counters 256 bytes apart
constexpr size_t kQueueBytes = (size_t)kMaxQueues * kQueueStride * sizeof(unsigned long long);

// The walk order: queue range j (nq ranges of equal internal-face counts, in
// the spatial bisection order), then length class c (longest first), then
// spatial sub-bucket.  Taking the long rays of a range first keeps the last
// rays in flight short, so the waves drain quickly once the queues are empty.
// Length classes are octaves of |v|^2 below the longest ray of the call, from
// the difference of the float bit patterns (integer arithmetic, so every
// kernel that recomputes a ray's bucket gets the same one).
constexpr int kLenClasses = 8;
constexpr int kVmaxWord = kMaxBuckets + 1;   // cnt[kVmaxWord]: float bits of the longest |v|^2
constexpr int kLenBlocks = 1024;             // k_len_max blocks; their partial maxima follow kVmaxWord
constexpr int kCountWords = kMaxBuckets + 2 + kLenBlocks;   // words of the bucket-count array

struct RayOrder {
    int nq;    // queue ranges
    int sub;   // spatial sub-buckets per (range, class)
    int nb;    // nq * kLenClasses * sub + 1 buckets (the last: face id out of range)
};

inline RayOrder ray_order(int nq) {
    RayOrder o;
    o.nq = nq;
    o.sub = kMaxBuckets / (nq * kLenClasses);
    o.nb = nq * kLenClasses * o.sub + 1;
    return o;
}

SG_HD __forceinline__ float len2(const float* v) { return fmaf(v[0], v[0], fmaf(v[1], v[1], v[2] * v[2])); }

// fi: the internal id of the ray's start face (-1: out of range).
SG_HD __forceinline__ int ray_bucket_int(const DevMesh& M, int32_t fi, const float* v, const RayOrder& o,
                                         uint32_t vmax_bits) {
    if (fi < 0) return o.nb - 1;
    const int64_t x = (int64_t)fi * o.nq;
    const int64_t j = x / M.n_faces;
    const int64_t sb = ((x - j * M.n_faces) * o.sub) / M.n_faces;
    const float l2 = len2(v);
    int c = 0;
    if (l2 <= __uint_as_float(vmax_bits)) {   // (NaN, inf: class 0)
        const uint32_t d = (vmax_bits - __float_as_uint(l2)) >> 23;
        c = d < (uint32_t)kLenClasses ? (int)d : kLenClasses - 1;
    }
    return (int)((j * kLenClasses + c) * o.sub + sb);
}

SG_HD __forceinline__ int ray_bucket(const DevMesh& M, int32_t fu, const float* v, const RayOrder& o, uint32_t vmax_bits) {
    return ray_bucket_int(M, internal_face(M, fu), v, o, vmax_bits);
}

// Longest finite |v|^2 of a call, as float bits (which order like the values
// for non-negative floats): each block writes its partial maximum after
// cnt[kVmaxWord], and the blocks clear the bucket counts for k_bucket_count.
__global__ __launch_bounds__(256) void k_len_max(int64_t n, const float* v, uint32_t* cnt) {
    __shared__ uint32_t part[4];
    for (int j = (int)(blockIdx.x * blockDim.x + threadIdx.x); j <= kMaxBuckets; j += (int)(gridDim.x * blockDim.x))
        cnt[j] = 0u;
    uint32_t m = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {   // four rays in flight per thread
        float l2[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) l2[j] = len2(v + 3 * (i + j * stride));
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (l2[j] <= 3.0e38f) m = max(m, __float_as_uint(l2[j]));
    }
    for (; i < n; i += stride) {
        const float l2 = len2(v + 3 * i);
        if (l2 <= 3.0e38f) m = max(m, __float_as_uint(l2));
    }
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63u) == 0u) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) cnt[kVmaxWord + 1 + blockIdx.x] = max(max(part[0], part[1]), max(part[2], part[3]));
}

// Rank of each ray inside its bucket: a 1024-thread block counts its
// kBucketRays rays in LDS (the LDS atomic returns the local rank), then adds
// each nonzero local count to the bucket's global counter once (returning the
// block's base in the bucket).
constexpr int kBucketRays = 4096;   // 256 blocks for 1M rays, one per CU

__global__ __launch_bounds__(1024) void k_bucket_count(DevMesh M, int64_t n, const int32_t* f, const float* v,
                                                       uint32_t* cnt, int32_t* slot, RayOrder o, int nparts,
                                                       int32_t* fint) {
    __shared__ uint32_t local[kMaxBuckets + 1];
    const int nb = o.nb;
    // the call's longest |v|^2 from k_len_max's nparts partial maxima (block 0 keeps it for later kernels)
    __shared__ uint32_t vmax_s;
    if (threadIdx.x < 64u) {
        uint32_t m = 0u;
        for (int j = (int)threadIdx.x; j < nparts; j += 64) m = max(m, cnt[kVmaxWord + 1 + j]);
        for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
        if (threadIdx.x == 0u) {
            vmax_s = m;
            if (blockIdx.x == 0u) cnt[kVmaxWord] = m;
        }
    }
    __syncthreads();
    const uint32_t vmax = vmax_s;
    const int t = (int)threadIdx.x;
    for (int b = t; b < nb; b += 1024) local[b] = 0u;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kBucketRays;
    constexpr int kPer = kBucketRays / 1024;
    uint32_t rk[kPer];
    int bk[kPer];
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = i0 + (int64_t)j * 1024 + t;
        const int32_t fi = i < n ? internal_face(M, f[i]) : -1;
        if (fint && i < n) fint[i] = fi;
        bk[j] = i < n ? ray_bucket_int(M, fi, v + 3 * i, o, vmax) : -1;
        rk[j] = bk[j] >= 0 ? atomicAdd(&local[bk[j]], 1u) : 0u;
    }
    __syncthreads();
    for (int b = t; b < nb; b += 1024) {
        const uint32_t c = local[b];
        local[b] = c ? atomicAdd(&cnt[b], c) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t i = i0 + (int64_t)j * 1024 + t;
        if (bk[j] >= 0) slot[i] = (int32_t)(local[bk[j]] + rk[j]);
    }
}

// Exclusive scan of nb counts in place (one block of 1024 threads).
__global__ __launch_bounds__(1024) void k_bucket_scan(uint32_t* cnt, int nb) {
    __shared__ uint32_t part[1024];
    const int t = (int)threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
    uint32_t sum = 0u;
    for (int b = b0; b < b1; ++b) sum += cnt[b];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int b = b0; b < b1; ++b) {
        const uint32_t c = cnt[b];
        cnt[b] = run;
        run += c;
    }
}

// slot[i] = bucket start + rank inside the bucket.
__global__ __launch_bounds__(256) void k_slot_place(DevMesh M, int64_t n, const int32_t* f, const float* v,
                                                    const uint32_t* bstart, int32_t* slot, RayOrder o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) slot[i] = (int32_t)bstart[ray_bucket(M, f[i], v + 3 * i, o, bstart[kVmaxWord])] + slot[i];
}

// Initial chart state of every ray, stored at its walk slot (slot[i] becomes
// that slot); the epilogue's start-side terms (|v_t| and the extra vectors'
// components on the start frame) go to aux, so the epilogue does not revisit
// the start face.  With fin (final states by query index), the state's
// crossing count carries the query index i to the walk, and a query with no
// walk is marked in fin.
__global__ __launch_bounds__(256) void k_init(DevMesh M, ExpArgs a, StateRec* states, unsigned long long* counter,
                                              float* aux, const uint32_t* bstart, int32_t* slot, RayOrder o,
                                              Final* fin, const int32_t* fint) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMaxQueues) counter[i * kQueueStride] = 0ull;
    if (i >= a.n) return;
    // the internal face id from the bucket pass (a stream), not a second random lookup
    const int32_t fi = fint ? fint[i] : internal_face(M, a.f[i]);
    const int32_t at = (int32_t)bstart[ray_bucket_int(M, fi, a.v + 3 * i, o, bstart[kVmaxWord])] + slot[i];
    if (!fin) slot[i] = at;   // the slot-order epilogue needs it
    Ray st;
    float L = 0.f;
    const int ir = ray_init_int(M, fi, a.b + 3 * i, a.v + 3 * i, st, L);
    StateRec rec;
    if (ir != kInitOk) {
        write_unwalked(M, a, i, ir == kInitBad);
        rec.h = -1;
        rec.s = rec.t = rec.Lhi = rec.Llo = 0.f;
        rec.phi = rec.flags = 0u;
        rec.ncross = 0;
        if (fin) fin[i].h = -1;   // the epilogue skips it
    } else {
        rec = pack_state(st);
        if (fin) rec.ncross = (int32_t)i;   // a start state has crossed nothing: the field carries the query
        float* x = aux + i * (1 + 2 * (int64_t)a.K);
        x[0] = L;
        if (a.K > 0) {
            float3 d0, q0;
            start_tangent_frame_int(M, a, i, fi, d0, q0);
            for (int kk = 0; kk < a.K; ++kk) {
                const float3 w = ld3(a.W + 3 * (i * a.K + kk));
                x[1 + 2 * kk] = dot(w, d0);
                x[2 + 2 * kk] = dot(w, q0);
            }
        }
    }
    states[at] = rec;
}

// Float64 add into a global sum (the gradient accumulators).  hipMalloc'd
// memory is coarse-grained, where the hardware float64 atomic is exact.
SG_HD __forceinline__ void add_f64(double* p, double v) {
#if defined(__HIP_DEVICE_COMPILE__)
    unsafeAtomicAdd(p, v);
#else
    uint64_t* q = reinterpret_cast<uint64_t*>(p);
    uint64_t old = __atomic_load_n(q, __ATOMIC_RELAXED), nw;
    do {
        double d;
        __builtin_memcpy(&d, &old, 8);
        d += v;
        __builtin_memcpy(&nw, &d, 8);
    } while (!__atomic_compare_exchange_n(q, &old, nw, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED));
#endif
}

// Vertex-position gradient, per edge crossing: the adjoint lambda is
// constant in the development (it keeps its components c = (c_d, c_q, c_n)
// on the frame [d, nu x d, nu] of the tangent d and the carried normal nu).
// In the chart of the entered half-edge h, frame (u, m, n) = (x, y, z), it
// adds to h's sums the normal-and-apex-side components (l_m, l_n) of lambda
// and T = r x lambda, r = (s + l cos phi, l sin phi, 0) the virtual endpoint
// relative to the chart origin.
// One crossing's record: the entered half-edge and its five terms
// (l_m, l_n, T_u, T_m, T_n).
struct alignas(8) GxRec {
    int32_t h;
    float q[5];
};
static_assert(sizeof(GxRec) == 24, "grad-X record is 24 bytes");

// sn, cs: sin and cos of st.phi.
SG_HD __forceinline__ GxRec gx_terms(const Ray& st, const float4& c, float sn, float cs) {
    const float sg = (st.par & kParity) ? -1.f : 1.f;
    const float lu = fmaf(c.x, cs, -sg * c.y * sn);
    const float lm = fmaf(c.x, sn, sg * c.y * cs);
    const float ln = sg * c.z;
    const float Lr = st.Lhi + st.Llo;
    const float ru = fmaf(Lr, cs, st.s), rm = Lr * sn;
    GxRec r;
    r.h = st.h;
    r.q[0] = lm;
    r.q[1] = ln;
    r.q[2] = rm * ln;
    r.q[3] = -ru * ln;
    r.q[4] = fmaf(ru, lm, -rm * lu);
    return r;
}

SG_HD __forceinline__ void gx_cross(double* acc, const Ray& st, const float4& c, float sn, float cs) {
    const GxRec r = gx_terms(st, c, sn, cs);
    double* q = acc + 5 * (int64_t)r.h;
    for (int k = 0; k < 5; ++k) add_f64(q + k, (double)r.q[k]);
}

// Binned accumulation of the crossing terms.  Float64 atomics on the
// half-edge sums run at the memory-side atomic rate, five per crossing, so
// instead the walk appends each crossing's record to a chunk of a record
// buffer and counts the records per bin of 2^shift consecutive half-edges in
// LDS.  Every walk block owns a fixed range of chunks; its waves claim them
// with an LDS atomic and fill them with coalesced stores.  At its end the
// block writes its bin counts as one row of a (block, bin) matrix.  A column
// scan of that matrix gives each (block, bin) pair its place in bin order, so
// the scatter pass (one block per walk block) moves the records there with
// LDS cursors only, and a reduce pass sums each bin in LDS (float64) and adds
// the bin's totals to the half-edge sums once.  Crossings past a block's
// chunks fall back to the atomics.
constexpr int kGxChunk = 1024;            // records per chunk
constexpr int kGxMaxBins = 4096;          // bins (LDS counters of the walk and of the scatter)
constexpr int kGxWindow = 4096;           // half-edges summed in LDS at once by the reduce pass (160 KB)
constexpr int kGxShift0 = 12;             // log2 of the smallest bin: one reduce window
constexpr int64_t kGxMaxRecords = (int64_t)1 << 30;   // at most 48 GiB of records (bin starts are 32-bit)

// A record leaves the walk as a streaming (non-temporal) store, so the 24
// bytes per crossing do not displace the face records the walk re-reads
// from L2.
__device__ __forceinline__ void gx_store(GxRec* p, const GxRec& r) {
    // six 4-byte stores: three 8-byte ones at the records' 24-byte stride made the
    // walk 0.35 ms slower, and staging a wave's records in LDS for contiguous
    // stores gained nothing
    uint32_t* d = reinterpret_cast<uint32_t*>(p);
    __builtin_nontemporal_store((uint32_t)r.h, d);
    for (int k = 0; k < 5; ++k) __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, r.q[k]), d + 1 + k);
}

struct GxSink {
    GxRec* rec;       // record buffer, gridDim.x * per_block chunks of kGxChunk records; null: atomics only
    uint32_t* fill;   // records written into each claimed chunk
    int per_block;    // chunks owned by each walk block
    int shift;        // a bin is 2^shift consecutive half-edges
};

// Ray queues of the persistent walk.  The walk slots are in the order of
// ray_bucket, whose nq queue ranges are spatial regions (nq / 8 per XCD):
// blocks are dealt to the XCDs round-robin, so block b runs on XCD b % 8 and
// starts on queue b % 8, the first of that XCD's.  Each XCD then works through
// its own ranges one after another, long rays first within each, so its L2
// holds the face records of one range at a time (with many meshes in a batch,
// a range is about one mesh), and the claim atomics spread over eight counters
// on separate 256-byte lines instead of serializing on one address.  A wave
// whose queue runs dry moves on to the next one, first through its XCD's
// other queues, so every queue is drained.  Queue q serves range
// j = (q % 8) * (nq / 8) + q / 8, whose slots run from start[j * stride] to
// start[(j + 1) * stride] (bucket starts), times `per` states per ray.
struct QueueCursor {
    int q;      // queue this wave claims from
    int left;   // queues not yet seen empty; 0 once every queue is
    int nq;
};

struct QueueRanges {
    const uint32_t* start;   // scanned bucket starts
    int stride;              // buckets per queue range
    int per;                 // walk states per ray
};

SG_HD __forceinline__ QueueCursor queue_start(int nq) {
#if defined(__HIP_DEVICE_COMPILE__)
    return QueueCursor{(int)(blockIdx.x & 7u), nq, nq};
#else
    return QueueCursor{0, nq, nq};
#endif
}

SG_HD __forceinline__ int queue_range(int q, int nq) { return (q & 7) * (nq >> 3) + (q >> 3); }

// One claim of `want` consecutive slots by the whole wave (lane 0 does the
// atomic).  Returns the first slot; slots at or past *hi belong to another
// queue and are not this claim's.  When the claim reaches the end of its queue
// the cursor moves on.
__device__ __forceinline__ int64_t queue_claim(unsigned long long* ctr, const QueueRanges& R, int lane, int want,
                                               QueueCursor& c, int64_t& hi) {
    const int per = c.nq >> 3;
    const int j = queue_range(c.q, c.nq);
    const int64_t lo = (int64_t)R.start[j * R.stride] * R.per;
    hi = (int64_t)R.start[(j + 1) * R.stride] * R.per;
    unsigned long long b = 0ull;
    if (lane == 0) b = atomicAdd(ctr + (size_t)c.q * kQueueStride, (unsigned long long)want);
    b = __shfl(b, 0);
    const int64_t first = lo + (int64_t)b;
    if (first + want >= hi) {   // on to the next range in XCD-major order
        const int jn = j + 1 == c.nq ? 0 : j + 1;
        c.q = (jn % per) * 8 + jn / per;
        --c.left;
    }
    return first;
}

// Persistent walk: each wave keeps 64 rays in flight and refills finished
// lanes from the ray queues (one atomic per wave per refill, ballot for the
// lane ranks), so short and long rays share lanes instead of idling behind
// the longest ray of a fixed batch.  Between refills the wave runs a tight
// loop of walk steps and re-ballots only to see whether enough lanes are idle.
// With kGX every edge crossing also adds its vertex-gradient terms.
template <bool kHash, bool kFlip, bool kHole, bool kGX>
__device__ __forceinline__ void walk_loop(const DevMesh& M, StateRec* states, QueueRanges R, unsigned long long* counter,
                                          int32_t max_steps, float snap, int refill_min, int nq, const float4* cvec,
                                          double* acc, const GxSink& sink, uint32_t* lbins, Final* fin_out = nullptr) {
    const int lane = (int)(threadIdx.x & 63u);
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    // record chunk of this wave (wave-uniform): index, records written, or spilling to atomics
    int64_t chunk = -1;
    int used = kGxChunk;
    bool spill = sink.rec == nullptr;
    bool active = false;
    QueueCursor qc = queue_start(nq);
    int64_t q = 0;
    int32_t ray = 0;   // with fin_out: the query index, carried in the initial state's crossing count
    Ray st;
    st.h = 0; st.s = st.t = st.Lhi = st.Llo = st.bias = 0.f; st.phi = st.par = 0u; st.ncross = 0; st.hash = 0ull;
    float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
    float gsn = 0.f, gcs = 0.f;   // with kGX: sin and cos of st.phi, shared by the crossing's terms and the next step
    for (;;) {
        const uint64_t idle = __ballot(!active);
        const int nidle = __popcll(idle);
        if (nidle == 64 && qc.left == 0) break;
        if (qc.left > 0 && nidle >= refill_min) {
            int64_t hi = 0;
            const int64_t base = queue_claim(counter, R, lane, nidle, qc, hi);
            if (!active) {
                q = base + __popcll(idle & below);
                if (q < hi) {
                    const StateRec rec = states[q];
                    if (rec.h >= 0) {
                        unpack_state(rec, st);
                        if (fin_out) {
                            ray = rec.ncross;
                            st.ncross = 0;
                        }
                        st.hash = kHash ? fnv_face(14695981039346656037ull, (uint32_t)M.order[rec.h / 3]) : 0ull;
                        if (kGX) {
                            c = cvec[q];
                            sincos_fx(st.phi, gsn, gcs);
                        }
                        active = true;
                    }
                }
            }
        }
        // walk until enough lanes are idle to refill (all of them once the queues are empty)
        const int stop_at = qc.left == 0 ? 64 : refill_min;
        for (;;) {
            bool cross = false;
            if (active) {
                Final fin;
                if (walk_step<kHash, kFlip, kHole, kGX>(M, st, max_steps, snap, fin, true, gsn, gcs) == kStepDone) {
                    if (fin_out) fin_out[ray] = fin;
                    else *reinterpret_cast<Final*>(&states[q]) = fin;
                    active = false;
                } else if constexpr (kGX) {
                    sincos_fx(st.phi, gsn, gcs);
                    cross = st.bias == 0.f;   // an edge crossing (a vertex passage leaves a bias)
                }
            }
            if constexpr (kGX) {
                const uint64_t m = __ballot(cross);
                if (m) {
                    const int cw = __popcll(m);
                    if (!spill && used + cw > kGxChunk) {   // close this chunk, claim the block's next
                        if (chunk >= 0 && lane == 0) sink.fill[chunk] = (uint32_t)used;
                        uint32_t b = 0u;
                        if (lane == 0) b = atomicAdd(&lbins[kGxMaxBins], 1u);
                        b = (uint32_t)__shfl((int)b, 0);
                        if (b < (uint32_t)sink.per_block) {
                            chunk = (int64_t)blockIdx.x * sink.per_block + b;
                            used = 0;
                        } else {
                            chunk = -1;
                            spill = true;
                        }
                    }
                    if (cross) {
                        if (!spill) {
                            const GxRec r = gx_terms(st, c, gsn, gcs);
                            gx_store(sink.rec + chunk * kGxChunk + used + __popcll(m & below), r);
                            atomicAdd(&lbins[r.h >> sink.shift], 1u);
                        } else {
                            gx_cross(acc, st, c, gsn, gcs);
                        }
                    }
                    if (!spill) used += cw;
                }
            }
            if (__popcll(__ballot(!active)) >= stop_at) break;
        }
    }
    if (kGX && chunk >= 0 && lane == 0) sink.fill[chunk] = (uint32_t)used;
}

// Two rays per lane: both slots are stepped every iteration, branch-free, so
// each lane carries two independent dependency chains and two gathers in
// flight (the walk is bound by instruction latency at the occupancy where the
// memory system is not yet congested).  A slot without a ray steps a dummy
// state (alive = false) whose results are dropped.
template <bool kHash, bool kFlip, bool kHole>
__device__ __forceinline__ void walk_loop2(const DevMesh& M, StateRec* states, QueueRanges R,
                                           unsigned long long* counter, int32_t max_steps, float snap, int refill_min,
                                           int nq) {
    const int lane = (int)(threadIdx.x & 63u);
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    bool a0 = false, a1 = false;
    QueueCursor qc = queue_start(nq);
    int64_t q0 = 0, q1 = 0;
    Ray s0, s1;
    s0.h = 0; s0.s = s0.t = s0.Lhi = s0.Llo = s0.bias = 0.f; s0.phi = s0.par = 0u; s0.ncross = 0; s0.hash = 0ull;
    s1 = s0;
    for (;;) {
        const uint64_t i0 = __ballot(!a0), i1 = __ballot(!a1);
        const int n0 = __popcll(i0), nidle = n0 + __popcll(i1);
        if (nidle == 128 && qc.left == 0) break;
        if (qc.left > 0 && nidle >= refill_min) {
            int64_t hi = 0;
            const int64_t base = queue_claim(counter, R, lane, nidle, qc, hi);
            if (!a0) {
                q0 = base + __popcll(i0 & below);
                if (q0 < hi) {
                    const StateRec rec = states[q0];
                    if (rec.h >= 0) {
                        unpack_state(rec, s0);
                        s0.hash = kHash ? fnv_face(14695981039346656037ull, (uint32_t)M.order[rec.h / 3]) : 0ull;
                        a0 = true;
                    }
                }
            }
            if (!a1) {
                q1 = base + n0 + __popcll(i1 & below);
                if (q1 < hi) {
                    const StateRec rec = states[q1];
                    if (rec.h >= 0) {
                        unpack_state(rec, s1);
                        s1.hash = kHash ? fnv_face(14695981039346656037ull, (uint32_t)M.order[rec.h / 3]) : 0ull;
                        a1 = true;
                    }
                }
            }
        }
        const int stop_at = qc.left == 0 ? 128 : refill_min;
        for (;;) {
            Final f0, f1;
            const int e0 = walk_step<kHash, kFlip, kHole>(M, s0, max_steps, snap, f0, a0);
            const int e1 = walk_step<kHash, kFlip, kHole>(M, s1, max_steps, snap, f1, a1);
            if (a0 && e0 == kStepDone) {
                *reinterpret_cast<Final*>(&states[q0]) = f0;
                a0 = false;
            }
            if (a1 && e1 == kStepDone) {
                *reinterpret_cast<Final*>(&states[q1]) = f1;
                a1 = false;
            }
            if (__popcll(__ballot(!a0)) + __popcll(__ballot(!a1)) >= stop_at) break;
        }
    }
}

template <bool kHash, bool kFlip, bool kHole>
__global__ __launch_bounds__(256) void k_walk2(DevMesh M, StateRec* states, QueueRanges R, unsigned long long* counter,
                                               int32_t max_steps, float snap, int refill_min, int nq) {
    walk_loop2<kHash, kFlip, kHole>(M, states, R, counter, max_steps, snap, refill_min, nq);
}

template <bool kHash, bool kFlip, bool kHole>
__global__ __launch_bounds__(256) void k_walk(DevMesh M, StateRec* states, QueueRanges R, unsigned long long* counter,
                                              int32_t max_steps, float snap, int refill_min, int nq, Final* fin_out) {
    walk_loop<kHash, kFlip, kHole, false>(M, states, R, counter, max_steps, snap, refill_min, nq, nullptr, nullptr,
                                          GxSink{}, nullptr, fin_out);
}

// The same walk over the backward's stacked chart states (its own symbol, so
// profiles keep the forward's walk apart).
template <bool kHash, bool kFlip, bool kHole>
__global__ __launch_bounds__(256) void k_walk_bwd(DevMesh M, StateRec* states, QueueRanges R,
                                                  unsigned long long* counter, int32_t max_steps, float snap,
                                                  int refill_min, int nq) {
    walk_loop<false, kFlip, kHole, false>(M, states, R, counter, max_steps, snap, refill_min, nq, nullptr, nullptr,
                                          GxSink{}, nullptr);
}

template <bool kFlip, bool kHole>
__global__ __launch_bounds__(256) void k_walk_gx(DevMesh M, StateRec* states, QueueRanges R, unsigned long long* counter,
                                                 int32_t max_steps, float snap, int refill_min, int nq,
                                                 const float4* cvec, double* acc, GxSink sink, uint32_t* counts,
                                                 uint32_t* used, int nbins) {
    __shared__ uint32_t lbins[kGxMaxBins + 1];   // bin counts, then the block's chunk counter
    for (int b = (int)threadIdx.x; b < nbins; b += 256) lbins[b] = 0u;
    if (threadIdx.x == 0) lbins[kGxMaxBins] = 0u;
    __syncthreads();
    walk_loop<false, kFlip, kHole, true>(M, states, R, counter, max_steps, snap, refill_min, nq, cvec, acc, sink,
                                         lbins);
    __syncthreads();
    if (sink.rec == nullptr) return;
    uint32_t* row = counts + (size_t)blockIdx.x * nbins;
    for (int b = (int)threadIdx.x; b < nbins; b += 256) row[b] = lbins[b];
    if (threadIdx.x == 0) used[blockIdx.x] = min(lbins[kGxMaxBins], (uint32_t)sink.per_block);
}

// Column b of the (walk block, bin) count matrix to exclusive prefix sums
// over the blocks (in place), and the column total to total[b].
__global__ __launch_bounds__(1024) void k_gx_colscan(uint32_t* counts, int rows, int nbins, uint32_t* total) {
    __shared__ uint32_t part[1024];
    const int b = (int)blockIdx.x, t = (int)threadIdx.x;
    const int per = (rows + 1023) / 1024;
    const int r0 = min(rows, t * per), r1 = min(rows, r0 + per);
    uint32_t sum = 0u;
    for (int r = r0; r < r1; ++r) sum += counts[(size_t)r * nbins + b];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t x = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int r = r0; r < r1; ++r) {
        const uint32_t c = counts[(size_t)r * nbins + b];
        counts[(size_t)r * nbins + b] = run;
        run += c;
    }
    if (t == 1023) total[b] = part[1023];
    if (b == 0 && t == 0) total[nbins] = 0u;
}

// Moves walk block B's records to bin order: bin b's records of block B go
// to start[b] + (records of bin b in blocks before B) onward.  The block
// takes its records in tiles of four chunks, sorts each tile by bin in LDS
// (counting sort), and writes it out so that neighbouring lanes store
// neighbouring records of one bin: whole runs instead of 24-byte pieces.
constexpr int kGxTile = 4 * kGxChunk;

// Barrier for LDS traffic only: waits for this wave's LDS operations, not for
// its outstanding global loads and stores (which __syncthreads also drains).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Exclusive prefix sums of x[0, n) in place (n <= 4 * 1024, 1024 threads),
// visible to the whole block on return; returns the total to every thread.
__device__ __forceinline__ uint32_t block_scan4096(uint32_t* x, int n, uint32_t* wsum) {
    const int t = (int)threadIdx.x, lane = t & 63, wv = t >> 6;
    uint32_t v[4], sum = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = 4 * t + k < n ? x[4 * t + k] : 0u;
        sum += v[k];
    }
    uint32_t inc = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    lds_barrier();
    uint32_t base = 0u, total = 0u;
    for (int k = 0; k < 16; ++k) {
        const uint32_t w = wsum[k];
        base += k < wv ? w : 0u;
        total += w;
    }
    uint32_t run = base + inc - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (4 * t + k < n) {
            x[4 * t + k] = run;
            run += v[k];
        }
    lds_barrier();
    return total;
}

// Exclusive prefix sums of x[0, n) in place, in three launches: each block
// scans a tile of 4,096 entries and leaves its total in tile[b]; one block
// scans the totals; each block adds its tile's offset.
__global__ __launch_bounds__(1024) void k_scan_tiles(uint32_t* x, int64_t n, uint32_t* tile) {
    __shared__ uint32_t v[4096];
    __shared__ uint32_t wsum[16];
    const int64_t o = (int64_t)blockIdx.x * 4096;
    const int m = (int)std::min<int64_t>(4096, n - o);
    for (int k = (int)threadIdx.x; k < m; k += 1024) v[k] = x[o + k];
    __syncthreads();
    const uint32_t total = block_scan4096(v, m, wsum);
    for (int k = (int)threadIdx.x; k < m; k += 1024) x[o + k] = v[k];
    if (threadIdx.x == 0) tile[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void k_scan_add(uint32_t* x, int64_t n, const uint32_t* tile) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += tile[i >> 12];
}

__global__ __launch_bounds__(1024) void k_gx_scatter(const GxRec* __restrict__ rec, const uint32_t* __restrict__ fill,
                                                     const uint32_t* __restrict__ used, int per_block, int shift,
                                                     int nbins, const uint32_t* __restrict__ start,
                                                     const uint32_t* __restrict__ counts, GxRec* __restrict__ sorted) {
    __shared__ uint2 tile[3 * kGxTile];     // records as three 8-byte words
    __shared__ uint32_t cur[kGxMaxBins];    // next global place of each bin
    __shared__ uint32_t loff[kGxMaxBins];   // the tile's counts, then their exclusive sums
    __shared__ uint32_t wsum[16];
    const int t = (int)threadIdx.x;
    const uint32_t* row = counts + (size_t)blockIdx.x * nbins;
    for (int b = t; b < nbins; b += 1024) {
        cur[b] = start[b] + row[b];
        loff[b] = 0u;
    }
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * per_block, c1 = c0 + used[blockIdx.x];
    const uint2* src = reinterpret_cast<const uint2*>(rec);
    uint2* dst = reinterpret_cast<uint2*>(sorted);
    // the next tile's records are loaded while this one is sorted and written
    // (lanes past a chunk's fill load the block's first record and drop it)
    uint2 n0[4], n1[4], n2[4];
    bool okn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        okn[j] = c0 + j < c1 && t < (int)fill[c0 + j];
        const int64_t at = 3 * (okn[j] ? (c0 + j) * kGxChunk + t : c0 * kGxChunk);
        n0[j] = src[at];
        n1[j] = src[at + 1];
        n2[j] = src[at + 2];
    }
    for (int64_t c = c0; c < c1; c += 4) {
        uint2 r0[4], r1[4], r2[4];
        bool ok[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            r0[j] = n0[j];
            r1[j] = n1[j];
            r2[j] = n2[j];
            ok[j] = okn[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            okn[j] = c + 4 + j < c1 && t < (int)fill[c + 4 + j];
            const int64_t at = 3 * (okn[j] ? (c + 4 + j) * kGxChunk + t : c0 * kGxChunk);
            n0[j] = src[at];
            n1[j] = src[at + 1];
            n2[j] = src[at + 2];
        }
        uint32_t rk[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (ok[j]) rk[j] = atomicAdd(&loff[(int)r0[j].x >> shift], 1u);
        lds_barrier();
        const uint32_t nt = block_scan4096(loff, nbins, wsum);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (ok[j]) {
                const uint32_t k = 3 * (loff[(int)r0[j].x >> shift] + rk[j]);
                tile[k] = r0[j];
                tile[k + 1] = r1[j];
                tile[k + 2] = r2[j];
            }
        lds_barrier();
        for (uint32_t i = (uint32_t)t; i < nt; i += 1024u) {
            const uint2 q0 = tile[3 * i], q1 = tile[3 * i + 1], q2 = tile[3 * i + 2];
            const int b = (int)q0.x >> shift;
            const size_t at = 3 * (size_t)(cur[b] + (i - loff[b]));
            dst[at] = q0;   // ordinary stores: L2 merges a run's pieces into whole lines
            dst[at + 1] = q1;
            dst[at + 2] = q2;
        }
        lds_barrier();
        uint32_t k4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int b = t + 1024 * k;
            k4[k] = b < nbins ? (b + 1 < nbins ? loff[b + 1] : nt) - loff[b] : 0u;
        }
        lds_barrier();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int b = t + 1024 * k;
            if (b < nbins) {
                cur[b] += k4[k];
                loff[b] = 0u;
            }
        }
        lds_barrier();
    }
}

// Sums the records of one bin (one window of kGxWindow half-edges of it per
// block) in LDS in float64 and adds the totals to the half-edge sums.  Every
// bin has one owner here, so the adds need no atomics.
__global__ __launch_bounds__(1024) void k_gx_reduce(const GxRec* sorted, const uint32_t* start, int shift,
                                                    int64_t nh, double* acc) {
    __shared__ double s[5 * kGxWindow];
    const int wpb = (1 << shift) / kGxWindow;
    const int bin = (int)blockIdx.x / wpb, win = (int)blockIdx.x - bin * wpb;
    const int64_t h0 = ((int64_t)bin << shift) + (int64_t)win * kGxWindow;
    if (h0 >= nh) return;
    const int t = (int)threadIdx.x;
    for (int k = t; k < 5 * kGxWindow; k += 1024) s[k] = 0.0;
    __syncthreads();
    const uint32_t lo = start[bin], hi = start[bin + 1];
    // four records per thread in flight: one at a time leaves the loop bound by load latency
    uint32_t i = lo + (uint32_t)t;
    for (; i + 3u * 1024u < hi; i += 4u * 1024u) {
        GxRec r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) r[j] = sorted[i + (uint32_t)j * 1024u];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t d = (int64_t)r[j].h - h0;
            if (d >= 0 && d < kGxWindow)
                for (int k = 0; k < 5; ++k) atomicAdd(&s[5 * d + k], (double)r[j].q[k]);
        }
    }
    for (; i < hi; i += 1024u) {
        const GxRec r = sorted[i];
        const int64_t d = (int64_t)r.h - h0;
        if (d >= 0 && d < kGxWindow)
            for (int k = 0; k < 5; ++k) atomicAdd(&s[5 * d + k], (double)r.q[k]);
    }
    __syncthreads();
    const int64_t n5 = min((int64_t)5 * kGxWindow, 5 * (nh - h0));
    for (int64_t k = t; k < n5; k += 1024) {
        const double x = s[k];
        if (x != 0.0) acc[5 * h0 + k] += x;
    }
}

// ---------------------------------------------------------------- partitioned form
// The mesh is cut into kParts spatial parts (contiguous internal face
// ranges).  Blocks are dealt to the XCDs round-robin, so block b runs on XCD
// b % kParts and serves part b % kParts, whose records then stay in that XCD's
// L2.  The walk runs in rounds, one launch each.  Every ray carries a one-byte
// tag, (round << 3) | part of its current chart, or kTagDone.  In round r the
// waves of part p scan the tags in slices claimed from a per-part counter,
// collect the rays tagged (r, p) in a per-wave list in LDS, and walk each
// until it ends or leaves the part; a ray that leaves is tagged (r + 1, its
// new part).  The round stamp keeps a tag written during a round from being
// taken in the same round; the next launch sees the ray's state.  The last
// round walks every remaining ray to its end.
constexpr uint8_t kTagDone = 0xffu;
constexpr int kSlice = 2048;   // tags per claimed slice (also the per-wave list capacity)

SG_HD __forceinline__ int part_of(const DevMesh& M, int32_t h) {
    int p = 0;
#pragma unroll
    for (int k = 1; k < kParts; ++k) p += h >= M.part_he[k] ? 1 : 0;
    return p;
}

__global__ __launch_bounds__(256) void k_rounds_reset(unsigned long long* ctr, int n) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) ctr[i] = 0ull;
}

// Initial chart state of every ray (as k_init), tagged (0, part of its first chart).
template <bool kHash>
__global__ __launch_bounds__(256) void k_init_rounds(DevMesh M, ExpArgs a, StateRec* states, float* aux,
                                                     uint64_t* hashes, uint8_t* tags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    Ray st;
    float L = 0.f;
    const int ir = ray_init(M, a.f[i], a.b + 3 * i, a.v + 3 * i, st, L);
    StateRec rec;
    uint8_t tag = kTagDone;
    if (ir != kInitOk) {
        write_unwalked(M, a, i, ir == kInitBad);
        rec.h = -1;
        rec.s = rec.t = rec.Lhi = rec.Llo = 0.f;
        rec.phi = rec.flags = 0u;
        rec.ncross = 0;
    } else {
        rec = pack_state(st);
        float* x = aux + i * (1 + 2 * (int64_t)a.K);
        x[0] = L;
        if (a.K > 0) {
            float3 d0, q0;
            start_tangent_frame(M, a, i, d0, q0);
            for (int kk = 0; kk < a.K; ++kk) {
                const float3 w = ld3(a.W + 3 * (i * a.K + kk));
                x[1 + 2 * kk] = dot(w, d0);
                x[2 + 2 * kk] = dot(w, q0);
            }
        }
        if (kHash) hashes[i] = st.hash;
        tag = (uint8_t)part_of(M, st.h);
    }
    states[i] = rec;
    tags[i] = tag;
}

// One round (see above).  slice_ctr: this round's per-part slice counters.
template <bool kHash, bool kFlip, bool kHole>
__global__ __launch_bounds__(256) void k_walk_round(DevMesh M, StateRec* states, uint64_t* hashes, uint8_t* tags,
                                                    unsigned long long* slice_ctr, int64_t n, int32_t max_steps,
                                                    float snap, int refill_min, int round, int restrict_part) {
    __shared__ int32_t lists[4][kSlice];
    const int lane = (int)(threadIdx.x & 63u);
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int32_t* list = lists[threadIdx.x >> 6];
    const int home = (int)(blockIdx.x % kParts);
    const uint8_t want = (uint8_t)((round << 3) | home);
    const int32_t lo = M.part_he[home], hi = M.part_he[home + 1];
    bool active = false, exhausted = false;
    int list_n = 0, list_pos = 0;
    int32_t ray = 0;
    Ray st;
    st.h = 0; st.s = st.t = st.Lhi = st.Llo = st.bias = 0.f; st.phi = st.par = 0u; st.ncross = 0; st.hash = 0ull;
    for (;;) {
        const uint64_t idle = __ballot(!active);
        const int nidle = __popcll(idle);
        const bool drained = exhausted && list_pos == list_n;
        if (nidle == 64 && drained) break;
        if (!drained && nidle >= refill_min) {
            while (list_pos == list_n && !exhausted) {
                // claim a slice of tags and list the rays of this part and round
                unsigned long long base = 0ull;
                if (lane == 0) base = atomicAdd(&slice_ctr[home], (unsigned long long)kSlice);
                base = __shfl(base, 0);
                if (base >= (unsigned long long)n) {
                    exhausted = true;
                    break;
                }
                list_n = 0;
                list_pos = 0;
                for (int j = 0; j < kSlice; j += 64) {
                    const int64_t idx = (int64_t)base + j + lane;
                    const bool match = idx < n && tags[idx] == want;
                    const uint64_t m = __ballot(match);
                    if (match) list[list_n + __popcll(m & below)] = (int32_t)idx;
                    list_n += __popcll(m);
                }
            }
            if (!active) {
                const int k = list_pos + __popcll(idle & below);
                if (k < list_n) {
                    ray = list[k];
                    unpack_state(states[ray], st);
                    st.hash = kHash ? hashes[ray] : 0ull;
                    active = true;
                }
            }
            list_pos = min(list_n, list_pos + nidle);
        }
        const int stop_at = (exhausted && list_pos == list_n) ? 64 : refill_min;
        for (;;) {
            if (active) {
                Final fin;
                if (walk_step<kHash, kFlip, kHole>(M, st, max_steps, snap, fin) == kStepDone) {
                    *reinterpret_cast<Final*>(&states[ray]) = fin;
                    tags[ray] = kTagDone;
                    active = false;
                } else if (restrict_part && (st.h < lo || st.h >= hi)) {
                    states[ray] = pack_state(st);
                    if (kHash) hashes[ray] = st.hash;
                    tags[ray] = (uint8_t)(((round + 1) << 3) | part_of(M, st.h));
                    active = false;
                }
            }
            if (__popcll(__ballot(!active)) >= stop_at) break;
        }
    }
}

__global__ __launch_bounds__(256) void k_finish(DevMesh M, ExpArgs a, const StateRec* states, const uint64_t* hashes,
                                                const float* aux, const int32_t* slot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int64_t at = slot ? (int64_t)slot[i] : i;
    // every walk kernel runs each of its rays to a Final record (the step cap
    // included), which overwrites the start state in place; h < 0 marks a query
    // with no walk, whose outputs k_init wrote
    Final fin = *reinterpret_cast<const Final*>(&states[at]);
    if (fin.h < 0) return;
    if (hashes) fin.hash = hashes[i];
    if (aux) {
        const float* x = aux + i * (1 + 2 * (int64_t)a.K);
        write_final(M, a, i, fin, x[0], x);
    } else {
        write_final(M, a, i, fin, tangent_length(M, a, i));
    }
}


// ---------------------------------------------------------------- backward
// Point of a finished walk as an offset from `o` (a vertex near it): the
// finite differences of the geodesic scheme subtract nearby points, so they
// are formed from small local vectors rather than from rounded 3D positions.
SG_HD __forceinline__ float3 final_offset(const DevMesh& M, const Final& fin, float3 o, int32_t& fe_out) {
    const int32_t fe = fin.h / 3;
    const int ke = fin.h - 3 * fe;
    const HalfEdgeRec r = rec_geo(M, fin.h);
    const int64_t f3 = 3 * (int64_t)fe;
    const float3 y0 = sub(fvx(M, f3 / 3, 0), o);
    const float3 y1 = sub(fvx(M, f3 / 3, 1), o);
    const float3 y2 = sub(fvx(M, f3 / 3, 2), o);
    const float ell = r.lab;
    float b0, b1, b2;
    chart_bary(r, ell, fin.ex, fin.ey, ke, b0, b1, b2);
    fe_out = fe;
    return make_float3(fmaf(b0, y0.x, fmaf(b1, y1.x, b2 * y2.x)), fmaf(b0, y0.y, fmaf(b1, y1.y, b2 * y2.y)),
                       fmaf(b0, y0.z, fmaf(b1, y1.z, b2 * y2.z)));
}

// Tangent and orientation-consistent normal at the end of a walk.
SG_HD __forceinline__ void final_frame(const DevMesh& M, const Final& fin, float3& d3, float3& n3) {
    const int32_t fe = fin.h / 3;
    const int ke = fin.h - 3 * fe;
    const int64_t f3 = 3 * (int64_t)fe;
    const float3 ya = fvx(M, f3 / 3, ke);
    const float3 yb = fvx(M, f3 / 3, (ke + 1) % 3);
    const float3 yc = fvx(M, f3 / 3, (ke + 2) % 3);
    const float3 eab = sub(yb, ya);
    const float3 ex3 = nrm(eab);
    n3 = nrm(crs(eab, sub(yc, ya)));
    const float3 ey3 = crs(n3, ex3);
    float sn, cs;
    sincos_fx(fin.phi, sn, cs);
    d3 = make_float3(fmaf(cs, ex3.x, sn * ey3.x), fmaf(cs, ex3.y, sn * ey3.y), fmaf(cs, ex3.z, sn * ey3.z));
    if (fin.flags & kParity) n3 = scl(n3, -1.0f);
}

SG_HD __forceinline__ Final as_final(const StateRec& r) { return *reinterpret_cast<const Final*>(&r); }

SG_HD __forceinline__ StateRec dead_state() {
    StateRec r;
    r.h = -1; r.s = r.t = r.Lhi = r.Llo = 0.f; r.phi = r.flags = 0u; r.ncross = 0;
    return r;
}

// The query's start frame, direction angle phi0 (chart of half-edge 3 f) and
// length; |v_t| = 0 takes the chart's x-axis (e_u) as its direction.
SG_HD __forceinline__ int bwd_query(const DevMesh& M, const BwdArgs& a, int64_t i, StartFrame& S, uint32_t& phi0,
                                    float& L, float* Llo_out = nullptr) {
    if (start_frame(M, a.f[i], a.b + 3 * i, S) != kInitOk) return kInitBad;
    const float3 v = ld3(a.v + 3 * i);
    if (!__builtin_isfinite(v.x) || !__builtin_isfinite(v.y) || !__builtin_isfinite(v.z)) return kInitBad;
    float Llo;
    start_direction(M, S.f, v, L, Llo, phi0);
    if (Llo_out) *Llo_out = Llo;
    return kInitOk;
}

SG_HD __forceinline__ void nan_grads(const BwdArgs& a, int64_t i) {
    const float nan = __builtin_nanf("");
    for (int c = 0; c < 3; ++c) { a.grad_v[3 * i + c] = nan; a.grad_b[3 * i + c] = nan; }
    if (a.g_W)
        for (int k = 0; k < 3 * a.K; ++k) a.grad_W[3 * (i * a.K) + k] = nan;
}

// dL/dp' of query i, with the cotangent of the end barycentrics folded in:
// inside end face fe (internal id; vertices y0, y1, y2), b'_k has the in-plane
// gradient n x (y_{k+2} - y_{k+1}) / (2 A), n the unit normal of
// (y1 - y0) x (y2 - y0) and 2 A its length.
SG_HD __forceinline__ float3 load_g(const DevMesh& M, const BwdArgs& a, int64_t i, int32_t fe) {
    float3 g = a.g ? ld3(a.g + 3 * i) : make_float3(0.f, 0.f, 0.f);
    if (a.g_bo && fe >= 0) {
        const int64_t f3 = 3 * (int64_t)fe;
        const float3 y0 = fvx(M, f3 / 3, 0);
        const float3 y1 = fvx(M, f3 / 3, 1);
        const float3 y2 = fvx(M, f3 / 3, 2);
        const float3 c = crs(sub(y1, y0), sub(y2, y0));
        const float inv = 1.0f / dot(c, c);   // n / (2A) = c / |c|^2
        const float3 gb = ld3(a.g_bo + 3 * i);
        const float3 e = make_float3(gb.x * inv, gb.y * inv, gb.z * inv);
        const float3 t0 = crs(c, sub(y2, y1)), t1 = crs(c, sub(y0, y2)), t2 = crs(c, sub(y1, y0));
        g = make_float3(g.x + e.x * t0.x + e.y * t1.x + e.z * t2.x, g.y + e.x * t0.y + e.y * t1.y + e.z * t2.y,
                        g.z + e.x * t0.z + e.y * t1.z + e.z * t2.z);
    }
    return g;
}

// Cotangents of the transported outputs (an extension of the paper's
// backward).  The walk carries the frame (d, n x d) from (e_par, e_perp) at p
// to (d', q' = n' x d') at p' (Sec. 4 "Parallel Transport": a transported
// vector keeps its angle to the tangent), so W'_k = R W_k and v' = R v_t with
// R that frame map, constant wherever the face sequence is.  dL/dv gains
// R^T g_v and dL/dW_k = R^T g_Wk, both in the start face's plane (v and W are
// projected onto it first).  ident (|v_t| = 0: nothing moves): R = I, and
// the cotangents are projected with the start normal n0.
SG_HD __forceinline__ void transport_cot(const BwdArgs& a, int64_t i, bool ident, float3 epar, float3 eperp, float3 d3,
                                         float3 q3, float3 n0) {
    auto back = [&](float3 g) {
        if (ident) return sub(g, scl(n0, dot(g, n0)));
        const float c0 = dot(g, d3), c1 = dot(g, q3);
        return make_float3(fmaf(c0, epar.x, c1 * eperp.x), fmaf(c0, epar.y, c1 * eperp.y),
                           fmaf(c0, epar.z, c1 * eperp.z));
    };
    if (a.g_v) {
        const float3 t = back(ld3(a.g_v + 3 * i));
        a.grad_v[3 * i] += t.x; a.grad_v[3 * i + 1] += t.y; a.grad_v[3 * i + 2] += t.z;
    }
    if (a.g_W)
        for (int k = 0; k < a.K; ++k) {
            const int64_t j = 3 * (i * a.K + k);
            const float3 t = back(ld3(a.g_W + j));
            a.grad_W[j] = t.x; a.grad_W[j + 1] = t.y; a.grad_W[j + 2] = t.z;
        }
}

// Stage 1: the walks that start at p.  Slot 0 recomputes Exp(p, v) (unless
// the base geodesic's end is the forward's); for the geodesic finite
// differences (eqs. jv, jp) the next slot is Exp(p, v + eps_v e_perp), and the
// short walks Exp(p, eps_p e_u), Exp(p, eps_p e_v) go to sh[3 i], sh[3 i + 1]
// (query order), which a one-lane-per-walk kernel finishes: they rarely leave
// their face, and in the persistent pass each took a refill slot beside the
// long walks.  The perturbations are applied to the fixed-point angle and the
// compensated length, so the perturbed walks share the base walk's rounding.
// Position of query i in the backward's walk arrays (spatial order when sorted).
SG_HD __forceinline__ int64_t bwd_at(const BwdArgs& a, int64_t i) { return a.slot ? (int64_t)a.slot[i] : i; }

SG_HD void bwd_stage1(const DevMesh& M, const BwdArgs& a, StateRec* s1, int per_ray, StateRec* sh, int64_t i) {
    StateRec* out = s1 + (int64_t)per_ray * bwd_at(a, i);
    StartFrame S;
    uint32_t phi0;
    float L;
    Ray st;
    float Llo = 0.f;
    if (bwd_query(M, a, i, S, phi0, L, &Llo) != kInitOk) {
        for (int j = 0; j < per_ray; ++j) out[j] = dead_state();
        if (sh) sh[3 * i] = sh[3 * i + 1] = dead_state();
        return;
    }
    if (!sh || !a.gfd_saved) {   // the base geodesic (with GFD, unless its end is the forward's, saved)
        out[0] = enter_face(M, S.f, 0, S.l0, S.b0, S.b1, S.b2, phi0, L, Llo, st) == kInitOk ? pack_state(st)
                                                                                          : dead_state();
        if (!sh) return;
        ++out;
    }
    const float ev = a.eps_v, ep = a.eps_p;
    // |v + eps e_perp| = L + eps^2 / (L + sqrt(L^2 + eps^2)), angle + atan(eps / L)
    const float Lp = sqrtf(fmaf(L, L, ev * ev));
    const float dl = ev * ev / (L + Lp);
    const uint32_t dphi = rad_to_fx(atan2f(ev, L));
    out[0] = enter_face(M, S.f, 0, S.l0, S.b0, S.b1, S.b2, phi0 + dphi, L, Llo + dl, st) == kInitOk ? pack_state(st)
                                                                                                       : dead_state();
    sh[3 * i] = enter_face(M, S.f, 0, S.l0, S.b0, S.b1, S.b2, 0u, ep, 0.f, st) == kInitOk ? pack_state(st)
                                                                                          : dead_state();
    const uint32_t Av = rec_geo(M, 3 * S.f).A;   // angle of e_v = unit(x2 - x0) in the chart
    sh[3 * i + 1] = enter_face(M, S.f, 0, S.l0, S.b0, S.b1, S.b2, Av, ep, 0.f, st) == kInitOk ? pack_state(st)
                                                                                              : dead_state();
}

// The end of the base geodesic from the forward's saved outputs: the chart of
// half-edge 3 f' (x-axis along y1 - y0), the point from b' and the angle of
// v' in that chart (the start chart's x-axis when |v_t| = 0, as the walk
// keeps it); h < 0 when the saved end is unusable.
SG_HD __forceinline__ Final saved_final(const DevMesh& M, const BwdArgs& a, int64_t i) {
    Final F;
    F.h = -1;
    F.ex = F.ey = 0.f;
    F.phi = 0u;
    F.flags = 0u;
    F.ncross = 0;
    F.hash = 0ull;
    const int32_t fo = a.f_out[i];
    if (fo < 0 || (int64_t)fo >= M.n_faces) return F;
    const int32_t fe = M.perm[fo];
    const float b0 = a.b_out[3 * i], b1 = a.b_out[3 * i + 1], b2 = a.b_out[3 * i + 2];
    const float bs = b0 + b1 + b2;
    if (!(bs > 0.f) || !__builtin_isfinite(bs)) return F;
    const HalfEdgeRec r = rec_geo(M, 3 * fe);
    F.h = 3 * fe;
    F.ex = fmaf(b1 / bs, r.lab, (b2 / bs) * r.cx);
    F.ey = (b2 / bs) * r.cy;
    float Lo, Llo;
    uint32_t ph;
    start_direction(M, fe, ld3(a.v_out + 3 * i), Lo, Llo, ph);
    F.phi = Lo > 0.f ? ph : 0u;
    F.flags = kDoneBit | ((uint32_t)kRayOk << 8);
    return F;
}

// Stage 2: the walks that start where stage 1's ended.  With do_shift, the
// long Exp(p_u, v_u), Exp(p_v, v_v) from the ends of the two short start-point
// walks, with v transported along them (it keeps its angle to their tangent),
// to the last two of the query's per_ray long-walk slots; they need nothing
// from the base geodesic, so they join its pass.  With do_par, the short walk
// Exp(p', Pi(eps_v e_par)) along the transported tangent from the base's end
// (the forward's, or slot 0 once walked), to sh[3 i + 2].
SG_HD void bwd_stage2(const DevMesh& M, const BwdArgs& a, StateRec* s1, int per_ray, StateRec* sh, bool do_shift,
                      bool do_par, int64_t i) {
    const int64_t at = bwd_at(a, i);
    StateRec* out = s1 + (int64_t)per_ray * at + (per_ray - 2);
    StartFrame S;
    uint32_t phi0;
    float L;
    Ray st;
    Final F0{}, Fu{}, Fv{};
    if (do_par) F0 = a.gfd_saved ? saved_final(M, a, i) : as_final(s1[(int64_t)per_ray * at]);
    if (do_shift) {
        Fu = as_final(sh[3 * i]);
        Fv = as_final(sh[3 * i + 1]);
    }
    if (bwd_query(M, a, i, S, phi0, L) != kInitOk || F0.h < 0 || Fu.h < 0 || Fv.h < 0) {
        if (do_par) sh[3 * i + 2] = dead_state();
        if (do_shift) out[0] = out[1] = dead_state();
        return;
    }
    if (do_par)
        sh[3 * i + 2] = enter_chart(M, F0.h, F0.ex, F0.ey, F0.phi, a.eps_v, 0.f, st) == kInitOk ? pack_state(st)
                                                                                              : dead_state();
    if (!do_shift) return;
    const uint32_t psi_u = phi0;                              // v relative to e_u
    const uint32_t psi_v = phi0 - rec_geo(M, 3 * S.f).A;       // v relative to e_v
    const uint32_t du = (Fu.flags & kParity) ? Fu.phi - psi_u : Fu.phi + psi_u;
    const uint32_t dv = (Fv.flags & kParity) ? Fv.phi - psi_v : Fv.phi + psi_v;
    out[0] = enter_chart(M, Fu.h, Fu.ex, Fu.ey, du, L, 0.f, st) == kInitOk ? pack_state(st) : dead_state();
    out[1] = enter_chart(M, Fv.h, Fv.ex, Fv.ey, dv, L, 0.f, st) == kInitOk ? pack_state(st) : dead_state();
}

// Projection of an ambient vector onto the non-orthogonal frame [e_u, e_v]
// of face f (M^dagger = (M^T M)^-1 M^T, Sec. 4 "Differentiation via GFD").
SG_HD __forceinline__ float2 pinv_uv(float3 eu, float3 ev, float3 w) {
    const float a = dot(eu, eu), b = dot(eu, ev), d = dot(ev, ev);
    const float r1 = dot(eu, w), r2 = dot(ev, w);
    const float idet = 1.0f / fmaf(a, d, -b * b);
    return make_float2(fmaf(d, r1, -b * r2) * idet, fmaf(a, r2, -b * r1) * idet);
}

SG_HD __forceinline__ void face_uv(const DevMesh& M, int32_t f, float3& x0, float3& eu, float3& ev) {
    const int64_t f3 = 3 * (int64_t)f;
    x0 = fvx(M, f3 / 3, 0);
    eu = nrm(sub(fvx(M, f3 / 3, 1), x0));
    ev = nrm(sub(fvx(M, f3 / 3, 2), x0));
}

// Assembly (eqs. jv, jp, chain): finite-difference columns, projected on the
// end face's [e_u', e_v'] frame, contracted with the upstream gradient g.
SG_HD void gfd_assemble(const DevMesh& M, const BwdArgs& a, const StateRec* s1, const StateRec* sh, int64_t i) {
    StartFrame S;
    uint32_t phi0;
    float L;
    const int64_t at = bwd_at(a, i);
    // the long walks of a query: (base,) e_perp, the two shifted ones; the base's
    // end is the forward's when saved
    const int per = a.gfd_saved ? 3 : 4;
    const StateRec* q = s1 + (int64_t)per * at + (per - 3);
    const Final F0 = a.gfd_saved ? saved_final(M, a, i) : as_final(s1[(int64_t)per * at]);
    const Final Fp = as_final(q[0]), Fu = as_final(q[1]), Fv = as_final(q[2]);
    const Final Fq = as_final(sh[3 * i + 2]);
    if (bwd_query(M, a, i, S, phi0, L) != kInitOk || F0.h < 0 || Fp.h < 0 || Fq.h < 0 || Fu.h < 0 || Fv.h < 0) {
        nan_grads(a, i);
        return;
    }
    float3 o, eu2, ev2;
    face_uv(M, F0.h / 3, o, eu2, ev2);
    int32_t ft;
    const float3 q0 = final_offset(M, F0, o, ft);
    const float iv = 1.0f / a.eps_v, ip = 1.0f / a.eps_p;
    const float3 cpar = scl(sub(final_offset(M, Fq, o, ft), q0), iv);
    const float3 cperp = scl(sub(final_offset(M, Fp, o, ft), q0), iv);
    const float3 cu = scl(sub(final_offset(M, Fu, o, ft), q0), ip);
    const float3 cv = scl(sub(final_offset(M, Fv, o, ft), q0), ip);
    const float2 j0 = pinv_uv(eu2, ev2, cpar), j1 = pinv_uv(eu2, ev2, cperp);   // J^v columns
    const float2 k0 = pinv_uv(eu2, ev2, cu), k1 = pinv_uv(eu2, ev2, cv);         // J^p columns
    const float3 g = load_g(M, a, i, F0.h / 3);
    const float h0 = dot(eu2, g), h1 = dot(ev2, g);
    // J^T (M'^T g)
    const float c0 = fmaf(j0.x, h0, j0.y * h1), c1 = fmaf(j1.x, h0, j1.y * h1);
    const float d0 = fmaf(k0.x, h0, k0.y * h1), d1 = fmaf(k1.x, h0, k1.y * h1);
    float sn, cs;
    sincos_full(phi0, sn, cs);
    const float3 epar = make_float3(fmaf(cs, S.ex.x, sn * S.ey.x), fmaf(cs, S.ex.y, sn * S.ey.y),
                                    fmaf(cs, S.ex.z, sn * S.ey.z));
    const float3 eperp = crs(S.n, epar);
    for (int c = 0; c < 3; ++c) {
        const float ep_c = c == 0 ? epar.x : (c == 1 ? epar.y : epar.z);
        const float eq_c = c == 0 ? eperp.x : (c == 1 ? eperp.y : eperp.z);
        a.grad_v[3 * i + c] = fmaf(c0, ep_c, c1 * eq_c);
    }
    // start-point gradient G in the face plane with [e_u e_v]^T G = (d0, d1)
    const float3 su = S.ex;
    const int64_t f3 = 3 * (int64_t)S.f;
    const float3 x1 = fvx(M, f3 / 3, 1);
    const float3 x2 = fvx(M, f3 / 3, 2);
    const float3 sv = nrm(sub(x2, S.x0));
    const float ga = dot(su, su), gb = dot(su, sv), gd = dot(sv, sv);
    const float idet = 1.0f / fmaf(ga, gd, -gb * gb);
    const float y0 = fmaf(gd, d0, -gb * d1) * idet, y1 = fmaf(ga, d1, -gb * d0) * idet;
    const float3 G = make_float3(fmaf(y0, su.x, y1 * sv.x), fmaf(y0, su.y, y1 * sv.y), fmaf(y0, su.z, y1 * sv.z));
    a.grad_b[3 * i] = dot(G, S.x0);
    a.grad_b[3 * i + 1] = dot(G, x1);
    a.grad_b[3 * i + 2] = dot(G, x2);
    if (a.g_v || a.g_W) {
        float3 d3, n3;
        final_frame(M, F0, d3, n3);
        transport_cot(a, i, !(L > 0.f), epar, eperp, d3, crs(n3, d3), S.n);
    }
}

// Extrinsic proxy (eq. proxy_func): J^v = R = M_{p'} M_p^T with frames
// [e_par, e_perp, n], J^p = 0.  grad_v = R^T g = M_p (M_{p'}^T g).
SG_HD __forceinline__ void ep_grad(const DevMesh& M, const BwdArgs& a, int64_t i, const StartFrame& S, uint32_t phi0,
                                   float3 d3, float3 n3, int32_t fe) {
    const float3 g = load_g(M, a, i, fe);
    float sn, cs;
    sincos_full(phi0, sn, cs);
    const float3 epar = make_float3(fmaf(cs, S.ex.x, sn * S.ey.x), fmaf(cs, S.ex.y, sn * S.ey.y),
                                    fmaf(cs, S.ex.z, sn * S.ey.z));
    const float3 eperp = crs(S.n, epar);
    const float3 q = crs(n3, d3);
    const float a0 = dot(d3, g), a1 = dot(q, g), a2 = dot(n3, g);
    a.grad_v[3 * i] = fmaf(a0, epar.x, fmaf(a1, eperp.x, a2 * S.n.x));
    a.grad_v[3 * i + 1] = fmaf(a0, epar.y, fmaf(a1, eperp.y, a2 * S.n.y));
    a.grad_v[3 * i + 2] = fmaf(a0, epar.z, fmaf(a1, eperp.z, a2 * S.n.z));
    a.grad_b[3 * i] = a.grad_b[3 * i + 1] = a.grad_b[3 * i + 2] = 0.f;
    transport_cot(a, i, false, epar, eperp, d3, q, S.n);
}

// |v_t| = 0: nothing moves (R = I).
SG_HD __forceinline__ void ep_identity(const DevMesh& M, const BwdArgs& a, int64_t i, const StartFrame& S) {
    const float3 g = load_g(M, a, i, S.f);
    a.grad_v[3 * i] = g.x; a.grad_v[3 * i + 1] = g.y; a.grad_v[3 * i + 2] = g.z;
    a.grad_b[3 * i] = a.grad_b[3 * i + 1] = a.grad_b[3 * i + 2] = 0.f;
    const float3 z = make_float3(0.f, 0.f, 0.f);
    transport_cot(a, i, true, z, z, z, z, S.n);
}

// EP from the saved forward outputs (orientable meshes: the end normal is the
// end face's own normal).
SG_HD void ep_saved(const DevMesh& M, const BwdArgs& a, int64_t i) {
    StartFrame S;
    uint32_t phi0;
    float L;
    const int32_t fo = a.f_out[i];
    if (bwd_query(M, a, i, S, phi0, L) != kInitOk || fo < 0 || (int64_t)fo >= M.n_faces) {
        nan_grads(a, i);
        return;
    }
    const float3 vo = ld3(a.v_out + 3 * i);
    const float lo = sqrtf(dot(vo, vo));
    if (!(L > 0.f) || !(lo > 0.f)) {   // |v| = 0: R = I
        ep_identity(M, a, i, S);
        return;
    }
    const int64_t f3 = 3 * (int64_t)M.perm[fo];
    const float3 y0 = fvx(M, f3 / 3, 0);
    const float3 y1 = fvx(M, f3 / 3, 1);
    const float3 y2 = fvx(M, f3 / 3, 2);
    ep_grad(M, a, i, S, phi0, scl(vo, 1.0f / lo), nrm(crs(sub(y1, y0), sub(y2, y0))), M.perm[fo]);
}

// EP from a recomputed walk (meshes whose faces disagree in orientation: the
// end normal's sign comes from the walk's orientation parity).
SG_HD void ep_walked(const DevMesh& M, const BwdArgs& a, const StateRec* s1, int stride, int64_t i) {
    StartFrame S;
    uint32_t phi0;
    float L;
    const Final F0 = as_final(s1[(int64_t)stride * bwd_at(a, i)]);
    if (bwd_query(M, a, i, S, phi0, L) != kInitOk || F0.h < 0) {
        nan_grads(a, i);
        return;
    }
    if (!(L > 0.f)) {
        ep_identity(M, a, i, S);
        return;
    }
    float3 d3, n3;
    final_frame(M, F0, d3, n3);
    ep_grad(M, a, i, S, phi0, d3, n3, F0.h / 3);
}

// ---------------------------------------------------------------- vertex-position gradient
// (an extension: the paper differentiates in v and p only).  Away from
// vertices p' = H_m o ... o H_1(p + v_t), H_j the rigid unfolding about the
// j-th crossed edge, so for L = g . p'
//   dL = lambda_0 . d(p + v_t) + sum_j [ ((I - Q_j)^T lambda_j) . da_j
//                                         + dw_j . ((y_j - a_j) x lambda_j) ],
// lambda_j = Q_j ... Q_1 R^T g, dw_j the infinitesimal rotation of hinge j
// (the rotation rate of the entered face's edge frame minus that of the face
// left, carried over the hinge).  The walk adds each crossing's terms to sums
// of the entered half-edge; one pass over half-edges then maps the sums to
// the four hinge vertices in float64.

// Start term and the walk's initial state; c = components of g on the end frame
// [d', nu' x d', nu'] of the base walk (slot `stride * i` of s1).
// The start term (the query's terms on its start face's three vertices) goes
// to sterm[i] (nine floats), counted per start face in fcnt with the query's
// rank in srank[i] (-1: no start term), so the face pass can gather it.
SG_HD void gradx_init(const DevMesh& M, const BwdArgs& a, const StateRec* s1, int stride, StateRec* s3, float4* cvec,
                      float* sterm, int32_t* srank, uint32_t* fcnt, int64_t i) {
    const int64_t at = bwd_at(a, i);
    s3[at] = dead_state();
    srank[i] = -1;
    StartFrame S;
    uint32_t phi0;
    float L, Llo = 0.f;
    if (bwd_query(M, a, i, S, phi0, L, &Llo) != kInitOk) return;
    float3 d3, n3;
    int32_t fe;
    if (s1) {   // the end frame of the base re-walk
        const Final F0 = as_final(s1[(int64_t)stride * at]);
        if (F0.h < 0 || ((F0.flags >> 8) & 0xffu) != (uint32_t)kRayOk) return;
        if (F0.flags & kBndBit) return;   // slid along a boundary: not a chain of hinges
        final_frame(M, F0, d3, n3);
        fe = F0.h / 3;
    } else {    // the end frame from the forward's saved outputs (faces agree in orientation, no slides)
        if (a.status_in[i] != kRayOk) return;
        const int32_t fo = a.f_out[i];
        if (fo < 0 || (int64_t)fo >= M.n_faces) return;
        fe = M.perm[fo];
        const float3 vo = ld3(a.v_out + 3 * i);
        const float lo = sqrtf(dot(vo, vo));
        if (L > 0.f && lo > 0.f) {
            d3 = scl(vo, 1.0f / lo);
        } else {   // |v_t| = 0: the start chart's direction (phi0), as the base walk keeps it
            float sn, cs;
            sincos_full(phi0, sn, cs);
            d3 = make_float3(fmaf(cs, S.ex.x, sn * S.ey.x), fmaf(cs, S.ex.y, sn * S.ey.y),
                             fmaf(cs, S.ex.z, sn * S.ey.z));
        }
        const int64_t f3 = 3 * (int64_t)fe;
        const float3 y0 = fvx(M, f3 / 3, 0);
        n3 = nrm(crs(sub(fvx(M, f3 / 3, 1), y0), sub(fvx(M, f3 / 3, 2), y0)));
    }
    const float3 g = load_g(M, a, i, fe);
    const float4 c = make_float4(dot(g, d3), dot(g, crs(n3, d3)), dot(g, n3), 0.f);
    if (c.x == 0.f && c.y == 0.f && c.z == 0.f) return;   // g = 0: nothing to add
    float sn, cs;
    sincos_full(phi0, sn, cs);
    const float3 d0 = make_float3(fmaf(cs, S.ex.x, sn * S.ey.x), fmaf(cs, S.ex.y, sn * S.ey.y),
                                  fmaf(cs, S.ex.z, sn * S.ey.z));
    const float3 q0 = crs(S.n, d0);
    const float3 lam = make_float3(fmaf(c.x, d0.x, fmaf(c.y, q0.x, c.z * S.n.x)),
                                   fmaf(c.x, d0.y, fmaf(c.y, q0.y, c.z * S.n.y)),
                                   fmaf(c.x, d0.z, fmaf(c.y, q0.z, c.z * S.n.z)));
    // d(p + v_t): p = sum b_k x_k, and v_t = v - (v . n) n turns with the start
    // face's normal; with w = (lambda . n) v + (v . n) lambda its term is -w . dn,
    // dn = -alpha u - beta m for the plane tilt alpha = (h1 - h0)/l,
    // beta = (h2 - h0 - alpha cx)/cy of normal offsets h_k.
    const float3 v = ld3(a.v + 3 * i);
    const float vn = dot(v, S.n), ln = dot(lam, S.n);
    const float3 w = make_float3(fmaf(ln, v.x, vn * lam.x), fmaf(ln, v.y, vn * lam.y), fmaf(ln, v.z, vn * lam.z));
    const float wu = dot(w, S.ex), wm = dot(w, S.ey);
    const int64_t f3 = 3 * (int64_t)S.f;
    const float3 e2 = sub(fvx(M, f3 / 3, 2), S.x0);
    const float cx = dot(e2, S.ex), cy = dot(e2, S.ey);
    const float dh1 = wu / S.l0 - wm * cx / (S.l0 * cy);
    const float dh2 = wm / cy;
    const float dh[3] = {-(dh1 + dh2), dh1, dh2};
    const float bk[3] = {S.b0, S.b1, S.b2};
    float* q = sterm + 9 * i;
    for (int k = 0; k < 3; ++k) {
        q[3 * k] = fmaf(bk[k], lam.x, dh[k] * S.n.x);
        q[3 * k + 1] = fmaf(bk[k], lam.y, dh[k] * S.n.y);
        q[3 * k + 2] = fmaf(bk[k], lam.z, dh[k] * S.n.z);
    }
    srank[i] = (int32_t)atomicAdd(&fcnt[S.f], 1u);
    if (!(L > 0.f)) return;
    Ray st;
    if (enter_face(M, S.f, 0, S.l0, S.b0, S.b1, S.b2, phi0, L, Llo, st) != kInitOk) return;
    s3[at] = pack_state(st);
    cvec[at] = c;
}

struct D3 { double x, y, z; };
SG_HD __forceinline__ D3 dld(const float* p) { return D3{(double)p[0], (double)p[1], (double)p[2]}; }
SG_HD __forceinline__ D3 dsub(D3 a, D3 b) { return D3{a.x - b.x, a.y - b.y, a.z - b.z}; }
SG_HD __forceinline__ double ddot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
SG_HD __forceinline__ D3 dcrs(D3 a, D3 b) { return D3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
SG_HD __forceinline__ D3 dscl(D3 a, double s) { return D3{a.x * s, a.y * s, a.z * s}; }
SG_HD __forceinline__ D3 dmad(D3 a, double s, D3 b) { return D3{a.x + s * b.x, a.y + s * b.y, a.z + s * b.z}; }

// Edge pass: half-edge h (entered from its twin's face).  The rotation rate of
// a face's edge frame (u, m toward the apex, n = u x m) under normal offsets
// h_a, h_b, h_c of its vertices and an in-plane offset of b - a is
//   w.u = (h_c - h_a - (h_b - h_a) cx / l) / cy,  w.m = -(h_b - h_a) / l,
//   w.n = m . (db - da) / l,
// so T . w spreads over a, b and the apex; the face left enters with
// T' = (-T_u, T_m, T_n) (its frame is the unfolding's image of (u, -m, -n)).
// Returns false (nothing to add) for an edge without sums or without a twin;
// otherwise the terms of a, b, the entered face's apex c and the left face's
// apex p (vertex id ip).
SG_HD bool gradx_edge(const DevMesh& M, const double* acc, int64_t h, D3& ga_out, D3& gb_out, D3& gc_out,
                      D3& gp_out, int32_t& ip_out) {
    const double* q = acc + 5 * h;
    const double slm = q[0], sln = q[1], tu = q[2], tm = q[3], tn = q[4];
    if (slm == 0.0 && sln == 0.0 && tu == 0.0 && tm == 0.0 && tn == 0.0) return false;
    const int64_t t = M.twin[h];
    if (t < 0) return false;
    const int64_t f = h / 3, k = h - 3 * f, fg = t / 3, kt = t - 3 * fg;
    const int32_t ia = M.F[3 * f + k], ib = M.F[3 * f + (k + 1) % 3], ic = M.F[3 * f + (k + 2) % 3];
    const int32_t ip = M.F[3 * fg + (kt + 2) % 3];
    const D3 A = dld(M.X + 3 * (int64_t)ia), B = dld(M.X + 3 * (int64_t)ib);
    const D3 Cn = dld(M.X + 3 * (int64_t)ic), Cp = dld(M.X + 3 * (int64_t)ip);
    D3 u = dsub(B, A);
    const double l = sqrt(ddot(u, u));
    u = dscl(u, 1.0 / l);
    D3 wj = dsub(Cn, A);
    const double cx = ddot(wj, u);
    D3 mj = dmad(wj, -cx, u);
    const double cy = sqrt(ddot(mj, mj));
    mj = dscl(mj, 1.0 / cy);
    const D3 nj = dcrs(u, mj);
    D3 wp = dsub(Cp, A);
    const double cxp = ddot(wp, u);
    D3 mp = dmad(wp, -cxp, u);
    const double cyp = sqrt(ddot(mp, mp));
    mp = dscl(mp, 1.0 / cyp);
    const D3 np = dcrs(u, mp);
    // (I - Q)^T lambda = l_m (m_j + m') + l_n (n_j + n')
    D3 ga = D3{slm * (mj.x + mp.x) + sln * (nj.x + np.x), slm * (mj.y + mp.y) + sln * (nj.y + np.y),
               slm * (mj.z + mp.z) + sln * (nj.z + np.z)};
    D3 gb = D3{0.0, 0.0, 0.0};
    // entered face, T = (tu, tm, tn)
    const D3 gcn = dscl(nj, tu / cy);
    gb = dmad(gb, -tu * cx / (l * cy) - tm / l, nj);
    gb = dmad(gb, tn / l, mj);
    ga = dmad(ga, tu * (cx / l - 1.0) / cy + tm / l, nj);
    ga = dmad(ga, -tn / l, mj);
    // face left, T' = (-tu, tm, tn)
    const D3 gcp = dscl(np, -tu / cyp);
    gb = dmad(gb, tu * cxp / (l * cyp) - tm / l, np);
    gb = dmad(gb, tn / l, mp);
    ga = dmad(ga, -tu * (cxp / l - 1.0) / cyp + tm / l, np);
    ga = dmad(ga, -tn / l, mp);
    ga_out = ga;
    gb_out = gb;
    gc_out = gcn;
    gp_out = gcp;
    ip_out = ip;
    return true;
}

// Face pass: the terms of face f's three entered half-edges.  Those on f's own
// vertices (each edge's a and b, and the apex c) are summed per corner into
// own[f, k]; the term on the apex of the face across half-edge 3 f + k goes to
// far[3 f + k].  Every entry is written, so the buffer needs no clearing, and
// the vertex pass gathers them without atomics (float64 atomics to random
// addresses run at a fixed rate of about 2.3e10 per second).
SG_HD void gradx_face(const DevMesh& M, const BwdArgs& a, const double* acc, double* own, double* far, int64_t f) {
    D3 g[3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (uint32_t j = a.fstart[f]; j < a.fstart[f + 1]; ++j) {   // start terms of the queries that start in f
        const float* q = a.sterm + 9 * (int64_t)a.qlist[j];
        for (int k = 0; k < 3; ++k) g[k] = D3{g[k].x + (double)q[3 * k], g[k].y + (double)q[3 * k + 1], g[k].z + (double)q[3 * k + 2]};
    }
    for (int k = 0; k < 3; ++k) {
        D3 ga, gb, gc, gp = {0.0, 0.0, 0.0};
        int32_t ip;
        if (gradx_edge(M, acc, 3 * f + k, ga, gb, gc, gp, ip)) {
            const int kb = k == 2 ? 0 : k + 1, kc = k == 0 ? 2 : k - 1;
            g[k] = dmad(g[k], 1.0, ga);
            g[kb] = dmad(g[kb], 1.0, gb);
            g[kc] = dmad(g[kc], 1.0, gc);
        }
        double* q = far + 3 * (3 * f + k);
        q[0] = gp.x; q[1] = gp.y; q[2] = gp.z;
    }
    for (int k = 0; k < 3; ++k) {
        double* q = own + 3 * (3 * f + k);
        q[0] = g[k].x; q[1] = g[k].y; q[2] = g[k].z;
    }
}

// Vertex pass: vertex v sums own[f, k] over its corners (f, k) and far[h] over
// the half-edges h across the edge opposite each corner (their far apex is v),
// and adds the total to grad_X once.
SG_HD void gradx_vertex(const DevMesh& M, const BwdArgs& a, const double* own, const double* far, int64_t v) {
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int32_t j = a.vc_off[v]; j < a.vc_off[v + 1]; ++j) {
        const int32_t c = a.vc[j];
        const int32_t f = c / 3, k = c - 3 * f;
        const double* q = own + 3 * (int64_t)c;
        sx += q[0]; sy += q[1]; sz += q[2];
        const int32_t t = M.twin[3 * f + (k == 2 ? 0 : k + 1)];
        if (t >= 0) {
            const double* r = far + 3 * (int64_t)t;
            sx += r[0]; sy += r[1]; sz += r[2];
        }
    }
    if (sx != 0.0 || sy != 0.0 || sz != 0.0) {
        double* gx = a.grad_X + 3 * v;
        gx[0] += sx; gx[1] += sy; gx[2] += sz;
    }
}

// Walks one chart state to its end in place (sequential form of k_walk).
template <bool kFlip, bool kHole = false>
SG_HD void walk_state(const DevMesh& M, StateRec& r, int32_t max_steps, float snap) {
    if (r.h < 0) return;
    Ray st;
    unpack_state(r, st);
    st.hash = 0ull;
    Final fin;
    walk_to_end<false, kFlip, kHole>(M, st, max_steps, snap, fin);
    r = *reinterpret_cast<const StateRec*>(&fin);
}

// The short finite-difference walks, one lane each (sh[3 i + first] onward,
// count per query): most end in their first face.
template <bool kFlip, bool kHole>
__global__ __launch_bounds__(256) void k_walk_short(DevMesh M, StateRec* sh, int64_t n, int first, int count,
                                                    int32_t max_steps, float snap) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int j = 0; j < count; ++j) walk_state<kFlip, kHole>(M, sh[3 * i + first + j], max_steps, snap);
}

#define SG_ROW_KERNEL(name, body, ...)                                                   \
    __global__ __launch_bounds__(256) void name(DevMesh M, BwdArgs a, ##__VA_ARGS__) {   \
        const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;                \
        if (i < a.n) body;                                                               \
    }
SG_ROW_KERNEL(k_bwd_stage1, bwd_stage1(M, a, s1, per_ray, sh, i), StateRec* s1, int per_ray, StateRec* sh)
SG_ROW_KERNEL(k_bwd_stage2, bwd_stage2(M, a, s1, per_ray, sh, do_shift, do_par, i), StateRec* s1, int per_ray,
              StateRec* sh, bool do_shift, bool do_par)
SG_ROW_KERNEL(k_gfd_assemble, gfd_assemble(M, a, s1, sh, i), const StateRec* s1, const StateRec* sh)
SG_ROW_KERNEL(k_ep_saved, ep_saved(M, a, i))
SG_ROW_KERNEL(k_ep_walked, ep_walked(M, a, s1, stride, i), const StateRec* s1, int stride)
SG_ROW_KERNEL(k_gradx_init, gradx_init(M, a, s1, stride, s3, cvec, sterm, srank, fcnt, i), const StateRec* s1,
              int stride, StateRec* s3, float4* cvec, float* sterm, int32_t* srank, uint32_t* fcnt)
// qlist[fstart[f] + rank] = query: the queries of each start face, in a list
SG_ROW_KERNEL(k_gradx_start_place, if (a.srank[i] >= 0) a.qlist[a.fstart[M.perm[a.f[i]]] + a.srank[i]] = (int32_t)i)
#undef SG_ROW_KERNEL

__global__ __launch_bounds__(64) void k_reset_counter(unsigned long long* c) {
    if (threadIdx.x < (unsigned)kMaxQueues) c[threadIdx.x * kQueueStride] = 0ull;
}

__global__ __launch_bounds__(256) void k_zero_u32(uint32_t* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_zero_f64(double* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_gradx_faces(DevMesh M, BwdArgs a, const double* acc, double* gxv) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f < M.n_faces) gradx_face(M, a, acc, gxv, gxv + 9 * M.n_faces, f);
}

__global__ __launch_bounds__(256) void k_gradx_vertices(DevMesh M, BwdArgs a, const double* gxv) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < M.n_verts) gradx_vertex(M, a, gxv, gxv + 9 * M.n_faces, v);
}

}  // namespace

// Launches the kernel instance for the (hash, orientation-flip) combination in use.
// Launches the instantiation of KERNEL<kHash, kFlip, kHole> for the runtime
// flags; the hole-avoiding rare path is compiled only into kHole kernels.
#define SG_DISPATCH_H(KERNEL, HASH, FLIP, HOLE, GRID, BLOCK, STREAM, ...)                        \
    do {                                                                                         \
        if (HOLE) KERNEL<HASH, FLIP, true><<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__);       \
        else KERNEL<HASH, FLIP, false><<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__);           \
    } while (0)
#define SG_DISPATCH(KERNEL, HASH, FLIP, GRID, BLOCK, STREAM, ...)                                             \
    do {                                                                                                      \
        const bool hole_ = M.hole_avoid != 0;                                                                 \
        if (HASH) {                                                                                           \
            if (FLIP) SG_DISPATCH_H(KERNEL, true, true, hole_, GRID, BLOCK, STREAM, __VA_ARGS__);             \
            else SG_DISPATCH_H(KERNEL, true, false, hole_, GRID, BLOCK, STREAM, __VA_ARGS__);                 \
        } else {                                                                                              \
            if (FLIP) SG_DISPATCH_H(KERNEL, false, true, hole_, GRID, BLOCK, STREAM, __VA_ARGS__);            \
            else SG_DISPATCH_H(KERNEL, false, false, hole_, GRID, BLOCK, STREAM, __VA_ARGS__);                \
        }                                                                                                     \
    } while (0)

hipError_t launch_exp_plain(const DevMesh& M, const ExpArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    const int block = 256;
    const int64_t grid = (a.n + block - 1) / block;
    SG_DISPATCH(k_exp_plain, (a.debug & 2u) != 0u, M.has_flip != 0, dim3((unsigned)grid), dim3(block), s, M, a);
    return hipGetLastError();
}

// walk states (slot order) | final states (query order) | epilogue terms |
// slots | internal start-face ids | bucket counts | queue counters
struct PersistentLayout {
    size_t fin, aux, slot, fint, cnt, counter, total;
};
static PersistentLayout persistent_layout(int64_t n, int32_t K) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    PersistentLayout L{};
    size_t o = al((size_t)n * sizeof(StateRec));
    L.fin = o; o = al(o + (size_t)n * sizeof(Final));
    L.aux = o; o = al(o + (size_t)n * (1 + 2 * (size_t)K) * sizeof(float));
    L.slot = o; o = al(o + (size_t)n * sizeof(int32_t));
    L.fint = o; o = al(o + (size_t)n * sizeof(int32_t));
    L.cnt = o; o = al(o + (size_t)kCountWords * sizeof(uint32_t));
    L.counter = o; o = al(o + kQueueBytes);
    L.total = o;
    return L;
}
size_t exp_persistent_workspace(int64_t n, int32_t K) { return persistent_layout(n, K).total; }

// Bucket counts of the walk order (ray_bucket) and each ray's rank in its
// bucket; cnt (kCountWords words) ends with the exclusive bucket starts.
static void order_rays(const DevMesh& M, int64_t n, const int32_t* f, const float* v, uint32_t* cnt, int32_t* slot,
                       const RayOrder& ord, hipStream_t s, int32_t* fint = nullptr) {
    const int nparts = (int)std::min<int64_t>((n + 255) / 256, kLenBlocks);
    hipLaunchKernelGGL(k_len_max, dim3((unsigned)nparts), dim3(256), 0, s, n, v, cnt);
    hipLaunchKernelGGL(k_bucket_count, dim3((unsigned)((n + kBucketRays - 1) / kBucketRays)), dim3(1024), 0, s, M, n, f,
                       v, cnt, slot, ord, nparts, fint);
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, cnt, ord.nb);
}

hipError_t launch_exp_persistent(const DevMesh& M, const ExpArgs& a, void* ws, const WalkSched& w, hipStream_t s,
                                 hipEvent_t ev0, hipEvent_t ev1) {
    if (a.n <= 0) return hipSuccess;
    const int block = 256;
    const int64_t grid = (a.n + block - 1) / block;
    const PersistentLayout L = persistent_layout(a.n, a.K);
    char* p = reinterpret_cast<char*>(ws);
    auto* states = reinterpret_cast<StateRec*>(p);
    auto* aux = reinterpret_cast<float*>(p + L.aux);
    auto* slot = reinterpret_cast<int32_t*>(p + L.slot);
    auto* cnt = reinterpret_cast<uint32_t*>(p + L.cnt);
    auto* counter = reinterpret_cast<unsigned long long*>(p + L.counter);
    // the one-ray-per-lane walk writes each final state at its query's index,
    // so the epilogue streams them; the two-ray form leaves them in the slots
    const bool by_query = a.rays_per_lane != 2;
    auto* fin = by_query ? reinterpret_cast<Final*>(p + L.fin) : nullptr;
    const RayOrder ord = ray_order(w.queues);
    auto* fint = reinterpret_cast<int32_t*>(p + L.fint);
    order_rays(M, a.n, a.f, a.v, cnt, slot, ord, s, fint);
    hipLaunchKernelGGL(k_init, dim3((unsigned)grid), dim3(block), 0, s, M, a, states, counter, aux,
                       (const uint32_t*)cnt, slot, ord, fin, (const int32_t*)fint);
    const QueueRanges R{cnt, kLenClasses * ord.sub, 1};
    if (ev0) (void)hipEventRecord(ev0, s);
    if (!by_query)
        SG_DISPATCH(k_walk2, (a.debug & 2u) != 0u, M.has_flip != 0, dim3((unsigned)w.blocks), dim3(block), s, M,
                    states, R, counter, a.max_steps, a.snap, w.refill_min, w.queues);
    else
        SG_DISPATCH(k_walk, (a.debug & 2u) != 0u, M.has_flip != 0, dim3((unsigned)w.blocks), dim3(block), s, M,
                    states, R, counter, a.max_steps, a.snap, w.refill_min, w.queues, fin);
    if (ev1) (void)hipEventRecord(ev1, s);
    if (by_query)
        hipLaunchKernelGGL(k_finish, dim3((unsigned)grid), dim3(block), 0, s, M, a,
                           reinterpret_cast<const StateRec*>(fin), (const uint64_t*)nullptr, (const float*)aux,
                           (const int32_t*)nullptr);
    else
        hipLaunchKernelGGL(k_finish, dim3((unsigned)grid), dim3(block), 0, s, M, a, states, (const uint64_t*)nullptr,
                           (const float*)aux, (const int32_t*)slot);
    return hipGetLastError();
}

// ---------------------------------------------------------------- allocation-free forward
// Scratch of the allocation-free forward: the persistent walk's workspace
// (walk states, final states, epilogue terms, slots, bucket counts, queue
// counters) for callers that cannot allocate.  Every device the library runs
// on holds its own copy from the load of this code object until the process
// ends.  In host code the array's name is a host-side stand-in, never a
// device address: host code reaches the array only through the address
// hipGetSymbolAddress returns for the current device, looked up once per
// device.  The walk's kernels clear the counts and counters they use, so the
// previous call's contents do no harm; calls that overlap on one device race.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** out) {
    static std::mutex mu;
    static void* addr[kNoAllocMaxDevices] = {};
    *out = nullptr;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

// Rounds of the partitioned walk: all but the last stop rays at part borders
// (the round stamp in a tag has 5 bits).
constexpr int kRounds = 4;
static_assert(kRounds <= 30, "round stamps must stay below the done tag");

// states [n] | epilogue terms [n, 1 + 2K] | hashes [n] (debug) | tags [n] | slice counters [kRounds, kParts]
struct RoundsLayout {
    size_t aux, hashes, tags, ctr, total;
};
static RoundsLayout rounds_layout(int64_t n, int32_t K, bool hash) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    RoundsLayout L{};
    size_t o = al((size_t)n * sizeof(StateRec));
    L.aux = o; o = al(o + (size_t)n * (1 + 2 * (size_t)K) * sizeof(float));
    L.hashes = o; o = al(o + (hash ? (size_t)n * 8 : 0));
    L.tags = o; o = al(o + (size_t)n);
    L.ctr = o; o = al(o + (size_t)kRounds * kParts * sizeof(unsigned long long));
    L.total = o;
    return L;
}

size_t exp_partitioned_workspace(int64_t n, int32_t K, bool hashes) { return rounds_layout(n, K, hashes).total; }

hipError_t launch_exp_partitioned(const DevMesh& M, const ExpArgs& a, void* ws, int grid_blocks, int refill_min,
                                  hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (a.n <= 0) return hipSuccess;
    const int block = 256;
    const int64_t grid = (a.n + block - 1) / block;
    const bool hash = (a.debug & 2u) != 0u;
    const RoundsLayout L = rounds_layout(a.n, a.K, hash);
    char* p = reinterpret_cast<char*>(ws);
    auto* states = reinterpret_cast<StateRec*>(p);
    auto* aux = reinterpret_cast<float*>(p + L.aux);
    auto* hashes = hash ? reinterpret_cast<uint64_t*>(p + L.hashes) : nullptr;
    auto* tags = reinterpret_cast<uint8_t*>(p + L.tags);
    auto* ctr = reinterpret_cast<unsigned long long*>(p + L.ctr);
    hipLaunchKernelGGL(k_rounds_reset, dim3(1), dim3(kRounds * kParts), 0, s, ctr, kRounds * kParts);
    if (hash)
        hipLaunchKernelGGL(k_init_rounds<true>, dim3((unsigned)grid), dim3(block), 0, s, M, a, states, aux, hashes, tags);
    else
        hipLaunchKernelGGL(k_init_rounds<false>, dim3((unsigned)grid), dim3(block), 0, s, M, a, states, aux, hashes,
                           tags);
    if (ev0) (void)hipEventRecord(ev0, s);
    const int blocks = (grid_blocks + kParts - 1) / kParts * kParts;   // every part gets the same number of blocks
    for (int r = 0; r < kRounds; ++r) {
        SG_DISPATCH(k_walk_round, hash, M.has_flip != 0, dim3((unsigned)blocks), dim3(block), s, M, states, hashes,
                    tags, ctr + (size_t)r * kParts, (int64_t)a.n, a.max_steps, a.snap, refill_min, r,
                    r + 1 < kRounds ? 1 : 0);
    }
    if (ev1) (void)hipEventRecord(ev1, s);
    hipLaunchKernelGGL(k_finish, dim3((unsigned)grid), dim3(block), 0, s, M, a, states, (const uint64_t*)nullptr,
                       (const float*)aux, (const int32_t*)nullptr);
    return hipGetLastError();
}

// Backward workspace, carved in this order (each part 256-byte aligned):
// the long-walk states (per1 per query), GFD's short-walk states (3 per
// query), grad-X walk states and adjoint coefficients, grad-X half-edge sums
// (15 per face) and per-face corner terms (18 per face), the start terms,
// their ranks and the per-face query lists (offsets, tile sums, entries),
// walk slots and bucket counts, queue counters, then the grad-X records (walk
// order and bin order), the chunk fills and the bin words (nbins + 1 bin
// totals scanned into starts, chunks used per walk block, the (walk block,
// bin) count matrix).
struct BwdLayout {
    size_t s1, sh, s3, cvec, acc, gxv, sterm, srank, fstart, ftile, qlist, slot, cnt, counter, rec, sorted, fill,
        bins, total;
    int per_block;   // record chunks per walk block (0: no records)
    int shift, nbins;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// What a backward call walks.  The forward's saved outputs replace the base
// geodesic's walk (Appendix "Speed-up GFD and EP through batching": Exp(p, v)
// is the forward's) where the faces agree in orientation (the end normal's
// sign needs no walk) and hole avoidance is off: GFD then walks six
// geodesics per query (given f', b', v'), and the vertex gradient takes its
// end frame from f', v' and the status.
struct BwdPlan {
    bool gfd, walk, gfd_saved, gx_saved, base_walk;
    int per1;   // long-walk states per query (0: no walk pass)
};

static BwdPlan bwd_plan(int32_t mode, bool has_flip, bool hole, bool vjp, bool gradx, bool have_f, bool have_b,
                        bool have_v, bool have_status) {
    BwdPlan P{};
    P.gfd = vjp && mode == 1;
    P.walk = gradx || P.gfd || (vjp && has_flip);
    const bool plain = !has_flip && !hole;
    const bool end_ok = plain && have_f && have_v && have_status;   // end frame and status of every ray
    P.gfd_saved = P.gfd && plain && have_f && have_b && have_v && (!gradx || end_ok);
    P.gx_saved = gradx && end_ok && (!P.gfd || P.gfd_saved);
    // one persistent pass walks the long geodesics: the base (unless its end is
    // the forward's) and, for GFD, the e_perp one and the two start-shifted ones
    P.base_walk = (P.gfd && !P.gfd_saved) || (vjp && has_flip) || (gradx && !P.gx_saved);
    P.per1 = P.gfd ? (P.gfd_saved ? 3 : 4) : (P.base_walk ? 1 : 0);
    return P;
}

static BwdLayout bwd_layout(int64_t n, const BwdPlan& P, bool gradx, int64_t n_faces, int32_t gx_records,
                            int walk_blocks) {
    const bool gfd = P.gfd, walk = P.walk;
    const size_t per1 = P.per1;
    BwdLayout L{};
    size_t o = 0;
    L.s1 = o; o = align256(o + per1 * (size_t)n * sizeof(StateRec));
    L.sh = o; o = align256(o + (gfd ? 3 * (size_t)n * sizeof(StateRec) : 0));
    L.s3 = o; o = align256(o + (gradx ? (size_t)n * sizeof(StateRec) : 0));
    L.cvec = o; o = align256(o + (gradx ? (size_t)n * sizeof(float4) : 0));
    L.acc = o; o = align256(o + (gradx ? 15 * (size_t)n_faces * sizeof(double) : 0));
    L.gxv = o; o = align256(o + (gradx ? 18 * (size_t)n_faces * sizeof(double) : 0));
    L.sterm = o; o = align256(o + (gradx ? 9 * (size_t)n * sizeof(float) : 0));
    L.srank = o; o = align256(o + (gradx ? (size_t)n * sizeof(int32_t) : 0));
    L.fstart = o; o = align256(o + (gradx ? ((size_t)n_faces + 1) * sizeof(uint32_t) : 0));
    L.ftile = o; o = align256(o + (gradx ? (((size_t)n_faces + 1 + 4095) / 4096) * sizeof(uint32_t) : 0));
    L.qlist = o; o = align256(o + (gradx ? (size_t)n * sizeof(int32_t) : 0));
    L.slot = o; o = align256(o + (walk ? (size_t)n * sizeof(int32_t) : 0));
    L.cnt = o; o = align256(o + (walk ? (size_t)kCountWords * sizeof(uint32_t) : 0));
    L.counter = o; o = align256(o + kQueueBytes);
    const int64_t nh = 3 * n_faces;
    L.shift = kGxShift0;
    while (((nh + ((int64_t)1 << L.shift) - 1) >> L.shift) > kGxMaxBins) ++L.shift;
    const int64_t nblk = std::max(walk_blocks, 1);
    if (gradx && gx_records > 0 && nh > 0) {
        // about gx_records per query, shared evenly by the walk blocks (the
        // persistent walk balances crossings across them), plus one partly
        // filled chunk per wave
        const int64_t want = ((int64_t)n * gx_records + kGxChunk - 1) / kGxChunk;
        L.per_block = (int)std::min<int64_t>((want + nblk - 1) / nblk + 4, kGxMaxRecords / kGxChunk / nblk);
        L.nbins = (int)((nh + ((int64_t)1 << L.shift) - 1) >> L.shift);
    }
    const int64_t nchunks = L.per_block * nblk;
    const size_t recs = (size_t)nchunks * kGxChunk;
    L.rec = o; o = align256(o + recs * sizeof(GxRec));
    L.sorted = o; o = align256(o + recs * sizeof(GxRec));
    L.fill = o; o = align256(o + (size_t)nchunks * sizeof(uint32_t));
    L.bins = o; o = align256(o + (nchunks ? (size_t)(L.nbins + 1 + nblk + nblk * L.nbins) * sizeof(uint32_t) : 0));
    L.total = (walk || gradx) ? o : 0;
    return L;
}

size_t bwd_workspace(int64_t n, int32_t mode, bool has_flip, bool vjp, bool gradx, int64_t n_faces,
                     int32_t gx_records, int walk_blocks, bool hole, bool have_f, bool have_b, bool have_v,
                     bool have_status) {
    const BwdPlan P = bwd_plan(mode, has_flip, hole, vjp, gradx, have_f, have_b, have_v, have_status);
    return bwd_layout(n, P, gradx, n_faces, gx_records, walk_blocks).total;
}

hipError_t launch_backward(const DevMesh& M, const BwdArgs& a_in, void* ws, const WalkSched& w, hipStream_t s) {
    BwdArgs a = a_in;
    if (a.n <= 0) return hipSuccess;
    const int block = 256;
    const int64_t grid = (a.n + block - 1) / block;
    const bool vjp = a.grad_v != nullptr;
    const bool gfd = vjp && a.mode == 1;
    const bool gradx = a.grad_X != nullptr;
    const bool flip = M.has_flip != 0;
    if (vjp && a.mode == 0 && !flip) hipLaunchKernelGGL(k_ep_saved, dim3((unsigned)grid), dim3(block), 0, s, M, a);
    if (!(gradx || gfd || (vjp && flip))) return hipGetLastError();
    const BwdPlan P = bwd_plan(a.mode, flip, M.hole_avoid != 0, vjp, gradx, a.f_out != nullptr, a.b_out != nullptr,
                               a.v_out != nullptr, a.status_in != nullptr);
    a.gfd_saved = P.gfd_saved ? 1 : 0;
    const BwdLayout L = bwd_layout(a.n, P, gradx, M.n_faces, a.gx_records, w.blocks);
    char* base = reinterpret_cast<char*>(ws);
    auto* s1 = reinterpret_cast<StateRec*>(base + L.s1);
    auto* sh = gfd ? reinterpret_cast<StateRec*>(base + L.sh) : nullptr;
    auto* s3 = reinterpret_cast<StateRec*>(base + L.s3);
    auto* cvec = reinterpret_cast<float4*>(base + L.cvec);
    auto* acc = reinterpret_cast<double*>(base + L.acc);
    auto* counter = reinterpret_cast<unsigned long long*>(base + L.counter);
    const int per1 = P.per1;
    auto* cnt = reinterpret_cast<uint32_t*>(base + L.cnt);
    const RayOrder ord = ray_order(w.queues);
    {   // walk the queries in the order of ray_bucket (region, longest first, start face)
        auto* slot = reinterpret_cast<int32_t*>(base + L.slot);
        order_rays(M, a.n, a.f, a.v, cnt, slot, ord, s);
        hipLaunchKernelGGL(k_slot_place, dim3((unsigned)grid), dim3(block), 0, s, M, a.n, a.f, a.v,
                           (const uint32_t*)cnt, slot, ord);
        a.slot = slot;
    }
    // the short walks, one lane each, in the variant the persistent walks use
    auto walk_short = [&](int first, int count) {
        const dim3 g((unsigned)grid), b(block);
        if (flip && M.hole_avoid) k_walk_short<true, true><<<g, b, 0, s>>>(M, sh, a.n, first, count, a.max_steps, a.snap);
        else if (flip) k_walk_short<true, false><<<g, b, 0, s>>>(M, sh, a.n, first, count, a.max_steps, a.snap);
        else if (M.hole_avoid) k_walk_short<false, true><<<g, b, 0, s>>>(M, sh, a.n, first, count, a.max_steps, a.snap);
        else k_walk_short<false, false><<<g, b, 0, s>>>(M, sh, a.n, first, count, a.max_steps, a.snap);
    };
    // the long walks' start states (GFD: the two short start-point steps walk
    // first, one lane each, and the start-shifted long walks begin at their
    // ends), then one persistent pass over all of them
    const int stride = kLenClasses * ord.sub;
    if (per1 > 0) hipLaunchKernelGGL(k_bwd_stage1, dim3((unsigned)grid), dim3(block), 0, s, M, a, s1, per1, sh);
    if (gfd) {
        walk_short(0, 2);
        // with the base's end saved, the e_par step can start now as well
        hipLaunchKernelGGL(k_bwd_stage2, dim3((unsigned)grid), dim3(block), 0, s, M, a, s1, per1, sh, true,
                           P.gfd_saved);
        if (P.gfd_saved) walk_short(2, 1);
    }
    if (per1 > 0) {
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, counter);
        SG_DISPATCH(k_walk_bwd, false, flip, dim3((unsigned)w.blocks), dim3(block), s, M, s1,
                    QueueRanges{cnt, stride, per1}, counter, a.max_steps, a.snap, w.refill_min, w.queues);
    }
    if (vjp && a.mode == 0 && flip)   // (consistent orientation: k_ep_saved above)
        hipLaunchKernelGGL(k_ep_walked, dim3((unsigned)grid), dim3(block), 0, s, M, a, s1, per1);
    if (gfd) {
        if (!P.gfd_saved) {   // the e_par step from the walked base's end
            hipLaunchKernelGGL(k_bwd_stage2, dim3((unsigned)grid), dim3(block), 0, s, M, a, s1, per1, sh, false,
                               true);
            walk_short(2, 1);
        }
        hipLaunchKernelGGL(k_gfd_assemble, dim3((unsigned)grid), dim3(block), 0, s, M, a, s1, (const StateRec*)sh);
    }
    if (gradx) {
        const int64_t nacc = 15 * M.n_faces;
        hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)std::min<int64_t>((nacc + block - 1) / block, 8192)), dim3(block),
                           0, s, acc, nacc);
        auto* sterm = reinterpret_cast<float*>(base + L.sterm);
        auto* srank = reinterpret_cast<int32_t*>(base + L.srank);
        auto* fstart = reinterpret_cast<uint32_t*>(base + L.fstart);
        a.sterm = sterm;
        a.srank = srank;
        a.fstart = fstart;
        a.qlist = reinterpret_cast<int32_t*>(base + L.qlist);
        const int64_t nfs = M.n_faces + 1;
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)std::min<int64_t>((nfs + block - 1) / block, 8192)), dim3(block),
                           0, s, fstart, nfs);
        hipLaunchKernelGGL(k_gradx_init, dim3((unsigned)grid), dim3(block), 0, s, M, a,
                           P.gx_saved ? (const StateRec*)nullptr : (const StateRec*)s1, per1, s3, cvec, sterm, srank,
                           fstart);
        // each start face's queries as one list (counts to offsets, then the ranks place them)
        const int64_t ntile = (nfs + 4095) / 4096;
        auto* tile = reinterpret_cast<uint32_t*>(base + L.ftile);
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntile), dim3(1024), 0, s, fstart, nfs, tile);
        hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, tile, (int)ntile);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((nfs + block - 1) / block)), dim3(block), 0, s, fstart, nfs,
                           (const uint32_t*)tile);
        hipLaunchKernelGGL(k_gradx_start_place, dim3((unsigned)grid), dim3(block), 0, s, M, a);
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, counter);
        const int64_t nh = 3 * M.n_faces;
        GxSink sink{};
        auto* bins = reinterpret_cast<uint32_t*>(base + L.bins);   // [bin totals / starts, used, count matrix]
        uint32_t* used = bins + L.nbins + 1;
        uint32_t* counts = used + w.blocks;
        if (L.per_block > 0) {
            sink.rec = reinterpret_cast<GxRec*>(base + L.rec);
            sink.fill = reinterpret_cast<uint32_t*>(base + L.fill);
            sink.per_block = L.per_block;
            sink.shift = L.shift;
        }
        const QueueRanges R3{cnt, stride, 1};
        const dim3 gw((unsigned)w.blocks), bw(block);
        if (flip) {
            if (M.hole_avoid) k_walk_gx<true, true><<<gw, bw, 0, s>>>(M, s3, R3, counter, a.max_steps, a.snap,
                                                                       w.refill_min, w.queues, cvec, acc, sink,
                                                                       counts, used, L.nbins);
            else k_walk_gx<true, false><<<gw, bw, 0, s>>>(M, s3, R3, counter, a.max_steps, a.snap, w.refill_min,
                                                            w.queues, cvec, acc, sink, counts, used, L.nbins);
        } else {
            if (M.hole_avoid) k_walk_gx<false, true><<<gw, bw, 0, s>>>(M, s3, R3, counter, a.max_steps, a.snap,
                                                                        w.refill_min, w.queues, cvec, acc, sink,
                                                                        counts, used, L.nbins);
            else k_walk_gx<false, false><<<gw, bw, 0, s>>>(M, s3, R3, counter, a.max_steps, a.snap, w.refill_min,
                                                             w.queues, cvec, acc, sink, counts, used, L.nbins);
        }
        if (L.per_block > 0) {
            hipLaunchKernelGGL(k_gx_colscan, dim3((unsigned)L.nbins), dim3(1024), 0, s, counts, w.blocks, L.nbins,
                               bins);
            hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, bins, L.nbins + 1);
            hipLaunchKernelGGL(k_gx_scatter, dim3((unsigned)w.blocks), dim3(1024), 0, s, (const GxRec*)sink.rec,
                               (const uint32_t*)sink.fill, (const uint32_t*)used, L.per_block, L.shift, L.nbins,
                               (const uint32_t*)bins, (const uint32_t*)counts,
                               reinterpret_cast<GxRec*>(base + L.sorted));
            const int wpb = (1 << L.shift) / kGxWindow;
            hipLaunchKernelGGL(k_gx_reduce, dim3((unsigned)(L.nbins * wpb)), dim3(1024), 0, s,
                               (const GxRec*)(base + L.sorted), (const uint32_t*)bins, L.shift, nh, acc);
        }
        auto* gxv = reinterpret_cast<double*>(base + L.gxv);
        hipLaunchKernelGGL(k_gradx_faces, dim3((unsigned)((M.n_faces + block - 1) / block)), dim3(block), 0, s, M, a,
                           (const double*)acc, gxv);
        hipLaunchKernelGGL(k_gradx_vertices, dim3((unsigned)((M.n_verts + block - 1) / block)), dim3(block), 0, s,
                           M, a, (const double*)gxv);
    }
    return hipGetLastError();
}

hipError_t launch_ep_saved(const DevMesh& M, const BwdArgs& a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ep_saved, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, M, a);
    return hipGetLastError();
}

int walk_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk<false, false, false>, 256, 0) != hipSuccess || nb <= 0) nb = 1;
    return nb;
}

int part_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_walk_round<false, false, false>, 256, 0) != hipSuccess || nb <= 0)
        nb = 1;
    return nb;
}

}  // namespace sg
