// sg_internal.h -- data layout shared by the host packer and the gfx950 kernels.
//
// The walk is intrinsic: a ray inside a face is described in the chart of
// the half-edge it entered through.  For half-edge h = 3 f + k of face f the
// entry edge runs from a = F[f][k] to b = F[f][k+1]; the apex is
// c = F[f][k+2].  The chart puts a at the origin, b on the +x axis and the
// face in y > 0.  Unfolding across an edge (Sec. 4: the neighbourhood of an
// edge point is isometric to a plane) is then an exact change of chart, and
// the direction is carried as a fixed-point angle to the entry edge, so the
// angle-preserving transition is an integer add of a corner angle.
#pragma once
#include <stdint.h>

namespace sg {

// Fixed-point angles: 2^32 units = 2 pi.  Corner angles are rounded once from
// float64; their sums are exact integer arithmetic.
constexpr uint32_t kPiFx = 0x80000000u;
constexpr uint32_t kHalfPiFx = 0x40000000u;
constexpr double kFxPerRad = 4294967296.0 / 6.283185307179586476925286766559;
constexpr float kRadPerFx = 1.4629180792671596e-09f;   // 2 pi / 2^32

// One record per face (32 bytes, one aligned sector).  Edge k runs from
// vertex k to vertex k+1 of the face; corner k is the angle at vertex k.
struct alignas(32) FaceRec {
    float l[3];       // edge lengths |x_{k+1} - x_k|
    uint32_t c0, c1;  // corner angles at vertices 0 and 1 (fixed point); corner 2 = pi - c0 - c1
    int32_t nb[3];    // half-edge entered when crossing edge k: (id << 1) | flip, or -1 (boundary)
};
static_assert(sizeof(FaceRec) == 32, "record must be one 32-byte sector");

// The chart of half-edge h = 3 f + k as the walk sees it, rebuilt from the
// face record: a ray entering face f through edge k needs its exit test and
// its two onward links.
struct HalfEdgeRec {
    float cx, cy;     // apex c in the entry chart
    float lac, lbc;   // lengths |ac| and |bc|
    float lab;        // length |ab| of the entry edge
    uint32_t A, B;    // corner angles at a and b (fixed point)
    int32_t nca;      // half-edge entered when crossing edge c-a: (id << 1) | flip, or -1 (boundary)
    int32_t nbc;      // half-edge entered when crossing edge b-c, same encoding
};

// Faces are stored in a spatial (bisection) order cut into kParts contiguous
// parts, one per XCD of the MI355X, so that a part's records fit that XCD's L2.
constexpr int kParts = 8;

// Device view of a packed mesh handle.  Face ids inside the library are
// internal (bisection order); rays name faces by user id.
struct DevMesh {
    const FaceRec* face;        // [n_faces], internal order
    const int32_t* F;           // [n_faces, 3] global vertex ids, internal order
    const float* X;             // [n_verts, 3]
    const int64_t* half_theta;  // [n_verts] theta(x)/2 in fixed point, -1 on boundary vertices
    const int32_t* perm;        // [n_faces] user face id -> internal id
    const int32_t* order;       // [n_faces] internal face id -> user id
    int64_t n_faces;
    int64_t n_verts;
    int32_t has_flip;           // some adjacent faces disagree in orientation (non-orientable or mixed)
    int32_t part_he[kParts + 1];// half-edge id ranges of the parts
    const int32_t* twin;        // [3 n_faces] half-edge on the other side of each edge, -1 on the boundary
    int32_t hole_avoid;         // per call: 1 = trace along boundaries instead of stopping (Sec. 4)
    const float4* geo;          // [n_faces, 4]: the face's three vertex positions (w: its FaceRec's edge
                                // lengths l[0..2]), then (c0 bits, c1 bits, user face id bits, 0): one
                                // 64-byte record per face
};

// ---- projection integration (appendix "Projection Integration Exp Map"):
// the comparison Exp, whose steps project a point onto the nearest point of
// the mesh.  Faces are kept in user order (the tie rule takes the smallest
// user face id): the three vertex positions (float32, exact in float64) and
// the unit normal in float64.
struct alignas(16) PiFace {
    float x0[3], x1[3], x2[3];
    float pad;
    double n[3];
};
static_assert(sizeof(PiFace) == 64, "PiFace is one 64-byte segment");

// Uniform grid over one mesh of a handle: cell (ix, iy, iz) covers
// [o + i h, o + (i + 1) h] per axis (evaluated in float64) and lists every
// face whose bounding box, widened by a margin, meets it.  A nearest-point
// search visits cells in rings around the query's cell and skips those
// farther than the best distance found, so it returns what a scan over every
// face would.
struct PiGrid {
    float ox, oy, oz, h;      // origin and cell size
    int32_t nx, ny, nz;       // cells per axis
    uint32_t cell0;           // first cell of this mesh in the handle's cell arrays
    int32_t face0, face1;     // the mesh's user face range [face0, face1)
};

struct PiMesh {
    const PiFace* face;        // [n_faces] in user order
    const PiGrid* grid;        // [n_meshes]
    const uint32_t* cell_start;// [total cells + 1] offsets into cell_face
    const int32_t* cell_face;  // user face ids
    int64_t n_faces;
    int32_t n_meshes;
    double tie;                // distances within tie of the smallest are a tie (a shared nearest point)
    double slack;              // extra reach of the cell search over the tie (rounding of box distances)
};

enum RayStatus : int32_t { kRayOk = 0, kRayMaxSteps = 1, kRayBoundary = 2, kRayBadInput = 3 };

}  // namespace sg
