// Internal layouts shared by the host code and the HIP kernels of libptmi.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptmi {

// 4-wide BVH node, 80 bytes (five 16-byte loads per visit): the children's
// boxes as half-precision offsets from the node's origin, then the four
// child references.
//   o[a]      origin on axis a (the node's lower corner)
//   e         byte a = scale exponent of axis a, biased by 128:
//             plane = o[a] + h * 2^(e_a - 128), h a binary16 value
//   x, y, z   per axis four words of binary16 pairs: lower planes of
//             children (0, 1), (2, 3), then upper planes of (0, 1), (2, 3);
//             lower planes rounded down, upper planes up, so the decoded
//             box encloses the child's box
//   ref = index of an internal node            (bit 31 clear)
//   ref = LEAF | (count - 1) << 27 | first_tri (bit 31 set, 1..16 triangles)
//   ref = EMPTY (all ones) for an unused slot; its planes are +inf (lower)
//   and -inf (upper), an inverted box the slab test rejects.
struct alignas(16) Node4 {
    float o[3];
    uint32_t e;
    uint32_t x[4], y[4], z[4];
    uint32_t ref[4];
};
static_assert(sizeof(Node4) == 80, "node must be 80 bytes");
constexpr int kNodeGridMinExp = -100;  // smallest grid step exponent

constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kEmptyRef = 0xFFFFFFFFu;
constexpr int kLeafCountShift = 27;
constexpr uint32_t kLeafFirstMask = (1u << kLeafCountShift) - 1u;
constexpr int kMaxLeaf = 8;
constexpr int64_t kMaxTris = int64_t(kLeafFirstMask) + 1;

// Triangle in leaf order, 48 bytes: three float4 = (v0, input id bits),
// (v1, material index | light flag bit 31), (v2, 0).
constexpr uint32_t kLightFlag = 0x80000000u;
// The triangle array ends with kTriPad zero float4 after the last record, so
// a traversal step may read five float4 from any record (see fetch_item).
constexpr int kTriPad = 2;

// Light table entry, 16 bytes: leaf-order triangle index, the u32 CDF word,
// the input triangle index (which addresses the emission array), zero.
struct LightEntry {
    uint32_t tri;
    uint32_t cdf;
    uint32_t id;
    uint32_t pad;
};

// triangles of largest area whose adjoint gradients are summed per
// workgroup (many paths reach them: a ground plane, area lights)
constexpr int kHotTris = 64;

// Instance record of a two-level scene, kInstRecord float4 (112 bytes), in
// the top-level BVH's leaf order: rows 0-2 the world-to-object map (3x4,
// row-major, a float4 per row), rows 3-5 the object-to-world map, row 6 =
// (root node of the instance's mesh, input instance index, 0, 0) as bits.
// A top-level leaf reference holds the record index (one instance per leaf).
// In a two-level scene the light table's last word is the light's record.
constexpr int kInstRecord = 7;
// traversal stack entry that marks the return from an instance's mesh to
// the top level (never a node or leaf reference of a valid scene)
constexpr uint32_t kInstMarker = 0xFFFFFFFEu;

// Vertex attribute record of a triangle, kAttrRecord float4 (64 bytes), in
// leaf order like the triangle records: (n0.xyz, u0), (n1.xyz, v0),
// (n2.xyz, u1), (v1, u2, v2, 0).  SceneView::attr_flags says which of the
// two kinds the scene has.
constexpr int kAttrRecord = 4;
constexpr int32_t kAttrNormals = 1;
constexpr int32_t kAttrUV = 2;
// a material of the scene is coated: the shading kernels' extended variant
// (the one that also handles attributes) is needed
constexpr int32_t kAttrCoat = 4;

struct SceneView {
    const float4* __restrict__ nodes;
    const float4* __restrict__ tris;
    const LightEntry* __restrict__ lights;
    const float4* __restrict__ mats;
    const float* __restrict__ albedo;    // input order, nt*3
    const float* __restrict__ emission;  // input order, nt*3
    int32_t nl;
    int32_t nt;
    int32_t n_nodes;
    float area_total;
    float sky0, sky1, sky2;
    float cx, cy, cz;  // centre of the scene's bounding box (ray sort key)
    // the largest triangles (input ids by slot): a triangle record's third
    // word w holds its slot + 1 (0 = not one of them); the adjoint sums
    // their gradients per workgroup before adding them to global memory
    const uint32_t* __restrict__ hot_ids;
    int32_t n_hot;
    // two-level scene: instance records (kInstRecord float4 each) and their
    // count (0 for a flat scene); vertex attributes (kAttrRecord float4 per
    // triangle, leaf order) and which kinds are present (kAttrNormals |
    // kAttrUV; 0 = none).  The two pointers precede the two counts so the
    // struct has no padding: kernels that keep a scene per lane in
    // registers (the batched traversal) fit their register budget.
    const float4* __restrict__ insts;
    const float4* __restrict__ attrs;
    int32_t n_inst;
    int32_t attr_flags;
};

struct CamView {
    float E[3], R[3], U[3], F[3];
    int32_t W, H;
};

struct PathParams {
    int32_t spp, D, nee, rr_start;
    uint64_t seed;
    uint32_t frame, job;
    int32_t sampler;  // camera jitter: 0 Philox, 1 Halton(2,3) with a per-pixel rotation
};

}  // namespace ptmi
