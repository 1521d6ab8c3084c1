// Host-side scene packing for libptmi (BVH4 build, leaf-order triangles,
// light CDF).
#pragma once
#include <vector>

#include "ptmi_internal.h"

namespace ptmi {

struct BuildResult {
    std::vector<Node4> nodes;
    std::vector<float4> tris;        // 3 per triangle, leaf order, then kTriPad zero float4
    std::vector<float4> insts;       // two-level scenes: kInstRecord per instance, top-level leaf order
    std::vector<LightEntry> lights;  // input order of the light triangles
    std::vector<uint32_t> hot_ids;   // input ids of the largest triangles, by slot (at most kHotTris)
    float area_total = 0.f;
    float max_coord = 0.f;  // largest absolute vertex coordinate
    float center[3] = {0.f, 0.f, 0.f};  // centre of the scene's bounding box
    int depth = 0;
    int stack_entries = 0;
};

// tri_v: nt*9 vertex coordinates (v0, v1, v2) in input order.
BuildResult build_scene(const std::vector<float>& tri_v, const std::vector<int32_t>& tri_mat,
                        const std::vector<float>& emission, int max_leaf, int threads);

// Two-level scene: meshes are ranges of the triangles (object space),
// instances place them by 3x4 row-major affine maps (o2w; w2o its inverse
// for rays), 12 floats per instance.
struct InstanceSet {
    std::vector<int32_t> mesh_first, mesh_count, inst_mesh;
    std::vector<float> o2w, w2o;
};

// One BVH4 per mesh over its object-space triangles and a top-level BVH4
// over the instances' world boxes (node 0 is the top-level root); the
// instance records in top-level leaf order; the light set over every
// (instance, emissive triangle) pair in instance order with world-space
// areas.
BuildResult build_instanced(const std::vector<float>& tri_v, const std::vector<int32_t>& tri_mat,
                            const std::vector<float>& emission, const InstanceSet& inst, int max_leaf, int threads);

// world-space vertices of a triangle placed by a 3x4 row-major map M, in the
// renderer's arithmetic (((M0 x + M1 y) + M2 z) + M3 per row, binary32)
void xform_tri(const float* M, const float* v, float* out);

}  // namespace ptmi
