// Host-side scene packing for libptmi (BVH4 build, leaf-order triangles,
// light CDF).
#pragma once
#include <vector>

#include "ptmi_internal.h"

namespace ptmi {

struct BuildResult {
    std::vector<Node4> nodes;
    std::vector<float4> tris;        // 3 per triangle, leaf order
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

}  // namespace ptmi
