// Host-side scene packing for libptmi: binned-SAH binary BVH collapsed to a
// 4-wide BVH with 80-byte nodes (binary16 child boxes), triangles reordered to leaf order, and the
// area-proportional light CDF.  The paper builds its acceleration
// structures through the Vulkan driver (Sec. 3); this is the software
// counterpart for traversal on the compute units.
#include "bvh_build.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <deque>
#include <future>
#include <limits>
#include <memory>
#include <mutex>
#include <thread>

namespace ptmi {
namespace {

struct PrimInfo {
    float lo[3], hi[3], c[3];
};

struct BNode {
    float lo[3], hi[3];
    BNode* kid[2];
    int32_t first, count;  // count > 0: leaf
};

struct Arena {
    std::deque<BNode> nodes;
    BNode* make() {
        nodes.emplace_back();
        return &nodes.back();
    }
};

constexpr int kBins = 64;

float area_of(const float lo[3], const float hi[3]) {
    float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    if (!(dx >= 0.f) || !(dy >= 0.f) || !(dz >= 0.f)) return 0.f;
    return 2.f * (dx * dy + dy * dz + dz * dx);
}

class BinaryBuilder {
   public:
    BinaryBuilder(const std::vector<PrimInfo>& info, std::vector<int32_t>& order, int max_leaf, int threads)
        : info_(info), order_(order), max_leaf_(max_leaf), budget_(threads > 1 ? threads - 1 : 0) {}

    BNode* build() { return build(0, (int32_t)order_.size()); }
    // over order[first, first + count) only
    BNode* build(int32_t first, int32_t count) {
        arenas_.emplace_back(new Arena());
        return rec(first, count, arenas_.back().get());
    }

   private:
    const std::vector<PrimInfo>& info_;
    std::vector<int32_t>& order_;
    int max_leaf_;
    std::atomic<int> budget_;
    std::mutex mu_;
    std::vector<std::unique_ptr<Arena>> arenas_;

    Arena* new_arena() {
        std::lock_guard<std::mutex> g(mu_);
        arenas_.emplace_back(new Arena());
        return arenas_.back().get();
    }

    BNode* leaf(BNode* n, int32_t first, int32_t count) {
        n->first = first;
        n->count = count;
        n->kid[0] = n->kid[1] = nullptr;
        return n;
    }

    BNode* rec(int32_t first, int32_t count, Arena* arena) {
        BNode* n = arena->make();
        float clo[3], chi[3];
        for (int a = 0; a < 3; ++a) {
            n->lo[a] = INFINITY; n->hi[a] = -INFINITY;
            clo[a] = INFINITY; chi[a] = -INFINITY;
        }
        for (int32_t i = first; i < first + count; ++i) {
            const PrimInfo& p = info_[order_[i]];
            for (int a = 0; a < 3; ++a) {
                n->lo[a] = std::min(n->lo[a], p.lo[a]);
                n->hi[a] = std::max(n->hi[a], p.hi[a]);
                clo[a] = std::min(clo[a], p.c[a]);
                chi[a] = std::max(chi[a], p.c[a]);
            }
        }
        if (count <= 1) return leaf(n, first, count);

        // binned SAH over the three axes
        float best_cost = INFINITY;
        int best_axis = -1, best_split = -1;
        for (int a = 0; a < 3; ++a) {
            float ext = chi[a] - clo[a];
            if (!(ext > 0.f)) continue;
            float scale = kBins / ext;
            int cnt[kBins] = {0};
            float blo[kBins][3], bhi[kBins][3];
            for (int b = 0; b < kBins; ++b)
                for (int k = 0; k < 3; ++k) { blo[b][k] = INFINITY; bhi[b][k] = -INFINITY; }
            for (int32_t i = first; i < first + count; ++i) {
                const PrimInfo& p = info_[order_[i]];
                int b = std::min(kBins - 1, (int)((p.c[a] - clo[a]) * scale));
                cnt[b]++;
                for (int k = 0; k < 3; ++k) {
                    blo[b][k] = std::min(blo[b][k], p.lo[k]);
                    bhi[b][k] = std::max(bhi[b][k], p.hi[k]);
                }
            }
            float rarea[kBins];
            int rcnt[kBins];
            float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            int c = 0;
            for (int b = kBins - 1; b > 0; --b) {
                c += cnt[b];
                for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], blo[b][k]); hi[k] = std::max(hi[k], bhi[b][k]); }
                rarea[b] = area_of(lo, hi);
                rcnt[b] = c;
            }
            for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
            c = 0;
            for (int b = 0; b < kBins - 1; ++b) {
                c += cnt[b];
                for (int k = 0; k < 3; ++k) { lo[k] = std::min(lo[k], blo[b][k]); hi[k] = std::max(hi[k], bhi[b][k]); }
                if (c == 0 || rcnt[b + 1] == 0) continue;
                float cost = area_of(lo, hi) * c + rarea[b + 1] * rcnt[b + 1];
                if (cost < best_cost) { best_cost = cost; best_axis = a; best_split = b + 1; }
            }
        }
        float parea = area_of(n->lo, n->hi);
        float leaf_cost = (float)count;
        float split_cost = parea > 0.f ? 1.0f + best_cost / parea : INFINITY;
        if (count <= max_leaf_ && (best_axis < 0 || leaf_cost <= split_cost)) return leaf(n, first, count);

        int32_t mid;
        if (best_axis >= 0) {
            float ext = chi[best_axis] - clo[best_axis];
            float scale = kBins / ext;
            int a = best_axis, sb = best_split;
            float c0 = clo[a];
            auto it = std::partition(order_.begin() + first, order_.begin() + first + count, [&](int32_t t) {
                int b = std::min(kBins - 1, (int)((info_[t].c[a] - c0) * scale));
                return b < sb;
            });
            mid = (int32_t)(it - order_.begin());
            if (mid == first || mid == first + count) mid = first + count / 2;
        } else {
            mid = first + count / 2;  // all centroids coincide
        }
        int32_t nl = mid - first, nr = count - nl;
        n->first = -1;
        n->count = 0;
        bool spawn = false;
        if (count > 65536) {
            spawn = budget_.fetch_sub(1) > 0;
            if (!spawn) budget_.fetch_add(1);
        }
        if (spawn) {
            Arena* a2 = new_arena();
            auto fut = std::async(std::launch::async, [this, a2, first, nl]() { return rec(first, nl, a2); });
            n->kid[1] = rec(mid, nr, arena);
            n->kid[0] = fut.get();
            budget_.fetch_add(1);
        } else {
            n->kid[0] = rec(first, nl, arena);
            n->kid[1] = rec(mid, nr, arena);
        }
        return n;
    }
};

// binary16 encoding of x >= 0 (finite, below 65504), rounded down or up
uint16_t half_bits(double x, bool up) {
    if (!(x > 0.0)) return 0;
    int k;
    std::frexp(x, &k);  // x in [2^(k-1), 2^k)
    int ex = k - 1;
    double m;
    uint32_t bits;
    if (ex < -14) {  // subnormal: multiples of 2^-24
        m = x * std::ldexp(1.0, 24);
        double q = up ? std::ceil(m) : std::floor(m);
        bits = (uint32_t)q;  // 1024 (the smallest normal) when rounded up from the top
    } else {
        m = (x / std::ldexp(1.0, ex) - 1.0) * 1024.0;  // fraction in [0, 1024)
        double q = up ? std::ceil(m) : std::floor(m);
        bits = ((uint32_t)(ex + 15) << 10) + (uint32_t)q;  // a carry into the exponent stays exact
    }
    return (uint16_t)bits;
}

// Fills a node from its children's boxes (slots with ref == EMPTY unused):
// per axis the origin is the lowest child plane and the scale the power of
// two that brings the node's extent to at most 2^15; every plane offset is
// encoded as binary16, lower planes rounded down and upper planes up (from
// the exact offset in double), so every decoded box encloses its child's.
void quantize_node(Node4& q, const float lo[4][3], const float hi[4][3], const uint32_t ref[4]) {
    q = Node4{};
    float nlo[3] = {0.f, 0.f, 0.f}, nhi[3] = {0.f, 0.f, 0.f};
    bool any = false;
    for (int s = 0; s < 4; ++s) {
        if (ref[s] == kEmptyRef) continue;
        for (int a = 0; a < 3; ++a) {
            nlo[a] = any ? std::min(nlo[a], lo[s][a]) : lo[s][a];
            nhi[a] = any ? std::max(nhi[a], hi[s][a]) : hi[s][a];
        }
        any = true;
    }
    uint32_t* planes[3] = {q.x, q.y, q.z};
    for (int a = 0; a < 3; ++a) {
        const double ext = (double)nhi[a] - (double)nlo[a];
        int e = kNodeGridMinExp;
        if (ext > 0.0) {
            int k;
            std::frexp(ext, &k);  // ext < 2^k
            e = std::max(kNodeGridMinExp, k - 15);
            while (std::ldexp(32768.0, e) < ext) ++e;
        }
        q.o[a] = nlo[a];
        q.e |= (uint32_t)(e + 128) << (8 * a);
        const double scale = std::ldexp(1.0, e);
        uint16_t hl[4], hh[4];
        for (int s = 0; s < 4; ++s) {
            if (ref[s] == kEmptyRef) {
                hl[s] = 0x7C00;  // +inf
                hh[s] = 0xFC00;  // -inf
            } else {
                hl[s] = half_bits(((double)lo[s][a] - (double)nlo[a]) / scale, false);
                hh[s] = half_bits(((double)hi[s][a] - (double)nlo[a]) / scale, true);
            }
        }
        planes[a][0] = hl[0] | ((uint32_t)hl[1] << 16);
        planes[a][1] = hl[2] | ((uint32_t)hl[3] << 16);
        planes[a][2] = hh[0] | ((uint32_t)hh[1] << 16);
        planes[a][3] = hh[2] | ((uint32_t)hh[3] << 16);
    }
    for (int s = 0; s < 4; ++s) q.ref[s] = ref[s];
}

struct Collapser {
    std::vector<Node4>& out;
    float pad;
    int depth = 0;

    static bool is_leaf(const BNode* n) { return n->count > 0 || (n->kid[0] == nullptr); }

    // padded box of a child
    void child_box(const BNode* c, float lo[3], float hi[3]) const {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::nextafter(c->lo[a] - pad, -INFINITY);
            hi[a] = std::nextafter(c->hi[a] + pad, INFINITY);
        }
    }

    static uint32_t leaf_ref(const BNode* n) {
        return kLeafBit | (uint32_t(n->count - 1) << kLeafCountShift) | uint32_t(n->first);
    }

    // Writes node `idx` from the binary subtree rooted at internal node n.
    void emit(uint32_t idx, const BNode* n, int level) {
        depth = std::max(depth, level);
        const BNode* kids[4] = {n->kid[0], n->kid[1], nullptr, nullptr};
        int k = 2;
        while (k < 4) {
            int best = -1;
            float ba = -1.f;
            for (int i = 0; i < k; ++i) {
                if (is_leaf(kids[i])) continue;
                float a = area_of(kids[i]->lo, kids[i]->hi);
                if (a > ba) { ba = a; best = i; }
            }
            if (best < 0) break;
            const BNode* b = kids[best];
            kids[best] = b->kid[0];
            kids[k++] = b->kid[1];
        }
        // allocate the internal children first: emplace_back may move `out`
        uint32_t child_idx[4] = {0, 0, 0, 0};
        for (int s = 0; s < k; ++s) {
            if (is_leaf(kids[s])) continue;
            child_idx[s] = (uint32_t)out.size();
            out.emplace_back();
        }
        float lo[4][3], hi[4][3];
        uint32_t ref[4] = {kEmptyRef, kEmptyRef, kEmptyRef, kEmptyRef};
        for (int s = 0; s < k; ++s) {
            if (is_leaf(kids[s]) && kids[s]->count == 0) continue;  // empty leaf: slot stays empty
            child_box(kids[s], lo[s], hi[s]);
            ref[s] = is_leaf(kids[s]) ? leaf_ref(kids[s]) : child_idx[s];
        }
        quantize_node(out[idx], lo, hi, ref);
        for (int s = 0; s < k; ++s)
            if (!is_leaf(kids[s])) emit(child_idx[s], kids[s], level + 1);
    }
};

}  // namespace

BuildResult build_scene(const std::vector<float>& tri_v, const std::vector<int32_t>& tri_mat,
                        const std::vector<float>& emission, int max_leaf, int threads) {
    BuildResult r;
    const int32_t nt = (int32_t)tri_mat.size();
    max_leaf = std::max(1, std::min(kMaxLeaf, max_leaf));
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());

    std::vector<PrimInfo> info(nt);
    float M = 0.f;
    for (int32_t i = 0; i < nt; ++i) {
        const float* p = &tri_v[9 * (size_t)i];
        for (int a = 0; a < 3; ++a) {
            float lo = std::min(p[a], std::min(p[3 + a], p[6 + a]));
            float hi = std::max(p[a], std::max(p[3 + a], p[6 + a]));
            info[i].lo[a] = lo;
            info[i].hi[a] = hi;
            info[i].c[a] = 0.5f * (lo + hi);
            M = std::max(M, std::max(std::fabs(lo), std::fabs(hi)));
        }
    }
    // boxes are padded by 2^-18 of the largest coordinate so that the slab
    // test can never reject a triangle the watertight test accepts: the
    // padding absorbs the test's absolute rounding (a few ulps of the
    // coordinates), its relative slack the rest
    const float pad = M * 0x1p-18f;
    r.max_coord = M;
    if (nt > 0) {
        for (int a = 0; a < 3; ++a) {
            float lo = info[0].lo[a], hi = info[0].hi[a];
            for (int32_t i = 1; i < nt; ++i) {
                lo = std::min(lo, info[i].lo[a]);
                hi = std::max(hi, info[i].hi[a]);
            }
            r.center[a] = 0.5f * (lo + hi);
        }
    }

    std::vector<int32_t> order(nt);
    for (int32_t i = 0; i < nt; ++i) order[i] = i;
    r.nodes.reserve(nt / 2 + 1);
    r.nodes.emplace_back();
    Collapser col{r.nodes, pad};
    if (nt == 0) {
        const float lo[4][3] = {}, hi[4][3] = {};
        const uint32_t ref[4] = {kEmptyRef, kEmptyRef, kEmptyRef, kEmptyRef};
        quantize_node(r.nodes[0], lo, hi, ref);
        r.depth = 1;
    } else {
        BinaryBuilder bb(info, order, max_leaf, threads);
        BNode* root = bb.build();
        if (Collapser::is_leaf(root)) {
            // a single leaf: wrap it in a root node with one child
            float lo[4][3] = {}, hi[4][3] = {};
            const uint32_t ref[4] = {Collapser::leaf_ref(root), kEmptyRef, kEmptyRef, kEmptyRef};
            col.child_box(root, lo[0], hi[0]);
            quantize_node(r.nodes[0], lo, hi, ref);
            col.depth = 1;
        } else {
            col.emit(0, root, 1);
        }
        r.depth = col.depth;
    }
    r.stack_entries = 3 * r.depth + 1;

    // triangles in leaf order, then the padding
    r.tris.assign(3 * (size_t)nt + kTriPad, make_float4(0.f, 0.f, 0.f, 0.f));
    std::vector<uint8_t> is_light(nt);
    for (int32_t i = 0; i < nt; ++i) {
        const float* e = &emission[3 * (size_t)i];
        is_light[i] = (e[0] > 0.f || e[1] > 0.f || e[2] > 0.f);
    }
    std::vector<uint32_t> leaf_pos(nt);
    for (int32_t j = 0; j < nt; ++j) {
        int32_t t = order[j];
        leaf_pos[t] = (uint32_t)j;
        const float* p = &tri_v[9 * (size_t)t];
        uint32_t id = (uint32_t)t;
        uint32_t mi = (uint32_t)tri_mat[t] | (is_light[t] ? kLightFlag : 0u);
        float fid, fmi;
        std::memcpy(&fid, &id, 4);
        std::memcpy(&fmi, &mi, 4);
        r.tris[3 * (size_t)j + 0] = make_float4(p[0], p[1], p[2], fid);
        r.tris[3 * (size_t)j + 1] = make_float4(p[3], p[4], p[5], fmi);
        r.tris[3 * (size_t)j + 2] = make_float4(p[6], p[7], p[8], 0.f);
    }

    // the kHotTris triangles of largest area (ties to the smaller id), area
    // above zero: their slot + 1 goes into the w word of their third vertex
    {
        std::vector<std::pair<double, int32_t>> ar;
        ar.reserve(nt);
        for (int32_t i = 0; i < nt; ++i) {
            const float* p = &tri_v[9 * (size_t)i];
            double ax = (double)p[3] - (double)p[0], ay = (double)p[4] - (double)p[1], az = (double)p[5] - (double)p[2];
            double bx = (double)p[6] - (double)p[0], by = (double)p[7] - (double)p[1], bz = (double)p[8] - (double)p[2];
            double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
            double a2 = cx * cx + cy * cy + cz * cz;
            if (a2 > 0.0) ar.emplace_back(a2, i);
        }
        const size_t h = std::min<size_t>((size_t)kHotTris, ar.size());
        std::partial_sort(ar.begin(), ar.begin() + (std::ptrdiff_t)h, ar.end(), [](const auto& x, const auto& y) {
            return x.first > y.first || (x.first == y.first && x.second < y.second);
        });
        for (size_t k = 0; k < h; ++k) {
            const uint32_t id = (uint32_t)ar[k].second, slot1 = (uint32_t)k + 1u;
            r.hot_ids.push_back(id);
            float w;
            std::memcpy(&w, &slot1, 4);
            r.tris[3 * (size_t)leaf_pos[id] + 2].w = w;
        }
    }

    // light set in input order: fp64 prefix sums of the triangle areas,
    // quantised to u32 words (last word saturated)
    std::vector<double> cum;
    std::vector<uint32_t> ids;
    double acc = 0.0;
    for (int32_t i = 0; i < nt; ++i) {
        if (!is_light[i]) continue;
        const float* p = &tri_v[9 * (size_t)i];
        double ax = (double)p[3] - (double)p[0], ay = (double)p[4] - (double)p[1], az = (double)p[5] - (double)p[2];
        double bx = (double)p[6] - (double)p[0], by = (double)p[7] - (double)p[1], bz = (double)p[8] - (double)p[2];
        double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
        acc += 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
        cum.push_back(acc);
        ids.push_back((uint32_t)i);
    }
    r.area_total = (float)acc;
    if (acc > 0.0) {
        r.lights.resize(ids.size());
        for (size_t j = 0; j < ids.size(); ++j) {
            uint32_t w;
            if (j + 1 == ids.size()) {
                w = 0xFFFFFFFFu;
            } else {
                double q = std::floor(cum[j] / acc * 4294967296.0);
                w = q > 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)q;
            }
            r.lights[j].tri = leaf_pos[ids[j]];
            r.lights[j].cdf = w;
            r.lights[j].id = ids[j];
            r.lights[j].pad = 0u;
        }
    }
    return r;
}

void xform_tri(const float* M, const float* v, float* out) {
    for (int k = 0; k < 3; ++k) {
        const float x = v[3 * k], y = v[3 * k + 1], z = v[3 * k + 2];
        for (int r = 0; r < 3; ++r) out[3 * k + r] = ((M[4 * r] * x + M[4 * r + 1] * y) + M[4 * r + 2] * z) + M[4 * r + 3];
    }
}

namespace {

// A binary subtree collapsed into nodes[idx] (and nodes appended for its
// internal children); a single leaf is wrapped in a node with one child.
// Returns the depth in BVH4 levels.
int emit_tree(std::vector<Node4>& nodes, uint32_t idx, BNode* root, float pad) {
    Collapser col{nodes, pad};
    if (Collapser::is_leaf(root)) {
        float lo[4][3] = {}, hi[4][3] = {};
        const uint32_t ref[4] = {root->count > 0 ? Collapser::leaf_ref(root) : kEmptyRef, kEmptyRef, kEmptyRef,
                                 kEmptyRef};
        if (root->count > 0) col.child_box(root, lo[0], hi[0]);
        quantize_node(nodes[idx], lo, hi, ref);
        return 1;
    }
    col.emit(idx, root, 1);
    return col.depth;
}

double tri_area(const float* p) {
    double ax = (double)p[3] - (double)p[0], ay = (double)p[4] - (double)p[1], az = (double)p[5] - (double)p[2];
    double bx = (double)p[6] - (double)p[0], by = (double)p[7] - (double)p[1], bz = (double)p[8] - (double)p[2];
    double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    return 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
}

}  // namespace

BuildResult build_instanced(const std::vector<float>& tri_v, const std::vector<int32_t>& tri_mat,
                            const std::vector<float>& emission, const InstanceSet& is, int max_leaf, int threads) {
    BuildResult r;
    const int32_t nt = (int32_t)tri_mat.size();
    const int nmesh = (int)is.mesh_first.size(), ninst = (int)is.inst_mesh.size();
    max_leaf = std::max(1, std::min(kMaxLeaf, max_leaf));
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());

    std::vector<PrimInfo> info(nt);
    for (int32_t i = 0; i < nt; ++i) {
        const float* p = &tri_v[9 * (size_t)i];
        for (int a = 0; a < 3; ++a) {
            float lo = std::min(p[a], std::min(p[3 + a], p[6 + a]));
            float hi = std::max(p[a], std::max(p[3 + a], p[6 + a]));
            info[i].lo[a] = lo;
            info[i].hi[a] = hi;
            info[i].c[a] = 0.5f * (lo + hi);
        }
    }
    // leaf order: each mesh's triangles reordered within its own range
    std::vector<int32_t> order(nt);
    for (int32_t i = 0; i < nt; ++i) order[i] = i;
    r.nodes.emplace_back();  // node 0: the top-level root
    std::vector<uint32_t> mesh_root(nmesh, kEmptyRef);
    std::vector<double> mlo(3 * (size_t)nmesh), mhi(3 * (size_t)nmesh);
    int blas_depth = 0;
    for (int m = 0; m < nmesh; ++m) {
        const int32_t first = is.mesh_first[m], count = is.mesh_count[m];
        if (count == 0) continue;
        // object-space boxes padded by 2^-18 of the mesh's largest coordinate
        // (the flat scene's rule, per mesh)
        float M = 0.f;
        for (int32_t i = first; i < first + count; ++i)
            for (int a = 0; a < 3; ++a) M = std::max(M, std::max(std::fabs(info[i].lo[a]), std::fabs(info[i].hi[a])));
        const float pad = M * 0x1p-18f;
        BinaryBuilder bb(info, order, max_leaf, threads);
        BNode* root = bb.build(first, count);
        const uint32_t idx = (uint32_t)r.nodes.size();
        r.nodes.emplace_back();
        blas_depth = std::max(blas_depth, emit_tree(r.nodes, idx, root, pad));
        mesh_root[m] = idx;
        for (int a = 0; a < 3; ++a) {
            mlo[3 * m + a] = (double)std::nextafter(root->lo[a] - pad, -INFINITY);
            mhi[3 * m + a] = (double)std::nextafter(root->hi[a] + pad, INFINITY);
        }
    }
    // top level over the world boxes of the instances of non-empty meshes:
    // the eight corners of the mesh's padded box mapped by o2w in binary64,
    // then widened by 2^-12 of (extent + largest coordinate magnitude), which
    // covers the difference between the world ray and the rounded
    // object-space ray of an instance (a few ulps of the coordinates times
    // the transform's condition number) for rays within a few hundred scene
    // sizes
    std::vector<PrimInfo> iinfo(ninst);
    std::vector<int32_t> iorder;
    constexpr double kInf = std::numeric_limits<double>::infinity();
    double wlo[3] = {kInf, kInf, kInf}, whi[3] = {-kInf, -kInf, -kInf};
    for (int q = 0; q < ninst; ++q) {
        const int m = is.inst_mesh[q];
        if (mesh_root[m] == kEmptyRef) continue;
        const float* M = &is.o2w[12 * (size_t)q];
        double lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
        for (int c = 0; c < 8; ++c) {
            const double p[3] = {(c & 1) ? mhi[3 * m] : mlo[3 * m], (c & 2) ? mhi[3 * m + 1] : mlo[3 * m + 1],
                                 (c & 4) ? mhi[3 * m + 2] : mlo[3 * m + 2]};
            for (int a = 0; a < 3; ++a) {
                const double w = (double)M[4 * a] * p[0] + (double)M[4 * a + 1] * p[1] + (double)M[4 * a + 2] * p[2] +
                                 (double)M[4 * a + 3];
                lo[a] = std::min(lo[a], w);
                hi[a] = std::max(hi[a], w);
            }
        }
        double ext = 0.0, mag = 0.0;
        for (int a = 0; a < 3; ++a) {
            ext = std::max(ext, hi[a] - lo[a]);
            mag = std::max(mag, std::max(std::fabs(lo[a]), std::fabs(hi[a])));
        }
        const double pad = std::ldexp(ext + mag, -12);
        for (int a = 0; a < 3; ++a) {
            iinfo[q].lo[a] = std::nextafter((float)(lo[a] - pad), -INFINITY);
            iinfo[q].hi[a] = std::nextafter((float)(hi[a] + pad), INFINITY);
            iinfo[q].c[a] = 0.5f * (iinfo[q].lo[a] + iinfo[q].hi[a]);
            wlo[a] = std::min(wlo[a], (double)iinfo[q].lo[a]);
            whi[a] = std::max(whi[a], (double)iinfo[q].hi[a]);
        }
        iorder.push_back(q);
    }
    int tlas_depth = 1;
    if (iorder.empty()) {
        const float lo[4][3] = {}, hi[4][3] = {};
        const uint32_t ref[4] = {kEmptyRef, kEmptyRef, kEmptyRef, kEmptyRef};
        quantize_node(r.nodes[0], lo, hi, ref);
    } else {
        BinaryBuilder tb(iinfo, iorder, 1, threads);
        BNode* root = tb.build();
        tlas_depth = emit_tree(r.nodes, 0, root, 0.f);
        for (int a = 0; a < 3; ++a) {
            r.center[a] = (float)(0.5 * (wlo[a] + whi[a]));
            r.max_coord = std::max(r.max_coord, (float)std::max(std::fabs(wlo[a]), std::fabs(whi[a])));
        }
    }
    r.depth = tlas_depth + blas_depth;
    // top-level entries, the return marker, then the mesh's entries
    r.stack_entries = 3 * (tlas_depth + blas_depth) + 2;

    // instance records in top-level leaf order
    std::vector<uint32_t> rec_of(ninst, 0xFFFFFFFFu);
    r.insts.resize((size_t)kInstRecord * iorder.size());
    for (size_t pos = 0; pos < iorder.size(); ++pos) {
        const int q = iorder[pos];
        rec_of[q] = (uint32_t)pos;
        float4* rec = &r.insts[(size_t)kInstRecord * pos];
        const float* W = &is.w2o[12 * (size_t)q];
        const float* O = &is.o2w[12 * (size_t)q];
        for (int row = 0; row < 3; ++row) {
            rec[row] = make_float4(W[4 * row], W[4 * row + 1], W[4 * row + 2], W[4 * row + 3]);
            rec[3 + row] = make_float4(O[4 * row], O[4 * row + 1], O[4 * row + 2], O[4 * row + 3]);
        }
        const uint32_t root = mesh_root[is.inst_mesh[q]], qq = (uint32_t)q;
        float froot, fq;
        std::memcpy(&froot, &root, 4);
        std::memcpy(&fq, &qq, 4);
        rec[6] = make_float4(froot, fq, 0.f, 0.f);
    }

    // triangles in leaf order
    std::vector<uint8_t> is_light(nt);
    for (int32_t i = 0; i < nt; ++i) {
        const float* e = &emission[3 * (size_t)i];
        is_light[i] = (e[0] > 0.f || e[1] > 0.f || e[2] > 0.f);
    }
    r.tris.assign(3 * (size_t)nt + kTriPad, make_float4(0.f, 0.f, 0.f, 0.f));
    std::vector<uint32_t> leaf_pos(nt);
    for (int32_t j = 0; j < nt; ++j) {
        const int32_t t = order[j];
        leaf_pos[t] = (uint32_t)j;
        const float* p = &tri_v[9 * (size_t)t];
        const uint32_t id = (uint32_t)t, mi = (uint32_t)tri_mat[t] | (is_light[t] ? kLightFlag : 0u);
        float fid, fmi;
        std::memcpy(&fid, &id, 4);
        std::memcpy(&fmi, &mi, 4);
        r.tris[3 * (size_t)j + 0] = make_float4(p[0], p[1], p[2], fid);
        r.tris[3 * (size_t)j + 1] = make_float4(p[3], p[4], p[5], fmi);
        r.tris[3 * (size_t)j + 2] = make_float4(p[6], p[7], p[8], 0.f);
    }

    // lights: every (instance, emissive triangle) in instance order, areas of
    // the world-space triangles in binary64
    std::vector<double> cum;
    std::vector<LightEntry> ent;
    double acc = 0.0;
    for (int q = 0; q < ninst; ++q) {
        const int m = is.inst_mesh[q];
        for (int32_t i = is.mesh_first[m]; i < is.mesh_first[m] + is.mesh_count[m]; ++i) {
            if (!is_light[i]) continue;
            float w[9];
            xform_tri(&is.o2w[12 * (size_t)q], &tri_v[9 * (size_t)i], w);
            acc += tri_area(w);
            cum.push_back(acc);
            ent.push_back(LightEntry{leaf_pos[i], 0u, (uint32_t)i, rec_of[q]});
        }
    }
    r.area_total = (float)acc;
    if (acc > 0.0) {
        r.lights = ent;
        for (size_t j = 0; j < ent.size(); ++j) {
            if (j + 1 == ent.size()) {
                r.lights[j].cdf = 0xFFFFFFFFu;
            } else {
                double q = std::floor(cum[j] / acc * 4294967296.0);
                r.lights[j].cdf = q > 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)q;
            }
        }
    }
    return r;
}

}  // namespace ptmi
