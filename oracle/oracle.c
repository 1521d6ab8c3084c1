/*
 * CPU oracle for unidirectional Monte Carlo path tracing of triangle scenes.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark, never by the renderer.  It shares
 * no code with the HIP library.
 *
 * The estimator follows the paper's Sec. 2.2 (Eq. 3 and its five-step
 * forward path-tracing loop); points the paper leaves open (random number
 * generator, camera, intersection test, materials, next-event estimation,
 * roulette rule, ray offsets) are fixed by the readings written out next to
 * each function.  Path arithmetic is binary32 in source order with no
 * contraction, so that float-decided choices are taken in the renderer's
 * precision.  Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math.
 */
#define _GNU_SOURCE
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* small vector helpers (binary32, source-order evaluation)                  */
/* ------------------------------------------------------------------------ */
typedef struct { float x, y, z; } v3;

static v3 V(float x, float y, float z) { v3 r = {x, y, z}; return r; }
static v3 vadd(v3 a, v3 b) { return V(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vsub(v3 a, v3 b) { return V(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vscale(v3 a, float s) { return V(a.x * s, a.y * s, a.z * s); }
static v3 vneg(v3 a) { return V(-a.x, -a.y, -a.z); }
static float vdot(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static v3 vcross(v3 a, v3 b)
{
    return V(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
/* normalize: multiply by the correctly rounded 1/sqrt(|v|^2) */
static v3 vnorm(v3 a)
{
    float s = 1.0f / sqrtf(vdot(a, a));
    return vscale(a, s);
}
static float vget(v3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
static v3 vload(const float* p) { return V(p[0], p[1], p[2]); }
static void vstore(float* p, v3 a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }

#define PI_F ((float)3.14159265358979323846)
#define INV_PI_F ((float)(1.0 / 3.14159265358979323846))
#define SHADOW_TMAX 0.9999f
#define FRAG_EPS 1e-5f
/* fragility reasons (bit mask) */
#define FR_TIE 1
#define FR_EDGE 2
#define FR_NEARMISS 4
#define FR_THRESH 8
#define FR_GRAZE 16

float orc_unif(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC 2011): ten rounds of two 64x64->128      */
/* multiplies, the key bumped by the two Weyl constants between rounds.      */
/* ------------------------------------------------------------------------ */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Eight 32-bit words for (pixel, sample, bounce, job) under key (seed, 0):
 * word 2i is the low half of output i, word 2i+1 its high half. */
static void rng_words(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce,
                      uint32_t job, uint32_t w[8])
{
    uint64_t ctr[4] = {pixel, sample, bounce, job}, key[2] = {seed, 0}, out[4];
    orc_philox4x64(ctr, key, out);
    for (int i = 0; i < 4; ++i) {
        w[2 * i] = (uint32_t)out[i];
        w[2 * i + 1] = (uint32_t)(out[i] >> 32);
    }
}

/* ------------------------------------------------------------------------ */
/* Halton(2,3) camera jitter with a per-pixel Cranley-Patterson rotation     */
/* (the sampler of the paper's wavefront renderer).  The radical inverse     */
/* phi_b(n) = sum_i d_i b^-(i+1) of the base-b digits d_i of n, truncated to */
/* 24 bits: an integer q with q 2^-24 <= phi_b(n) < (q + 1) 2^-24.  The      */
/* rotation adds 24-bit offsets drawn once per pixel (Philox words 0 and 1   */
/* of the reserved sample index 0xFFFFFFFF) modulo 1.                        */
/* ------------------------------------------------------------------------ */
static uint32_t radical_inverse24(uint32_t n, int base)
{
    if (base == 2) {
        uint32_t rev = 0;
        for (int i = 0; i < 32; ++i) {  /* bit i of n becomes bit 31 - i */
            rev = (rev << 1) | (n & 1u);
            n >>= 1;
        }
        return rev >> 8;
    }
    /* base 3: R = sum_{i<21} d_i 3^(20-i) (3^21 > 2^32, so every digit of a
     * 32-bit n is included), phi_3(n) = R / 3^21 exactly */
    uint64_t R = 0, p21 = 1;
    for (int i = 0; i < 21; ++i) {
        R = R * 3u + (n % 3u);
        n /= 3u;
        p21 *= 3u;
    }
    return (uint32_t)((R << 24) / p21);
}

float orc_radical_inverse(uint32_t n, int32_t base)
{
    return (float)radical_inverse24(n, base == 2 ? 2 : 3) * 0x1p-24f;
}

void orc_halton_jitter(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t job, float out[2])
{
    uint32_t w[8];
    rng_words(seed, pixel, 0xFFFFFFFFu, 0, job, w);
    const uint32_t u0 = (radical_inverse24(sample, 2) + (w[0] >> 8)) & 0xFFFFFFu;
    const uint32_t u1 = (radical_inverse24(sample, 3) + (w[1] >> 8)) & 0xFFFFFFu;
    out[0] = (float)u0 * 0x1p-24f;
    out[1] = (float)u1 * 0x1p-24f;
}

/* ------------------------------------------------------------------------ */
/* scene                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    float lo[3], hi[3];
    int32_t left, right;  /* children (internal) */
    int32_t first, count; /* triangle range in order[] (leaf: count > 0) */
} onode;

struct orc_scene {
    int32_t nt, nm;
    float* v;          /* nt * 9: v0, v1, v2 */
    int32_t* tri_mat;  /* nt */
    float* mats;       /* nm * 4 */
    float* albedo;     /* nt * 3 */
    float* emission;   /* nt * 3 */
    uint8_t* is_light; /* nt */
    float sky[3];
    /* light set: area-proportional CDF in u32 fixed point */
    int32_t nl;
    int32_t* light_tri;
    uint32_t* light_cdf;
    float area_total;
    /* oracle BVH */
    onode* nodes;
    int32_t nnodes, depth;
    int32_t* order;
    /* two-level scene: ninst > 0 places meshes (ranges of the triangles, in
     * object space) by affine maps; the triangles alone are then no longer
     * world geometry.  o2w, w2o: 12 floats per instance (3x4, row-major). */
    int32_t nmesh, ninst;
    int32_t *mesh_first, *mesh_count, *mesh_root;
    int32_t* inst_mesh;
    float *o2w, *w2o;
    int32_t* light_inst; /* instance of each light */
    /* vertex attributes per triangle corner (NULL when absent): normals
     * nt * 9 (n0, n1, n2), texture coordinates nt * 6 (uv0, uv1, uv2) */
    float* nrm;
    float* uv;
};

/* Affine map by a 3x4 row-major matrix M (row r: linear part M[4r..4r+2],
 * translation M[4r+3]), in this order: ((M0 x + M1 y) + M2 z) + M3.  The
 * direction map drops the translation. */
static v3 xform_point(const float* M, v3 p)
{
    return V(((M[0] * p.x + M[1] * p.y) + M[2] * p.z) + M[3], ((M[4] * p.x + M[5] * p.y) + M[6] * p.z) + M[7],
             ((M[8] * p.x + M[9] * p.y) + M[10] * p.z) + M[11]);
}
static v3 xform_dir(const float* M, v3 d)
{
    return V((M[0] * d.x + M[1] * d.y) + M[2] * d.z, (M[4] * d.x + M[5] * d.y) + M[6] * d.z,
             (M[8] * d.x + M[9] * d.y) + M[10] * d.z);
}

/* World-space vertices (9 floats) of triangle tri, placed by instance inst
 * (the triangle itself in a flat scene): out, or the triangle's own array. */
static const float* world_tri(const orc_scene* s, int32_t inst, int32_t tri, float out[9])
{
    const float* p = s->v + 9 * (size_t)tri;
    if (s->ninst == 0) return p;
    const float* M = s->o2w + 12 * (size_t)inst;
    for (int k = 0; k < 3; ++k) {
        v3 w = xform_point(M, V(p[3 * k], p[3 * k + 1], p[3 * k + 2]));
        out[3 * k] = w.x; out[3 * k + 1] = w.y; out[3 * k + 2] = w.z;
    }
    return out;
}

static int finite3(const float* p) { return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]); }

/* Light set = triangles with some emission channel > 0 at creation time.
 * CDF: fp64 prefix sums of the areas 0.5 |(v1-v0) x (v2-v0)| in triangle
 * order, quantised as floor(cum/total * 2^32), the last entry forced to
 * 2^32-1.  A raw word w selects the first light j with w <= cdf[j]. */
/* In a two-level scene the light set is every (instance, emissive triangle of
 * its mesh) pair, in instance order, with the areas of the world-space
 * triangles (world_tri). */
static void build_lights(orc_scene* s)
{
    free(s->light_tri); free(s->light_cdf); free(s->light_inst);
    s->nl = 0;
    const int ninst = s->ninst > 0 ? s->ninst : 1;
    for (int q = 0; q < ninst; ++q) {
        int first = s->ninst > 0 ? s->mesh_first[s->inst_mesh[q]] : 0;
        int count = s->ninst > 0 ? s->mesh_count[s->inst_mesh[q]] : s->nt;
        for (int i = first; i < first + count; ++i) s->nl += s->is_light[i];
    }
    s->light_tri = (int32_t*)malloc(sizeof(int32_t) * (s->nl ? s->nl : 1));
    s->light_inst = (int32_t*)malloc(sizeof(int32_t) * (s->nl ? s->nl : 1));
    s->light_cdf = (uint32_t*)malloc(sizeof(uint32_t) * (s->nl ? s->nl : 1));
    double* cum = (double*)malloc(sizeof(double) * (s->nl ? s->nl : 1));
    double acc = 0.0;
    int j = 0;
    for (int q = 0; q < ninst; ++q) {
      int first = s->ninst > 0 ? s->mesh_first[s->inst_mesh[q]] : 0;
      int count = s->ninst > 0 ? s->mesh_count[s->inst_mesh[q]] : s->nt;
      for (int i = first; i < first + count; ++i) {
        if (!s->is_light[i]) continue;
        float tw[9];
        const float* t = world_tri(s, q, i, tw);
        double e1x = (double)t[3] - (double)t[0], e1y = (double)t[4] - (double)t[1],
               e1z = (double)t[5] - (double)t[2];
        double e2x = (double)t[6] - (double)t[0], e2y = (double)t[7] - (double)t[1],
               e2z = (double)t[8] - (double)t[2];
        double cx = e1y * e2z - e1z * e2y, cy = e1z * e2x - e1x * e2z, cz = e1x * e2y - e1y * e2x;
        double area = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
        acc += area;
        cum[j] = acc;
        s->light_tri[j] = i;
        s->light_inst[j] = s->ninst > 0 ? q : 0;
        ++j;
      }
    }
    s->area_total = (float)acc;
    for (j = 0; j < s->nl; ++j) {
        if (j == s->nl - 1 || acc <= 0.0) {
            s->light_cdf[j] = 0xFFFFFFFFu;
        } else {
            double q = floor(cum[j] / acc * 4294967296.0);
            if (q > 4294967295.0) q = 4294967295.0;
            s->light_cdf[j] = (uint32_t)q;
        }
    }
    if (acc <= 0.0) s->nl = 0;
    free(cum);
}

int32_t orc_pick_light(const orc_scene* s, uint32_t w)
{
    if (s->nl == 0) return -1;
    int lo = 0, hi = s->nl - 1; /* first j with w <= cdf[j] */
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (w <= s->light_cdf[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

/* ---- oracle BVH: binary, object-median split on the longest centroid axis,
 * leaves of at most two triangles.  Every box is padded by 2^-18 times the
 * largest absolute vertex coordinate so that the box test can never reject a
 * triangle the exact triangle test accepts (see box_test).             ---- */
typedef struct { const orc_scene* s; int axis; } sort_ctx;
static __thread sort_ctx g_sort;

static float centroid(const orc_scene* s, int t, int a)
{
    const float* p = s->v + 9 * (size_t)t;
    return (p[a] + p[3 + a] + p[6 + a]) / 3.0f;
}

static int cmp_centroid(const void* A, const void* B)
{
    int a = *(const int*)A, b = *(const int*)B;
    float ca = centroid(g_sort.s, a, g_sort.axis), cb = centroid(g_sort.s, b, g_sort.axis);
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return (a > b) - (a < b);
}

static int bvh_build_rec(orc_scene* s, int first, int count, int depth, float pad)
{
    int ni = s->nnodes++;
    onode nd;
    memset(&nd, 0, sizeof nd);
    for (int a = 0; a < 3; ++a) { nd.lo[a] = INFINITY; nd.hi[a] = -INFINITY; }
    for (int i = first; i < first + count; ++i) {
        const float* p = s->v + 9 * (size_t)s->order[i];
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) {
                if (p[3 * k + a] < nd.lo[a]) nd.lo[a] = p[3 * k + a];
                if (p[3 * k + a] > nd.hi[a]) nd.hi[a] = p[3 * k + a];
            }
    }
    for (int a = 0; a < 3; ++a) {
        nd.lo[a] = nextafterf(nd.lo[a] - pad, -INFINITY);
        nd.hi[a] = nextafterf(nd.hi[a] + pad, INFINITY);
    }
    if (depth + 1 > s->depth) s->depth = depth + 1;
    if (count <= 2) {
        nd.first = first;
        nd.count = count;
        nd.left = nd.right = -1;
        s->nodes[ni] = nd;
        return ni;
    }
    float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = first; i < first + count; ++i)
        for (int a = 0; a < 3; ++a) {
            float c = centroid(s, s->order[i], a);
            if (c < clo[a]) clo[a] = c;
            if (c > chi[a]) chi[a] = c;
        }
    int axis = 0;
    for (int a = 1; a < 3; ++a)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    g_sort.s = s;
    g_sort.axis = axis;
    qsort(s->order + first, (size_t)count, sizeof(int), cmp_centroid);
    int half = count / 2;
    nd.count = 0;
    nd.first = -1;
    s->nodes[ni] = nd;
    int l = bvh_build_rec(s, first, half, depth + 1, pad);
    int r = bvh_build_rec(s, first + half, count - half, depth + 1, pad);
    s->nodes[ni].left = l;
    s->nodes[ni].right = r;
    return ni;
}

static void build_bvh(orc_scene* s)
{
    free(s->order); free(s->nodes);
    s->order = (int32_t*)malloc(sizeof(int32_t) * (s->nt ? s->nt : 1));
    for (int i = 0; i < s->nt; ++i) s->order[i] = i;
    s->nodes = (onode*)malloc(sizeof(onode) * (size_t)(2 * (s->nt ? s->nt : 1)));
    s->nnodes = 0;
    s->depth = 0;
    if (s->nt == 0) return;
    /* one BVH over all triangles (flat scene), or one per mesh in object
     * space (two-level scene), each padded by 2^-18 of its own largest
     * coordinate */
    const int nb = s->ninst > 0 ? s->nmesh : 1;
    for (int b = 0; b < nb; ++b) {
        int first = s->ninst > 0 ? s->mesh_first[b] : 0, count = s->ninst > 0 ? s->mesh_count[b] : s->nt;
        float m = 0.0f;
        for (size_t i = 9 * (size_t)first; i < 9 * (size_t)(first + count); ++i)
            if (fabsf(s->v[i]) > m) m = fabsf(s->v[i]);
        int root = count > 0 ? bvh_build_rec(s, first, count, 0, m * 0x1p-18f) : -1;
        if (s->ninst > 0) s->mesh_root[b] = root;
    }
}

orc_scene* orc_scene_create(int32_t nv, const float* pos, int32_t nt, const int32_t* idx,
                            const int32_t* tri_mat, int32_t nm, const float* mats,
                            const float* albedo, const float* emission, const float* sky,
                            int32_t build)
{
    if (nv < 0 || nt < 0 || nm <= 0) return NULL;
    for (int i = 0; i < nv; ++i)
        if (!finite3(pos + 3 * (size_t)i)) return NULL;
    for (int i = 0; i < nt; ++i) {
        for (int k = 0; k < 3; ++k)
            if (idx[3 * (size_t)i + k] < 0 || idx[3 * (size_t)i + k] >= nv) return NULL;
        if (tri_mat[i] < 0 || tri_mat[i] >= nm) return NULL;
        if (!finite3(albedo + 3 * (size_t)i) || !finite3(emission + 3 * (size_t)i)) return NULL;
    }
    orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
    s->nt = nt;
    s->nm = nm;
    s->v = (float*)malloc(sizeof(float) * 9 * (size_t)(nt ? nt : 1));
    for (int i = 0; i < nt; ++i)
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a)
                s->v[9 * (size_t)i + 3 * k + a] = pos[3 * (size_t)idx[3 * (size_t)i + k] + a];
    s->tri_mat = (int32_t*)malloc(sizeof(int32_t) * (nt ? nt : 1));
    memcpy(s->tri_mat, tri_mat, sizeof(int32_t) * nt);
    s->mats = (float*)malloc(sizeof(float) * 4 * nm);
    memcpy(s->mats, mats, sizeof(float) * 4 * nm);
    s->albedo = (float*)malloc(sizeof(float) * 3 * (size_t)(nt ? nt : 1));
    s->emission = (float*)malloc(sizeof(float) * 3 * (size_t)(nt ? nt : 1));
    memcpy(s->albedo, albedo, sizeof(float) * 3 * (size_t)nt);
    memcpy(s->emission, emission, sizeof(float) * 3 * (size_t)nt);
    s->is_light = (uint8_t*)malloc(nt ? nt : 1);
    for (int i = 0; i < nt; ++i) {
        const float* e = emission + 3 * (size_t)i;
        s->is_light[i] = (e[0] > 0.0f || e[1] > 0.0f || e[2] > 0.0f);
    }
    s->sky[0] = sky[0]; s->sky[1] = sky[1]; s->sky[2] = sky[2];
    build_lights(s);
    if (build) build_bvh(s);
    return s;
}

void orc_scene_set_params(orc_scene* s, const float* albedo, const float* emission)
{
    memcpy(s->albedo, albedo, sizeof(float) * 3 * (size_t)s->nt);
    memcpy(s->emission, emission, sizeof(float) * 3 * (size_t)s->nt);
}

int32_t orc_scene_num_lights(const orc_scene* s) { return s->nl; }

void orc_scene_bvh_stats(const orc_scene* s, int32_t* nodes, int32_t* depth)
{
    *nodes = s->nodes ? s->nnodes : 0;
    *depth = s->nodes ? s->depth : 0;
}

void orc_scene_destroy(orc_scene* s)
{
    if (!s) return;
    free(s->v); free(s->tri_mat); free(s->mats); free(s->albedo); free(s->emission);
    free(s->is_light); free(s->light_tri); free(s->light_cdf); free(s->nodes); free(s->order);
    free(s->mesh_first); free(s->mesh_count); free(s->mesh_root); free(s->inst_mesh); free(s->o2w); free(s->w2o);
    free(s->light_inst);
    free(s->nrm); free(s->uv);
    free(s);
}

int32_t orc_scene_set_instances(orc_scene* s, int32_t n_meshes, const int32_t* mesh_first,
                                const int32_t* mesh_count, int32_t n_inst, const int32_t* inst_mesh,
                                const float* o2w, const float* w2o)
{
    if (n_meshes < 1 || n_inst < 1) return -1;
    for (int m = 0; m < n_meshes; ++m)
        if (mesh_first[m] < 0 || mesh_count[m] < 0 || (int64_t)mesh_first[m] + mesh_count[m] > s->nt) return -1;
    for (int q = 0; q < n_inst; ++q) {
        if (inst_mesh[q] < 0 || inst_mesh[q] >= n_meshes) return -1;
        for (int k = 0; k < 12; ++k)
            if (!isfinite(o2w[12 * (size_t)q + k]) || !isfinite(w2o[12 * (size_t)q + k])) return -1;
    }
    int had_bvh = s->nodes != NULL;
    s->nmesh = n_meshes;
    s->ninst = n_inst;
    s->mesh_first = (int32_t*)malloc(sizeof(int32_t) * n_meshes);
    s->mesh_count = (int32_t*)malloc(sizeof(int32_t) * n_meshes);
    s->mesh_root = (int32_t*)malloc(sizeof(int32_t) * n_meshes);
    memcpy(s->mesh_first, mesh_first, sizeof(int32_t) * n_meshes);
    memcpy(s->mesh_count, mesh_count, sizeof(int32_t) * n_meshes);
    s->inst_mesh = (int32_t*)malloc(sizeof(int32_t) * n_inst);
    memcpy(s->inst_mesh, inst_mesh, sizeof(int32_t) * n_inst);
    s->o2w = (float*)malloc(sizeof(float) * 12 * (size_t)n_inst);
    s->w2o = (float*)malloc(sizeof(float) * 12 * (size_t)n_inst);
    memcpy(s->o2w, o2w, sizeof(float) * 12 * (size_t)n_inst);
    memcpy(s->w2o, w2o, sizeof(float) * 12 * (size_t)n_inst);
    build_lights(s);
    if (had_bvh) build_bvh(s);
    return 0;
}

int32_t orc_scene_set_attributes(orc_scene* s, int32_t nv, const int32_t* idx, const float* normals,
                                 const float* uvs)
{
    for (int i = 0; i < s->nt; ++i)
        for (int k = 0; k < 3; ++k)
            if (idx[3 * (size_t)i + k] < 0 || idx[3 * (size_t)i + k] >= nv) return -1;
    for (int i = 0; i < nv; ++i) {
        if (normals && !finite3(normals + 3 * (size_t)i)) return -1;
        if (uvs && !(isfinite(uvs[2 * (size_t)i]) && isfinite(uvs[2 * (size_t)i + 1]))) return -1;
    }
    free(s->nrm); free(s->uv);
    s->nrm = NULL; s->uv = NULL;
    size_t nt = (size_t)(s->nt ? s->nt : 1);
    if (normals) {
        s->nrm = (float*)malloc(sizeof(float) * 9 * nt);
        for (int i = 0; i < s->nt; ++i)
            for (int k = 0; k < 3; ++k)
                for (int a = 0; a < 3; ++a)
                    s->nrm[9 * (size_t)i + 3 * k + a] = normals[3 * (size_t)idx[3 * (size_t)i + k] + a];
    }
    if (uvs) {
        s->uv = (float*)malloc(sizeof(float) * 6 * nt);
        for (int i = 0; i < s->nt; ++i)
            for (int k = 0; k < 3; ++k)
                for (int a = 0; a < 2; ++a)
                    s->uv[6 * (size_t)i + 2 * k + a] = uvs[2 * (size_t)idx[3 * (size_t)i + k] + a];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* camera (pinhole, box-filtered jitter)                                     */
/* Host constants in binary64, rounded once: F = unit(target - eye),         */
/* R = unit(F x up) * tan(vfov/2) * W/H, U = (R' x F) * tan(vfov/2).         */
/* ------------------------------------------------------------------------ */
void orc_camera(const double e[3], const double t[3], const double up[3], double vfov_deg,
                int32_t width, int32_t height, float out[12])
{
    double f[3] = {t[0] - e[0], t[1] - e[1], t[2] - e[2]};
    double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    f[0] = f[0] / fl; f[1] = f[1] / fl; f[2] = f[2] / fl;
    double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    double rl = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    r[0] = r[0] / rl; r[1] = r[1] / rl; r[2] = r[2] / rl;
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    double th = tan(0.5 * (vfov_deg * (3.14159265358979323846 / 180.0)));
    double asp = (double)width / (double)height;
    for (int a = 0; a < 3; ++a) {
        out[a] = (float)e[a];
        out[3 + a] = (float)(r[a] * (th * asp));
        out[6 + a] = (float)(u[a] * th);
        out[9 + a] = (float)f[a];
    }
}

/* Primary ray through pixel (px, py) (py = 0 is the top row) at sub-pixel
 * offset (u0, u1) in [0,1)^2. */
static void camera_ray(const float cam[12], int W, int H, int px, int py, float u0, float u1,
                       v3* o, v3* d)
{
    float sx = (((float)px + u0) / (float)W) * 2.0f - 1.0f;
    float sy = 1.0f - (((float)py + u1) / (float)H) * 2.0f;
    v3 R = vload(cam + 3), U = vload(cam + 6), F = vload(cam + 9);
    v3 dd = V((sx * R.x + sy * U.x) + F.x, (sx * R.y + sy * U.y) + F.y, (sx * R.z + sy * U.z) + F.z);
    *o = vload(cam);
    *d = vnorm(dd);
}

/* ------------------------------------------------------------------------ */
/* watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013)             */
/* ------------------------------------------------------------------------ */
typedef struct {
    v3 o, d;
    float inv[3];
    int kx, ky, kz;
    float Sx, Sy, Sz;
} ray_t;

static void ray_setup(ray_t* r, v3 o, v3 d)
{
    r->o = o;
    r->d = d;
    r->inv[0] = 1.0f / d.x; r->inv[1] = 1.0f / d.y; r->inv[2] = 1.0f / d.z;
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = 0;
    float m = ax;
    if (ay > m) { kz = 1; m = ay; }
    if (az > m) { kz = 2; }
    int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
    if (vget(d, kz) < 0.0f) { int tmp = kx; kx = ky; ky = tmp; }
    r->kx = kx; r->ky = ky; r->kz = kz;
    r->Sx = vget(d, kx) / vget(d, kz);
    r->Sy = vget(d, ky) / vget(d, kz);
    r->Sz = 1.0f / vget(d, kz);
}

/* Returns 1 on a hit with t > 0 (t, barycentrics of v1 and v2).  *margin
 * receives the smallest barycentric on a hit, or the relative size of the
 * wrong-signed edge functions on a miss (for fragility flags). */
static int tri_test(const ray_t* r, const float* p, float* t_out, float* b1, float* b2,
                    float* margin)
{
    v3 A = vsub(vload(p), r->o), B = vsub(vload(p + 3), r->o), C = vsub(vload(p + 6), r->o);
    float Ax = vget(A, r->kx) - r->Sx * vget(A, r->kz);
    float Ay = vget(A, r->ky) - r->Sy * vget(A, r->kz);
    float Bx = vget(B, r->kx) - r->Sx * vget(B, r->kz);
    float By = vget(B, r->ky) - r->Sy * vget(B, r->kz);
    float Cx = vget(C, r->kx) - r->Sx * vget(C, r->kz);
    float Cy = vget(C, r->ky) - r->Sy * vget(C, r->kz);
    float U = Cx * By - Cy * Bx;
    float Vv = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || Vv == 0.0f || W == 0.0f) {
        /* exact products of binary32 values, one rounding each */
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        Vv = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    *margin = 1.0f;
    if ((U < 0.0f || Vv < 0.0f || W < 0.0f) && (U > 0.0f || Vv > 0.0f || W > 0.0f)) {
        float pos = (U > 0.0f ? U : 0.0f) + (Vv > 0.0f ? Vv : 0.0f) + (W > 0.0f ? W : 0.0f);
        float neg = (U < 0.0f ? -U : 0.0f) + (Vv < 0.0f ? -Vv : 0.0f) + (W < 0.0f ? -W : 0.0f);
        float small = pos < neg ? pos : neg;
        *margin = -small / (pos + neg);
        *t_out = 0.0f;
        float dm = (U + Vv) + W;
        if (dm != 0.0f)
            *t_out = ((U * (r->Sz * vget(A, r->kz)) + Vv * (r->Sz * vget(B, r->kz))) + W * (r->Sz * vget(C, r->kz))) / dm;
        return 0;
    }
    float det = (U + Vv) + W;
    if (det == 0.0f) return 0;
    float Az = r->Sz * vget(A, r->kz);
    float Bz = r->Sz * vget(B, r->kz);
    float Cz = r->Sz * vget(C, r->kz);
    float T = (U * Az + Vv * Bz) + W * Cz;
    float t = T / det;
    if (!(t > 0.0f)) return 0;
    float q0 = U / det, q1 = Vv / det, q2 = W / det;
    *t_out = t;
    *b1 = q1;
    *b2 = q2;
    float mm = q0 < q1 ? q0 : q1;
    *margin = mm < q2 ? mm : q2;
    return 1;
}

int32_t orc_tri_test(const float o[3], const float d[3], const float v0[3], const float v1[3],
                     const float v2[3], float* t, float* b1, float* b2)
{
    ray_t r;
    ray_setup(&r, vload(o), vload(d));
    float p[9];
    memcpy(p, v0, 12); memcpy(p + 3, v1, 12); memcpy(p + 6, v2, 12);
    float m;
    *t = 0.0f; *b1 = 0.0f; *b2 = 0.0f;
    return tri_test(&r, p, t, b1, b2, &m);
}

typedef struct {
    float t, b1, b2;
    int32_t prim;
    int32_t inst; /* instance of the hit (0 in a flat scene) */
    float margin; /* smallest barycentric of the current best hit */
    float tie_t;  /* largest t of the closest pair of near-equal hits seen */
    float miss_t; /* smallest plane distance of a near-missed triangle */
} hit_t;

/* Candidate update with the (t, instance, id) lexicographic order (instance
 * 0 in a flat scene).  For the fragility flags it also remembers near-ties
 * (relative 2^-20) between distinct triangles and near-misses (within 1e-6
 * barycentric of an edge); they are judged against the final closest hit in
 * closest().  r is the ray in the triangle's own space (object space of the
 * instance), whose parameter t is the world ray's. */
static void consider(const orc_scene* s, const ray_t* r, int tri, int inst, float tmax, hit_t* h)
{
    float t, b1, b2, m;
    int ok = tri_test(r, s->v + 9 * (size_t)tri, &t, &b1, &b2, &m);
    if (!ok) {
        if (m < 0.0f && m > -1e-6f && t > 0.0f && t < h->miss_t) h->miss_t = t;
        return;
    }
    if (!(t < tmax)) return;
    if (h->prim >= 0 && fabsf(t - h->t) <= h->t * 0x1p-20f) {
        float hi = t > h->t ? t : h->t;
        if (hi < h->tie_t) h->tie_t = hi;
    }
    if (t < h->t || (t == h->t && (inst < h->inst || (inst == h->inst && tri < h->prim)))) {
        h->t = t; h->b1 = b1; h->b2 = b2; h->prim = tri; h->inst = inst; h->margin = m;
    }
}

/* The ray in the object space of instance q: origin and direction mapped by
 * its world-to-object matrix (xform_point, xform_dir), not renormalised, so
 * that a point at parameter t is the image of the world ray's point at t. */
static void object_ray(const orc_scene* s, int q, const ray_t* r, ray_t* ro)
{
    const float* M = s->w2o + 12 * (size_t)q;
    ray_setup(ro, xform_point(M, r->o), xform_dir(M, r->d));
}

/* Conservative slab test: entry <= exit * (1 + 2^-16), entry clamped at 0
 * and exit at tlim.  A zero direction component keeps the slab unbounded
 * when the origin lies inside it. */
static int box_test(const onode* nd, const ray_t* r, float tlim, float* tnear)
{
    float t0 = 0.0f, t1 = tlim;
    for (int a = 0; a < 3; ++a) {
        float o = vget(r->o, a), d = vget(r->d, a);
        if (d == 0.0f) {
            if (o < nd->lo[a] || o > nd->hi[a]) return 0;
            continue;
        }
        float ta = (nd->lo[a] - o) * r->inv[a];
        float tb = (nd->hi[a] - o) * r->inv[a];
        float tn = ta < tb ? ta : tb, tf = ta < tb ? tb : ta;
        if (tn > t0) t0 = tn;
        if (tf < t1) t1 = tf;
    }
    *tnear = t0;
    return t0 <= t1 * (1.0f + 0x1p-16f);
}

static void bvh_closest_rec(const orc_scene* s, int ni, const ray_t* r, int inst, float tmax, hit_t* h)
{
    const onode* nd = &s->nodes[ni];
    float tn;
    float lim = h->prim >= 0 ? h->t : tmax;
    if (!box_test(nd, r, lim, &tn)) return;
    if (nd->count > 0) {
        for (int i = nd->first; i < nd->first + nd->count; ++i) consider(s, r, s->order[i], inst, tmax, h);
        return;
    }
    float tl = INFINITY, tr = INFINITY;
    int hl = box_test(&s->nodes[nd->left], r, lim, &tl);
    int hr = box_test(&s->nodes[nd->right], r, lim, &tr);
    if (hl && hr && tr < tl) {
        bvh_closest_rec(s, nd->right, r, inst, tmax, h);
        bvh_closest_rec(s, nd->left, r, inst, tmax, h);
    } else {
        if (hl) bvh_closest_rec(s, nd->left, r, inst, tmax, h);
        if (hr) bvh_closest_rec(s, nd->right, r, inst, tmax, h);
    }
}

static void closest(const orc_scene* s, const ray_t* r, float tmax, int use_bvh, hit_t* h, int* frag)
{
    h->t = tmax; h->b1 = 0.0f; h->b2 = 0.0f; h->prim = -1; h->inst = 0;
    h->margin = 1.0f; h->tie_t = INFINITY; h->miss_t = INFINITY;
    if (s->nt == 0) return;
    if (s->ninst > 0) {
        /* every instance, in its object space (no world-space culling: the
         * result cannot depend on instance boxes) */
        for (int q = 0; q < s->ninst; ++q) {
            const int m = s->inst_mesh[q];
            if (s->mesh_count[m] == 0) continue;
            ray_t ro;
            object_ray(s, q, r, &ro);
            if (use_bvh && s->nodes) bvh_closest_rec(s, s->mesh_root[m], &ro, q, tmax, h);
            else
                for (int i = s->mesh_first[m]; i < s->mesh_first[m] + s->mesh_count[m]; ++i) consider(s, &ro, i, q, tmax, h);
        }
    } else if (use_bvh && s->nodes) {
        bvh_closest_rec(s, 0, r, 0, tmax, h);
    } else {
        for (int i = 0; i < s->nt; ++i) consider(s, r, i, 0, tmax, h);
    }
    if (!frag) return;
    if (h->prim >= 0) {
        float lim = h->t * (1.0f + 0x1p-20f);
        if (h->margin < 1e-6f) *frag |= FR_EDGE;
        if (h->tie_t <= lim) *frag |= FR_TIE;
        if (h->miss_t <= lim) *frag |= FR_NEARMISS;
    } else if (h->miss_t < tmax) {
        *frag |= FR_NEARMISS;
    }
}

static int any_tri(const orc_scene* s, const ray_t* r, int tri, float tmax, int* frag)
{
    float t, b1, b2, m;
    int ok = tri_test(r, s->v + 9 * (size_t)tri, &t, &b1, &b2, &m);
    if (!ok) {
        if (frag && m < 0.0f && m > -1e-6f) *frag |= FR_NEARMISS;
        return 0;
    }
    if (!(t < tmax)) {
        if (frag && t < tmax * (1.0f + 0x1p-20f)) *frag |= FR_TIE;
        return 0;
    }
    if (frag && m < 1e-6f) *frag |= FR_EDGE;
    if (frag && t > tmax * (1.0f - 0x1p-20f)) *frag |= FR_TIE;
    return 1;
}

static int bvh_any_rec(const orc_scene* s, int ni, const ray_t* r, float tmax, int* frag)
{
    const onode* nd = &s->nodes[ni];
    float tn;
    if (!box_test(nd, r, tmax, &tn)) return 0;
    if (nd->count > 0) {
        for (int i = nd->first; i < nd->first + nd->count; ++i)
            if (any_tri(s, r, s->order[i], tmax, frag)) return 1;
        return 0;
    }
    if (bvh_any_rec(s, nd->left, r, tmax, frag)) return 1;
    return bvh_any_rec(s, nd->right, r, tmax, frag);
}

static int occluded(const orc_scene* s, const ray_t* r, float tmax, int use_bvh, int* frag)
{
    if (s->nt == 0) return 0;
    if (s->ninst > 0) {
        for (int q = 0; q < s->ninst; ++q) {
            const int m = s->inst_mesh[q];
            if (s->mesh_count[m] == 0) continue;
            ray_t ro;
            object_ray(s, q, r, &ro);
            if (use_bvh && s->nodes) {
                if (bvh_any_rec(s, s->mesh_root[m], &ro, tmax, frag)) return 1;
            } else {
                for (int i = s->mesh_first[m]; i < s->mesh_first[m] + s->mesh_count[m]; ++i)
                    if (any_tri(s, &ro, i, tmax, frag)) return 1;
            }
        }
        return 0;
    }
    if (use_bvh && s->nodes) return bvh_any_rec(s, 0, r, tmax, frag);
    for (int i = 0; i < s->nt; ++i)
        if (any_tri(s, r, i, tmax, frag)) return 1;
    return 0;
}

int32_t orc_closest(const orc_scene* s, int32_t n, const float* o, const float* d, float tmax,
                    int32_t mode, float* t, int32_t* prim, float* b1, float* b2, int32_t* inst)
{
    for (int i = 0; i < n; ++i) {
        ray_t r;
        ray_setup(&r, vload(o + 3 * (size_t)i), vload(d + 3 * (size_t)i));
        hit_t h;
        closest(s, &r, tmax, mode, &h, NULL);
        t[i] = h.t; prim[i] = h.prim; b1[i] = h.b1; b2[i] = h.b2;
        if (inst) inst[i] = h.prim >= 0 ? h.inst : -1;
    }
    return 0;
}

int32_t orc_anyhit(const orc_scene* s, int32_t n, const float* o, const float* d, float tmax,
                   int32_t mode, uint8_t* occ)
{
    for (int i = 0; i < n; ++i) {
        ray_t r;
        ray_setup(&r, vload(o + 3 * (size_t)i), vload(d + 3 * (size_t)i));
        occ[i] = (uint8_t)occluded(s, &r, tmax, mode, NULL);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* geometry helpers                                                          */
/* ------------------------------------------------------------------------ */
/* Offset of a surface point off its plane along n: o = p + (2^-15 m) n per
 * coordinate, m the largest coordinate magnitude of the triangle the point
 * lies on (at least 2^-7).  The offset follows the scale idea of Waechter and
 * Binder (Ray Tracing Gems ch. 6, 2019: about 256 ulps of the coordinates),
 * but measures it on the triangle rather than on the point: the hit point and
 * the next ray's intersection test with the same triangle carry rounding
 * errors of a few ulps of the triangle's vertex coordinates, which on a large
 * triangle near a coordinate plane (a ground plane at y = 0) exceed a step
 * measured on the point's own small coordinates. */
static float tri_extent(const float* p)
{
    float m = 0x1p-7f;
    for (int i = 0; i < 9; ++i) m = fabsf(p[i]) > m ? fabsf(p[i]) : m;
    return m;
}
static v3 offset_point(v3 p, v3 n, float m)
{
    float dl = 0x1p-15f * m;
    return V(p.x + dl * n.x, p.y + dl * n.y, p.z + dl * n.z);
}

void orc_offset(const float p[3], const float n[3], const float tri[9], float out[3])
{
    vstore(out, offset_point(vload(p), vload(n), tri_extent(tri)));
}

/* Uniform point on a triangle: b1 = sqrt(u1)(1-u2), b2 = sqrt(u1) u2,
 * y = (v0 + b1 (v1-v0)) + b2 (v2-v0). */
static v3 tri_point(const float* p, float u1, float u2)
{
    v3 v0 = vload(p), e1 = vsub(vload(p + 3), v0), e2 = vsub(vload(p + 6), v0);
    float su = sqrtf(u1);
    float b1 = su * (1.0f - u2), b2 = su * u2;
    return V((v0.x + b1 * e1.x) + b2 * e2.x, (v0.y + b1 * e1.y) + b2 * e2.y,
             (v0.z + b1 * e1.z) + b2 * e2.z);
}

void orc_sample_triangle(const float v0[3], const float v1[3], const float v2[3], float u1,
                         float u2, float out[3])
{
    float p[9];
    memcpy(p, v0, 12); memcpy(p + 3, v1, 12); memcpy(p + 6, v2, 12);
    vstore(out, tri_point(p, u1, u2));
}

/* Geometric normal unit((v1-v0) x (v2-v0)); (0,0,1) for a zero-area one. */
static v3 tri_normal(const float* p)
{
    v3 v0 = vload(p), e1 = vsub(vload(p + 3), v0), e2 = vsub(vload(p + 6), v0);
    v3 c = vcross(e1, e2);
    if (vdot(c, c) == 0.0f) return V(0.0f, 0.0f, 1.0f);
    return vnorm(c);
}

/* Orthonormal basis around unit n (Duff et al., JCGT 2017). */
typedef struct { v3 t, b, n; } frame_t;
static frame_t make_frame(v3 n)
{
    float sign = copysignf(1.0f, n.z);
    float a = -1.0f / (sign + n.z);
    float b = n.x * n.y * a;
    frame_t f;
    f.t = V(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
    f.b = V(b, sign + n.y * n.y * a, -n.y);
    f.n = n;
    return f;
}
void orc_frame(const float n[3], float t[3], float b[3])
{
    frame_t f = make_frame(vload(n));
    vstore(t, f.t);
    vstore(b, f.b);
}
static v3 to_local(const frame_t* f, v3 w) { return V(vdot(f->t, w), vdot(f->b, w), vdot(f->n, w)); }
static v3 to_world(const frame_t* f, v3 l)
{
    return V((f->t.x * l.x + f->b.x * l.y) + f->n.x * l.z, (f->t.y * l.x + f->b.y * l.y) + f->n.y * l.z,
             (f->t.z * l.x + f->b.z * l.y) + f->n.z * l.z);
}

/* ------------------------------------------------------------------------ */
/* vertex attributes at a hit (paper Sec. 2.3: the shading stage rebuilds    */
/* the hit's attributes from the triangle and its barycentrics)              */
/* Reading: weights (w0, b1, b2) with w0 = (1 - b1) - b2 for (v0, v1, v2),   */
/* the sum ((w0 a0 + b1 a1) + b2 a2) per component.                          */
/* ------------------------------------------------------------------------ */
static float interp3(float a0, float a1, float a2, float w0, float b1, float b2)
{
    return (w0 * a0 + b1 * a1) + b2 * a2;
}

/* Shading normal: the interpolated vertex normal; in a two-level scene it is
 * an object-space normal and maps by the inverse transpose of the
 * instance's object-to-world map, i.e. by the columns of w2o's linear part;
 * normalised once; turned to the side of the geometric normal ng (vertex
 * normals and winding may disagree); ng itself when the scene has no
 * normals or the interpolant is zero or not finite. */
static v3 shading_normal(const orc_scene* s, int32_t inst, int32_t tri, float b1, float b2, v3 ng)
{
    if (!s->nrm) return ng;
    const float* n = s->nrm + 9 * (size_t)tri;
    float w0 = (1.0f - b1) - b2;
    v3 m = V(interp3(n[0], n[3], n[6], w0, b1, b2), interp3(n[1], n[4], n[7], w0, b1, b2),
             interp3(n[2], n[5], n[8], w0, b1, b2));
    if (s->ninst > 0) {
        const float* M = s->w2o + 12 * (size_t)inst;
        m = V((M[0] * m.x + M[4] * m.y) + M[8] * m.z, (M[1] * m.x + M[5] * m.y) + M[9] * m.z,
              (M[2] * m.x + M[6] * m.y) + M[10] * m.z);
    }
    float l2 = vdot(m, m);
    if (!(l2 > 0.0f && l2 <= FLT_MAX)) return ng;
    v3 ns = vnorm(m);
    return vdot(ns, ng) < 0.0f ? vneg(ns) : ns;
}

/* Checker texture of the albedo (a synthetic stand-in for the paper's
 * base-colour textures): cell (floor(u f), floor(v f)); the factor is
 * CHECKER_DARK on cells whose two indices differ in parity, else 1.  Parity
 * of floor(x): floor(x)/2 is an integer or a half, both exact in binary32. */
#define CHECKER_DARK 0.25f
static int odd_cell(float x)
{
    float f = floorf(x);
    float h = f * 0.5f;
    return floorf(h) != h;
}
static float texture(const orc_scene* s, int32_t tri, float b1, float b2, float freq)
{
    if (!s->uv || !(freq > 0.0f)) return 1.0f;
    const float* q = s->uv + 6 * (size_t)tri;
    float w0 = (1.0f - b1) - b2;
    float u = interp3(q[0], q[2], q[4], w0, b1, b2), v = interp3(q[1], q[3], q[5], w0, b1, b2);
    return odd_cell(u * freq) != odd_cell(v * freq) ? CHECKER_DARK : 1.0f;
}

/* cos and sin of 2 pi u, evaluated in binary64 and rounded to binary32. */
static void cos_sin_2pi(float u, float* c, float* s)
{
    double ph = (2.0 * 3.14159265358979323846) * (double)u;
    *c = (float)cos(ph);
    *s = (float)sin(ph);
}

/* ------------------------------------------------------------------------ */
/* BSDFs                                                                     */
/* ------------------------------------------------------------------------ */
static float ggx_alpha(float rough)
{
    float a = rough * rough;
    return a < 1e-4f ? 1e-4f : a;
}
/* GGX normal distribution for a unit half vector h.  The denominator uses
 * hx^2 + hy^2 + a2 hz^2, equal to cos^2 (a2 - 1) + 1 for unit h but free of
 * the cancellation that form suffers near the lobe peak in binary32. */
static float ggx_D(v3 h, float a2)
{
    float den = (h.x * h.x + h.y * h.y) + a2 * (h.z * h.z);
    return a2 / ((PI_F * den) * den);
}
static float ggx_lambda(v3 w, float a2)
{
    float t2 = (w.x * w.x + w.y * w.y) / (w.z * w.z);
    return (sqrtf(1.0f + a2 * t2) - 1.0f) * 0.5f;
}
/* visible-normal sampling (Heitz, JCGT 2018), wo in the local frame */
static v3 ggx_vndf(v3 wo, float alpha, float u5, float u6)
{
    v3 Vh = vnorm(V(alpha * wo.x, alpha * wo.y, wo.z));
    float lensq = Vh.x * Vh.x + Vh.y * Vh.y;
    v3 T1 = lensq > 0.0f ? vscale(V(-Vh.y, Vh.x, 0.0f), 1.0f / sqrtf(lensq)) : V(1.0f, 0.0f, 0.0f);
    v3 T2 = vcross(Vh, T1);
    float r = sqrtf(u5), c, s;
    cos_sin_2pi(u6, &c, &s);
    float t1 = r * c, t2 = r * s;
    float sh = 0.5f * (1.0f + Vh.z);
    t2 = (1.0f - sh) * sqrtf(1.0f - t1 * t1) + sh * t2;
    float nz2 = (1.0f - t1 * t1) - t2 * t2;
    float nz = sqrtf(nz2 > 0.0f ? nz2 : 0.0f);
    v3 Nh = V((t1 * T1.x + t2 * T2.x) + nz * Vh.x, (t1 * T1.y + t2 * T2.y) + nz * Vh.y,
              (t1 * T1.z + t2 * T2.z) + nz * Vh.z);
    return vnorm(V(alpha * Nh.x, alpha * Nh.y, Nh.z > 0.0f ? Nh.z : 0.0f));
}
static float pow5(float m) { return ((m * m) * (m * m)) * m; }

/* Scatter record: the pieces of f and of the sampling weight that do not
 * depend on the albedo, for the gradient. */
typedef struct {
    int type;
    float m5; /* Schlick (1 - cos)^5 (conductor) */
    float k;  /* Lambert: f = albedo k; conductor: D G2 / (4 cos_o cos_i) in f = F k;
                 dielectric: weight; coated: the base's factor in f = albedo k + b */
    float b;  /* coated: the coat's specular term (albedo-free) */
} lobe_t;

/* Coated material (a two-lobe subset of a layered model such as OpenPBR's
 * coat over a base; reading, the paper names the layered model but not its
 * evaluation): a GGX dielectric coat of index ior over a Lambertian base,
 *   f = F(wo.h) D G2 / (4 cos_o cos_i) + (1 - F(cos_o)) (1 - F(cos_i)) albedo / pi
 * with F the exact unpolarised Fresnel reflectance of the coat (its
 * specular reflection, Walter et al. 2007) and the base seen through two
 * coat crossings at the macro-surface angles (no interreflection between
 * the layers).  Symmetric in (wo, wi).  Sampling takes the coat's visible
 * normals with probability F(cos_o) (u4 < F(cos_o)), else the base's cosine
 * lobe; the pdf is the mixture of the two, and the weight f cos_i / pdf. */
static float fresnel_dielectric(float ci, float eta);
static void eval_coat(float rough, float ior, float tex, v3 alb, v3 wo, v3 wi, v3* f, float* pdf, lobe_t* lb)
{
    float alpha = ggx_alpha(rough), a2 = alpha * alpha;
    v3 h = vnorm(vadd(wo, wi));
    float D = ggx_D(h, a2);
    float lo = ggx_lambda(wo, a2), li = ggx_lambda(wi, a2);
    float G1 = 1.0f / (1.0f + lo);
    float G2 = 1.0f / ((1.0f + lo) + li);
    float Fh = fresnel_dielectric(vdot(wo, h), ior);
    float fs = ((Fh * D) * G2) / ((4.0f * wo.z) * wi.z);
    float Fo = fresnel_dielectric(wo.z, ior), Fi = fresnel_dielectric(wi.z, ior);
    float kd = (((1.0f - Fo) * (1.0f - Fi)) * tex) * INV_PI_F;
    *f = V(alb.x * kd + fs, alb.y * kd + fs, alb.z * kd + fs);
    *pdf = Fo * ((G1 * D) / (4.0f * wo.z)) + (1.0f - Fo) * (wi.z * INV_PI_F);
    lb->k = kd;
    lb->b = fs;
}

/* Evaluate f and the solid-angle pdf for an opaque material (Lambert or
 * conductor) with wo, wi in the local frame of the normal on wo's side. */
static void eval_opaque(int type, float rough, float ior, float tex, v3 alb, v3 wo, v3 wi, v3* f, float* pdf,
                        lobe_t* lb)
{
    *f = V(0.0f, 0.0f, 0.0f);
    *pdf = 0.0f;
    lb->type = type; lb->m5 = 0.0f; lb->k = 0.0f; lb->b = 0.0f;
    if (wi.z <= 0.0f || wo.z <= 0.0f) return;
    if (type == ORC_LAMBERT) {
        float k = tex * INV_PI_F;
        *f = V(alb.x * k, alb.y * k, alb.z * k);
        *pdf = wi.z * INV_PI_F;
        lb->k = k;
        return;
    }
    if (type == ORC_COATED) {
        eval_coat(rough, ior, tex, alb, wo, wi, f, pdf, lb);
        return;
    }
    float alpha = ggx_alpha(rough), a2 = alpha * alpha;
    v3 h = vnorm(vadd(wo, wi));
    float D = ggx_D(h, a2);
    float lo = ggx_lambda(wo, a2), li = ggx_lambda(wi, a2);
    float G1 = 1.0f / (1.0f + lo);
    float G2 = 1.0f / ((1.0f + lo) + li);
    float m5 = pow5(1.0f - vdot(wi, h));
    float k = (D * G2) / ((4.0f * wo.z) * wi.z);
    *f = V((alb.x + (1.0f - alb.x) * m5) * k, (alb.y + (1.0f - alb.y) * m5) * k,
           (alb.z + (1.0f - alb.z) * m5) * k);
    *pdf = (G1 * D) / (4.0f * wo.z);
    lb->m5 = m5;
    lb->k = k;
}

/* Exact unpolarised Fresnel reflectance; eta = eta_t / eta_i. */
static float fresnel_dielectric(float ci, float eta)
{
    float s2 = (1.0f - ci * ci) / (eta * eta);
    if (s2 >= 1.0f) return 1.0f;
    float ct = sqrtf(1.0f - s2);
    float rs = (ci - eta * ct) / (ci + eta * ct);
    float rp = (eta * ci - ct) / (eta * ci + ct);
    return 0.5f * (rs * rs + rp * rp);
}

/* Sample a direction.  wo is in the local frame (z = normal on the side the
 * sampling happens: wo side for opaque, the side of wo for the dielectric).
 * Returns 0 if rejected.  weight = f |cos| / pdf. */
/* cosine-weighted direction about +z from (u5, u6) */
static v3 cosine_dir(float u5, float u6)
{
    float r = sqrtf(u5), c, s;
    cos_sin_2pi(u6, &c, &s);
    float z2 = 1.0f - u5;
    return V(r * c, r * s, sqrtf(z2 > 0.0f ? z2 : 0.0f));
}

static int sample_local(int type, float rough, float ior, float tex, int entering, v3 alb, v3 wo, float u4,
                        float u5, float u6, v3* wi, v3* weight, float* pdf, lobe_t* lb, int* frag)
{
    lb->type = type; lb->m5 = 0.0f; lb->k = 0.0f; lb->b = 0.0f;
    if (type == ORC_LAMBERT) {
        *wi = cosine_dir(u5, u6);
        *weight = V(alb.x * tex, alb.y * tex, alb.z * tex);
        *pdf = wi->z * INV_PI_F;
        lb->k = tex;
        return 1;
    }
    if (wo.z <= 0.0f) return 0;
    if (frag && wo.z < FRAG_EPS) *frag |= FR_GRAZE;
    float alpha = ggx_alpha(rough), a2 = alpha * alpha;
    if (type == ORC_COATED) {
        float Fo = fresnel_dielectric(wo.z, ior);
        if (frag && fabsf(u4 - Fo) < 0x1p-20f) *frag |= FR_THRESH;
        v3 w;
        if (u4 < Fo) {
            v3 m = ggx_vndf(wo, alpha, u5, u6);
            float com = vdot(wo, m);
            w = V((2.0f * com) * m.x - wo.x, (2.0f * com) * m.y - wo.y, (2.0f * com) * m.z - wo.z);
        } else {
            w = cosine_dir(u5, u6);
        }
        if (frag && fabsf(w.z) < FRAG_EPS) *frag |= FR_GRAZE;
        if (w.z <= 0.0f) return 0;
        v3 f;
        float p;
        eval_coat(rough, ior, tex, alb, wo, w, &f, &p, lb);
        if (!(p > 0.0f)) return 0;
        float sc = w.z / p;
        lb->k = lb->k * sc;
        lb->b = lb->b * sc;
        *wi = w;
        *weight = V(alb.x * lb->k + lb->b, alb.y * lb->k + lb->b, alb.z * lb->k + lb->b);
        *pdf = p;
        return 1;
    }
    v3 m = ggx_vndf(wo, alpha, u5, u6);
    float com = vdot(wo, m);
    float lo = ggx_lambda(wo, a2);
    float G1 = 1.0f / (1.0f + lo);
    if (type == ORC_CONDUCTOR) {
        v3 w = V((2.0f * com) * m.x - wo.x, (2.0f * com) * m.y - wo.y, (2.0f * com) * m.z - wo.z);
        if (frag && fabsf(w.z) < FRAG_EPS) *frag |= FR_GRAZE;
        if (w.z <= 0.0f) return 0;
        float li = ggx_lambda(w, a2);
        float G2 = 1.0f / ((1.0f + lo) + li);
        float g = G2 / G1;
        float m5 = pow5(1.0f - com);
        *wi = w;
        *weight = V((alb.x + (1.0f - alb.x) * m5) * g, (alb.y + (1.0f - alb.y) * m5) * g,
                    (alb.z + (1.0f - alb.z) * m5) * g);
        *pdf = (G1 * ggx_D(m, a2)) / (4.0f * wo.z);
        lb->m5 = m5;
        lb->k = g;
        return 1;
    }
    /* rough dielectric (Walter et al. 2007) */
    float eta = entering ? ior : 1.0f / ior;
    float F = fresnel_dielectric(com, eta);
    if (frag && fabsf(u4 - F) < 0x1p-20f) *frag |= FR_THRESH;
    v3 w;
    float scale;
    if (u4 < F) {
        w = V((2.0f * com) * m.x - wo.x, (2.0f * com) * m.y - wo.y, (2.0f * com) * m.z - wo.z);
        if (frag && fabsf(w.z) < FRAG_EPS) *frag |= FR_GRAZE;
        if (w.z <= 0.0f) return 0;
        scale = 1.0f;
    } else {
        float s2 = (1.0f - com * com) / (eta * eta);
        float ct = sqrtf(1.0f - s2);
        float a = com / eta - ct;
        w = V(-wo.x / eta + a * m.x, -wo.y / eta + a * m.y, -wo.z / eta + a * m.z);
        if (frag && fabsf(w.z) < FRAG_EPS) *frag |= FR_GRAZE;
        if (w.z >= 0.0f) return 0;
        scale = 1.0f / (eta * eta);
    }
    float li = ggx_lambda(w, a2);
    float G2 = 1.0f / ((1.0f + lo) + li);
    float g = (G2 / G1) * scale;
    *wi = w;
    *weight = V(g, g, g);
    *pdf = 0.0f; /* not used: no light sampling at dielectric vertices */
    lb->k = g;
    return 1;
}

void orc_bsdf_eval(int32_t type, float rough, float ior, float tex, const float alb[3], const float n[3],
                   const float wo[3], const float wi[3], float f[3], float* pdf)
{
    frame_t fr = make_frame(vload(n));
    v3 ff;
    lobe_t lb;
    eval_opaque(type, rough, ior, tex, vload(alb), to_local(&fr, vload(wo)), to_local(&fr, vload(wi)), &ff, pdf,
                &lb);
    vstore(f, ff);
}

int32_t orc_bsdf_sample(int32_t type, float rough, float ior, float tex, const float alb[3],
                        const float n[3], const float wo[3], float u4, float u5, float u6,
                        float wi[3], float weight[3], float* pdf)
{
    v3 nn = vload(n);
    int entering = 1;
    if (type == ORC_DIELECTRIC) {
        entering = vdot(nn, vload(wo)) > 0.0f;
        if (!entering) nn = vneg(nn);
    }
    frame_t fr = make_frame(nn);
    v3 w, W;
    lobe_t lb;
    int ok = sample_local(type, rough, ior, tex, entering, vload(alb), to_local(&fr, vload(wo)), u4, u5, u6,
                          &w, &W, pdf, &lb, NULL);
    vstore(wi, ok ? to_world(&fr, w) : V(0.0f, 0.0f, 0.0f));
    vstore(weight, ok ? W : V(0.0f, 0.0f, 0.0f));
    if (!ok) *pdf = 0.0f;
    return ok;
}

void orc_shading_normal(const orc_scene* s, int32_t inst, int32_t tri, float b1, float b2, float out[3])
{
    float tw[9];
    const float* tp = world_tri(s, inst, tri, tw);
    vstore(out, shading_normal(s, inst, tri, b1, b2, tri_normal(tp)));
}

float orc_texture(const orc_scene* s, int32_t tri, float b1, float b2, float freq)
{
    return texture(s, tri, b1, b2, freq);
}

/* ------------------------------------------------------------------------ */
/* path tracer                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t tri;       /* triangle at this vertex */
    int emit;          /* emission term counted (front face) */
    float w_emit;      /* its MIS weight */
    int nee;           /* light-sample term counted (unoccluded) */
    int32_t ltri;      /* light triangle */
    float G;           /* |cos_x| * w_light / p_light */
    lobe_t nee_lobe;   /* f = lobe(albedo) */
    int scat;          /* path continued from here */
    lobe_t scat_lobe;  /* weight = lobe(albedo) */
} vrec;

typedef struct {
    const orc_scene* s;
    const float* cam;
    int W, H, D, nee, rr_start, use_bvh;
    uint64_t seed;
    uint32_t job;
    int sampler; /* camera jitter: 0 Philox, 1 Halton(2,3) + rotation */
} pt_args;

static float maxc(v3 a) { float m = a.x > a.y ? a.x : a.y; return m > a.z ? m : a.z; }

/* One camera path.  Returns L; fills rec[0..*nrec) if rec != NULL and sets
 * *escaped when the last event was an escape to the sky. */
static v3 trace_path(const pt_args* a, int pix, uint32_t sample, int* frag, vrec* rec, int* nrec)
{
    const orc_scene* s = a->s;
    uint32_t w[8];
    v3 L = V(0.0f, 0.0f, 0.0f), beta = V(1.0f, 1.0f, 1.0f);
    int px = pix % a->W, py = pix / a->W;
    rng_words(a->seed, (uint32_t)pix, sample, 0, a->job, w);
    ray_t r;
    v3 o, d;
    float jit[2] = {orc_unif(w[0]), orc_unif(w[1])};
    if (a->sampler == 1) orc_halton_jitter(a->seed, (uint32_t)pix, sample, a->job, jit);
    camera_ray(a->cam, a->W, a->H, px, py, jit[0], jit[1], &o, &d);
    ray_setup(&r, o, d);
    float p_prev = 0.0f;
    int prev_smooth = 0; /* previous vertex sampled a light (MIS applies) */
    int nr = 0;
    for (int k = 1;; ++k) {
        hit_t h;
        closest(s, &r, INFINITY, a->use_bvh, &h, frag);
        if (h.prim < 0) {
            L = V(L.x + beta.x * s->sky[0], L.y + beta.y * s->sky[1], L.z + beta.z * s->sky[2]);
            break;
        }
        float tw[9];
        const float* tp = world_tri(s, h.inst, h.prim, tw);
        v3 v0 = vload(tp), e1 = vsub(vload(tp + 3), v0), e2 = vsub(vload(tp + 6), v0);
        v3 x = V((v0.x + h.b1 * e1.x) + h.b2 * e2.x, (v0.y + h.b1 * e1.y) + h.b2 * e2.y,
                 (v0.z + h.b1 * e1.z) + h.b2 * e2.z);
        v3 ng = tri_normal(tp);
        v3 wo = vneg(r.d);
        float cos_e = vdot(ng, wo);
        vrec* vr = rec ? &rec[nr] : NULL;
        if (vr) { memset(vr, 0, sizeof *vr); vr->tri = h.prim; }
        ++nr;
        if (frag && cos_e != 0.0f && fabsf(cos_e) < FRAG_EPS) *frag |= FR_GRAZE;
        /* emitted radiance, front face only */
        if (cos_e > 0.0f) {
            float wgt = 1.0f;
            if (k > 1 && a->nee && prev_smooth && s->is_light[h.prim] && s->nl > 0) {
                float pl = (h.t * h.t) / (s->area_total * cos_e);
                wgt = (p_prev * p_prev) / (p_prev * p_prev + pl * pl);
            }
            const float* Le = s->emission + 3 * (size_t)h.prim;
            L = V(L.x + beta.x * (wgt * Le[0]), L.y + beta.y * (wgt * Le[1]), L.z + beta.z * (wgt * Le[2]));
            if (vr) { vr->emit = 1; vr->w_emit = wgt; }
        }
        if (k == a->D + 1) break;
        rng_words(a->seed, (uint32_t)pix, sample, (uint32_t)k, a->job, w);
        int mt = s->tri_mat[h.prim];
        const float* mat = s->mats + 4 * (size_t)mt;
        int type = (int)mat[0];
        float rough = mat[1], ior = mat[2];
        v3 alb = vload(s->albedo + 3 * (size_t)h.prim);
        float tex = (type == ORC_LAMBERT || type == ORC_COATED) ? texture(s, h.prim, h.b1, h.b2, mat[3]) : 1.0f;
        /* BSDF frame: the shading normal turned to wo's side of the surface
         * (the geometric normal when the scene has no vertex normals) */
        v3 ns = shading_normal(s, h.inst, h.prim, h.b1, h.b2, ng);
        int entering = 1;
        v3 n, ngf;
        if (type == ORC_DIELECTRIC) {
            entering = cos_e > 0.0f;
            n = entering ? ns : vneg(ns);
            ngf = entering ? ng : vneg(ng);
        } else {
            n = cos_e > 0.0f ? ns : vneg(ns);
            ngf = cos_e > 0.0f ? ng : vneg(ng);
        }
        frame_t fr = make_frame(n);
        v3 wo_l = to_local(&fr, wo);
        /* shading normals (reading): a vertex seen from below its shading
         * horizon scatters nothing; a light or continuation direction must
         * also lie on the geometric side its lobe implies (reflection: wo's
         * side, transmission: the other), so that no light leaks through
         * the surface */
        if (frag && s->nrm && fabsf(wo_l.z) < FRAG_EPS) *frag |= FR_GRAZE;
        if (s->nrm && wo_l.z <= 0.0f) break;
        /* next-event estimation at opaque vertices */
        if (a->nee && s->nl > 0 && type != ORC_DIELECTRIC) {
            int j = orc_pick_light(s, w[0]);
            if (frag) {
                uint32_t hi = s->light_cdf[j], lo = j > 0 ? s->light_cdf[j - 1] : 0u;
                if (hi - w[0] < 4096u || (j > 0 && w[0] - lo < 4096u)) *frag |= FR_THRESH;
            }
            int lt = s->light_tri[j];
            float lw[9];
            const float* lp = world_tri(s, s->light_inst[j], lt, lw);
            v3 y = tri_point(lp, orc_unif(w[1]), orc_unif(w[2]));
            v3 ny = tri_normal(lp);
            v3 dv = vsub(y, x);
            float d2 = vdot(dv, dv);
            if (d2 > 0.0f) {
                v3 wl = vscale(dv, 1.0f / sqrtf(d2));
                float cos_y = -vdot(ny, wl);
                float cos_x = vdot(n, wl);
                if (frag && ((cos_y != 0.0f && fabsf(cos_y) < FRAG_EPS) || (cos_x != 0.0f && fabsf(cos_x) < FRAG_EPS))) *frag |= FR_GRAZE;
                int side = 1;
                if (s->nrm) {
                    float cg = vdot(ngf, wl);
                    if (frag && fabsf(cg) < FRAG_EPS) *frag |= FR_GRAZE;
                    side = cg > 0.0f;
                }
                if (cos_y > 0.0f && cos_x > 0.0f && side) {
                    v3 f;
                    float pb;
                    lobe_t lb;
                    eval_opaque(type, rough, ior, tex, alb, wo_l, to_local(&fr, wl), &f, &pb, &lb);
                    float pl = d2 / (s->area_total * cos_y);
                    if (lb.k > 0.0f && pl > 0.0f) {
                        float wmis = (pl * pl) / (pl * pl + pb * pb);
                        float G = (cos_x * wmis) / pl;
                        const float* Le = s->emission + 3 * (size_t)lt;
                        v3 C = V((f.x * Le[0]) * G, (f.y * Le[1]) * G, (f.z * Le[2]) * G);
                        v3 so = offset_point(x, vdot(ng, wl) > 0.0f ? ng : vneg(ng), tri_extent(tp));
                        v3 sy = offset_point(y, ny, tri_extent(lp));
                        ray_t sr;
                        ray_setup(&sr, so, vsub(sy, so));
                        if (!occluded(s, &sr, SHADOW_TMAX, a->use_bvh, frag)) {
                            L = V(L.x + beta.x * C.x, L.y + beta.y * C.y, L.z + beta.z * C.z);
                            if (vr) { vr->nee = 1; vr->ltri = lt; vr->G = G; vr->nee_lobe = lb; }
                        }
                    }
                }
            }
        }
        /* continue the path by sampling the BSDF */
        v3 wi_l, W;
        float pb;
        lobe_t lb;
        int ok = sample_local(type, rough, ior, tex, entering, alb, wo_l, orc_unif(w[4]), orc_unif(w[5]),
                              orc_unif(w[6]), &wi_l, &W, &pb, &lb, frag);
        if (!ok) break;
        if (W.x == 0.0f && W.y == 0.0f && W.z == 0.0f) break;
        if (type != ORC_DIELECTRIC && !(pb > 0.0f)) break;
        v3 wi = to_world(&fr, wi_l);
        if (s->nrm) {
            float cg = vdot(ngf, wi);
            if (frag && fabsf(cg) < FRAG_EPS) *frag |= FR_GRAZE;
            if (wi_l.z > 0.0f ? !(cg > 0.0f) : !(cg < 0.0f)) break;
        }
        beta = V(beta.x * W.x, beta.y * W.y, beta.z * W.z);
        if (a->rr_start >= 0 && k >= a->rr_start) {
            float q = maxc(beta);
            q = q < 1.0f ? q : 1.0f;
            float u7 = orc_unif(w[7]);
            if (frag && fabsf(u7 - q) < 0x1p-20f) *frag |= FR_THRESH;
            if (u7 >= q) break;
            beta = V(beta.x / q, beta.y / q, beta.z / q);
        }
        if (vr) { vr->scat = 1; vr->scat_lobe = lb; }
        v3 no = vdot(ng, wi) > 0.0f ? ng : vneg(ng);
        ray_setup(&r, offset_point(x, no, tri_extent(tp)), wi);
        p_prev = pb;
        prev_smooth = type != ORC_DIELECTRIC;
    }
    if (nrec) *nrec = nr;
    return L;
}

/* ------------------------------------------------------------------------ */
/* threads: static row-interleaved partition of the pixel list               */
/* ------------------------------------------------------------------------ */
typedef struct {
    const pt_args* a;
    const int32_t* pixels;
    int n, spp, tid, nth;
    uint32_t frame;
    float* out;
    uint8_t* frag;
    float* per_sample;
    /* backward */
    const float* dimg;
    double *ga, *ge, *aa, *ae;
    int err;
} job_t;

static void* render_worker(void* p)
{
    job_t* j = (job_t*)p;
    for (int i = j->tid; i < j->n; i += j->nth) {
        int pix = j->pixels[i];
        int fr = 0;
        v3 acc = V(0.0f, 0.0f, 0.0f);
        for (int smp = 0; smp < j->spp; ++smp) {
            uint32_t sg = j->frame * (uint32_t)j->spp + (uint32_t)smp;
            v3 Ls = trace_path(j->a, pix, sg, &fr, NULL, NULL);
            if (j->per_sample) vstore(j->per_sample + 3 * ((size_t)i * j->spp + smp), Ls);
            acc = smp == 0 ? Ls : vadd(acc, Ls);
        }
        float sp = (float)j->spp;
        vstore(j->out + 3 * (size_t)i, V(acc.x / sp, acc.y / sp, acc.z / sp));
        if (j->frag) j->frag[i] = (uint8_t)fr;
    }
    return NULL;
}

static int run_threads(job_t* base, int threads, void* (*fn)(void*))
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < threads; ++t) {
        jobs[t] = *base;
        jobs[t].tid = t;
        jobs[t].nth = threads;
    }
    for (int t = 1; t < threads; ++t) pthread_create(&th[t], NULL, fn, &jobs[t]);
    fn(&jobs[0]);
    for (int t = 1; t < threads; ++t) pthread_join(th[t], NULL);
    return 0;
}

int32_t orc_render(const orc_scene* s, const float cam[12], int32_t width, int32_t height,
                   const int32_t* pixels, int32_t n, int32_t spp, int32_t max_depth,
                   uint64_t seed, uint32_t frame, uint32_t job, int32_t nee, int32_t rr_start,
                   int32_t sampler, int32_t use_bvh, int32_t threads, float* out, uint8_t* fragile,
                   float* per_sample)
{
    if (!s || width <= 0 || height <= 0 || spp <= 0 || max_depth < 0 || n < 0) return -1;
    if (sampler != 0 && sampler != 1) return -1;
    for (int i = 0; i < n; ++i)
        if (pixels[i] < 0 || pixels[i] >= width * height) return -1;
    pt_args a = {s, cam, width, height, max_depth, nee, rr_start, use_bvh, seed, job, sampler};
    job_t b;
    memset(&b, 0, sizeof b);
    b.a = &a; b.pixels = pixels; b.n = n; b.spp = spp; b.frame = frame;
    b.out = out; b.frag = fragile; b.per_sample = per_sample;
    return run_threads(&b, threads, render_worker);
}

/* ------------------------------------------------------------------------ */
/* gradient: stored path, suffix radiance in binary64                        */
/* For a path with scatter vertices k = 1..K, emission terms e_k = w_k Le,   */
/* light-sample terms n_k = f_k Le_y G_k and sampling weights W_k:           */
/*   R_k = e_k + n_k + W_k R_{k+1},  L = R_1,  beta_k = prod_{j<k} W_j,      */
/*   dL/d albedo(tri_k) = beta_k (dn_k/dalbedo + dW_k/dalbedo R_{k+1}),      */
/*   dL/d Le(tri)      = sum over emission and light-sample events.          */
/* ------------------------------------------------------------------------ */
static double lobe_val(const lobe_t* lb, double rho)
{
    if (lb->type == ORC_LAMBERT) return rho * (double)lb->k;
    if (lb->type == ORC_CONDUCTOR) return (rho + (1.0 - rho) * (double)lb->m5) * (double)lb->k;
    if (lb->type == ORC_COATED) return rho * (double)lb->k + (double)lb->b;
    return (double)lb->k;
}
static double lobe_der(const lobe_t* lb)
{
    if (lb->type == ORC_LAMBERT || lb->type == ORC_COATED) return (double)lb->k;
    if (lb->type == ORC_CONDUCTOR) return (1.0 - (double)lb->m5) * (double)lb->k;
    return 0.0;
}

#define MAX_VERTS 1024

static void* backward_worker(void* p)
{
    job_t* j = (job_t*)p;
    const orc_scene* s = j->a->s;
    vrec* rec = (vrec*)malloc(sizeof(vrec) * MAX_VERTS);
    double (*R)[3] = malloc(sizeof(double[3]) * (MAX_VERTS + 1));
    for (int i = j->tid; i < j->n; i += j->nth) {
        int pix = j->pixels[i];
        for (int smp = 0; smp < j->spp; ++smp) {
            uint32_t sg = j->frame * (uint32_t)j->spp + (uint32_t)smp;
            int nr = 0;
            trace_path(j->a, pix, sg, NULL, rec, &nr);
            if (nr >= MAX_VERTS) { j->err = 1; continue; }
            double delta[3];
            for (int c = 0; c < 3; ++c) delta[c] = (double)j->dimg[3 * (size_t)i + c] / (double)j->spp;
            /* suffix radiance per unit throughput */
            for (int c = 0; c < 3; ++c) R[nr][c] = 0.0;
            int escaped = nr == 0 || rec[nr - 1].scat; /* last vertex continued => escape */
            if (escaped)
                for (int c = 0; c < 3; ++c) R[nr][c] = (double)s->sky[c];
            for (int k = nr - 1; k >= 0; --k) {
                const vrec* v = &rec[k];
                for (int c = 0; c < 3; ++c) {
                    double acc = 0.0;
                    if (v->emit) acc += (double)v->w_emit * (double)s->emission[3 * (size_t)v->tri + c];
                    if (v->nee) {
                        double rho = (double)s->albedo[3 * (size_t)v->tri + c];
                        acc += lobe_val(&v->nee_lobe, rho) * (double)s->emission[3 * (size_t)v->ltri + c] *
                               (double)v->G;
                    }
                    if (v->scat) {
                        double rho = (double)s->albedo[3 * (size_t)v->tri + c];
                        acc += lobe_val(&v->scat_lobe, rho) * R[k + 1][c];
                    }
                    R[k][c] = acc;
                }
            }
            /* forward pass with throughput */
            double beta[3] = {1.0, 1.0, 1.0};
            for (int k = 0; k < nr; ++k) {
                const vrec* v = &rec[k];
                for (int c = 0; c < 3; ++c) {
                    size_t ti = 3 * (size_t)v->tri + c;
                    if (v->emit) {
                        double g = delta[c] * beta[c] * (double)v->w_emit;
                        j->ge[ti] += g;
                        if (j->ae) j->ae[ti] += fabs(g);
                    }
                    if (v->nee) {
                        double rho = (double)s->albedo[ti];
                        double Le = (double)s->emission[3 * (size_t)v->ltri + c];
                        double ge = delta[c] * beta[c] * lobe_val(&v->nee_lobe, rho) * (double)v->G;
                        j->ge[3 * (size_t)v->ltri + c] += ge;
                        if (j->ae) j->ae[3 * (size_t)v->ltri + c] += fabs(ge);
                        double ga = delta[c] * beta[c] * lobe_der(&v->nee_lobe) * Le * (double)v->G;
                        j->ga[ti] += ga;
                        if (j->aa) j->aa[ti] += fabs(ga);
                    }
                    if (v->scat) {
                        double ga = delta[c] * beta[c] * lobe_der(&v->scat_lobe) * R[k + 1][c];
                        j->ga[ti] += ga;
                        if (j->aa) j->aa[ti] += fabs(ga);
                        beta[c] *= lobe_val(&v->scat_lobe, (double)s->albedo[ti]);
                    }
                }
            }
        }
    }
    free(rec);
    free(R);
    return NULL;
}

int32_t orc_backward(const orc_scene* s, const float cam[12], int32_t width, int32_t height,
                     const int32_t* pixels, int32_t n, int32_t spp, int32_t max_depth,
                     uint64_t seed, uint32_t frame, uint32_t job, int32_t nee, int32_t sampler,
                     int32_t use_bvh, int32_t threads, const float* d_image, double* g_albedo,
                     double* g_emission, double* abs_albedo, double* abs_emission)
{
    if (!s || width <= 0 || height <= 0 || spp <= 0 || max_depth < 0 || n < 0) return -1;
    if (sampler != 0 && sampler != 1) return -1;
    if (max_depth + 2 > MAX_VERTS) return -1;
    for (int i = 0; i < n; ++i)
        if (pixels[i] < 0 || pixels[i] >= width * height) return -1;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    size_t m = 3 * (size_t)s->nt;
    pt_args a = {s, cam, width, height, max_depth, nee, -1, use_bvh, seed, job, sampler};
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < threads; ++t) {
        memset(&jobs[t], 0, sizeof(job_t));
        jobs[t].a = &a; jobs[t].pixels = pixels; jobs[t].n = n; jobs[t].spp = spp;
        jobs[t].frame = frame; jobs[t].dimg = d_image; jobs[t].tid = t; jobs[t].nth = threads;
        jobs[t].ga = (double*)calloc(m ? m : 1, sizeof(double));
        jobs[t].ge = (double*)calloc(m ? m : 1, sizeof(double));
        jobs[t].aa = abs_albedo ? (double*)calloc(m ? m : 1, sizeof(double)) : NULL;
        jobs[t].ae = abs_emission ? (double*)calloc(m ? m : 1, sizeof(double)) : NULL;
    }
    for (int t = 1; t < threads; ++t) pthread_create(&th[t], NULL, backward_worker, &jobs[t]);
    backward_worker(&jobs[0]);
    for (int t = 1; t < threads; ++t) pthread_join(th[t], NULL);
    int err = 0;
    for (size_t i = 0; i < m; ++i) {
        double sa = 0, se = 0, saa = 0, sae = 0;
        for (int t = 0; t < threads; ++t) {
            sa += jobs[t].ga[i];
            se += jobs[t].ge[i];
            if (abs_albedo) saa += jobs[t].aa[i];
            if (abs_emission) sae += jobs[t].ae[i];
        }
        g_albedo[i] = sa;
        g_emission[i] = se;
        if (abs_albedo) abs_albedo[i] = saa;
        if (abs_emission) abs_emission[i] = sae;
    }
    for (int t = 0; t < threads; ++t) {
        err |= jobs[t].err;
        free(jobs[t].ga); free(jobs[t].ge); free(jobs[t].aa); free(jobs[t].ae);
    }
    return err ? -2 : 0;
}
