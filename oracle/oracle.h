/*
 * CPU oracle for unidirectional Monte Carlo path tracing of triangle scenes.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain reference that the HIP
 * renderer is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code with the HIP
 * library.
 *
 * What it computes (paper, Sec. 2.1-2.2, Eq. 1-3 and the five-step forward
 * path-tracing loop): for every requested pixel p the estimator
 *     I(p) = (1/spp) * sum_{s<spp} L(p, s)
 * where L(p, s) is one camera path traced vertex by vertex: extend by the
 * closest hit, add emitted radiance times the path throughput, sample a new
 * direction and multiply the throughput by f |n . w| / p.  Next-event
 * estimation with the power heuristic and Russian roulette are options.  All
 * random numbers come from a counter-based Philox4x64-10 generator keyed by
 * (pixel, sample, bounce, job), so any path can be replayed exactly.
 *
 * Precision: the path arithmetic is IEEE binary32 with no contraction
 * (compiled with -ffp-contract=off), so every decision taken on a float
 * (closest hit, light pick, roulette, lobe) is taken in the renderer's
 * precision.  Gradients (orc_backward) are accumulated in binary64.
 */
#ifndef PTMI_ORACLE_H
#define PTMI_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_scene orc_scene;

/* Material types of the material table (type, roughness, ior, checker
 * frequency).  ORC_COATED: a dielectric coat (GGX roughness, ior) over a
 * Lambertian base of the triangle's albedo.  The checker frequency (> 0)
 * textures the albedo of Lambertian and coated materials through the
 * vertex texture coordinates (orc_scene_set_attributes); 0 = untextured. */
enum { ORC_LAMBERT = 0, ORC_CONDUCTOR = 1, ORC_DIELECTRIC = 2, ORC_COATED = 3 };

/* Build a scene from indexed triangles.  Arrays are copied.  build_bvh != 0
 * also builds the oracle's own binary BVH (object-median splits).
 * Returns NULL on invalid input (out-of-range index, non-finite value). */
orc_scene* orc_scene_create(int32_t nv, const float* pos, int32_t nt, const int32_t* idx,
                            const int32_t* tri_mat, int32_t nm, const float* mats,
                            const float* albedo, const float* emission, const float* sky,
                            int32_t build_bvh);
void orc_scene_destroy(orc_scene* s);
/* Replace albedo / emission (nt*3 each).  The light set stays the one fixed
 * at creation (triangles with some emission channel > 0). */
void orc_scene_set_params(orc_scene* s, const float* albedo, const float* emission);
int32_t orc_scene_num_lights(const orc_scene* s);
/* Two-level scene (paper Sec. 2.3 and 3: a top-level structure over
 * instances of bottom-level meshes).  Mesh m is the triangle range
 * [mesh_first[m], mesh_first[m] + mesh_count[m]) of the scene, in object
 * space; instance q places mesh inst_mesh[q] in the world by the affine map
 * o2w[12q .. 12q + 11] (3x4 row-major: row r = linear row r, translation r),
 * and w2o (same layout) maps world rays into its object space.  From then on
 * the world is the instances: a ray is tested against each instance's mesh
 * with the object-space ray ((M0 x + M1 y) + M2 z) + M3 per row, direction
 * without translation, not renormalised, so t is the world ray's parameter;
 * the closest hit is the smallest t, ties to the smaller instance and then
 * the smaller triangle; shading, light sampling and areas use the world-space
 * vertices o2w(v) in the same arithmetic; per-triangle parameters (material,
 * albedo, emission) are shared by all instances of a mesh; the light set is
 * every (instance, emissive triangle) pair.  Returns 0, or -1 on invalid
 * input (out-of-range ranges or indices, non-finite matrices). */
int32_t orc_scene_set_instances(orc_scene* s, int32_t n_meshes, const int32_t* mesh_first,
                                const int32_t* mesh_count, int32_t n_inst, const int32_t* inst_mesh,
                                const float* o2w, const float* w2o);
/* Vertex attributes (paper Sec. 2.3: the shading stage interpolates the
 * hit triangle's vertex attributes).  normals (nv*3, may be NULL) and uvs
 * (nv*2, may be NULL) are per vertex, taken through idx (nt*3, the scene's
 * indices; in a two-level scene they are in object space).  The shading
 * normal at barycentrics (b1, b2) is the interpolation
 * ((w0 n0 + b1 n1) + b2 n2), w0 = (1 - b1) - b2, mapped to world space by
 * the columns of w2o's linear part in a two-level scene, normalised, and
 * turned to the geometric normal's side; a zero or non-finite interpolant
 * falls back to the geometric normal.  Texture: the checker factor of
 * orc_texture.  Returns 0, or -1 on a non-finite value or an index out of
 * range. */
int32_t orc_scene_set_attributes(orc_scene* s, int32_t nv, const int32_t* idx, const float* normals,
                                 const float* uvs);
/* Shading normal of triangle tri (instance inst in a two-level scene) at
 * barycentrics (b1, b2), before it is turned towards the outgoing
 * direction; the geometric normal when the scene has no normals. */
void orc_shading_normal(const orc_scene* s, int32_t inst, int32_t tri, float b1, float b2, float out[3]);
/* Albedo factor of the checker texture of frequency freq at (b1, b2) of
 * triangle tri: with (u, v) interpolated like the normals, 1/4 where
 * floor(u freq) + floor(v freq) is odd, else 1 (1 without texture
 * coordinates or with freq <= 0). */
float orc_texture(const orc_scene* s, int32_t tri, float b1, float b2, float freq);
/* BVH statistics: node count and maximum depth (0 if no BVH). */
void orc_scene_bvh_stats(const orc_scene* s, int32_t* nodes, int32_t* depth);

/* Pinhole camera constants: out = E[3], R[3], U[3], F[3] (binary32). */
void orc_camera(const double eye[3], const double target[3], const double up[3],
                double vfov_deg, int32_t width, int32_t height, float out[12]);

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011). */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Render the listed pixels.  out: n*3 floats, the per-pixel mean over spp.
 * fragile (may be NULL): n bytes, nonzero where some decision along one of
 * the pixel's paths was within rounding distance of flipping.
 * per_sample (may be NULL): n*spp*3 floats, L of each sample.
 * use_bvh: 0 = brute force, 1 = oracle BVH.  rr_start < 0 disables roulette.
 * sampler: camera jitter of sample n of a pixel, 0 = Philox words 0, 1 of
 * the path's first block, 1 = Halton(2,3) point n with the pixel's
 * Cranley-Patterson rotation (orc_halton_jitter).
 * Returns 0 or a negative error code. */
int32_t orc_render(const orc_scene* s, const float cam[12], int32_t width, int32_t height,
                   const int32_t* pixels, int32_t n, int32_t spp, int32_t max_depth,
                   uint64_t seed, uint32_t frame, uint32_t job, int32_t nee, int32_t rr_start,
                   int32_t sampler, int32_t use_bvh, int32_t threads, float* out, uint8_t* fragile,
                   float* per_sample);

/* Gradient of sum_p sum_c d_image[p,c] * I(p,c) with respect to per-triangle
 * albedo and emission, for the fixed-sample estimator (same seed/frame).
 * Binary64 accumulation; outputs are overwritten (nt*3 each).  abs_* (may be
 * NULL) receive the sum of absolute values of the individual terms.
 * Roulette must be off (its survival probability depends on albedo). */
int32_t orc_backward(const orc_scene* s, const float cam[12], int32_t width, int32_t height,
                     const int32_t* pixels, int32_t n, int32_t spp, int32_t max_depth,
                     uint64_t seed, uint32_t frame, uint32_t job, int32_t nee, int32_t sampler,
                     int32_t use_bvh, int32_t threads, const float* d_image, double* g_albedo,
                     double* g_emission, double* abs_albedo, double* abs_emission);

/* Radical inverse of n in base 2 or 3, truncated to 24 bits (exact integer
 * digit reversal, so the value is q 2^-24 with q 2^-24 <= phi_b(n)). */
float orc_radical_inverse(uint32_t n, int32_t base);
/* Camera jitter of sample `sample` of `pixel` with sampler 1: the Halton
 * (2,3) point of that index rotated by the pixel's offsets, modulo 1. */
void orc_halton_jitter(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t job, float out[2]);

/* Closest hit (mode 0 brute force, 1 BVH) for n rays o[3n], d[3n] with
 * t in (0, tmax).  prim = -1 on a miss; inst (may be NULL) receives the
 * instance of the hit in a two-level scene (0 in a flat one, -1 on a miss). */
int32_t orc_closest(const orc_scene* s, int32_t n, const float* o, const float* d, float tmax,
                    int32_t mode, float* t, int32_t* prim, float* b1, float* b2, int32_t* inst);
/* Any hit in (0, tmax): occluded[i] = 0/1. */
int32_t orc_anyhit(const orc_scene* s, int32_t n, const float* o, const float* d, float tmax,
                   int32_t mode, uint8_t* occluded);

/* Single-triangle watertight test (for pins): returns 1 on a hit. */
int32_t orc_tri_test(const float o[3], const float d[3], const float v0[3], const float v1[3],
                     const float v2[3], float* t, float* b1, float* b2);

/* BSDF pieces, for pins.  n is the unit surface normal on the side of wo
 * (for the dielectric: the outside normal); tex is the texture factor of
 * the albedo (Lambertian and coated base).  eval writes f[3] and *pdf
 * (solid angle).  sample writes wi, the weight f|n.wi|/pdf and *pdf and
 * returns 0 when the sample is rejected. */
void orc_bsdf_eval(int32_t type, float rough, float ior, float tex, const float alb[3], const float n[3],
                   const float wo[3], const float wi[3], float f[3], float* pdf);
int32_t orc_bsdf_sample(int32_t type, float rough, float ior, float tex, const float alb[3],
                        const float n[3], const float wo[3], float u4, float u5, float u6,
                        float wi[3], float weight[3], float* pdf);

/* Local frame of the BSDFs around the unit normal n (Duff et al., JCGT 2017):
 * tangent t and bitangent b, so that (t, b, n) is right-handed. */
void orc_frame(const float n[3], float t[3], float b[3]);
/* Uniform point on a triangle from (u1, u2); out = point. */
void orc_sample_triangle(const float v0[3], const float v1[3], const float v2[3], float u1,
                         float u2, float out[3]);
/* Self-intersection offset of p along n; tri = the 9 vertex coordinates of
 * the triangle p lies on (the offset scales with their magnitude). */
void orc_offset(const float p[3], const float n[3], const float tri[9], float out[3]);
/* Light pick: index of the light chosen by raw word w (-1 if no lights). */
int32_t orc_pick_light(const orc_scene* s, uint32_t w);
/* u32 -> [0,1) conversion used for every uniform variate. */
float orc_unif(uint32_t w);

#ifdef __cplusplus
}
#endif
#endif
