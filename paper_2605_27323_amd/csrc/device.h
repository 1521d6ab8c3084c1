// Device functions of the path tracer (gfx950, wave64).
//
// Arithmetic is binary32 in source order; the library is compiled with
// -ffp-contract=off and IEEE division/square root, so every float decision
// (closest hit, light pick, roulette, lobe) is reproducible on any IEEE
// machine that evaluates the same expressions.  Formulas follow the paper's
// estimator (Sec. 2.2, Eq. 3) with the readings fixed in the design notes:
// Philox4x64-10 random numbers keyed by (pixel, sample, bounce, job),
// pinhole camera with box-filter jitter, watertight ray/triangle test,
// Lambertian / GGX conductor / rough dielectric materials, next-event
// estimation with the power heuristic, roulette after the throughput update.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "ptmi.h"
#include "ptmi_internal.h"

namespace ptmi {

// Every function here is also compiled for the host, so that the exact
// kernel arithmetic can be run on the CPU by the test emulator.
#define PT_DEV __host__ __device__ __forceinline__

PT_DEV uint32_t f2u(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __float_as_uint(x);
#else
    uint32_t u;
    memcpy(&u, &x, 4);
    return u;
#endif
}
PT_DEV float u2f(uint32_t u) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __uint_as_float(u);
#else
    float x;
    memcpy(&x, &u, 4);
    return x;
#endif
}
PT_DEV uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

constexpr float kPi = (float)3.14159265358979323846;
constexpr float kInvPi = (float)(1.0 / 3.14159265358979323846);
constexpr float kShadowTmax = 0.9999f;
constexpr float kBoxSlack = 1.0f + 0x1p-16f;

struct f3 {
    float x, y, z;
};
PT_DEV f3 mk3(float x, float y, float z) { return f3{x, y, z}; }
PT_DEV f3 add3(f3 a, f3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
PT_DEV f3 sub3(f3 a, f3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
PT_DEV f3 scl3(f3 a, float s) { return mk3(a.x * s, a.y * s, a.z * s); }
PT_DEV f3 neg3(f3 a) { return mk3(-a.x, -a.y, -a.z); }
PT_DEV f3 mul3(f3 a, f3 b) { return mk3(a.x * b.x, a.y * b.y, a.z * b.z); }
PT_DEV float dot3(f3 a, f3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
PT_DEV f3 cross3(f3 a, f3 b) {
    return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// v * (1 / sqrt(|v|^2)), IEEE division and square root
PT_DEV f3 normalize3(f3 a) {
    float s = 1.0f / sqrtf(dot3(a, a));
    return scl3(a, s);
}
PT_DEV float comp3(f3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }
PT_DEV f3 xyz(float4 v) { return mk3(v.x, v.y, v.z); }
PT_DEV float max3c(f3 a) {
    float m = a.x > a.y ? a.x : a.y;
    return m > a.z ? m : a.z;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011)
// ---------------------------------------------------------------------------
struct Rng8 {
    uint32_t w[8];
};

PT_DEV Rng8 philox8(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce, uint32_t job) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = pixel, c1 = sample, c2 = bounce, c3 = job;
    uint64_t k0 = seed, k1 = 0;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0 = mulhi64(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = mulhi64(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    Rng8 r;
    r.w[0] = (uint32_t)c0; r.w[1] = (uint32_t)(c0 >> 32);
    r.w[2] = (uint32_t)c1; r.w[3] = (uint32_t)(c1 >> 32);
    r.w[4] = (uint32_t)c2; r.w[5] = (uint32_t)(c2 >> 32);
    r.w[6] = (uint32_t)c3; r.w[7] = (uint32_t)(c3 >> 32);
    return r;
}
// top 24 bits scaled by 2^-24: exact, in [0, 1)
PT_DEV float unif(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

// cos and sin of 2 pi u, evaluated in binary64 and rounded once
PT_DEV void cos_sin_2pi(float u, float& c, float& s) {
    double ph = (2.0 * 3.14159265358979323846) * (double)u;
#if defined(__HIP_DEVICE_COMPILE__)
    double sd, cd;
    sincos(ph, &sd, &cd);
#else
    double sd = ::sin(ph), cd = ::cos(ph);
#endif
    c = (float)cd;
    s = (float)sd;
}

// ---------------------------------------------------------------------------
// camera
// ---------------------------------------------------------------------------
PT_DEV void camera_ray(const CamView& cam, int px, int py, float u0, float u1, f3& o, f3& d) {
    float sx = (((float)px + u0) / (float)cam.W) * 2.0f - 1.0f;
    float sy = 1.0f - (((float)py + u1) / (float)cam.H) * 2.0f;
    f3 dd = mk3((sx * cam.R[0] + sy * cam.U[0]) + cam.F[0], (sx * cam.R[1] + sy * cam.U[1]) + cam.F[1],
                (sx * cam.R[2] + sy * cam.U[2]) + cam.F[2]);
    o = mk3(cam.E[0], cam.E[1], cam.E[2]);
    d = normalize3(dd);
}

// Radical inverse phi_b(n) = sum_i d_i b^-(i+1) of the base-b digits of n
// (b = 2 or 3), truncated to 24 bits: q with q 2^-24 <= phi_b(n).  Base 2
// reverses the bits; base 3 forms R = sum_{i<21} d_i 3^(20-i) (3^21 > 2^32
// covers every digit of a 32-bit n), so phi_3(n) = R / 3^21 exactly.
PT_DEV uint32_t radical_inverse24(uint32_t n, int base) {
    if (base == 2) return __builtin_bitreverse32(n) >> 8;
    uint64_t R = 0;
#pragma unroll
    for (int i = 0; i < 21; ++i) {
        R = R * 3u + (n % 3u);
        n /= 3u;
    }
    return (uint32_t)((R << 24) / 10460353203ull);  // 3^21
}

// Camera ray of sample `sample` of pixel `pix`.  The pixel jitter is Philox
// words 0, 1 of the path's first block, or with sampler 1 (the paper's
// wavefront sampler) the Halton(2,3) point of the sample index rotated by
// the pixel's Cranley-Patterson offsets (words 0, 1 of the reserved sample
// index 0xFFFFFFFF), modulo 1 on the 2^-24 grid.
PT_DEV void camera_sample(const CamView& cam, const PathParams& pp, uint32_t pix, uint32_t sample, f3& o, f3& d) {
    float u0, u1;
    if (pp.sampler == 1) {
        const Rng8 c = philox8(pp.seed, pix, 0xFFFFFFFFu, 0u, pp.job);
        u0 = (float)((radical_inverse24(sample, 2) + (c.w[0] >> 8)) & 0xFFFFFFu) * 0x1p-24f;
        u1 = (float)((radical_inverse24(sample, 3) + (c.w[1] >> 8)) & 0xFFFFFFu) * 0x1p-24f;
    } else {
        const Rng8 r0 = philox8(pp.seed, pix, sample, 0u, pp.job);
        u0 = unif(r0.w[0]);
        u1 = unif(r0.w[1]);
    }
    camera_ray(cam, (int)(pix % (uint32_t)cam.W), (int)(pix / (uint32_t)cam.W), u0, u1, o, d);
}

// ---------------------------------------------------------------------------
// rays: watertight triangle test (Woop, Benthin, Wald, JCGT 2013)
// ---------------------------------------------------------------------------
struct Ray {
    f3 o, d;
    f3 inv;  // 1/d for the slab test, components below 2^-80 in magnitude replaced by +-2^-80
    f3 oi;   // o * inv, rounded: slab distances are p * inv - oi, one fused multiply-add
    uint32_t k;  // axis permutation of the watertight test: kx | ky << 2 | kz << 4
    float Sx, Sy, Sz;
};

PT_DEV void set_shear(Ray& r, f3 d);

// Ray setup: inv = 1/d for the slab test (slab4_q bounds its errors, oi =
// o * inv rounded is its origin term).  A direction component below 2^-80
// is replaced by +-2^-80: over any hit distance the ray moves far less than
// the boxes' padding along that axis, so the smaller inverse keeps every
// distance's sign and leaves the test conservative.
PT_DEV Ray make_ray(f3 o, f3 d) {
    Ray r;
    r.o = o;
    r.d = d;
    r.inv = mk3(1.0f / (fabsf(d.x) >= 0x1p-80f ? d.x : copysignf(0x1p-80f, d.x)),
                1.0f / (fabsf(d.y) >= 0x1p-80f ? d.y : copysignf(0x1p-80f, d.y)),
                1.0f / (fabsf(d.z) >= 0x1p-80f ? d.z : copysignf(0x1p-80f, d.z)));
    r.oi = mk3(o.x * r.inv.x, o.y * r.inv.y, o.z * r.inv.z);
    set_shear(r, d);
    return r;
}

// The watertight test's axis permutation and shear constants of direction d
PT_DEV void set_shear(Ray& r, f3 d) {
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    int kz = 0;
    float m = ax;
    if (ay > m) {
        kz = 1;
        m = ay;
    }
    if (az > m) kz = 2;
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    float dkz = comp3(d, kz);
    if (dkz < 0.0f) {
        int t = kx;
        kx = ky;
        ky = t;
    }
    r.k = (uint32_t)kx | ((uint32_t)ky << 2) | ((uint32_t)kz << 4);
    r.Sx = comp3(d, kx) / dkz;
    r.Sy = comp3(d, ky) / dkz;
    r.Sz = 1.0f / dkz;
}

// Returns true on a hit with t > 0: t, and the barycentrics of v1 and v2
// undivided, as Vn / det and Wn / det (the traversal divides only for the
// hit it keeps).
PT_DEV bool tri_test(const Ray& r, f3 v0, f3 v1, f3 v2, float& t, float& Vn, float& Wn, float& dn) {
    const int kx = (int)(r.k & 3u), ky = (int)((r.k >> 2) & 3u), kz = (int)(r.k >> 4);
    f3 A = sub3(v0, r.o), B = sub3(v1, r.o), C = sub3(v2, r.o);
    float Akz = comp3(A, kz), Bkz = comp3(B, kz), Ckz = comp3(C, kz);
    float Ax = comp3(A, kx) - r.Sx * Akz;
    float Ay = comp3(A, ky) - r.Sy * Akz;
    float Bx = comp3(B, kx) - r.Sx * Bkz;
    float By = comp3(B, ky) - r.Sy * Bkz;
    float Cx = comp3(C, kx) - r.Sx * Ckz;
    float Cy = comp3(C, ky) - r.Sy * Ckz;
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        // exact binary32 products in binary64, one rounding each
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = (U + V) + W;
    if (det == 0.0f) return false;
    float Az = r.Sz * Akz;
    float Bz = r.Sz * Bkz;
    float Cz = r.Sz * Ckz;
    float T = (U * Az + V * Bz) + W * Cz;
    float tt = T / det;
    if (!(tt > 0.0f)) return false;
    t = tt;
    Vn = V;
    Wn = W;
    dn = det;
    return true;
}

// Returns true on a hit with t > 0; t and the barycentrics of v1, v2.
PT_DEV bool tri_intersect(const Ray& r, f3 v0, f3 v1, f3 v2, float& t, float& b1, float& b2) {
    float V, W, det;
    if (!tri_test(r, v0, v1, v2, t, V, W, det)) return false;
    b1 = V / det;
    b2 = W / det;
    return true;
}

// ---------------------------------------------------------------------------
// traversal stack: per-lane entries in LDS (stride = block size, so the 64
// lanes of a wave hit 64 consecutive 8-byte words), deeper entries spill to
// a per-lane global area (stride = number of lanes).  The LDS pointer
// carries the local address space so that pushes and pops compile to
// ds_write_b64 / ds_read_b64 rather than flat accesses.
//
// Each lane owns LDS + 1 LDS entries: entry LDS is a discard slot.  A node
// visit pushes its (up to three) farther children with push3, which writes
// all three candidates without branches, the invalid ones into the discard
// slot, as long as no lane of the wave is within three entries of the LDS
// limit (a wave-uniform test); otherwise it takes the per-entry path that
// spills to global memory.
// ---------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(3))) uint2 lds_uint2;
// product of two values below 2^24 (full-rate 24-bit multiply on the GPU)
__device__ __forceinline__ uint32_t mul24(uint32_t a, uint32_t b) { return __umul24(a, b); }
// true when the condition holds on no active lane of the wave
__device__ __forceinline__ bool wave_none(bool c) { return __ballot(c) == 0ull; }
#else
typedef uint2 lds_uint2;
inline uint32_t mul24(uint32_t a, uint32_t b) { return (a & 0xFFFFFFu) * (b & 0xFFFFFFu); }
inline bool wave_none(bool c) { return !c; }
#endif

// LDS bytes of a block's traversal stacks: LDS entries plus the discard slot
// per lane, 8 bytes each
PT_DEV constexpr size_t trav_stack_lds_bytes(int lds, int block) {
    return (size_t)(lds + 1) * sizeof(uint2) * (size_t)block;
}

template <int LDS, bool COUNT = false>
struct TravStack {
    static_assert(LDS >= 3, "push3 needs at least three LDS entries");
    lds_uint2* lds;  // (reference, entry distance bits), one 64-bit LDS access per push / pop
    uint2* gbl;      // spill area of all lanes (uniform); this lane's entry LDS + k is gbl[glane + k * gstride]
    uint32_t glane;
    int lstride;
    int gstride;
    int gcap;
    int sp;
    bool overflow;
    uint32_t nodes, tris;  // node visits and triangle tests of this lane (counted when COUNT)

    PT_DEV void push(uint32_t ref, float t) {
        const uint2 e = make_uint2(ref, f2u(t));
        if (sp < LDS) {
            lds[mul24((uint32_t)sp, (uint32_t)lstride)] = e;
        } else if (sp - LDS < gcap) {
            gbl[glane + (size_t)(sp - LDS) * (uint32_t)gstride] = e;
        } else {
            overflow = true;
            return;
        }
        ++sp;
    }
    // push e0, e1, e2 in this order, each only where its flag is set
    PT_DEV void push3(uint2 e0, bool v0, uint2 e1, bool v1, uint2 e2, bool v2) {
        if (wave_none(sp > LDS - 3)) {
            uint32_t s = (uint32_t)sp;
            const uint32_t a0 = v0 ? s : (uint32_t)LDS;
            s += v0 ? 1u : 0u;
            const uint32_t a1 = v1 ? s : (uint32_t)LDS;
            s += v1 ? 1u : 0u;
            const uint32_t a2 = v2 ? s : (uint32_t)LDS;
            s += v2 ? 1u : 0u;
            lds[mul24(a0, (uint32_t)lstride)] = e0;
            lds[mul24(a1, (uint32_t)lstride)] = e1;
            lds[mul24(a2, (uint32_t)lstride)] = e2;
            sp = (int)s;
        } else {
            if (v0) push(e0.x, u2f(e0.y));
            if (v1) push(e1.x, u2f(e1.y));
            if (v2) push(e2.x, u2f(e2.y));
        }
    }
    PT_DEV void pop(uint32_t& ref, float& t) {
        --sp;
        uint2 e;
        if (wave_none(sp >= LDS)) {
            e = lds[mul24((uint32_t)sp, (uint32_t)lstride)];
        } else if (sp < LDS) {
            e = lds[mul24((uint32_t)sp, (uint32_t)lstride)];
        } else {
            // a distinct load kind keeps the compiler from merging the two
            // branches into one flat load through a selected pointer
            const uint64_t g = __builtin_nontemporal_load(
                reinterpret_cast<const uint64_t*>(gbl + glane + (size_t)(sp - LDS) * (uint32_t)gstride));
            e = make_uint2((uint32_t)g, (uint32_t)(g >> 32));
        }
        ref = e.x;
        t = u2f(e.y);
    }
};

// lds_lane: this lane's first LDS entry (entry k at lds_lane[k * lstride],
// k = 0 .. LDS, the last one the discard slot);
// gbl: the spill area, where this lane's entry LDS + k is gbl[glane + k * gstride]
template <int LDS, bool COUNT = false>
PT_DEV TravStack<LDS, COUNT> make_trav_stack(uint2* lds_lane, int lstride, uint2* gbl, uint32_t glane, int gstride,
                                             int gcap) {
    TravStack<LDS, COUNT> st;
    st.lds = (lds_uint2*)lds_lane;
    st.lstride = lstride;
    st.gbl = gbl;
    st.glane = glane;
    st.gstride = gstride;
    st.gcap = gcap;
    st.sp = 0;
    st.overflow = false;
    st.nodes = st.tris = 0u;
    return st;
}

// During a traversal b1 and b2 hold the undivided barycentrics and det
// their denominator; closest_hit divides once at the end (hit_finish).
struct Hit {
    float t, b1, b2;
    float det;
    uint32_t tri;   // leaf-order index, ~0u on a miss
    uint32_t id;    // input id (tie-break)
    uint32_t inst;  // two-level scenes: instance record of the hit
    uint32_t iid;   // and its input index (tie-break before id)
};

PT_DEV void hit_finish(Hit& h) {
    if (h.tri != 0xFFFFFFFFu) {
        h.b1 = h.b1 / h.det;
        h.b2 = h.b2 / h.det;
    }
}

// plane offset c (0..3) of a word pair (w0: children 0, 1; w1: 2, 3) as float
PT_DEV float half_of(uint32_t w0, uint32_t w1, int c) {
    const uint32_t w = c < 2 ? w0 : w1;
    const uint16_t b = (uint16_t)((c & 1) ? (w >> 16) : (w & 0xFFFFu));
#if defined(__HIP_DEVICE_COMPILE__)
    return (float)__builtin_bit_cast(_Float16, b);
#else
    // binary16 to binary32 (exact)
    const uint32_t sgn = (uint32_t)(b >> 15) << 31, ex = (b >> 10) & 31u, man = b & 1023u;
    if (ex == 31u) return u2f(sgn | 0x7F800000u | (man << 13));
    if (ex == 0u) return man ? (b >> 15 ? -1.0f : 1.0f) * ldexpf((float)man, -24) : u2f(sgn);
    return u2f(sgn | ((ex + 112u) << 23) | (man << 13));
#endif
}

// Conservative slab test of the four children of a node against (0, tlim]:
// entry <= exit * (1 + 2^-16).  Writes the entry distances; returns a 4-bit
// hit mask.
// A plane at o_a + h 2^e (o_a the node's origin, h a binary16 offset) is at
// distance h (2^e inv_a) + (o_a inv_a - RN(o inv_a)): one fused
// multiply-add per plane (the binary16 operand read in place) after three
// per axis, with 2^e inv_a exact.  Besides the relative rounding of each
// result (covered by the slack), the errors are the roundings of o inv_a
// (make_ray) and of the per-axis term, at most 2^-24 of |o_a - o| in
// position: a part relative to the plane's distance and a part below 2^-23
// of the scene's largest coordinate, inside the builder's padding of every
// box.  The encoding only widens the boxes (planes rounded outward).  Per
// lane the near and far planes of an axis are chosen by the sign of its
// inverse direction, so the entry and exit distances per axis need no
// min/max.  Empty slots (planes +inf / -inf) are inverted boxes, also masked
// out by their reference.  A NaN distance is ignored by fmaxf / fminf,
// which keeps the test conservative.
PT_DEV unsigned slab4_q(const Ray& r, const float4 q[5], float tlim, float tn[4]) {
    const uint32_t e = f2u(q[0].w);
    const float Ax = ldexpf(r.inv.x, (int)(e & 255u) - 128);
    const float Ay = ldexpf(r.inv.y, (int)((e >> 8) & 255u) - 128);
    const float Az = ldexpf(r.inv.z, (int)((e >> 16) & 255u) - 128);
    const float Bx = fmaf(q[0].x, r.inv.x, -r.oi.x);
    const float By = fmaf(q[0].y, r.inv.y, -r.oi.y);
    const float Bz = fmaf(q[0].z, r.inv.z, -r.oi.z);
    const bool sx = (f2u(r.inv.x) >> 31) != 0u, sy = (f2u(r.inv.y) >> 31) != 0u, sz = (f2u(r.inv.z) >> 31) != 0u;
    // near / far word pairs per axis: lower planes (words 0, 1) or upper (2, 3)
    const uint32_t nx0 = f2u(sx ? q[1].z : q[1].x), nx1 = f2u(sx ? q[1].w : q[1].y);
    const uint32_t fx0 = f2u(sx ? q[1].x : q[1].z), fx1 = f2u(sx ? q[1].y : q[1].w);
    const uint32_t ny0 = f2u(sy ? q[2].z : q[2].x), ny1 = f2u(sy ? q[2].w : q[2].y);
    const uint32_t fy0 = f2u(sy ? q[2].x : q[2].z), fy1 = f2u(sy ? q[2].y : q[2].w);
    const uint32_t nz0 = f2u(sz ? q[3].z : q[3].x), nz1 = f2u(sz ? q[3].w : q[3].y);
    const uint32_t fz0 = f2u(sz ? q[3].x : q[3].z), fz1 = f2u(sz ? q[3].y : q[3].w);
    unsigned mask = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float ax = fmaf(half_of(nx0, nx1, c), Ax, Bx), bx = fmaf(half_of(fx0, fx1, c), Ax, Bx);
        float ay = fmaf(half_of(ny0, ny1, c), Ay, By), by = fmaf(half_of(fy0, fy1, c), Ay, By);
        float az = fmaf(half_of(nz0, nz1, c), Az, Bz), bz = fmaf(half_of(fz0, fz1, c), Az, Bz);
        float t0 = fmaxf(fmaxf(ax, ay), fmaxf(az, 0.0f));
        float t1 = fminf(fminf(bx, by), fminf(bz, tlim));
        tn[c] = t0;
        const float cref = c == 0 ? q[4].x : (c == 1 ? q[4].y : (c == 2 ? q[4].z : q[4].w));
        if (t0 <= t1 * kBoxSlack && f2u(cref) != kEmptyRef) mask |= 1u << c;
    }
    return mask;
}


// sort four (ref, t) pairs by t (ascending), invalid entries (t = +inf)
// last; a select network, no branches
PT_DEV void cswap(uint32_t& ra, float& ta, uint32_t& rb, float& tb) {
    const bool s = tb < ta;
    const float t0 = s ? tb : ta, t1 = s ? ta : tb;
    const uint32_t r0 = s ? rb : ra, r1 = s ? ra : rb;
    ta = t0;
    tb = t1;
    ra = r0;
    rb = r1;
}

PT_DEV void sort4(uint32_t ref[4], float t[4]) {
    cswap(ref[0], t[0], ref[1], t[1]);
    cswap(ref[2], t[2], ref[3], t[3]);
    cswap(ref[0], t[0], ref[2], t[2]);
    cswap(ref[1], t[1], ref[3], t[3]);
    cswap(ref[1], t[1], ref[2], t[2]);
}

// One fetch per lane and traversal step: five float4 from the node (an
// inner node) or from the leaf's first triangle record (a leaf: its three
// float4, then two that are not used; the triangle array's padding keeps
// the last record readable), issued by the same instructions for every
// lane before any lane uses them.  A wave whose lanes are at inner nodes
// and at leaves then waits for memory once per step, not once per branch.
// `ok` = the reference is in range (else node 0 is read and ignored).
PT_DEV void fetch_item(const SceneView& sc, uint32_t ref, bool ok, float4 q[5]) {
    const uint32_t r = ok ? ref : 0u;
    const float4* p = (r & kLeafBit) ? sc.tris + (size_t)(r & kLeafFirstMask) * 3 : sc.nodes + (size_t)mul24(r, 5u);
    q[0] = p[0];
    q[1] = p[1];
    q[2] = p[2];
    q[3] = p[3];
    q[4] = p[4];
}

// Closest hit in (0, tmax): smallest t, ties to the smaller input id.
// References outside the node or triangle arrays are skipped, so a damaged
// BVH cannot make a lane read out of bounds.
//
// The traversal is written as a resumable step (closest_step), so that a
// persistent kernel can run one step per loop trip and hand a finished
// lane a new ray while the others are still traversing.  closest_hit runs
// the steps to the end.

template <int LDS, bool COUNT = false>
PT_DEV void closest_begin(float tmax, Hit& h, uint32_t& ref, TravStack<LDS, COUNT>& st) {
    h.t = tmax;
    h.b1 = 0.0f;
    h.b2 = 0.0f;
    h.det = 1.0f;
    h.tri = 0xFFFFFFFFu;
    h.id = 0xFFFFFFFFu;
    st.sp = 0;
    ref = 0;  // root
}

// Visit `ref` (an inner node: push the farther hit children, move to the
// nearest; a leaf: test its triangles), then pop the next entry that can
// still hold a closer hit.  Returns false when the traversal is finished.
template <int LDS, bool COUNT = false>
PT_DEV bool closest_step(const SceneView& sc, const Ray& r, float tmax, Hit& h, uint32_t& ref, TravStack<LDS, COUNT>& st) {
    const bool leaf = (ref & kLeafBit) != 0;
    const uint32_t first = ref & kLeafFirstMask;
    const uint32_t cnt = ((ref >> kLeafCountShift) & 15u) + 1u;
    const bool ok = leaf ? first + cnt <= (uint32_t)sc.nt : ref < (uint32_t)sc.n_nodes;
    float4 q[5];
    fetch_item(sc, ref, ok, q);
    if (!leaf) {
        if (ok) {
            if constexpr (COUNT) ++st.nodes;
            float tn[4];
            unsigned m = slab4_q(r, q, h.t, tn);
            if (m) {
                uint32_t rr[4];
                float tt[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    bool hit = (m >> c) & 1u;
                    const float cref = c == 0 ? q[4].x : (c == 1 ? q[4].y : (c == 2 ? q[4].z : q[4].w));
                    rr[c] = hit ? f2u(cref) : kEmptyRef;
                    tt[c] = hit ? tn[c] : INFINITY;
                }
                sort4(rr, tt);
                // push the farther hits (farthest first), descend into the nearest
                st.push3(make_uint2(rr[3], f2u(tt[3])), rr[3] != kEmptyRef, make_uint2(rr[2], f2u(tt[2])),
                         rr[2] != kEmptyRef, make_uint2(rr[1], f2u(tt[1])), rr[1] != kEmptyRef);
                ref = rr[0];
                return true;
            }
        }
    } else {
        if (ok) {
            if constexpr (COUNT) st.tris += cnt;
            for (uint32_t i = first; i < first + cnt; ++i) {
                float4 a = q[0], b = q[1], c = q[2];  // the first triangle came with the fetch
                if (i != first) {
                    const float4* tp = sc.tris + (size_t)i * 3;
                    a = tp[0];
                    b = tp[1];
                    c = tp[2];
                }
                float t, vn, wn, dn;
                if (tri_test(r, xyz(a), xyz(b), xyz(c), t, vn, wn, dn) && t < tmax) {
                    uint32_t id = f2u(a.w);
                    if (t < h.t || (t == h.t && id < h.id)) {
                        h.t = t;
                        h.b1 = vn;
                        h.b2 = wn;
                        h.det = dn;
                        h.tri = i;
                        h.id = id;
                    }
                }
            }
        }
    }
    while (st.sp > 0) {
        float t;
        st.pop(ref, t);
        if (t <= h.t * kBoxSlack) return true;
    }
    return false;
}

template <int LDS, bool COUNT = false>
PT_DEV Hit closest_hit(const SceneView& sc, const Ray& r, float tmax, TravStack<LDS, COUNT>& st) {
    Hit h;
    uint32_t ref;
    closest_begin<LDS>(tmax, h, ref, st);
    while (closest_step<LDS>(sc, r, tmax, h, ref, st)) {
    }
    hit_finish(h);
    return h;
}

// Barycentrics of the closest hit h of the ray (o, d), when the stage that
// found it kept only t and the triangle (the stage kernels' hit record):
// the watertight test of that triangle again, on the same inputs, so the
// values are the ones the traversal had.
PT_DEV void hit_barycentrics(const SceneView& sc, f3 o, f3 d, Hit& h) {
    h.b1 = 0.0f;
    h.b2 = 0.0f;
    if (h.tri >= (uint32_t)sc.nt) return;
    Ray r;
    r.o = o;
    set_shear(r, d);
    const float4* tp = sc.tris + (size_t)h.tri * 3;
    float t;
    tri_intersect(r, xyz(tp[0]), xyz(tp[1]), xyz(tp[2]), t, h.b1, h.b2);
}

// Any hit in (0, tmax), as resumable steps: any_step visits `ref` and pops
// the next entry; it returns false when the traversal is finished, with
// `occluded` set if a triangle was hit.
template <int LDS, bool COUNT = false>
PT_DEV void any_begin(uint32_t& ref, TravStack<LDS, COUNT>& st) {
    st.sp = 0;
    ref = 0;
}

template <int LDS, bool COUNT = false>
PT_DEV bool any_step(const SceneView& sc, const Ray& r, float tmax, uint32_t& ref, TravStack<LDS, COUNT>& st,
                     bool& occluded) {
    const bool leaf = (ref & kLeafBit) != 0;
    const uint32_t first = ref & kLeafFirstMask;
    const uint32_t cnt = ((ref >> kLeafCountShift) & 15u) + 1u;
    const bool ok = leaf ? first + cnt <= (uint32_t)sc.nt : ref < (uint32_t)sc.n_nodes;
    float4 q[5];
    fetch_item(sc, ref, ok, q);
    if (!leaf) {
        if (ok) {
            if constexpr (COUNT) ++st.nodes;
            float tn[4];
            unsigned m = slab4_q(r, q, tmax, tn);
            if (m) {
                // descend into the last hit child, push the other hit ones
                const uint32_t cr[4] = {f2u(q[4].x), f2u(q[4].y), f2u(q[4].z), f2u(q[4].w)};
                const uint32_t last = 31u - (uint32_t)__builtin_clz(m);
                st.push3(make_uint2(cr[0], f2u(tn[0])), (m & 1u) && last > 0u, make_uint2(cr[1], f2u(tn[1])),
                         ((m >> 1) & 1u) && last > 1u, make_uint2(cr[2], f2u(tn[2])), ((m >> 2) & 1u) && last > 2u);
                ref = last == 0u ? cr[0] : (last == 1u ? cr[1] : (last == 2u ? cr[2] : cr[3]));
                return true;
            }
        }
    } else {
        if (ok) {
            for (uint32_t i = first; i < first + cnt; ++i) {
                if constexpr (COUNT) ++st.tris;
                float4 a = q[0], b = q[1], c = q[2];  // the first triangle came with the fetch
                if (i != first) {
                    const float4* tp = sc.tris + (size_t)i * 3;
                    a = tp[0];
                    b = tp[1];
                    c = tp[2];
                }
                float t, vn, wn, dn;
                if (tri_test(r, xyz(a), xyz(b), xyz(c), t, vn, wn, dn) && t < tmax) {
                    occluded = true;
                    return false;
                }
            }
        }
    }
    if (st.sp == 0) return false;
    float t;
    st.pop(ref, t);
    return true;
}

template <int LDS, bool COUNT = false>
PT_DEV bool any_hit(const SceneView& sc, const Ray& r, float tmax, TravStack<LDS, COUNT>& st) {
    uint32_t ref;
    any_begin<LDS>(ref, st);
    bool occluded = false;
    while (any_step<LDS>(sc, r, tmax, ref, st, occluded)) {
    }
    return occluded;
}

// ---------------------------------------------------------------------------
// two-level traversal (paper Sec. 2.3 and 3: a top-level structure over
// instances of per-mesh bottom-level structures)
// ---------------------------------------------------------------------------
// Affine map by a 3x4 matrix given as three float4 rows (linear part xyz,
// translation w): ((r.x x + r.y y) + r.z z) + r.w per row; directions drop
// the translation.
PT_DEV f3 xform_point(float4 r0, float4 r1, float4 r2, f3 p) {
    return mk3(((r0.x * p.x + r0.y * p.y) + r0.z * p.z) + r0.w, ((r1.x * p.x + r1.y * p.y) + r1.z * p.z) + r1.w,
               ((r2.x * p.x + r2.y * p.y) + r2.z * p.z) + r2.w);
}
PT_DEV f3 xform_dir(float4 r0, float4 r1, float4 r2, f3 d) {
    return mk3((r0.x * d.x + r0.y * d.y) + r0.z * d.z, (r1.x * d.x + r1.y * d.y) + r1.z * d.z,
               (r2.x * d.x + r2.y * d.y) + r2.z * d.z);
}

// The ray of a two-level traversal.  At a top-level leaf the active Ray
// becomes the instance's object-space ray (origin and direction mapped by
// its world-to-object rows, not renormalised, so a point at parameter t is
// the image of the world ray's point at t and distances stay comparable
// across instances) and a marker entry is pushed; popping the marker
// restores the world ray kept here.
struct InstTrav {
    f3 o, d;       // the world ray
    uint32_t rec;  // instance record while inside a mesh
    uint32_t iid;  // its input index
    bool obj;      // inside a mesh
};

PT_DEV void inst_begin(f3 o, f3 d, InstTrav& it) {
    it.o = o;
    it.d = d;
    it.rec = 0u;
    it.iid = 0u;
    it.obj = false;
}

// Enter the instance of top-level leaf `ref`: object-space ray, marker, the
// mesh's root as the next reference.  False for a reference outside the
// instance records.
template <int LDS, bool COUNT>
PT_DEV bool inst_enter(const SceneView& sc, Ray& r, InstTrav& it, uint32_t& ref, TravStack<LDS, COUNT>& st) {
    const uint32_t rec = ref & kLeafFirstMask;
    if (rec >= (uint32_t)sc.n_inst) return false;
    const float4* ip = sc.insts + (size_t)rec * kInstRecord;
    const float4 w0 = ip[0], w1 = ip[1], w2 = ip[2], meta = ip[6];
    r = make_ray(xform_point(w0, w1, w2, it.o), xform_dir(w0, w1, w2, it.d));
    it.obj = true;
    it.rec = rec;
    it.iid = f2u(meta.y);
    st.push(kInstMarker, 0.0f);
    ref = f2u(meta.x);
    return true;
}

// closest_step over a two-level scene; closest-hit key (t, input instance,
// input triangle)
template <int LDS, bool COUNT = false, bool SPLIT = false>
PT_DEV bool closest_step_inst(const SceneView& sc, Ray& r, InstTrav& it, float tmax, Hit& h, uint32_t& ref,
                              TravStack<LDS, COUNT>& st) {
    // one fetch as in closest_step (an instance leaf fetches its record in
    // inst_enter instead); SPLIT: each branch fetches its own (the
    // megakernel's two-level traversal, whose register budget the single
    // fetch exceeds)
    const bool leaf = (ref & kLeafBit) != 0;
    const uint32_t first = ref & kLeafFirstMask;
    const uint32_t cnt = ((ref >> kLeafCountShift) & 15u) + 1u;
    const bool ok = leaf ? it.obj && first + cnt <= (uint32_t)sc.nt : ref < (uint32_t)sc.n_nodes;
    float4 q[5];
    if constexpr (!SPLIT) fetch_item(sc, ref, ok, q);
    if (!leaf) {
        if (ok) {
            if constexpr (SPLIT) fetch_item(sc, ref, true, q);
            if constexpr (COUNT) ++st.nodes;
            float tn[4];
            unsigned m = slab4_q(r, q, h.t, tn);
            if (m) {
                uint32_t rr[4];
                float tt[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    bool hit = (m >> c) & 1u;
                    const float cref = c == 0 ? q[4].x : (c == 1 ? q[4].y : (c == 2 ? q[4].z : q[4].w));
                    rr[c] = hit ? f2u(cref) : kEmptyRef;
                    tt[c] = hit ? tn[c] : INFINITY;
                }
                sort4(rr, tt);
                st.push3(make_uint2(rr[3], f2u(tt[3])), rr[3] != kEmptyRef, make_uint2(rr[2], f2u(tt[2])),
                         rr[2] != kEmptyRef, make_uint2(rr[1], f2u(tt[1])), rr[1] != kEmptyRef);
                ref = rr[0];
                return true;
            }
        }
    } else if (!it.obj) {
        if (inst_enter<LDS, COUNT>(sc, r, it, ref, st)) return true;
    } else {
        if (ok) {
            if constexpr (SPLIT) fetch_item(sc, ref, true, q);
            if constexpr (COUNT) st.tris += cnt;
            for (uint32_t i = first; i < first + cnt; ++i) {
                float4 a = q[0], b = q[1], c = q[2];  // the first triangle came with the fetch
                if (i != first) {
                    const float4* tp = sc.tris + (size_t)i * 3;
                    a = tp[0];
                    b = tp[1];
                    c = tp[2];
                }
                float t, vn, wn, dn;
                if (tri_test(r, xyz(a), xyz(b), xyz(c), t, vn, wn, dn) && t < tmax) {
                    uint32_t id = f2u(a.w);
                    if (t < h.t || (t == h.t && (it.iid < h.iid || (it.iid == h.iid && id < h.id)))) {
                        h.t = t;
                        h.b1 = vn;
                        h.b2 = wn;
                        h.det = dn;
                        h.tri = i;
                        h.id = id;
                        h.inst = it.rec;
                        h.iid = it.iid;
                    }
                }
            }
        }
    }
    while (st.sp > 0) {
        float t;
        st.pop(ref, t);
        if (ref == kInstMarker) {
            r = make_ray(it.o, it.d);
            it.obj = false;
            continue;
        }
        if (t <= h.t * kBoxSlack) return true;
    }
    return false;
}

template <int LDS, bool COUNT = false>
PT_DEV void closest_begin_inst(f3 o, f3 d, float tmax, Ray& r, InstTrav& it, Hit& h, uint32_t& ref,
                               TravStack<LDS, COUNT>& st) {
    closest_begin<LDS>(tmax, h, ref, st);
    h.inst = 0u;
    h.iid = 0xFFFFFFFFu;
    inst_begin(o, d, it);
    r = make_ray(o, d);
}

// any_step over a two-level scene
template <int LDS, bool COUNT = false, bool SPLIT = false>
PT_DEV bool any_step_inst(const SceneView& sc, Ray& r, InstTrav& it, float tmax, uint32_t& ref,
                          TravStack<LDS, COUNT>& st, bool& occluded) {
    const bool leaf = (ref & kLeafBit) != 0;
    const uint32_t first = ref & kLeafFirstMask;
    const uint32_t cnt = ((ref >> kLeafCountShift) & 15u) + 1u;
    const bool ok = leaf ? it.obj && first + cnt <= (uint32_t)sc.nt : ref < (uint32_t)sc.n_nodes;
    float4 q[5];
    if constexpr (!SPLIT) fetch_item(sc, ref, ok, q);
    if (!leaf) {
        if (ok) {
            if constexpr (SPLIT) fetch_item(sc, ref, true, q);
            if constexpr (COUNT) ++st.nodes;
            float tn[4];
            unsigned m = slab4_q(r, q, tmax, tn);
            if (m) {
                const uint32_t cr[4] = {f2u(q[4].x), f2u(q[4].y), f2u(q[4].z), f2u(q[4].w)};
                const uint32_t last = 31u - (uint32_t)__builtin_clz(m);
                st.push3(make_uint2(cr[0], f2u(tn[0])), (m & 1u) && last > 0u, make_uint2(cr[1], f2u(tn[1])),
                         ((m >> 1) & 1u) && last > 1u, make_uint2(cr[2], f2u(tn[2])), ((m >> 2) & 1u) && last > 2u);
                ref = last == 0u ? cr[0] : (last == 1u ? cr[1] : (last == 2u ? cr[2] : cr[3]));
                return true;
            }
        }
    } else if (!it.obj) {
        if (inst_enter<LDS, COUNT>(sc, r, it, ref, st)) return true;
    } else {
        if (ok) {
            if constexpr (SPLIT) fetch_item(sc, ref, true, q);
            for (uint32_t i = first; i < first + cnt; ++i) {
                if constexpr (COUNT) ++st.tris;
                float4 a = q[0], b = q[1], c = q[2];  // the first triangle came with the fetch
                if (i != first) {
                    const float4* tp = sc.tris + (size_t)i * 3;
                    a = tp[0];
                    b = tp[1];
                    c = tp[2];
                }
                float t, vn, wn, dn;
                if (tri_test(r, xyz(a), xyz(b), xyz(c), t, vn, wn, dn) && t < tmax) {
                    occluded = true;
                    return false;
                }
            }
        }
    }
    while (st.sp > 0) {
        float t;
        st.pop(ref, t);
        if (ref == kInstMarker) {
            r = make_ray(it.o, it.d);
            it.obj = false;
            continue;
        }
        return true;
    }
    return false;
}

// Closest hit and any hit in (0, tmax) of the world ray (o, d): the flat
// traversal, or with INST the two-level one
template <int LDS, bool COUNT = false, bool INST = false>
PT_DEV Hit closest_hit_t(const SceneView& sc, f3 o, f3 d, float tmax, TravStack<LDS, COUNT>& st) {
    if constexpr (INST) {
        Hit h;
        Ray r;
        InstTrav it;
        uint32_t ref;
        closest_begin_inst<LDS>(o, d, tmax, r, it, h, ref, st);
        while (closest_step_inst<LDS, COUNT, true>(sc, r, it, tmax, h, ref, st)) {
        }
        hit_finish(h);
        return h;
    } else {
        return closest_hit<LDS>(sc, make_ray(o, d), tmax, st);
    }
}
template <int LDS, bool COUNT = false, bool INST = false>
PT_DEV bool any_hit_t(const SceneView& sc, f3 o, f3 d, float tmax, TravStack<LDS, COUNT>& st) {
    if constexpr (INST) {
        Ray r = make_ray(o, d);
        InstTrav it;
        inst_begin(o, d, it);
        uint32_t ref;
        any_begin<LDS>(ref, st);
        bool occluded = false;
        while (any_step_inst<LDS, COUNT, true>(sc, r, it, tmax, ref, st, occluded)) {
        }
        return occluded;
    } else {
        return any_hit<LDS>(sc, make_ray(o, d), tmax, st);
    }
}

// World-space vertices of the hit triangle: the record's vertices, mapped by
// the object-to-world rows of instance record `rec` in a two-level scene
PT_DEV void inst_vertices(const SceneView& sc, uint32_t rec, float4& a, float4& b, float4& c) {
    const float4* ip = sc.insts + (size_t)rec * kInstRecord;
    const float4 o0 = ip[3], o1 = ip[4], o2 = ip[5];
    const f3 wa = xform_point(o0, o1, o2, xyz(a)), wb = xform_point(o0, o1, o2, xyz(b)),
             wc = xform_point(o0, o1, o2, xyz(c));
    a = make_float4(wa.x, wa.y, wa.z, a.w);
    b = make_float4(wb.x, wb.y, wb.z, b.w);
    c = make_float4(wc.x, wc.y, wc.z, c.w);
}

// hit_barycentrics in a two-level scene: the same test in the object space
// of the hit's instance record h.inst, with the object-space ray of the
// traversal
PT_DEV void hit_barycentrics_inst(const SceneView& sc, f3 o, f3 d, Hit& h) {
    h.b1 = 0.0f;
    h.b2 = 0.0f;
    if (h.tri >= (uint32_t)sc.nt || h.inst >= (uint32_t)sc.n_inst) return;
    const float4* ip = sc.insts + (size_t)h.inst * kInstRecord;
    const float4 w0 = ip[0], w1 = ip[1], w2 = ip[2];
    Ray r;
    r.o = xform_point(w0, w1, w2, o);
    set_shear(r, xform_dir(w0, w1, w2, d));
    const float4* tp = sc.tris + (size_t)h.tri * 3;
    float t;
    tri_intersect(r, xyz(tp[0]), xyz(tp[1]), xyz(tp[2]), t, h.b1, h.b2);
}

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
// Self-intersection offset: p + (2^-15 m) n per coordinate, m the largest
// coordinate magnitude of the triangle p lies on (at least 2^-7).  The scale
// is that of Waechter and Binder (Ray Tracing Gems ch. 6: about 256 ulps),
// measured on the triangle: the hit point and the next intersection test
// with the same triangle err by a few ulps of its vertex coordinates, which
// on a large triangle near a coordinate plane exceed a step measured on the
// point's own small coordinates.
PT_DEV float tri_extent(f3 v0, f3 v1, f3 v2) {
    const float c[9] = {v0.x, v0.y, v0.z, v1.x, v1.y, v1.z, v2.x, v2.y, v2.z};
    float m = 0x1p-7f;
#pragma unroll
    for (int i = 0; i < 9; ++i) m = fabsf(c[i]) > m ? fabsf(c[i]) : m;
    return m;
}
PT_DEV f3 offset_point(f3 p, f3 n, float m) {
    const float dl = 0x1p-15f * m;
    return mk3(p.x + dl * n.x, p.y + dl * n.y, p.z + dl * n.z);
}

PT_DEV f3 tri_normal(f3 v0, f3 v1, f3 v2) {
    f3 c = cross3(sub3(v1, v0), sub3(v2, v0));
    if (dot3(c, c) == 0.0f) return mk3(0.0f, 0.0f, 1.0f);
    return normalize3(c);
}

// uniform point: b1 = sqrt(u1)(1-u2), b2 = sqrt(u1) u2 on edges e1, e2
PT_DEV f3 tri_point(f3 v0, f3 v1, f3 v2, float u1, float u2) {
    f3 e1 = sub3(v1, v0), e2 = sub3(v2, v0);
    float su = sqrtf(u1);
    float b1 = su * (1.0f - u2), b2 = su * u2;
    return mk3((v0.x + b1 * e1.x) + b2 * e2.x, (v0.y + b1 * e1.y) + b2 * e2.y, (v0.z + b1 * e1.z) + b2 * e2.z);
}

// Orthonormal basis (Duff et al., JCGT 2017).
struct Frame {
    f3 t, b, n;
};
PT_DEV Frame make_frame(f3 n) {
    float sign = copysignf(1.0f, n.z);
    float a = -1.0f / (sign + n.z);
    float b = n.x * n.y * a;
    Frame f;
    f.t = mk3(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
    f.b = mk3(b, sign + n.y * n.y * a, -n.y);
    f.n = n;
    return f;
}
PT_DEV f3 to_local(const Frame& f, f3 w) { return mk3(dot3(f.t, w), dot3(f.b, w), dot3(f.n, w)); }
PT_DEV f3 to_world(const Frame& f, f3 l) {
    return mk3((f.t.x * l.x + f.b.x * l.y) + f.n.x * l.z, (f.t.y * l.x + f.b.y * l.y) + f.n.y * l.z,
               (f.t.z * l.x + f.b.z * l.y) + f.n.z * l.z);
}

// ---------------------------------------------------------------------------
// vertex attributes at a hit (paper Sec. 2.3: the shading stage rebuilds the
// hit's attributes from its triangle and barycentrics): weights
// (w0, b1, b2), w0 = (1 - b1) - b2, summed as ((w0 a0 + b1 a1) + b2 a2)
// ---------------------------------------------------------------------------
PT_DEV float interp3(float a0, float a1, float a2, float w0, float b1, float b2) {
    return (w0 * a0 + b1 * a1) + b2 * a2;
}

// Shading normal of hit h: the interpolated vertex normal (object space in a
// two-level scene, mapped by the inverse transpose of the instance's
// object-to-world map = the columns of its world-to-object rows),
// normalised once and turned to the side of the geometric normal ng; ng
// itself when the interpolant is zero or not finite.
template <bool INST>
PT_DEV f3 shading_normal(const SceneView& sc, const Hit& h, f3 ng) {
    const float4* ap = sc.attrs + (size_t)h.tri * kAttrRecord;
    const float4 a0 = ap[0], a1 = ap[1], a2 = ap[2];
    const float w0 = (1.0f - h.b1) - h.b2;
    f3 m = mk3(interp3(a0.x, a1.x, a2.x, w0, h.b1, h.b2), interp3(a0.y, a1.y, a2.y, w0, h.b1, h.b2),
               interp3(a0.z, a1.z, a2.z, w0, h.b1, h.b2));
    if constexpr (INST) {
        const float4* ip = sc.insts + (size_t)h.inst * kInstRecord;
        const float4 r0 = ip[0], r1 = ip[1], r2 = ip[2];
        m = mk3((r0.x * m.x + r1.x * m.y) + r2.x * m.z, (r0.y * m.x + r1.y * m.y) + r2.y * m.z,
                (r0.z * m.x + r1.z * m.y) + r2.z * m.z);
    }
    const float l2 = dot3(m, m);
    if (!(l2 > 0.0f && l2 <= 3.40282347e38f)) return ng;
    const f3 ns = normalize3(m);
    return dot3(ns, ng) < 0.0f ? neg3(ns) : ns;
}

// Checker texture of the albedo: cell (floor(u f), floor(v f)) of the
// interpolated texture coordinates; the factor is 1/4 where the two cell
// indices differ in parity, else 1.  Parity of floor(x): floor(x) / 2 is an
// integer or a half, both exact in binary32.
constexpr float kCheckerDark = 0.25f;
PT_DEV bool odd_cell(float x) {
    const float f = floorf(x);
    const float hf = f * 0.5f;
    return floorf(hf) != hf;
}
PT_DEV float checker(const SceneView& sc, const Hit& h, float freq) {
    const float4* ap = sc.attrs + (size_t)h.tri * kAttrRecord;
    const float4 a0 = ap[0], a1 = ap[1], a2 = ap[2], a3 = ap[3];
    const float w0 = (1.0f - h.b1) - h.b2;
    const float u = interp3(a0.w, a2.w, a3.y, w0, h.b1, h.b2), v = interp3(a1.w, a3.x, a3.z, w0, h.b1, h.b2);
    return odd_cell(u * freq) != odd_cell(v * freq) ? kCheckerDark : 1.0f;
}

// ---------------------------------------------------------------------------
// materials
// ---------------------------------------------------------------------------
PT_DEV float ggx_alpha(float rough) {
    float a = rough * rough;
    return a < 1e-4f ? 1e-4f : a;
}
// GGX D for a unit half vector; hx^2 + hy^2 + a2 hz^2 avoids the
// cancellation of cos^2 (a2 - 1) + 1 near the peak
PT_DEV float ggx_D(f3 h, float a2) {
    float den = (h.x * h.x + h.y * h.y) + a2 * (h.z * h.z);
    return a2 / ((kPi * den) * den);
}
PT_DEV float ggx_lambda(f3 w, float a2) {
    float t2 = (w.x * w.x + w.y * w.y) / (w.z * w.z);
    return (sqrtf(1.0f + a2 * t2) - 1.0f) * 0.5f;
}
// visible-normal sampling (Heitz, JCGT 2018)
PT_DEV f3 ggx_vndf(f3 wo, float alpha, float u5, float u6) {
    f3 Vh = normalize3(mk3(alpha * wo.x, alpha * wo.y, wo.z));
    float lensq = Vh.x * Vh.x + Vh.y * Vh.y;
    f3 T1 = lensq > 0.0f ? scl3(mk3(-Vh.y, Vh.x, 0.0f), 1.0f / sqrtf(lensq)) : mk3(1.0f, 0.0f, 0.0f);
    f3 T2 = cross3(Vh, T1);
    float r = sqrtf(u5), c, s;
    cos_sin_2pi(u6, c, s);
    float t1 = r * c, t2 = r * s;
    float sh = 0.5f * (1.0f + Vh.z);
    t2 = (1.0f - sh) * sqrtf(1.0f - t1 * t1) + sh * t2;
    float nz2 = (1.0f - t1 * t1) - t2 * t2;
    float nz = sqrtf(nz2 > 0.0f ? nz2 : 0.0f);
    f3 Nh = mk3((t1 * T1.x + t2 * T2.x) + nz * Vh.x, (t1 * T1.y + t2 * T2.y) + nz * Vh.y,
                (t1 * T1.z + t2 * T2.z) + nz * Vh.z);
    return normalize3(mk3(alpha * Nh.x, alpha * Nh.y, Nh.z > 0.0f ? Nh.z : 0.0f));
}
PT_DEV float pow5(float m) { return ((m * m) * (m * m)) * m; }

// Albedo-free factors of a lobe, kept for the adjoint: f (or the sampling
// weight) = Lambert: albedo * k (k holds the texture factor); conductor:
// (albedo + (1 - albedo) m5) * k; dielectric: k, untinted; coated:
// albedo * k + m5 (k: the base seen through the coat, m5: the coat's
// specular term).
struct Lobe {
    int type;
    float m5, k;
};

// value and albedo derivative of a lobe at albedo rho (one channel)
PT_DEV float lobe_value(const Lobe& lb, float rho) {
    if (lb.type == PT_LAMBERT) return rho * lb.k;
    if (lb.type == PT_CONDUCTOR) return (rho + (1.0f - rho) * lb.m5) * lb.k;
    if (lb.type == PT_COATED) return rho * lb.k + lb.m5;
    return lb.k;
}
PT_DEV float lobe_der(const Lobe& lb) {
    if (lb.type == PT_LAMBERT || lb.type == PT_COATED) return lb.k;
    if (lb.type == PT_CONDUCTOR) return (1.0f - lb.m5) * lb.k;
    return 0.0f;
}

PT_DEV float fresnel_dielectric(float ci, float eta);

// Coated material: a GGX dielectric coat of index ior over a Lambertian base,
// f = F(wo.h) D G2 / (4 cos_o cos_i) + (1 - F(cos_o)) (1 - F(cos_i)) tex
// albedo / pi, pdf = F(cos_o) G1 D / (4 cos_o) + (1 - F(cos_o)) cos_i / pi
// (the mixture the sampler draws from).  wo, wi above the surface.
PT_DEV void eval_coat(float rough, float ior, float tex, f3 alb, f3 wo, f3 wi, f3& f, float& pdf, Lobe& lb) {
    const float alpha = ggx_alpha(rough), a2 = alpha * alpha;
    const f3 h = normalize3(add3(wo, wi));
    const float D = ggx_D(h, a2);
    const float lo = ggx_lambda(wo, a2), li = ggx_lambda(wi, a2);
    const float G1 = 1.0f / (1.0f + lo);
    const float G2 = 1.0f / ((1.0f + lo) + li);
    const float Fh = fresnel_dielectric(dot3(wo, h), ior);
    const float fs = ((Fh * D) * G2) / ((4.0f * wo.z) * wi.z);
    const float Fo = fresnel_dielectric(wo.z, ior), Fi = fresnel_dielectric(wi.z, ior);
    const float kd = (((1.0f - Fo) * (1.0f - Fi)) * tex) * kInvPi;
    f = mk3(alb.x * kd + fs, alb.y * kd + fs, alb.z * kd + fs);
    pdf = Fo * ((G1 * D) / (4.0f * wo.z)) + (1.0f - Fo) * (wi.z * kInvPi);
    lb.k = kd;
    lb.m5 = fs;
}

// cosine-weighted direction about +z
PT_DEV f3 cosine_dir(float u5, float u6) {
    float r = sqrtf(u5), c, s;
    cos_sin_2pi(u6, c, s);
    float z2 = 1.0f - u5;
    return mk3(r * c, r * s, sqrtf(z2 > 0.0f ? z2 : 0.0f));
}

// f and the solid-angle pdf of an opaque material, wo and wi in the local
// frame of the normal on wo's side.  EXT: the scene may hold coated
// materials (else their case is compiled out).
template <bool EXT = true>
PT_DEV void eval_opaque(int type, float rough, float ior, float tex, f3 alb, f3 wo, f3 wi, f3& f, float& pdf,
                        Lobe& lb) {
    f = mk3(0.0f, 0.0f, 0.0f);
    pdf = 0.0f;
    lb.type = type;
    lb.m5 = 0.0f;
    lb.k = 0.0f;
    if (wi.z <= 0.0f || wo.z <= 0.0f) return;
    if (type == PT_LAMBERT) {
        const float k = tex * kInvPi;
        f = mk3(alb.x * k, alb.y * k, alb.z * k);
        pdf = wi.z * kInvPi;
        lb.k = k;
        return;
    }
    if (EXT && type == PT_COATED) {
        eval_coat(rough, ior, tex, alb, wo, wi, f, pdf, lb);
        return;
    }
    float alpha = ggx_alpha(rough), a2 = alpha * alpha;
    f3 h = normalize3(add3(wo, wi));
    float D = ggx_D(h, a2);
    float lo = ggx_lambda(wo, a2), li = ggx_lambda(wi, a2);
    float G1 = 1.0f / (1.0f + lo);
    float G2 = 1.0f / ((1.0f + lo) + li);
    float m5 = pow5(1.0f - dot3(wi, h));
    float k = (D * G2) / ((4.0f * wo.z) * wi.z);
    f = mk3((alb.x + (1.0f - alb.x) * m5) * k, (alb.y + (1.0f - alb.y) * m5) * k, (alb.z + (1.0f - alb.z) * m5) * k);
    pdf = (G1 * D) / (4.0f * wo.z);
    lb.m5 = m5;
    lb.k = k;
}

// exact unpolarised Fresnel reflectance, eta = eta_t / eta_i
PT_DEV float fresnel_dielectric(float ci, float eta) {
    float s2 = (1.0f - ci * ci) / (eta * eta);
    if (s2 >= 1.0f) return 1.0f;
    float ct = sqrtf(1.0f - s2);
    float rs = (ci - eta * ct) / (ci + eta * ct);
    float rp = (eta * ci - ct) / (eta * ci + ct);
    return 0.5f * (rs * rs + rp * rp);
}

// Sample a continuation direction in the local frame; false = rejected.
// EXT as for eval_opaque.
template <bool EXT = true>
PT_DEV bool sample_local(int type, float rough, float ior, float tex, bool entering, f3 alb, f3 wo, float u4,
                         float u5, float u6, f3& wi, f3& weight, float& pdf, Lobe& lb) {
    lb.type = type;
    lb.m5 = 0.0f;
    lb.k = 0.0f;
    if (type == PT_LAMBERT) {
        wi = cosine_dir(u5, u6);
        weight = mk3(alb.x * tex, alb.y * tex, alb.z * tex);
        pdf = wi.z * kInvPi;
        lb.k = tex;
        return true;
    }
    if (wo.z <= 0.0f) return false;
    float alpha = ggx_alpha(rough), a2 = alpha * alpha;
    if (EXT && type == PT_COATED) {
        // the coat's visible normals with probability F(cos_o), else the
        // base's cosine lobe; weight f cos_i / (mixture pdf)
        const float Fo = fresnel_dielectric(wo.z, ior);
        f3 w;
        if (u4 < Fo) {
            const f3 m = ggx_vndf(wo, alpha, u5, u6);
            const float com = dot3(wo, m);
            w = mk3((2.0f * com) * m.x - wo.x, (2.0f * com) * m.y - wo.y, (2.0f * com) * m.z - wo.z);
        } else {
            w = cosine_dir(u5, u6);
        }
        if (w.z <= 0.0f) return false;
        f3 f;
        float p;
        eval_coat(rough, ior, tex, alb, wo, w, f, p, lb);
        if (!(p > 0.0f)) return false;
        const float sc = w.z / p;
        lb.k = lb.k * sc;
        lb.m5 = lb.m5 * sc;
        wi = w;
        weight = mk3(alb.x * lb.k + lb.m5, alb.y * lb.k + lb.m5, alb.z * lb.k + lb.m5);
        pdf = p;
        return true;
    }
    f3 m = ggx_vndf(wo, alpha, u5, u6);
    float com = dot3(wo, m);
    float lo = ggx_lambda(wo, a2);
    float G1 = 1.0f / (1.0f + lo);
    if (type == PT_CONDUCTOR) {
        f3 w = mk3((2.0f * com) * m.x - wo.x, (2.0f * com) * m.y - wo.y, (2.0f * com) * m.z - wo.z);
        if (w.z <= 0.0f) return false;
        float li = ggx_lambda(w, a2);
        float G2 = 1.0f / ((1.0f + lo) + li);
        float g = G2 / G1;
        float m5 = pow5(1.0f - com);
        wi = w;
        weight = mk3((alb.x + (1.0f - alb.x) * m5) * g, (alb.y + (1.0f - alb.y) * m5) * g,
                     (alb.z + (1.0f - alb.z) * m5) * g);
        pdf = (G1 * ggx_D(m, a2)) / (4.0f * wo.z);
        lb.m5 = m5;
        lb.k = g;
        return true;
    }
    // rough dielectric (Walter et al., EGSR 2007)
    float eta = entering ? ior : 1.0f / ior;
    float F = fresnel_dielectric(com, eta);
    f3 w;
    float scale;
    if (u4 < F) {
        w = mk3((2.0f * com) * m.x - wo.x, (2.0f * com) * m.y - wo.y, (2.0f * com) * m.z - wo.z);
        if (w.z <= 0.0f) return false;
        scale = 1.0f;
    } else {
        float s2 = (1.0f - com * com) / (eta * eta);
        float ct = sqrtf(1.0f - s2);
        float a = com / eta - ct;
        w = mk3(-wo.x / eta + a * m.x, -wo.y / eta + a * m.y, -wo.z / eta + a * m.z);
        if (w.z >= 0.0f) return false;
        scale = 1.0f / (eta * eta);
    }
    float li = ggx_lambda(w, a2);
    float G2 = 1.0f / ((1.0f + lo) + li);
    float g = (G2 / G1) * scale;
    wi = w;
    weight = mk3(g, g, g);
    pdf = 0.0f;
    lb.k = g;
    return true;
}

// ---------------------------------------------------------------------------
// one path vertex (shared by the megakernel, the wavefront and the adjoint)
// ---------------------------------------------------------------------------
struct PathState {
    f3 beta;
    f3 L;
    float p_prev;
    int prev_smooth;
};

struct ShadowReq {
    bool valid;
    f3 o, d;     // segment origin and unnormalised direction to the light
    f3 C;        // f Le_y G: contribution per unit throughput if visible
    f3 contrib;  // beta * C with the throughput arriving at the vertex
    uint32_t light_id;  // input id of the light triangle
    uint32_t light_idx; // its index in the light table
    float G;
    Lobe lobe;   // f = lobe(albedo)
};

struct VertexOut {
    bool cont;          // the path continues
    f3 o, d;            // continuation ray
    uint32_t id;        // input id of the hit triangle (~0u on a miss)
    uint32_t hot;       // its slot among the largest triangles + 1 (0 = not one of them)
    bool emitted;       // emission term counted at this vertex
    float w_emit;       // its MIS weight
    Lobe scat;          // sampling weight = lobe(albedo) when cont
    bool addL;          // radiance to add at this vertex (emission or sky) ...
    f3 Ladd;            // ... this much: L becomes L + Ladd (see add_radiance)
};

// apply a vertex's emission / sky term to the path radiance
PT_DEV void add_radiance(PathState& ps, const VertexOut& vo) {
    if (vo.addL) ps.L = mk3(ps.L.x + vo.Ladd.x, ps.L.y + vo.Ladd.y, ps.L.z + vo.Ladd.z);
}

// Light table staged in LDS by a kernel (CDF words, leaf-order triangle and
// input indices of the n lights); n = 0: read the table from global memory.
#if defined(__HIP_DEVICE_COMPILE__)
typedef __attribute__((address_space(3))) uint32_t lds_u32;
#else
typedef uint32_t lds_u32;
#endif
constexpr int kLdsLights = 1024;

struct LightCache {
    const lds_u32* cdf;
    const lds_u32* tri;
    const lds_u32* id;
    int n;
};

PT_DEV LightCache no_light_cache() {
    LightCache lc;
    lc.cdf = lc.tri = lc.id = nullptr;
    lc.n = 0;
    return lc;
}

// first light whose CDF word is >= w (the last word is 2^32 - 1)
PT_DEV uint32_t pick_light(const SceneView& sc, const LightCache& lc, uint32_t w) {
    int lo = 0, hi = sc.nl - 1;
    if (lc.n) {
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (w <= lc.cdf[mid]) hi = mid;
            else lo = mid + 1;
        }
    } else {
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (w <= sc.lights[mid].cdf) hi = mid;
            else lo = mid + 1;
        }
    }
    return (uint32_t)lo;
}

PT_DEV f3 load3(const float* __restrict__ p, uint32_t i) {
    return mk3(p[3 * (size_t)i], p[3 * (size_t)i + 1], p[3 * (size_t)i + 2]);
}

// Shade vertex k of a path: add emission (MIS-weighted after a light-sampled
// vertex), build the light-sample request, sample the continuation and
// apply roulette.  The emission (or sky) term is returned in out.Ladd for
// the caller to add to the path radiance (add_radiance), so that the
// radiance is needed only where it is updated; the light-sample
// contribution beta * C is added by the caller once the segment is found
// unoccluded (megakernel: at once; wavefront: in the shadow stage).
//
// Memory access order is arranged for latency: the hit triangle, the
// random numbers, the light choice and the light triangle and emission do
// not depend on each other, so all their loads are issued before any of
// them is waited for; only the per-triangle albedo, emission and material
// wait for the hit triangle.  Values fetched this way are used under the
// same conditions as before, so the arithmetic is unchanged.
//
// INST (two-level scene): the hit triangle's vertices are mapped to world
// space by its instance record's object-to-world rows, and so are the
// sampled light's (its instance record is the light table's last word).
// ATTR: the scene may have vertex attributes (shading normals, texture
// coordinates) or coated materials; without it that code is compiled out,
// so scenes without them keep the smaller register budget.
template <bool INST = false, bool ATTR = false>
PT_DEV VertexOut shade_vertex(const SceneView& sc, const PathParams& pp, uint32_t pixel, uint32_t sample, int k,
                              f3 rd, const Hit& h, PathState& ps, ShadowReq& sh,
                              const LightCache& lc = no_light_cache()) {
    VertexOut out;
    out.cont = false;
    out.id = 0xFFFFFFFFu;
    out.hot = 0u;
    out.emitted = false;
    out.w_emit = 0.0f;
    out.addL = false;
    sh.valid = false;
    if (h.tri >= (uint32_t)sc.nt) {
        out.addL = true;
        out.Ladd = mk3(ps.beta.x * sc.sky0, ps.beta.y * sc.sky1, ps.beta.z * sc.sky2);
        return out;
    }
    const float4* tp = sc.tris + (size_t)h.tri * 3;
    float4 ta = tp[0], tb = tp[1], tc = tp[2];
    if constexpr (INST) inst_vertices(sc, h.inst, ta, tb, tc);
    const bool more = k != pp.D + 1;
    Rng8 rn;
    float4 la, lb4, lc4;
    f3 Le_l;
    const bool nee = more && pp.nee && sc.nl > 0;
    if (more) rn = philox8(pp.seed, pixel, sample, (uint32_t)k, pp.job);
    uint32_t lj = 0;
    if (nee) {
        const uint32_t j = pick_light(sc, lc, rn.w[0]);
        lj = j;
        const uint32_t lt = lc.n ? lc.tri[j] : sc.lights[j].tri;
        const uint32_t lid = lc.n ? lc.id[j] : sc.lights[j].id;
        const float4* lp = sc.tris + (size_t)lt * 3;
        la = lp[0];
        lb4 = lp[1];
        lc4 = lp[2];
        Le_l = load3(sc.emission, lid);
        if constexpr (INST) inst_vertices(sc, sc.lights[j].pad, la, lb4, lc4);
    }
    f3 v0 = xyz(ta), v1 = xyz(tb), v2 = xyz(tc);
    uint32_t id = f2u(ta.w);
    uint32_t minfo = f2u(tb.w);
    const f3 Le = load3(sc.emission, id);
    const f3 alb = load3(sc.albedo, id);
    const float4 mat = sc.mats[minfo & ~kLightFlag];
    out.id = id;
    out.hot = f2u(tc.w);
    f3 e1 = sub3(v1, v0), e2 = sub3(v2, v0);
    f3 x = mk3((v0.x + h.b1 * e1.x) + h.b2 * e2.x, (v0.y + h.b1 * e1.y) + h.b2 * e2.y,
               (v0.z + h.b1 * e1.z) + h.b2 * e2.z);
    f3 ng = tri_normal(v0, v1, v2);
    f3 wo = neg3(rd);
    float cos_e = dot3(ng, wo);
    if (cos_e > 0.0f) {
        float w = 1.0f;
        if (k > 1 && pp.nee && ps.prev_smooth && (minfo & kLightFlag) && sc.nl > 0) {
            float pl = (h.t * h.t) / (sc.area_total * cos_e);
            w = (ps.p_prev * ps.p_prev) / (ps.p_prev * ps.p_prev + pl * pl);
        }
        out.addL = true;
        out.Ladd = mk3(ps.beta.x * (w * Le.x), ps.beta.y * (w * Le.y), ps.beta.z * (w * Le.z));
        out.emitted = true;
        out.w_emit = w;
    }
    if (!more) return out;
    int type = (int)mat.x;
    float rough = mat.y, ior = mat.z;
    // vertex attributes: the shading normal (the BSDF frame) and the
    // checker factor of the albedo
    const bool nrm = ATTR && (sc.attr_flags & kAttrNormals) != 0;
    float tex = 1.0f;
    if (ATTR && (sc.attr_flags & kAttrUV) && (type == PT_LAMBERT || type == PT_COATED) && mat.w > 0.0f)
        tex = checker(sc, h, mat.w);
    const f3 ns = nrm ? shading_normal<INST>(sc, h, ng) : ng;
    bool entering = true;
    f3 n, ngf;
    if (type == PT_DIELECTRIC) {
        entering = cos_e > 0.0f;
        n = entering ? ns : neg3(ns);
        ngf = entering ? ng : neg3(ng);
    } else {
        n = cos_e > 0.0f ? ns : neg3(ns);
        ngf = cos_e > 0.0f ? ng : neg3(ng);
    }
    Frame fr = make_frame(n);
    f3 wo_l = to_local(fr, wo);
    // with shading normals: nothing scatters from below the shading
    // horizon, and directions on the wrong geometric side for their lobe
    // are dropped (no light leaks through the surface)
    if (nrm && wo_l.z <= 0.0f) return out;
    if (nee && type != PT_DIELECTRIC) {
        f3 y = tri_point(xyz(la), xyz(lb4), xyz(lc4), unif(rn.w[1]), unif(rn.w[2]));
        f3 ny = tri_normal(xyz(la), xyz(lb4), xyz(lc4));
        f3 dv = sub3(y, x);
        float d2 = dot3(dv, dv);
        if (d2 > 0.0f) {
            f3 wl = scl3(dv, 1.0f / sqrtf(d2));
            float cos_y = -dot3(ny, wl);
            float cos_x = dot3(n, wl);
            if (cos_y > 0.0f && cos_x > 0.0f && (!nrm || dot3(ngf, wl) > 0.0f)) {
                f3 f;
                float pb;
                Lobe lob;
                eval_opaque<ATTR>(type, rough, ior, tex, alb, wo_l, to_local(fr, wl), f, pb, lob);
                float pl = d2 / (sc.area_total * cos_y);
                if (lob.k > 0.0f && pl > 0.0f) {
                    float wmis = (pl * pl) / (pl * pl + pb * pb);
                    float G = (cos_x * wmis) / pl;
                    uint32_t lid = f2u(la.w);
                    sh.C = mk3((f.x * Le_l.x) * G, (f.y * Le_l.y) * G, (f.z * Le_l.z) * G);
                    sh.contrib = mk3(ps.beta.x * sh.C.x, ps.beta.y * sh.C.y, ps.beta.z * sh.C.z);
                    sh.o = offset_point(x, dot3(ng, wl) > 0.0f ? ng : neg3(ng), tri_extent(v0, v1, v2));
                    f3 sy = offset_point(y, ny, tri_extent(xyz(la), xyz(lb4), xyz(lc4)));
                    sh.d = sub3(sy, sh.o);
                    sh.valid = true;
                    sh.light_id = lid;
                    sh.light_idx = lj;
                    sh.G = G;
                    sh.lobe = lob;
                }
            }
        }
    }
    f3 wi_l, W;
    float pb;
    Lobe lb;
    bool ok = sample_local<ATTR>(type, rough, ior, tex, entering, alb, wo_l, unif(rn.w[4]), unif(rn.w[5]), unif(rn.w[6]),
                           wi_l, W, pb, lb);
    if (!ok) return out;
    if (W.x == 0.0f && W.y == 0.0f && W.z == 0.0f) return out;
    if (type != PT_DIELECTRIC && !(pb > 0.0f)) return out;
    f3 wi = to_world(fr, wi_l);
    if (nrm) {
        const float cg = dot3(ngf, wi);
        if (wi_l.z > 0.0f ? !(cg > 0.0f) : !(cg < 0.0f)) return out;
    }
    ps.beta = mk3(ps.beta.x * W.x, ps.beta.y * W.y, ps.beta.z * W.z);
    if (pp.rr_start >= 0 && k >= pp.rr_start) {
        float q = max3c(ps.beta);
        q = q < 1.0f ? q : 1.0f;
        float u7 = unif(rn.w[7]);
        if (u7 >= q) return out;
        ps.beta = mk3(ps.beta.x / q, ps.beta.y / q, ps.beta.z / q);
    }
    f3 no = dot3(ng, wi) > 0.0f ? ng : neg3(ng);
    out.o = offset_point(x, no, tri_extent(v0, v1, v2));
    out.d = wi;
    out.cont = true;
    out.scat = lb;
    ps.p_prev = pb;
    ps.prev_smooth = type != PT_DIELECTRIC;
    return out;
}

// A camera path traced vertex by vertex (megakernel): path_begin generates
// the camera ray, path_vertex extends it to the next vertex, shades it and
// traces the light-sample segment at once; it returns false when the path
// has ended (its radiance is then in pr.ps.L).  Extension and shadow rays
// are counted in n_ext / n_sh.
struct PathRun {
    f3 o, d;
    PathState ps;
    int k;
};

PT_DEV void path_begin(const CamView& cam, const PathParams& pp, uint32_t pix, uint32_t sample, PathRun& pr) {
    camera_sample(cam, pp, pix, sample, pr.o, pr.d);
    pr.ps.beta = mk3(1.f, 1.f, 1.f);
    pr.ps.L = mk3(0.f, 0.f, 0.f);
    pr.ps.p_prev = 0.f;
    pr.ps.prev_smooth = 0;
    pr.k = 1;
}

template <int LDS, bool COUNT = false, bool INST = false, bool ATTR = false>
PT_DEV bool path_vertex(const SceneView& sc, const PathParams& pp, uint32_t pix, uint32_t sample, PathRun& pr,
                        TravStack<LDS, COUNT>& st, uint32_t& n_ext, uint32_t& n_sh,
                        const LightCache& lc = no_light_cache()) {
    Hit h = closest_hit_t<LDS, COUNT, INST>(sc, pr.o, pr.d, INFINITY, st);
    ++n_ext;
    ShadowReq sh;
    VertexOut vo = shade_vertex<INST, ATTR>(sc, pp, pix, sample, pr.k, pr.d, h, pr.ps, sh, lc);
    add_radiance(pr.ps, vo);
    if (sh.valid) {
        ++n_sh;
        if (!any_hit_t<LDS, COUNT, INST>(sc, sh.o, sh.d, kShadowTmax, st))
            pr.ps.L = mk3(pr.ps.L.x + sh.contrib.x, pr.ps.L.y + sh.contrib.y, pr.ps.L.z + sh.contrib.z);
    }
    if (!vo.cont) return false;
    pr.o = vo.o;
    pr.d = vo.d;
    ++pr.k;
    return true;
}

// One complete camera path: its radiance.
template <int LDS, bool COUNT = false, bool INST = false, bool ATTR = false>
PT_DEV f3 trace_path(const SceneView& sc, const CamView& cam, const PathParams& pp, uint32_t pix, uint32_t sample,
                     TravStack<LDS, COUNT>& st, uint32_t& n_ext, uint32_t& n_sh, const LightCache& lc = no_light_cache()) {
    PathRun pr;
    path_begin(cam, pp, pix, sample, pr);
    while (path_vertex<LDS, COUNT, INST, ATTR>(sc, pp, pix, sample, pr, st, n_ext, n_sh, lc)) {
    }
    return pr.ps.L;
}

}  // namespace ptmi
