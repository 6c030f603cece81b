// Internal helpers of the HIP library: storage-type loads and stores,
// luminance, the empty-pixel test, argument checks and launch plumbing.
// Device code targets gfx950 (CDNA4, 64-lane wavefronts).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sv.h"

namespace sv {

// ---- storage types ------------------------------------------------------

typedef _Float16 half_t;

template <typename T> __device__ __forceinline__ float ld(const T *p);
template <> __device__ __forceinline__ float ld<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float ld<half_t>(const half_t *p) { return (float)*p; }

// Round-to-nearest-even conversion to the storage type.
template <typename T> __device__ __forceinline__ void st(T *p, float v);
template <> __device__ __forceinline__ void st<float>(float *p, float v) { *p = v; }
template <> __device__ __forceinline__ void st<half_t>(half_t *p, float v) { *p = (half_t)v; }

// ---- shared arithmetic ----------------------------------------------------

// Rec. 709 luminance, fixed evaluation order.
__device__ __forceinline__ float luma(float r, float g, float b) {
    return fmaf(0.0722f, b, fmaf(0.7152f, g, 0.2126f * r));
}

// No surface: depth not > 0 or not finite.
__device__ __forceinline__ bool empty_px(float z) { return !(z > 0.0f) || !(z < INFINITY); }

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

constexpr float kLog2e = 1.4426950408889634f;

// ---- normal edge weight ----------------------------------------------------
//
// The weight is max(0, cos)^sigma_n with the cosine of two unit normals
// taken as 1 - s2/2, s2 = |n(p) - n(q)|^2.  Its base-2 logarithm
// sigma_n log2(1 - s2/2) is added to a tap's exponent.  For sigma_n >= 64
// the logarithm is its series -(t + t^2/2 + t^3/3 + t^4/4), t = s2/2: the
// weights that matter have t small, where the first omitted term
// sigma_n t^5/5 times the weight exp(-sigma_n t) stays below
// e^-5 5^4 / sigma_n^4 (2.5e-7 at sigma_n = 64, 1.6e-8 at 128), and it
// avoids rounding 1 - s2/2 near 1, which sigma_n would amplify.  Below 64 the
// logarithm of the rounded u = 1 - s2/2 is corrected by the rounding error
// of u.
enum { kNormalOff = 0, kNormalPoly = 1, kNormalLog = 2 };

struct NormalCoef {
    float c1, c2, c3, c4;  // sigma_n log2(e) times the series coefficients in s2
    float sn;              // sigma_n
    float snl;             // sigma_n log2(e)
};

inline NormalCoef make_normal_coef(float sigma_n) {
    const float k = sigma_n * 1.4426950408889634f;
    // -(t + t^2/2 + t^3/3 + t^4/4) with t = s2/2
    return NormalCoef{-k / 2.0f, -k / 8.0f, -k / 24.0f, -k / 64.0f, sigma_n, k};
}

inline int normal_mode(float sigma_n) {
    return sigma_n == 0.0f ? kNormalOff : (sigma_n >= 64.0f ? kNormalPoly : kNormalLog);
}

template <int NM>
__device__ __forceinline__ float add_normal_term(float e, float s2, const NormalCoef &k) {
    if (NM == kNormalPoly) {
        float p = fmaf(s2, k.c4, k.c3);
        p = fmaf(s2, p, k.c2);
        p = fmaf(s2, p, k.c1);
        return fmaf(s2, p, e);
    } else if (NM == kNormalLog) {
        const float u = fmaf(-0.5f, s2, 1.0f);
        const float r = fmaf(-0.5f, s2, 1.0f - u);  // (1 - s2/2) - u, exact
        e = fmaf(k.sn, __builtin_amdgcn_logf(fmaxf(u, 0.0f)), e);
        return fmaf(k.snl, r, e);
    }
    return e;
}

__device__ __forceinline__ float chord2(float ax, float ay, float az, float bx, float by,
                                        float bz) {
    const float dx = ax - bx, dy = ay - by, dz = az - bz;
    return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

// Exact inverse of the LUMA tone map, denominator floored at 2^-20.
__device__ __forceinline__ void inv_tonemap(float &r, float &g, float &b, float k) {
    float L = luma(r, g, b);
    float den = fmaxf(1.0f - k * L, 0x1p-20f);
    r = r / den;
    g = g / den;
    b = b / den;
}

// ---- host-side checks -----------------------------------------------------

constexpr int32_t kMaxDim = 32768;

inline size_t elem_size(sv_dtype t) { return t == SV_F16 ? 2 : 4; }

inline bool valid_dtype(sv_dtype t) { return t == SV_F32 || t == SV_F16; }

// 0: fine and non-empty; 1: valid empty call; -1: invalid.
inline int check_dims(sv_dims d) {
    if (d.w < 0 || d.h < 0 || d.w > kMaxDim || d.h > kMaxDim) return -1;
    if (d.w == 0 || d.h == 0) return 1;
    if (d.pitch < d.w) return -1;
    if ((int64_t)d.pitch * d.h >= ((int64_t)1 << 31)) return -1;
    return 0;
}

struct span {
    uintptr_t lo, hi;  // [lo, hi)
};

inline span plane_span(const void *p, sv_dims d, size_t esz) {
    uintptr_t a = (uintptr_t)p;
    size_t bytes = ((size_t)(d.h - 1) * (size_t)d.pitch + (size_t)d.w) * esz;
    return span{a, a + bytes};
}

inline bool overlaps(span a, span b) { return a.lo < b.hi && b.lo < a.hi; }

// Records the error of the last launch on this thread.
int hip_status(hipError_t e);

inline hipStream_t as_stream(sv_stream s) { return (hipStream_t)s; }

}  // namespace sv
