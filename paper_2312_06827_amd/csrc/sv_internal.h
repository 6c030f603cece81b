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
