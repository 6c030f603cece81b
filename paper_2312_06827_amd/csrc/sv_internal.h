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

// Plane element `idx` addressed by a 32-bit byte offset from the plane's
// base (an SGPR pair): loads and stores then need no 64-bit address
// arithmetic.  The host limits pitch * h to 2^29 elements, so every byte
// offset fits in 32 bits.
template <typename T>
__device__ __forceinline__ float ldo(const void *base, uint32_t idx) {
    return ld((const T *)((const char *)base + idx * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void sto(void *base, uint32_t idx, float v) {
    st((T *)((char *)base + idx * (uint32_t)sizeof(T)), v);
}
__device__ __forceinline__ float ldf(const float *base, uint32_t idx) {
    return *(const float *)((const char *)base + idx * 4u);
}
__device__ __forceinline__ void stf(float *base, uint32_t idx, float v) {
    *(float *)((char *)base + idx * 4u) = v;
}

// An element offset shared by loads or stores of several planes, made
// opaque to the optimiser: an empty asm statement (no instruction) that
// pins it as a 32-bit value in a VGPR.  Each access is then addressed as
// plane base (SGPRs) + this offset, which the memory instruction adds by
// itself; left visible, the compiler tends to widen the offset once and
// form a 64-bit address per plane with a VALU add.
__device__ __forceinline__ uint32_t vofs(uint32_t o) {
    asm volatile("" : "+v"(o));
    return o;
}

// ---- shared arithmetic ----------------------------------------------------

// Rec. 709 luminance, fixed evaluation order, written as
// g + 0.2126 (r - g) + 0.0722 (b - g) (the weights sum to one): exact for
// grey colours, so the luminance difference of two grey pixels is their
// exact difference.  The luminance edge weight divides that difference by
// sigma_l sqrt(g) + eps_l, which is tiny where the variance vanishes (e.g.
// a binary visibility signal away from its edges); with the plain form the
// rounding of each pixel's luminance (an ulp of L) then moves weights by
// percents.
__device__ __forceinline__ float luma(float r, float g, float b) {
    // no contraction of the differences into a producer's product: every
    // caller gets the same bits for the same colour
    return fmaf(0.0722f, __fsub_rn(b, g), fmaf(0.2126f, __fsub_rn(r, g), g));
}

// n / d from inv ~ 1 / d (rounded, or the hardware reciprocal within an
// ulp) with one correction step: the residual n - q d is exact in an fma,
// so the quotient is correctly rounded but in rare hard cases, and n == d
// gives exactly 1, n == 0 gives 0.  Weighted means thus
// keep a flat region exactly flat, which the luminance edge weight needs:
// where the variance vanishes it is a near step function of the luminance
// difference (scale eps_l), and a flat value off by an ulp would cut its
// neighbours off.
__device__ __forceinline__ float quot(float n, float d, float inv) {
    const float q = n * inv;
    return fmaf(fmaf(-q, d, n), inv, q);
}

// No surface: depth not > 0 or not finite.
__device__ __forceinline__ bool empty_px(float z) { return !(z > 0.0f) || !(z < INFINITY); }

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;  // 1 / log2(e)

// ---- normal edge weight ----------------------------------------------------
//
// The weight is max(0, cos)^sigma_n with the cosine of two unit normals
// taken as u = 1 - s2/2, s2 = |n(p) - n(q)|^2 (accurate where the normals
// are close, unlike 1 - rounded dot products).  Its base-2 logarithm
// sigma_n log2(u) is added to a tap's exponent.  u is rounded once; sigma_n
// (128) would amplify that rounding into the weight, so the exact residual
// r = (1 - s2/2) - u is added as sigma_n log2(e) r (the first-order term of
// log(u + r) - log(u) near u = 1, where every weight that matters lies).
// sigma_n == 0 (normal weight off) uses the same code with u floored at 1:
// both terms are then exactly 0.
struct NormalCoef {
    float sn;    // sigma_n
    float snl;   // sigma_n log2(e)
    float umin;  // 0, or 1 when sigma_n == 0
    int series;  // sigma_n >= kSeriesMinSigmaN: the a-trous levels use the series form
};

__device__ __forceinline__ float add_normal_term(float e, float s2, const NormalCoef &k) {
    const float u = fmaf(-0.5f, s2, 1.0f);
    const float r = fmaf(-0.5f, s2, 1.0f - u);  // (1 - s2/2) - u, exact for u >= 1/2
    e = fmaf(k.sn, __builtin_amdgcn_logf(fmaxf(u, k.umin)), e);
    return fmaf(k.snl, r, e);
}

// From this sigma_n on, the a-trous levels take the normal term as a
// truncated series (add_normal_series), with no logarithm.
constexpr float kSeriesMinSigmaN = 96.0f;

inline NormalCoef make_normal_coef(float sigma_n) {
    return NormalCoef{sigma_n, sigma_n * 1.4426950408889634f, sigma_n == 0.0f ? 1.0f : 0.0f,
                      sigma_n >= kSeriesMinSigmaN ? 1 : 0};
}

// The same term for large sigma_n without the logarithm.  With x = s2/2,
// log2(1 - x) = -log2(e) (x + x^2/2 + ... + x^6/6 + R), taken through x^6/6
// and evaluated by Horner in s2 (x^k/k = s2^k / (k 2^k)):
//   sigma_n log2(1 - s2/2) ~ sigma_n s2 P(s2),  P(s2) = -log2(e) sum_k s2^(k-1) / (k 2^k).
// The remainder R <= x^7 / (7 (1 - x)) is dropped; sigma_n R is the relative
// error it leaves in the weight.  At sigma_n = 128 that stays below the
// binary32 evaluation's own error (about 1e-6 relative) for every weight
// above 1e-3 of the centre's and below 4e-6 for weights above 1e-6 (at 96:
// 1.4e-6 and 1.5e-5), comparable to the log form's 5e-7 and 1.1e-6.  Where
// x is large the series gives an exponentially small weight, as the exact
// one is (or zero: for x >= 1 the exact weight is 0 and the series' exp2
// underflows), so no clamp is needed; and no 1 - s2/2 is rounded, so no
// residual term either.
__device__ __forceinline__ float add_normal_series(float e, float s2, const NormalCoef &k) {
    constexpr float L = 1.4426950408889634f;
    float p = fmaf(s2, -L / 384.0f, -L / 160.0f);  // 1/(6 2^6), 1/(5 2^5)
    p = fmaf(p, s2, -L / 64.0f);
    p = fmaf(p, s2, -L / 24.0f);
    p = fmaf(p, s2, -L / 8.0f);
    p = fmaf(p, s2, -L / 2.0f);
    return fmaf(p * s2, k.sn, e);
}

// The depth difference p's gradient (gx, gy) predicts over an offset
// (a, b) of integers (held as floats): gx a + gy b, rounded about once.
// The rounding error of gy b is recovered with an fma and added back, so
// an offset nearly orthogonal to the gradient, where the two terms almost
// cancel, keeps its significant bits (the depth weight divides by this
// difference).  Where both products are exact (offsets of 1 or 2 times a
// power of two) it is the single rounding of one fma.
__device__ __forceinline__ float grad_offset(float gx, float gy, float a, float b) {
    const float p = gy * b;
    return fmaf(gx, a, p) + fmaf(gy, b, -p);
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

// ---- XCD-aware tile order ----------------------------------------------------
//
// The 256 CUs sit in 8 XCDs, each with its own L2, and workgroups are handed
// to the XCDs round-robin by workgroup index.  Tile kernels launch a 1-D
// grid of 8 * ceil(tiles / 8) workgroups and map workgroup b to tile
// (b % 8) * ceil(tiles / 8) + b / 8: every XCD then sweeps one contiguous
// range of tiles in order, so the halos that neighbouring tiles share are
// re-read from its own L2.  Returns -1 for the padding workgroups (which
// must return before any barrier).
constexpr int kXCD = 8;

__device__ __forceinline__ int xcd_tile(int tiles) {
    const int per = (tiles + kXCD - 1) / kXCD;
    const int b = (int)blockIdx.x;
    const int t = (b % kXCD) * per + b / kXCD;
    return t < tiles ? t : -1;
}

inline unsigned xcd_grid(int tiles) { return (unsigned)(((tiles + kXCD - 1) / kXCD) * kXCD); }

// ---- short-history list of the variance estimate ---------------------------
//
// Pixels whose history is too short for the temporal variance are listed
// for a spatial estimate.  Workspace: eight 128-byte lines of counters,
// then eight sublists; the 64x4-pixel tile t appends to sublist t % 8, so a
// sublist holds at most ceil(tiles / 8) tiles' pixels (its capacity `cap`)
// whichever workgroup runs the tile.  Entries are (y << 15) | x.
//
// The counters are never reset.  Line k holds three words of sublist k:
//   kCount  the number of appends so far (atomic, wraps modulo 2^32);
//   kNext   its value when the last reading pass ran: an appending pass
//           stores entry i of its own appends at slot i = count - next;
//   kBase   the same value, copied by the appending pass's tile 0 for the
//           reading pass, which lists the count - base entries and then
//           sets next = count.
// Each word is written by one kind of pass and read only by the other, and
// passes are ordered on one stream, so no pass reads a word that another
// workgroup of the same launch writes.  A zeroed workspace is consistent.
constexpr int kVX = 64, kVY = 4;
constexpr int kLines = 32;
constexpr int kCount = 0, kBase = 1, kNext = 2;

struct VarWork {
    uint32_t count[kXCD * kLines];  // count[k * kLines + kCount | kBase | kNext]
    uint32_t list[1];               // sublist k at list + k * cap
};

inline uint32_t point_grid(sv_dims d) {
    return xcd_grid(((d.w + kVX - 1) / kVX) * ((d.h + kVY - 1) / kVY));
}

// Appends this thread's pixel (x, y) if `spatial`: one atomic per
// workgroup.  Every thread of the 256-thread workgroup must call it (it
// holds two barriers); tile is this workgroup's 64x4 tile index.
__device__ __forceinline__ void list_short_pixel(VarWork *work, uint32_t cap, int tile,
                                                 bool spatial, int x, int y, uint32_t *wave_n,
                                                 uint32_t &base_sh) {
    const uint64_t mask = __ballot(spatial);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wave_n[wave] = (uint32_t)__popcll(mask);
    // tile 0 (every launch has it) hands each sublist's start to the
    // reading pass, also for sublists that no tile of this launch reaches
    if (tile == 0 && threadIdx.x < kXCD)
        work->count[threadIdx.x * kLines + kBase] = work->count[threadIdx.x * kLines + kNext];
    __syncthreads();
    const uint32_t n0 = wave_n[0], n1 = wave_n[1], n2 = wave_n[2], n3 = wave_n[3];
    const uint32_t total = n0 + n1 + n2 + n3;
    if (total == 0) return;  // uniform over the workgroup
    const uint32_t k = (uint32_t)tile % kXCD;
    if (threadIdx.x == 0)
        base_sh = atomicAdd(&work->count[k * kLines + kCount], total) -
                  work->count[k * kLines + kNext];
    __syncthreads();
    const uint32_t before = (wave > 0 ? n0 : 0u) + (wave > 1 ? n1 : 0u) + (wave > 2 ? n2 : 0u);
    const uint32_t slot = base_sh + before + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    // a workspace that was not zeroed cannot push a store past the sublist
    if (spatial && slot < cap) work->list[k * cap + slot] = ((uint32_t)y << 15) | (uint32_t)x;
}

// ---- batched passes (many independent streams, one launch per pass) ----------
//
// A batched pass runs the tiles of n streams as one global list: stream s
// owns tiles prefix[s] .. prefix[s+1]-1 and its own argument struct.  One
// workgroup per tile, mapped as in xcd_tile, so each XCD sweeps one
// contiguous eighth of the list in order (a stream's tiles stay on one or
// two XCDs and neighbouring tiles share that XCD's L2), exactly as the
// single-stream launches do.  Every tile is computed by the same device
// code as the single-stream kernel, so each stream's result is bitwise the
// same.

// Stream that owns global tile t (prefix has n + 1 entries; n is small and
// the loop is uniform across the workgroup).
__device__ __forceinline__ int batch_stream(const int *prefix, int n, int t) {
    int s = 0;
    while (s + 1 < n && prefix[s + 1] <= t) ++s;
    return s;
}

// This workgroup's tile within its stream s, or -1 for a padding workgroup.
__device__ __forceinline__ int batch_tile(const int *prefix, int n, int total, int &s) {
    const int t = xcd_tile(total);
    if (t < 0) return -1;
    s = batch_stream(prefix, n, t);
    return t - prefix[s];
}

// Launcher of one batched pass: `args` holds n argument structs (device),
// `prefix` n + 1 tile offsets (device), total = prefix[n].
typedef void (*BatchLaunch)(const void *args, const int *prefix, int n, int total,
                            hipStream_t s);

// While a recorder is installed on the calling thread, the pass launchers
// append (launcher, argument struct, tile count) here instead of
// launching: the batch plan records each stream's frame this way and
// replays the passes batched.
struct PassRecord {
    BatchLaunch fn;
    size_t arg_size;
    int tiles;
    unsigned char args[512];
};

struct Recorder {
    PassRecord *passes;
    int cap, count;
    bool overflow;
};

inline Recorder *&recorder() {
    static thread_local Recorder *r = nullptr;
    return r;
}

template <class A>
inline bool record_pass(BatchLaunch fn, const A &a, int tiles) {
    static_assert(sizeof(A) <= sizeof(PassRecord::args), "argument struct too large");
    Recorder *r = recorder();
    if (!r) return false;
    if (r->count >= r->cap) {
        r->overflow = true;
        return true;
    }
    PassRecord &p = r->passes[r->count++];
    p.fn = fn;
    p.arg_size = sizeof(A);
    p.tiles = tiles;
    const unsigned char *src = (const unsigned char *)&a;
    for (size_t i = 0; i < sizeof(A); ++i) p.args[i] = src[i];
    return true;
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
    if ((int64_t)d.pitch * d.h > ((int64_t)1 << 29)) return -1;
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
