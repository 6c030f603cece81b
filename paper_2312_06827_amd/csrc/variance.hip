// Variance estimate (Section 2): the temporal variance of the luminance
// moments where the history is long enough, a depth- and normal-weighted
// spatial estimate where it is not.  The second moment arrives as the
// central moment m2c = E[L^2] - E[L]^2, so neither branch cancels.
//
// Pass 1 (pointwise) writes the temporal estimate and lists the pixels
// whose history is short; pass 2 computes the spatial estimate of the
// listed pixels, eight lanes per pixel, spread over every CU.
#include <mutex>

#include "sv_internal.h"

namespace sv {

constexpr int kSpatialBlocks = 1024;  // pass-2 grid (grid-stride over the list)

struct VarianceArgs {
    const float *m1, *m2c;
    const uint8_t *n;
    const void *z, *dzdx, *dzdy, *nx, *ny, *nz;
    float *var;
    VarWork *work;
    uint32_t cap;  // entries per sublist
    int w, h, pitch;
    float sigma_z, eps_z;
    NormalCoef nc;
    int min_hist;
};

// Tile `tile` (-1: a padding workgroup, which still takes the barriers).
template <typename T>
__device__ __forceinline__ void variance_point_tile(const VarianceArgs &a, int tile,
                                                    uint32_t *wave_n, uint32_t &base_sh) {
    const int gxt = (a.w + kVX - 1) / kVX;
    const int byt = tile / gxt, bxt = tile - byt * gxt;
    const int x = bxt * kVX + (threadIdx.x & 63), y = byt * kVY + (threadIdx.x >> 6);
    const bool inside = tile >= 0 && x < a.w && y < a.h;
    const uint32_t o = vofs(inside ? (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x : 0u);
    // all three loads issued together (the address is in the image)
    const int nn = a.n[o];
    const float zp = ldo<T>(a.z, o), m2 = ldf(a.m2c, o);
    const int n = inside ? nn : 0;
    const bool live = inside && n >= 1 && !empty_px(zp);
    const bool spatial = live && n < a.min_hist;
    if (inside && !spatial) stf(a.var, o, live ? fmaxf(0.f, m2) : 0.f);
    list_short_pixel(a.work, a.cap, tile, spatial, x, y, wave_n, base_sh);
}

template <typename T>
__global__ __launch_bounds__(256) void variance_point_k(VarianceArgs a) {
    __shared__ uint32_t wave_n[4], base_sh;
    const int gxt = (a.w + kVX - 1) / kVX;
    variance_point_tile<T>(a, xcd_tile(gxt * ((a.h + kVY - 1) / kVY)), wave_n, base_sh);
}

template <typename T>
__global__ __launch_bounds__(256) void variance_point_batch_k(const VarianceArgs *args,
                                                              const int *prefix, int n, int total) {
    __shared__ uint32_t wave_n[4], base_sh;
    int s = 0;
    const int lt = batch_tile(prefix, n, total, s);
    if (lt < 0) return;
    const VarianceArgs a = args[s];
    variance_point_tile<T>(a, lt, wave_n, base_sh);
}

// Zero state of a workspace's counters (the allocation-free entry point's
// shared array, which another call may have left in any state).
__global__ __launch_bounds__(64) void variance_reset_k(VarWork *w) {
    if (threadIdx.x < kXCD) {
        w->count[threadIdx.x * kLines + kCount] = 0;
        w->count[threadIdx.x * kLines + kBase] = 0;
        w->count[threadIdx.x * kLines + kNext] = 0;
    }
}

// Sum over the 8 lanes of an aligned lane group (butterfly: a fixed order,
// so the result is the same on every run).
__device__ __forceinline__ float group8_sum(float v) {
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 1, 64);
    return v;
}

// Window of radius R, eight lanes per listed pixel: lane `sub` takes taps
// sub, sub + 8, ...  Every tap's loads are issued before any weight is
// formed, and the weights and m1 stay in registers for the second pass.
template <typename T, int R>
__device__ __forceinline__ void variance_spatial_stream(const VarianceArgs &a) {
    constexpr int D = 2 * R + 1, NT = D * D, PER = (NT + 7) / 8, CTR = R * D + R;
    uint32_t pre[kXCD + 1];
    pre[0] = 0;
#pragma unroll
    for (int k = 0; k < kXCD; ++k)
        pre[k + 1] = pre[k] + min(a.work->count[k * kLines + kCount] -
                                      a.work->count[k * kLines + kBase],
                                  a.cap);
    const uint32_t count = pre[kXCD];
    // the list is consumed: the next appending pass starts after it (no
    // workgroup of this pass reads kNext)
    if (blockIdx.x == 0 && threadIdx.x < kXCD)
        a.work->count[threadIdx.x * kLines + kNext] = a.work->count[threadIdx.x * kLines + kCount];
    const int sub = threadIdx.x & 7;
    const uint32_t groups = gridDim.x * (blockDim.x / 8);
    for (uint32_t e = blockIdx.x * (blockDim.x / 8) + (threadIdx.x >> 3); e < count; e += groups) {
        int k = 0;
#pragma unroll
        for (int j = 1; j < kXCD; ++j) k += e >= pre[j] ? 1 : 0;
        const uint32_t packed = a.work->list[k * a.cap + (e - pre[k])];
        const int x = (int)(packed & 32767u), y = (int)(packed >> 15);
        if (x >= a.w || y >= a.h) continue;  // only a stale entry can be outside
        const uint32_t po = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
        const float zc = ldo<T>(a.z, po), gx = ldo<T>(a.dzdx, po), gy = ldo<T>(a.dzdy, po);
        const float nxp = ldo<T>(a.nx, po), nyp = ldo<T>(a.ny, po), nzp = ldo<T>(a.nz, po);
        float zq[PER], qx_[PER], qy_[PER], qz_[PER], m1q[PER], m2q[PER];
        bool ok[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int t = sub + 8 * j;
            const int dx = t % D - R, dy = t / D - R;
            const int qx = x + dx, qy = y + dy;
            ok[j] = t < NT && qx >= 0 && qx < a.w && qy >= 0 && qy < a.h;
            const uint32_t q = vofs(ok[j] ? (uint32_t)qy * (uint32_t)a.pitch + (uint32_t)qx : po);
            zq[j] = ldo<T>(a.z, q);
            qx_[j] = ldo<T>(a.nx, q);
            qy_[j] = ldo<T>(a.ny, q);
            qz_[j] = ldo<T>(a.nz, q);
            m1q[j] = ldf(a.m1, q);
            m2q[j] = ldf(a.m2c, q);
        }
        // pass 1: weights and weighted sums of m1 and m2c
        float wt[PER];
        float sw = 0.f, s1 = 0.f, sm = 0.f;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int t = sub + 8 * j;
            const int dx = t % D - R, dy = t / D - R;
            float w;
            if (t == CTR) {
                w = 1.f;
            } else {
                const float s2 = chord2(nxp, nyp, nzp, qx_[j], qy_[j], qz_[j]);
                const float den = fmaf(
                    a.sigma_z, fabsf(grad_offset(gx, gy, (float)dx, (float)dy)), a.eps_z);
                float ex = -fabsf(zc - zq[j]) * (kLog2e / den);
                ex = add_normal_term(ex, s2, a.nc);
                w = empty_px(zq[j]) ? 0.f : __builtin_amdgcn_exp2f(ex);
            }
            w = ok[j] ? w : 0.f;
            wt[j] = w;
            if (ok[j]) {
                sw += w;
                s1 = fmaf(w, m1q[j], s1);
                sm = fmaf(w, m2q[j], sm);
            }
        }
        sw = group8_sum(sw);
        s1 = group8_sum(s1);
        sm = group8_sum(sm);
        const float mean1 = s1 / sw;
        // pass 2: spread of m1 about its weighted mean
        float spread = 0.f;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const float d = m1q[j] - mean1;
            if (ok[j]) spread = fmaf(wt[j] * d, d, spread);
        }
        spread = group8_sum(spread);
        if (sub == 0) stf(a.var, po, fmaxf(0.f, (sm + spread) / sw));
    }
}

template <typename T, int R>
__global__ __launch_bounds__(256) void variance_spatial_k(VarianceArgs a) {
    variance_spatial_stream<T, R>(a);
}

template <typename T, int R>
__global__ __launch_bounds__(256) void variance_spatial_batch_k(const VarianceArgs *args, int n) {
    for (int s = 0; s < n; ++s) {
        const VarianceArgs a = args[s];
        variance_spatial_stream<T, R>(a);
    }
}

template <typename T>
static void point_batch_launch(const void *args, const int *prefix, int n, int total,
                               hipStream_t s) {
    hipLaunchKernelGGL(variance_point_batch_k<T>, dim3(xcd_grid(total)), dim3(256), 0, s,
                       (const VarianceArgs *)args, prefix, n, total);
}

template <typename T, int R>
static void spatial_batch_launch(const void *args, const int *, int n, int, hipStream_t s) {
    hipLaunchKernelGGL((variance_spatial_batch_k<T, R>), dim3(kSpatialBlocks), dim3(256), 0, s,
                       (const VarianceArgs *)args, n);
}

template <typename T, int R>
void launch_spatial(const VarianceArgs &a, hipStream_t s) {
    if (record_pass(&spatial_batch_launch<T, R>, a, 0)) return;
    hipLaunchKernelGGL((variance_spatial_k<T, R>), dim3(kSpatialBlocks), dim3(256), 0, s, a);
}

template <typename T>
void launch_variance(const VarianceArgs &a, unsigned grid, int radius, bool listed,
                     hipStream_t s) {
    const int tiles = ((a.w + kVX - 1) / kVX) * ((a.h + kVY - 1) / kVY);
    if (!listed && !record_pass(&point_batch_launch<T>, a, tiles))
        hipLaunchKernelGGL(variance_point_k<T>, dim3(grid), dim3(256), 0, s, a);
    switch (radius) {
    case 0: launch_spatial<T, 0>(a, s); break;
    case 1: launch_spatial<T, 1>(a, s); break;
    case 2: launch_spatial<T, 2>(a, s); break;
    case 3: launch_spatial<T, 3>(a, s); break;
    case 4: launch_spatial<T, 4>(a, s); break;
    case 5: launch_spatial<T, 5>(a, s); break;
    case 6: launch_spatial<T, 6>(a, s); break;
    default: launch_spatial<T, 7>(a, s); break;
    }
}

}  // namespace sv

// ---- the variance estimate without a caller workspace -------------------------
//
// For callers that cannot allocate (code under graph capture, tight serving
// loops): the workspace is one file-scope device array, kNoAllocBytes
// long, which each GPU holds for the life of the process.  Host code never
// passes the array's name to a kernel (in host code it is a stand-in, not a
// device address): the device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is used.

namespace sv {

// 32 MiB: the eight counters and the pixel list of a 3840x2160 frame
// (sv_variance_work_bytes gives 33,178,624 bytes there).
constexpr size_t kNoAllocBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_scratch_lock;
static void *g_scratch_ptr[kMaxDevices];

// This device's address of the array, looked up on the first call on the
// device (with the device current); nullptr on failure.
static void *scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_lock);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace sv

extern "C" int sv_variance_noalloc(const float *m1, const float *m2c, const uint8_t *n,
                                   const sv_gbuf *g, float *var, sv_dims d, sv_dtype t,
                                   const sv_variance_params *p, sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    const int dc = check_dims(d);
    if (dc < 0 || !p) return SV_EINVAL;
    if (p->flags & SV_V_LISTED) return SV_EINVAL;  // a list lives in the caller's workspace
    if (dc == 1) return SV_OK;
    if (sv_variance_work_bytes(d) > kNoAllocBytes) return SV_ETOOBIG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SV_EHIP;
    void *work = scratch_ptr(dev);
    if (!work) return SV_EHIP;
    // every call shares this device's array and finds what the last call
    // left there: its counters are cleared first (a kernel, not a memset,
    // so that a captured graph holds kernel nodes only)
    hipLaunchKernelGGL(variance_reset_k, dim3(1), dim3(64), 0, as_stream(stream),
                       (VarWork *)work);
    const int rc = hip_status(hipGetLastError());
    if (rc != SV_OK) return rc;
    return sv_variance(m1, m2c, n, g, var, work, d, t, p, stream);
}

extern "C" size_t sv_variance_work_bytes(sv_dims d) {
    if (sv::check_dims(d) < 0) return 0;
    return offsetof(sv::VarWork, list) + sizeof(uint32_t) * 256 * (size_t)sv::point_grid(d);
}

extern "C" int sv_variance(const float *m1, const float *m2c, const uint8_t *n, const sv_gbuf *g,
                           float *var, void *work, sv_dims d, sv_dtype t,
                           const sv_variance_params *p, sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    int dc = check_dims(d);
    if (dc < 0 || !g || !p) return SV_EINVAL;
    if (p->radius < 0 || p->radius > 7 || p->min_hist < 0) return SV_EINVAL;
    if (!(p->sigma_n >= 0.f)) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    if (!m1 || !m2c || !n || !var || !work || !g->z || !g->dzdx || !g->dzdy || !g->nx || !g->ny ||
        !g->nz)
        return SV_EINVAL;
    const size_t es = elem_size(t);
    const span ins[] = {plane_span(m1, d, 4), plane_span(m2c, d, 4), plane_span(n, d, 1),
                        plane_span(g->z, d, es), plane_span(g->dzdx, d, es),
                        plane_span(g->dzdy, d, es), plane_span(g->nx, d, es),
                        plane_span(g->ny, d, es), plane_span(g->nz, d, es)};
    const span so = plane_span(var, d, 4);
    const span sw{(uintptr_t)work, (uintptr_t)work + sv_variance_work_bytes(d)};
    for (const span &si : ins)
        if (overlaps(so, si) || overlaps(sw, si)) return SV_EALIAS;
    if (overlaps(so, sw)) return SV_EALIAS;
    const unsigned grid = point_grid(d);
    VarianceArgs a{m1, m2c, n, g->z, g->dzdx, g->dzdy, g->nx, g->ny, g->nz, var,
                   (VarWork *)work, (grid / kXCD) * 256u, d.w, d.h, d.pitch, p->sigma_z,
                   p->eps_z, make_normal_coef(p->sigma_n), p->min_hist};
    hipStream_t s = as_stream(stream);
    const bool listed = (p->flags & SV_V_LISTED) != 0;
    if (t == SV_F32)
        launch_variance<float>(a, grid, p->radius, listed, s);
    else
        launch_variance<half_t>(a, grid, p->radius, listed, s);
    return hip_status(hipGetLastError());
}
