// Status strings, version, error capture, the copy bandwidth probe and the
// issue-rate probe.
#include "sv_internal.h"

namespace sv {

static thread_local int g_last_hip_error = 0;

int hip_status(hipError_t e) {
    if (e == hipSuccess) return SV_OK;
    g_last_hip_error = (int)e;
    return SV_EHIP;
}

// Streaming copy: 16 bytes per lane per iteration, grid-stride.
__global__ __launch_bounds__(256) void probe_copy_k(uint4 *__restrict__ dst,
                                                    const uint4 *__restrict__ src, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

// Issue-rate probe: eight independent chains per lane, each link one
// operation under test beside full-rate ones (KIND 0: fma with literal
// operands, which issues at the full rate; 1: exp2, mul;
// 2: add, log2, mul; 3: add, rcp, mul; 4: add, sqrt, mul).  The values
// stay bounded (exp2 of [0, 1/2], log2 / rcp / sqrt of [1.5, 2.5]), and
// each lane writes its one sum, so nothing is optimised away.
template <int KIND>
__global__ __launch_bounds__(256) void probe_issue_k(float *out, int iters) {
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = 0.0625f * (float)((threadIdx.x + j) & 7);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (KIND == 0) x[j] = fmaf(x[j], 0.5f, 0.25f);
            if (KIND == 1) x[j] = __builtin_amdgcn_exp2f(x[j]) * 0.25f;
            if (KIND == 2) x[j] = __builtin_amdgcn_logf(x[j] + 1.5f) * 0.5f;
            if (KIND == 3) x[j] = __builtin_amdgcn_rcpf(x[j] + 1.5f) * 0.5f;
            if (KIND == 4) x[j] = __builtin_amdgcn_sqrtf(x[j] + 1.5f) * 0.5f;
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += x[j];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

}  // namespace sv

extern "C" {

const char *sv_status_str(int status) {
    switch (status) {
    case SV_OK: return "ok";
    case SV_EINVAL: return "invalid argument";
    case SV_EALIAS: return "an output overlaps an input";
    case SV_EDTYPE: return "unknown storage type";
    case SV_EHIP: return "HIP launch error";
    case SV_EUNSUPPORTED: return "unsupported combination";
    case SV_ETOOBIG: return "larger than the fixed workspace of the allocation-free call";
    default: return "unknown status";
    }
}

int sv_version(void) { return 1; }

int sv_last_hip_error(void) { return sv::g_last_hip_error; }

int sv_probe_copy(void *dst, const void *src, size_t bytes, sv_stream stream) {
    if (!dst || !src) return SV_EINVAL;
    if (bytes % 16 != 0 || ((uintptr_t)dst % 16) != 0 || ((uintptr_t)src % 16) != 0)
        return SV_EINVAL;
    if (bytes == 0) return SV_OK;
    uintptr_t a = (uintptr_t)dst, b = (uintptr_t)src;
    if (a < b + bytes && b < a + bytes) return SV_EALIAS;
    size_t n = bytes / 16;
    size_t blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;  // 64 workgroups per CU, grid-stride beyond
    hipLaunchKernelGGL(sv::probe_copy_k, dim3((unsigned)blocks), dim3(256), 0,
                       sv::as_stream(stream), (uint4 *)dst, (const uint4 *)src, n);
    return sv::hip_status(hipGetLastError());
}

int sv_probe_issue(int32_t kind, int32_t iters, float *out, int32_t blocks, sv_stream stream) {
    if (!out || kind < 0 || kind > 4 || iters < 1 || iters > (1 << 20) || blocks < 1 ||
        blocks > 65536)
        return SV_EINVAL;
    hipStream_t s = sv::as_stream(stream);
    const dim3 g((unsigned)blocks), b(256);
    switch (kind) {
    case 0: hipLaunchKernelGGL(sv::probe_issue_k<0>, g, b, 0, s, out, (int)iters); break;
    case 1: hipLaunchKernelGGL(sv::probe_issue_k<1>, g, b, 0, s, out, (int)iters); break;
    case 2: hipLaunchKernelGGL(sv::probe_issue_k<2>, g, b, 0, s, out, (int)iters); break;
    case 3: hipLaunchKernelGGL(sv::probe_issue_k<3>, g, b, 0, s, out, (int)iters); break;
    default: hipLaunchKernelGGL(sv::probe_issue_k<4>, g, b, 0, s, out, (int)iters); break;
    }
    return sv::hip_status(hipGetLastError());
}

}  // extern "C"

extern "C" int sv_struct_sizes(size_t *sizes, int32_t n) {
    const size_t all[] = {sizeof(sv_dims),          sizeof(sv_rgb),
                          sizeof(sv_gbuf),          sizeof(sv_tm_params),
                          sizeof(sv_temporal_io),   sizeof(sv_temporal_params),
                          sizeof(sv_variance_params), sizeof(sv_atrous_params),
                          sizeof(sv_denoiser),      sizeof(sv_frame_in),
                          sizeof(sv_frame_params),  sizeof(sv_mlp),
                          sizeof(sv_adam_params),   sizeof(sv_blur_rule),
                          sizeof(sv_grad_params)};
    const int32_t k = (int32_t)(sizeof(all) / sizeof(all[0]));
    if (!sizes || n < 0) return SV_EINVAL;
    for (int32_t i = 0; i < n && i < k; ++i) sizes[i] = all[i];
    return k;
}
