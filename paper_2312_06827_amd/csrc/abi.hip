// Status strings, version, error capture and the copy bandwidth probe.
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
