// Variance estimate (Section 2): the temporal variance of the luminance
// moments where the history is long enough, a depth- and normal-weighted
// spatial estimate where it is not.  The second moment arrives as the
// central moment m2c = E[L^2] - E[L]^2, so neither branch cancels.
#include "sv_internal.h"

namespace sv {

constexpr int kVX = 64, kVY = 4;

struct VarianceArgs {
    const float *m1, *m2c;
    const uint8_t *n;
    const void *z, *dzdx, *dzdy, *nx, *ny, *nz;
    float *var;
    int w, h, pitch;
    float sigma_z, eps_z;
    NormalCoef nc;
    int min_hist, radius;
};

// Sum over the 64 lanes of a wavefront (butterfly: a fixed order, so the
// result is the same on every run).
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One workgroup covers 64x4 pixels.  The temporal estimate is pointwise.
// Pixels with a short history (1 <= n < min_hist) are rare (disocclusions)
// and scattered; instead of letting each of them hold its whole wavefront
// through a (2R+1)^2 loop, the workgroup lists them and each wavefront takes
// one listed pixel at a time with one window tap per lane, combining the
// lanes by wavefront sums.  The window (tile plus an R apron) is staged in
// LDS only when the list is not empty: m1, m2c, z, nx, ny, nz per pixel,
// z = 0 outside the image or empty.
template <typename T, int NM>
__global__ __launch_bounds__(256) void variance_k(VarianceArgs a) {
    extern __shared__ float s_win[];
    __shared__ int s_count;
    __shared__ int s_list[256];
    __shared__ float s_res[256];
    const int lx = threadIdx.x & 63, ly = threadIdx.x >> 6;
    const int x = blockIdx.x * kVX + lx, y = blockIdx.y * kVY + ly;
    const bool inside = x < a.w && y < a.h;
    const uint32_t o = inside ? (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x : 0;
    int n = 0;
    float zp = 0.f;
    if (inside) {
        n = a.n[o];
        zp = ldo<T>(a.z, o);
    }
    const bool live = inside && n >= 1 && !empty_px(zp);
    const bool spatial = live && n < a.min_hist;
    float v = 0.f;
    if (live && !spatial) v = fmaxf(0.f, ldf(a.m2c, o));
    if (threadIdx.x == 0) s_count = 0;
    __syncthreads();
    if (spatial) s_list[atomicAdd(&s_count, 1)] = threadIdx.x;
    __syncthreads();
    const int cnt = s_count;
    if (cnt > 0) {
        const int R = a.radius, D = 2 * R + 1, NT = D * D;
        const int WX = kVX + 2 * R, WY = kVY + 2 * R, NW = WX * WY;
        float *s_m1 = s_win, *s_m2 = s_win + NW, *s_z = s_win + 2 * NW;
        float *s_nx = s_win + 3 * NW, *s_ny = s_win + 4 * NW, *s_nz = s_win + 5 * NW;
        const int gx0 = blockIdx.x * kVX - R, gy0 = blockIdx.y * kVY - R;
        for (int i = threadIdx.x; i < NW; i += 256) {
            const int r = i / WX, c = i - r * WX;
            const int gx = gx0 + c, gy = gy0 + r;
            float m1 = 0.f, m2 = 0.f, zz = 0.f, nx = 0.f, ny = 0.f, nz = 0.f;
            if (gx >= 0 && gx < a.w && gy >= 0 && gy < a.h) {
                const uint32_t q = (uint32_t)gy * (uint32_t)a.pitch + (uint32_t)gx;
                zz = ldo<T>(a.z, q);
                if (empty_px(zz)) zz = 0.f;
                m1 = ldf(a.m1, q);
                m2 = ldf(a.m2c, q);
                nx = ldo<T>(a.nx, q);
                ny = ldo<T>(a.ny, q);
                nz = ldo<T>(a.nz, q);
            }
            s_m1[i] = m1;
            s_m2[i] = m2;
            s_z[i] = zz;
            s_nx[i] = nx;
            s_ny[i] = ny;
            s_nz[i] = nz;
        }
        __syncthreads();
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        for (int e = wave; e < cnt; e += 4) {
            const int pt = s_list[e];
            const int px = pt & 63, py = pt >> 6;
            const uint32_t po = (uint32_t)(blockIdx.y * kVY + py) * (uint32_t)a.pitch + (uint32_t)(blockIdx.x * kVX + px);
            const float gx = ldo<T>(a.dzdx, po), gy = ldo<T>(a.dzdy, po);
            const int ci = (py + R) * WX + px + R;
            const float zc = s_z[ci], nxp = s_nx[ci], nyp = s_ny[ci], nzp = s_nz[ci];
            // pass 1: per-lane taps (lane, lane + 64, ...) then wavefront sums
            float w[4], m1v[4];
            float sw = 0.f, s1 = 0.f, sm = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int t = lane + 64 * k;
                w[k] = 0.f;
                m1v[k] = 0.f;
                if (t < NT) {
                    const int dx = t % D - R, dy = t / D - R;
                    const int qi = ci + dy * WX + dx;
                    const float zq = s_z[qi];
                    if (dx == 0 && dy == 0) {
                        w[k] = 1.f;
                    } else if (zq > 0.f) {
                        const float den = fmaf(a.sigma_z, fabsf(fmaf(gx, (float)dx, gy * (float)dy)),
                                               a.eps_z);
                        float ex = -fabsf(zc - zq) * (kLog2e / den);
                        ex = add_normal_term<NM>(
                            ex, chord2(nxp, nyp, nzp, s_nx[qi], s_ny[qi], s_nz[qi]), a.nc);
                        w[k] = __builtin_amdgcn_exp2f(ex);
                    }
                    m1v[k] = s_m1[qi];
                    sw += w[k];
                    s1 = fmaf(w[k], m1v[k], s1);
                    sm = fmaf(w[k], s_m2[qi], sm);
                }
            }
            sw = wave_sum(sw);
            s1 = wave_sum(s1);
            sm = wave_sum(sm);
            const float mean1 = s1 / sw;
            // pass 2: spread of m1 about its weighted mean
            float spread = 0.f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float d = m1v[k] - mean1;
                spread = fmaf(w[k] * d, d, spread);
            }
            spread = wave_sum(spread);
            if (lane == 0) s_res[pt] = fmaxf(0.f, (sm + spread) / sw);
        }
        __syncthreads();
        if (spatial) v = s_res[threadIdx.x];
    }
    if (inside) stf(a.var, o, v);
}

template <typename T>
static void launch_variance(const VarianceArgs &a, int nm, dim3 grid, size_t lds,
                            hipStream_t s) {
    switch (nm) {
    case kNormalOff:
        hipLaunchKernelGGL((variance_k<T, kNormalOff>), grid, dim3(256), lds, s, a);
        break;
    default:
        hipLaunchKernelGGL((variance_k<T, kNormalLog>), grid, dim3(256), lds, s, a);
    }
}

}  // namespace sv

extern "C" int sv_variance(const float *m1, const float *m2c, const uint8_t *n, const sv_gbuf *g,
                           float *var, sv_dims d, sv_dtype t, const sv_variance_params *p,
                           sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    int dc = check_dims(d);
    if (dc < 0 || !g || !p) return SV_EINVAL;
    if (p->radius < 0 || p->radius > 7 || p->min_hist < 0) return SV_EINVAL;
    if (!(p->sigma_n >= 0.f)) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    if (!m1 || !m2c || !n || !var || !g->z || !g->dzdx || !g->dzdy || !g->nx || !g->ny || !g->nz)
        return SV_EINVAL;
    const size_t es = elem_size(t);
    const span ins[] = {plane_span(m1, d, 4), plane_span(m2c, d, 4), plane_span(n, d, 1),
                        plane_span(g->z, d, es), plane_span(g->dzdx, d, es),
                        plane_span(g->dzdy, d, es), plane_span(g->nx, d, es),
                        plane_span(g->ny, d, es), plane_span(g->nz, d, es)};
    const span so = plane_span(var, d, 4);
    for (const span &si : ins)
        if (overlaps(so, si)) return SV_EALIAS;
    VarianceArgs a{m1, m2c, n, g->z, g->dzdx, g->dzdy, g->nx, g->ny, g->nz, var,
                   d.w, d.h, d.pitch, p->sigma_z, p->eps_z, make_normal_coef(p->sigma_n),
                   p->min_hist, p->radius};
    const size_t lds = sizeof(float) * 6 * (kVX + 2 * p->radius) * (kVY + 2 * p->radius);
    dim3 grid((d.w + kVX - 1) / kVX, (d.h + kVY - 1) / kVY);
    const int nm = normal_mode(p->sigma_n);
    if (t == SV_F32) launch_variance<float>(a, nm, grid, lds, as_stream(stream));
    else launch_variance<half_t>(a, nm, grid, lds, as_stream(stream));
    return hip_status(hipGetLastError());
}
