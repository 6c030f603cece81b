// Learned blend factor and edge scale: a 14 -> 32 -> 32 -> 2 per-pixel
// network on the matrix cores (bfloat16 operands, binary32 accumulation),
// its backward pass, Adam, and the two truncated loss gradients that train
// it (through the temporal blend and through each a-trous level).
//
// The forward pass and the matrix layout are in mlp_impl.h.
#include "mlp_impl.h"

namespace sv {

struct MlpArgs {
    const float *params;
    const uint16_t *wq;
    const uint4 *feat;  // 2 x 16 bytes per pixel
    float *alpha, *kappa;
    const float *d_alpha, *d_kappa;
    float *part;  // backward: per-wave partial gradients
    int w, h, pitch;
    int npix, nblk;  // pixels, 32-pixel blocks
};

__device__ __forceinline__ void load_x(const MlpArgs &a, int p, int hf, bf16x4 (&x)[2]) {
    // features 8 kb + 4 hf .. + 3 of pixel p: 8 bytes inside its 32-byte row
    const uint2 *row = (const uint2 *)(a.feat + 2 * (size_t)p);
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        const uint2 v = row[2 * kb + hf];
        x[kb][0] = (short)(v.x & 0xFFFFu);
        x[kb][1] = (short)(v.x >> 16);
        x[kb][2] = (short)(v.y & 0xFFFFu);
        x[kb][3] = (short)(v.y >> 16);
    }
}

__device__ __forceinline__ uint32_t plane_off(const MlpArgs &a, int p) {
    const int y = p / a.w, x = p - y * a.w;
    return (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
}

__global__ __launch_bounds__(256) void mlp_forward_k(MlpArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, hf = lane >> 5;
    FwdW f;
    load_fwd(a.params, a.wq, col, hf, f);
    for (int blk = blockIdx.x * 4 + wave; blk < a.nblk; blk += gridDim.x * 4) {
        const int p = blk * 32 + col;
        const bool valid = p < a.npix;
        bf16x4 x[2];
        load_x(a, valid ? p : a.npix - 1, hf, x);
        FwdOut r;
        forward_block(a.params, f, x, hf, r);
        if (valid && hf == 0) {
            const uint32_t o = plane_off(a, p);
            float al, ka;
            mlp_heads(r.o0, r.o1, al, ka);
            if (a.alpha) a.alpha[o] = al;
            if (a.kappa) a.kappa[o] = ka;
        }
    }
}

// ---- backward ------------------------------------------------------------

constexpr int kTP = 36;  // LDS tile row pitch in bfloat16 (32 + 4: fewer bank conflicts)

// Sum over the 32 lanes of one half-wave (butterfly, fixed order).
__device__ __forceinline__ float half_sum(float v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 16, 64);
    return v;
}

__device__ __forceinline__ bf16x4 tile_read(const uint16_t *t, int row, int k0) {
    const uint2 v = *(const uint2 *)(t + row * kTP + k0);
    bf16x4 r;
    r[0] = (short)(v.x & 0xFFFFu);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xFFFFu);
    r[3] = (short)(v.y >> 16);
    return r;
}

// Every wave of a workgroup runs the same number of iterations (a wave
// whose block is past the end works on an empty block), so the workgroup
// barriers around the LDS transposes are uniform.
__global__ __launch_bounds__(256) void mlp_backward_k(MlpArgs a) {
    // per wave: tiles [unit or feature][pixel] of g_h2, h1, g_h1, x
    __shared__ __align__(16) uint16_t lds[4][4][32 * kTP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 31, hf = lane >> 5;
    uint16_t *t_gh2 = lds[wave][0], *t_h1 = lds[wave][1], *t_gh1 = lds[wave][2],
             *t_x = lds[wave][3];
    // rows 16..31 of the x tile stay zero: the feature dimension is padded
    for (int i = lane; i < 32 * kTP; i += 64) t_x[i] = 0;
    FwdW f;
    load_fwd(a.params, a.wq, col, hf, f);
    bf16x4 w2t[4];  // A operand of W2^T: [h1 unit = col][h2 unit]
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            w2t[kb][i] = (short)a.wq[kOffW2 + (8 * kb + 4 * hf + i) * SV_MLP_HIDDEN + col];
    f32x16 dw1, dw2;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        dw1[i] = 0.f;
        dw2[i] = 0.f;
    }
    float dw3a[16], dw3b[16], db1[16], db2[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) dw3a[i] = dw3b[i] = db1[i] = db2[i] = 0.f;
    float db3a = 0.f, db3b = 0.f;
    const int stride = gridDim.x * 4;
    for (int base = blockIdx.x * 4; base < a.nblk; base += stride) {
        const int blk = base + wave;
        const int p = blk * 32 + col;
        const bool valid = blk < a.nblk && p < a.npix;
        bf16x4 x[2];
        load_x(a, valid ? p : 0, hf, x);
        FwdOut r;
        forward_block(a.params, f, x, hf, r);
        // gradients of the outputs
        float da = 0.f, dk = 0.f;
        if (valid) {
            const uint32_t o = plane_off(a, p);
            da = a.d_alpha ? a.d_alpha[o] : 0.f;
            dk = a.d_kappa ? a.d_kappa[o] : 0.f;
        }
        // the heads' slopes without cancellation: sigmoid' = e / (1 + e)^2
        // with e = exp(-|o|), and 1 - tanh^2 = 4 e / (1 + e)^2 with
        // e = exp(-2|o|) (1 - sg and 1 - th^2 would lose every digit once
        // the heads saturate)
        const float e0 = expf(-fabsf(r.o0)), d0 = 1.0f / (1.0f + e0);
        const float e1 = expf(-2.0f * fabsf(r.o1)), d1 = 1.0f / (1.0f + e1);
        const float kap = exp2f(2.0f * tanhf(r.o1));
        const float g0 = da * (1.0f - kAlphaMin) * (e0 * d0 * d0);
        const float g1 = dk * kap * 0.69314718055994531f * 2.0f * (4.0f * e1 * d1 * d1);
        const float g0q = from_bf16(to_bf16(g0)), g1q = from_bf16(to_bf16(g1));
        if (hf == 0) {
            db3a += g0;
            db3b += g1;
        }
        // layer 3 and the gradient reaching layer 2
        float gh2[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            dw3a[i] = fmaf(g0q, r.h2[i], dw3a[i]);
            dw3b[i] = fmaf(g1q, r.h2[i], dw3b[i]);
            gh2[i] = r.a2[i] > 0.f ? fmaf(f.w3a[i], g0q, f.w3b[i] * g1q) : 0.f;
            db2[i] += gh2[i];
        }
        bf16x4 gb[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
#pragma unroll
            for (int i = 0; i < 4; ++i) gb[kb][i] = (short)to_bf16(gh2[4 * kb + i]);
        // gradient reaching layer 1: W2^T g_h2, masked by a1 > 0
        f32x16 g1acc;
#pragma unroll
        for (int i = 0; i < 16; ++i) g1acc[i] = 0.f;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) g1acc = mfma(w2t[kb], gb[kb], g1acc);
        float gh1[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            gh1[i] = r.a1[i] > 0.f ? g1acc[i] : 0.f;
            db1[i] += gh1[i];
        }
        // transposes for the weight gradients (contractions over pixels)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int u = drow(i, hf);
            t_gh2[u * kTP + col] = (uint16_t)gb[i >> 2][i & 3];
            t_h1[u * kTP + col] = (uint16_t)r.h1[i >> 2][i & 3];
            t_gh1[u * kTP + col] = to_bf16(gh1[i]);
        }
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int i = 0; i < 4; ++i) t_x[(8 * kb + 4 * hf + i) * kTP + col] = (uint16_t)x[kb][i];
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const int k0 = 8 * kb + 4 * hf;
            dw2 = mfma(tile_read(t_gh2, col, k0), tile_read(t_h1, col, k0), dw2);
            dw1 = mfma(tile_read(t_gh1, col, k0), tile_read(t_x, col, k0), dw1);
        }
        __syncthreads();
    }
    // this wave's partial gradient, flat order
    float *out = a.part + (size_t)(blockIdx.x * 4 + wave) * SV_MLP_PARAMS;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int u = drow(i, hf);
        out[kOffW2 + u * SV_MLP_HIDDEN + col] = dw2[i];
        if (col < SV_MLP_IN) out[kOffW1 + u * SV_MLP_IN + col] = dw1[i];
        const float s3a = half_sum(dw3a[i]), s3b = half_sum(dw3b[i]);
        const float s1 = half_sum(db1[i]), s2 = half_sum(db2[i]);
        if (col == 0) {
            out[kOffW3 + u] = s3a;
            out[kOffW3 + SV_MLP_HIDDEN + u] = s3b;
            out[kOffB1 + u] = s1;
            out[kOffB2 + u] = s2;
        }
    }
    db3a = half_sum(db3a);
    db3b = half_sum(db3b);
    db3a += __shfl_xor(db3a, 32, 64);
    db3b += __shfl_xor(db3b, 32, 64);
    if (lane == 0) {
        out[kOffB3] = db3a;
        out[kOffB3 + 1] = db3b;
    }
}

__global__ __launch_bounds__(256) void mlp_reduce_k(const float *part, int nw, float scale,
                                                    float *grad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= SV_MLP_PARAMS) return;
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += part[(size_t)w * SV_MLP_PARAMS + j];
    grad[j] = s * scale;
}

__global__ __launch_bounds__(256) void adam_k(float *params, uint16_t *wq, float *m, float *v,
                                              const float *g, int n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j];
    const float mj = fmaf(b1, m[j], (1.0f - b1) * gj);
    const float vj = fmaf(b2, v[j], (1.0f - b2) * gj * gj);
    m[j] = mj;
    v[j] = vj;
    const float pj = params[j] - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
    params[j] = pj;
    if (wq) wq[j] = to_bf16(pj);
}

// ---- truncated loss gradients ---------------------------------------------

struct AlphaGradArgs {
    const void *ctr, *ctg, *ctb, *cr, *cg, *cb;
    const float *hr, *hg, *hb, *yr, *yg, *yb, *alpha;
    const uint8_t *n;
    const void *z;
    float *d_alpha;
    int w, h, pitch;
    float tm_k;
};

// The two loss gradients are training-only passes, off the measured path.
// Their results are sums over channels (and, for kappa, over taps) of terms
// of either sign, so binary32 would lose digits to cancellation wherever the
// terms nearly balance; they are evaluated in binary64 from the stored
// (binary32 or binary16) inputs, like the definition they implement.
__device__ __forceinline__ double luma_d(double r, double g, double b) {
    return 0.2126 * r + 0.7152 * g + 0.0722 * b;
}

template <typename T>
__global__ __launch_bounds__(256) void alpha_grad_k(AlphaGradArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.w || y >= a.h) return;
    const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    const int n = a.n[o];
    double g = 0.0;
    if (!empty_px(ldo<T>(a.z, o)) && n >= 1 && a.alpha[o] >= 1.0f / (float)n) {
        double c[3] = {ldo<T>(a.cr, o), ldo<T>(a.cg, o), ldo<T>(a.cb, o)};
        if (a.tm_k > 0.f) {
            const double sc = 1.0 / (1.0 + (double)a.tm_k * luma_d(c[0], c[1], c[2]));
            c[0] *= sc;
            c[1] *= sc;
            c[2] *= sc;
        }
        const double ct[3] = {ldo<T>(a.ctr, o), ldo<T>(a.ctg, o), ldo<T>(a.ctb, o)};
        const double hh[3] = {ldf(a.hr, o), ldf(a.hg, o), ldf(a.hb, o)};
        const double yy[3] = {ldf(a.yr, o), ldf(a.yg, o), ldf(a.yb, o)};
#pragma unroll
        for (int k = 0; k < 3; ++k) g += (ct[k] - yy[k]) / (yy[k] * yy[k] + 0.01) * (c[k] - hh[k]);
        g *= 2.0 / 3.0;
    }
    a.d_alpha[o] = (float)g;
}

struct KappaGradArgs {
    const void *cr, *cg, *cb;
    const float *var;
    const void *z, *dzdx, *dzdy, *nx, *ny, *nz;
    const float *kappa;
    const float *yr, *yg, *yb;
    const float *rr, *rg, *rb;  // optional: the colour whose residual is used
    float *d_kappa;
    int w, h, pitch, step;
    float sigma_z, sigma_n, sigma_l, eps_z, eps_l;
};

// One pixel per thread, taps read directly, in binary64 (see alpha_grad_k).
// The 3x3 variance prefilter runs over the in-image, non-empty taps, as in
// the level itself.
template <typename T>
__global__ __launch_bounds__(256) void kappa_grad_k(KappaGradArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63), y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.w || y >= a.h) return;
    const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    const double zp = ldo<T>(a.z, o);
    if (empty_px((float)zp)) return;
    double gs = 0.0, gw = 0.0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            const int qx = x + dx, qy = y + dy;
            if (qx < 0 || qx >= a.w || qy < 0 || qy >= a.h) continue;
            const uint32_t q = (uint32_t)qy * (uint32_t)a.pitch + (uint32_t)qx;
            if (empty_px(ldo<T>(a.z, q))) continue;
            const double k = (dx == 0 ? 0.5 : 0.25) * (dy == 0 ? 0.5 : 0.25);
            gs += k * (double)ldf(a.var, q);
            gw += k;
        }
    const double sg = sqrt(gs / gw);
    const double sl = a.sigma_l;
    const double dl = sl * (double)ldf(a.kappa, o) * sg + (double)a.eps_l;
    const double cp[3] = {ldo<T>(a.cr, o), ldo<T>(a.cg, o), ldo<T>(a.cb, o)};
    const double lp = luma_d(cp[0], cp[1], cp[2]);
    const double gx = ldo<T>(a.dzdx, o), gy = ldo<T>(a.dzdy, o);
    const double np_[3] = {ldo<T>(a.nx, o), ldo<T>(a.ny, o), ldo<T>(a.nz, o)};
    const double h1[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    double sw = 0.0, sd = 0.0, sc[3] = {0.0, 0.0, 0.0}, sdc[3] = {0.0, 0.0, 0.0};
    for (int b = -2; b <= 2; ++b)
        for (int aa = -2; aa <= 2; ++aa) {
            const int qx = x + aa * a.step, qy = y + b * a.step;
            if (qx < 0 || qx >= a.w || qy < 0 || qy >= a.h) continue;
            const uint32_t q = (uint32_t)qy * (uint32_t)a.pitch + (uint32_t)qx;
            const double hh = h1[aa + 2] * h1[b + 2];
            const double cq[3] = {ldo<T>(a.cr, q), ldo<T>(a.cg, q), ldo<T>(a.cb, q)};
            double w = 1.0, d = 0.0;
            if (aa != 0 || b != 0) {
                const float zq32 = ldo<T>(a.z, q);
                if (empty_px(zq32)) continue;
                const double zq = zq32;
                const double den = (double)a.sigma_z *
                                       fabs(gx * (double)(a.step * aa) + gy * (double)(a.step * b)) +
                                   (double)a.eps_z;
                const double wz = exp(-fabs(zp - zq) / den);
                const double ex = np_[0] - (double)ldo<T>(a.nx, q);
                const double ey = np_[1] - (double)ldo<T>(a.ny, q);
                const double ez = np_[2] - (double)ldo<T>(a.nz, q);
                const double cs = 1.0 - 0.5 * (ex * ex + ey * ey + ez * ez);
                const double wn = pow(cs > 0.0 ? cs : 0.0, (double)a.sigma_n);
                const double adl = fabs(lp - luma_d(cq[0], cq[1], cq[2]));
                w = wz * wn * exp(-adl / dl);
                d = w * adl * sl * sg / (dl * dl);
            }
            sw += hh * w;
            sd += hh * d;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                sc[k] += hh * w * cq[k];
                sdc[k] += hh * d * cq[k];
            }
        }
    const double yy[3] = {ldf(a.yr, o), ldf(a.yg, o), ldf(a.yb, o)};
    const float *rp[3] = {a.rr, a.rg, a.rb};
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double out = sc[k] / sw;
        const double der = (sdc[k] - out * sd) / sw;
        const double res = (a.rr ? (double)ldf(rp[k], o) : out) - yy[k];
        g += res / (yy[k] * yy[k] + 0.01) * der;
    }
    a.d_kappa[o] += (float)(g * (2.0 / 3.0));
}

inline unsigned mlp_grid(int nblk) {
    const int wgs = (nblk + 3) / 4;
    return (unsigned)std::max(1, std::min(wgs, 256 * 8));
}

inline bool valid_mlp(const sv_mlp *w) { return w && w->params && w->wq; }

}  // namespace sv

extern "C" int sv_mlp_forward(const sv_mlp *w, const void *feat, float *alpha, float *kappa,
                              sv_dims d, sv_stream stream) {
    using namespace sv;
    const int dc = check_dims(d);
    if (dc < 0 || !valid_mlp(w)) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    if (!feat || ((uintptr_t)feat & 15u)) return SV_EINVAL;
    const span fs{(uintptr_t)feat, (uintptr_t)feat + (size_t)d.w * (size_t)d.h * 32u};
    if ((alpha && overlaps(plane_span(alpha, d, 4), fs)) ||
        (kappa && overlaps(plane_span(kappa, d, 4), fs)) ||
        (alpha && kappa && overlaps(plane_span(alpha, d, 4), plane_span(kappa, d, 4))))
        return SV_EALIAS;
    MlpArgs a{};
    a.params = w->params;
    a.wq = w->wq;
    a.feat = (const uint4 *)feat;
    a.alpha = alpha;
    a.kappa = kappa;
    a.w = d.w;
    a.h = d.h;
    a.pitch = d.pitch;
    a.npix = d.w * d.h;
    a.nblk = (a.npix + 31) / 32;
    hipLaunchKernelGGL(mlp_forward_k, dim3(mlp_grid(a.nblk)), dim3(256), 0, as_stream(stream), a);
    return hip_status(hipGetLastError());
}

extern "C" size_t sv_mlp_backward_work_bytes(sv_dims d) {
    using namespace sv;
    if (check_dims(d) < 0) return 0;
    const int nblk = (d.w * d.h + 31) / 32;
    return (size_t)mlp_grid(nblk) * 4u * SV_MLP_PARAMS * sizeof(float);
}

extern "C" int sv_mlp_backward(const sv_mlp *w, const void *feat, const float *d_alpha,
                               const float *d_kappa, float scale, float *grad, void *work,
                               sv_dims d, sv_stream stream) {
    using namespace sv;
    const int dc = check_dims(d);
    if (dc < 0 || !valid_mlp(w) || !grad) return SV_EINVAL;
    if (dc == 1) {  // no pixels: a zero gradient (a fill kernel, not a memset node)
        hipLaunchKernelGGL(mlp_reduce_k, dim3((SV_MLP_PARAMS + 255) / 256), dim3(256), 0,
                           as_stream(stream), (const float *)nullptr, 0, 0.f, grad);
        return hip_status(hipGetLastError());
    }
    if (!feat || ((uintptr_t)feat & 15u) || !work) return SV_EINVAL;
    MlpArgs a{};
    a.params = w->params;
    a.wq = w->wq;
    a.feat = (const uint4 *)feat;
    a.d_alpha = d_alpha;
    a.d_kappa = d_kappa;
    a.part = (float *)work;
    a.w = d.w;
    a.h = d.h;
    a.pitch = d.pitch;
    a.npix = d.w * d.h;
    a.nblk = (a.npix + 31) / 32;
    const span ws{(uintptr_t)work, (uintptr_t)work + sv_mlp_backward_work_bytes(d)};
    const span gs{(uintptr_t)grad, (uintptr_t)grad + SV_MLP_PARAMS * sizeof(float)};
    const span fs{(uintptr_t)feat, (uintptr_t)feat + (size_t)d.w * (size_t)d.h * 32u};
    if (overlaps(ws, gs) || overlaps(ws, fs) || overlaps(gs, fs) ||
        (d_alpha && (overlaps(ws, plane_span(d_alpha, d, 4)) || overlaps(gs, plane_span(d_alpha, d, 4)))) ||
        (d_kappa && (overlaps(ws, plane_span(d_kappa, d, 4)) || overlaps(gs, plane_span(d_kappa, d, 4)))))
        return SV_EALIAS;
    const unsigned grid = mlp_grid(a.nblk);
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(mlp_backward_k, dim3(grid), dim3(256), 0, s, a);
    hipLaunchKernelGGL(mlp_reduce_k, dim3((SV_MLP_PARAMS + 255) / 256), dim3(256), 0, s,
                       (const float *)work, (int)grid * 4, scale, grad);
    return hip_status(hipGetLastError());
}

extern "C" int sv_adam(float *params, uint16_t *wq, float *m, float *v, const float *grad,
                       int32_t n, int32_t t, const sv_adam_params *p, sv_stream stream) {
    using namespace sv;
    if (!params || !m || !v || !grad || !p || n < 0 || t < 1) return SV_EINVAL;
    if (n == 0) return SV_OK;
    const float c1 = 1.0f - powf(p->beta1, (float)t), c2 = 1.0f - powf(p->beta2, (float)t);
    hipLaunchKernelGGL(adam_k, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), params, wq,
                       m, v, grad, n, p->lr, p->beta1, p->beta2, p->eps, c1, c2);
    return hip_status(hipGetLastError());
}

extern "C" int sv_mlp_alpha_grad(const sv_rgb *c_t, const sv_rgb *cur, const sv_rgb *hist,
                                 const sv_rgb *y, const float *alpha, const uint8_t *n,
                                 const void *z, float tm_k, float *d_alpha, sv_dims d, sv_dtype t,
                                 sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    const int dc = check_dims(d);
    if (dc < 0 || !c_t || !cur || !hist || !y) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    const void *req[] = {c_t->r, c_t->g, c_t->b, cur->r, cur->g, cur->b, hist->r, hist->g,
                         hist->b, y->r, y->g, y->b, alpha, n, z, d_alpha};
    for (const void *q : req)
        if (!q) return SV_EINVAL;
    const size_t es = elem_size(t);
    const span so = plane_span(d_alpha, d, 4);
    const span ins[] = {plane_span(c_t->r, d, es), plane_span(c_t->g, d, es),
                        plane_span(c_t->b, d, es), plane_span(cur->r, d, es),
                        plane_span(cur->g, d, es), plane_span(cur->b, d, es),
                        plane_span(hist->r, d, 4), plane_span(hist->g, d, 4),
                        plane_span(hist->b, d, 4), plane_span(y->r, d, 4),
                        plane_span(y->g, d, 4), plane_span(y->b, d, 4),
                        plane_span(alpha, d, 4), plane_span(n, d, 1), plane_span(z, d, es)};
    for (const span &si : ins)
        if (overlaps(so, si)) return SV_EALIAS;
    AlphaGradArgs a{c_t->r, c_t->g, c_t->b, cur->r, cur->g, cur->b,
                    (const float *)hist->r, (const float *)hist->g, (const float *)hist->b,
                    (const float *)y->r, (const float *)y->g, (const float *)y->b, alpha, n, z,
                    d_alpha, d.w, d.h, d.pitch, tm_k};
    dim3 grid((d.w + 63) / 64, (d.h + 3) / 4);
    if (t == SV_F32)
        hipLaunchKernelGGL(alpha_grad_k<float>, grid, dim3(256), 0, as_stream(stream), a);
    else
        hipLaunchKernelGGL(alpha_grad_k<half_t>, grid, dim3(256), 0, as_stream(stream), a);
    return hip_status(hipGetLastError());
}

extern "C" int sv_atrous_kappa_grad(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                                    const float *kappa, const sv_rgb *y, const sv_rgb *ref,
                                    float *d_kappa, int32_t step, sv_dims d, sv_dtype t,
                                    const sv_atrous_params *p, sv_stream stream) {
    using namespace sv;
    if (!valid_dtype(t)) return SV_EDTYPE;
    const int dc = check_dims(d);
    if (dc < 0 || !c_in || !g || !y || !p || step < 1 || step > kMaxDim) return SV_EINVAL;
    if (dc == 1) return SV_OK;
    const void *req[] = {c_in->r, c_in->g, c_in->b, var_in, g->z, g->dzdx, g->dzdy, g->nx,
                         g->ny, g->nz, kappa, y->r, y->g, y->b, d_kappa};
    for (const void *q : req)
        if (!q) return SV_EINVAL;
    if (!(p->sigma_n >= 0.f)) return SV_EINVAL;
    if (ref && (!ref->r || !ref->g || !ref->b)) return SV_EINVAL;
    const size_t es = elem_size(t);
    const span so = plane_span(d_kappa, d, 4);
    if (ref && (overlaps(so, plane_span(ref->r, d, 4)) || overlaps(so, plane_span(ref->g, d, 4)) ||
                overlaps(so, plane_span(ref->b, d, 4))))
        return SV_EALIAS;
    const span ins[] = {plane_span(c_in->r, d, es), plane_span(c_in->g, d, es),
                        plane_span(c_in->b, d, es), plane_span(var_in, d, 4),
                        plane_span(g->z, d, es), plane_span(g->dzdx, d, es),
                        plane_span(g->dzdy, d, es), plane_span(g->nx, d, es),
                        plane_span(g->ny, d, es), plane_span(g->nz, d, es),
                        plane_span(kappa, d, 4), plane_span(y->r, d, 4),
                        plane_span(y->g, d, 4), plane_span(y->b, d, 4)};
    for (const span &si : ins)
        if (overlaps(so, si)) return SV_EALIAS;
    KappaGradArgs a{c_in->r, c_in->g, c_in->b, var_in, g->z, g->dzdx, g->dzdy, g->nx, g->ny,
                    g->nz, kappa, (const float *)y->r, (const float *)y->g, (const float *)y->b,
                    ref ? (const float *)ref->r : nullptr, ref ? (const float *)ref->g : nullptr,
                    ref ? (const float *)ref->b : nullptr,
                    d_kappa, d.w, d.h, d.pitch, step, p->sigma_z, p->sigma_n, p->sigma_l,
                    p->eps_z, p->eps_l};
    dim3 grid((d.w + 63) / 64, (d.h + 3) / 4);
    if (t == SV_F32)
        hipLaunchKernelGGL(kappa_grad_k<float>, grid, dim3(256), 0, as_stream(stream), a);
    else
        hipLaunchKernelGGL(kappa_grad_k<half_t>, grid, dim3(256), 0, as_stream(stream), a);
    return hip_status(hipGetLastError());
}
