// Edge-avoiding a-trous wavelet levels guided by the variance (Section 2,
// Fig. 1) in 5x5 form, and the separable form of Section 3.3.
//
// Every tap's weight H(a,b) * w_z * w_n * w_l is evaluated as one
// exponential: log2 H - |dz| kz(a,b) - |dL| kl + sigma_n log2 max(0, cos)
// (the normal term as in sv_internal.h),
// with kz(a,b) = log2(e) / (sigma_z |grad z . step (a,b)| + eps_z) (12
// distinct values per pixel, the offsets pairing up as +-(a,b)) and
// kl = log2(e) / (sigma_l kappa sqrt(g) + eps_l).  A tap outside the image
// or on an empty pixel is staged with luminance +inf and zero colour,
// variance, depth and normal, which drives its exponent to -inf (weight 0)
// without a branch.
#include "sv_internal.h"

namespace sv {

struct AtrousArgs {
    const void *cr, *cg, *cb;
    const float *var;
    const void *z, *dzdx, *dzdy, *nx, *ny, *nz;
    const float *kappa;
    void *or_, *og, *ob;
    float *var_out;
    int w, h, pitch, step;
    float sigma_z, sigma_l, eps_z, eps_l, tm_k;
    NormalCoef nc;
    int inv_tm;
};

// Weight modes: every edge weight 1 (plain B3), or the full weight with the
// normal term off or on.
enum { kUnit = 3 };

// log2 of the B3-spline taps (1, 4, 6, 4, 1) / 16
__device__ constexpr float kLog2H1[5] = {-4.0f, -2.0f, -1.4150374992788438f, -2.0f, -4.0f};
__device__ constexpr float kH1[5] = {0.0625f, 0.25f, 0.375f, 0.25f, 0.0625f};
constexpr float kG3[3] = {0.25f, 0.5f, 0.25f};

// Index of the distinct depth denominator of offset (a, b): offsets +-(a,b)
// share one; the canonical one has b > 0, or b == 0 and a > 0.
// (Not recursive, so that it folds to a constant once the tap loops unroll.)
__host__ __device__ __forceinline__ constexpr int kz_index(int a, int b) {
    const bool flip = b < 0 || (b == 0 && a < 0);
    const int ca = flip ? -a : a, cb = flip ? -b : b;
    return cb == 0 ? ca - 1 : 2 + (cb - 1) * 5 + (ca + 2);
}
static_assert(kz_index(1, 0) == 0 && kz_index(-2, 0) == 1 && kz_index(-2, 1) == 2 &&
                  kz_index(2, -2) == 7 && kz_index(2, 2) == 11,
              "depth denominator indexing");

// 3x3 Gaussian of the variance around (x, y) over in-image, non-empty
// pixels, renormalised.  All nine loads are issued before any test.
template <typename T>
__device__ __forceinline__ float prefilter_global(const AtrousArgs &a, int x, int y) {
    float zq[9], vq[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int qx = x + i % 3 - 1, qy = y + i / 3 - 1;
        const bool in = qx >= 0 && qx < a.w && qy >= 0 && qy < a.h;
        const uint32_t q = in ? (uint32_t)qy * (uint32_t)a.pitch + (uint32_t)qx : (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
        zq[i] = in ? ldo<T>(a.z, q) : 0.f;
        vq[i] = ldf(a.var, q);
    }
    float s = 0.f, sw = 0.f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float k = empty_px(zq[i]) ? 0.f : kG3[i % 3] * kG3[i / 3];
        s = fmaf(k, vq[i], s);
        sw += k;
    }
    return s / sw;
}

__device__ __forceinline__ float luma_scale(const AtrousArgs &a, float g, uint32_t o) {
    const float kap = a.kappa ? ldf(a.kappa, o) : 1.0f;
    return kLog2e / fmaf(a.sigma_l * kap, sqrtf(g), a.eps_l);
}

struct Acc {
    float sw, sr, sg, sb, sv;
};

// One weighted tap (not the centre).  qc = (r, g, b, L), qg = (z, nx, ny, nz).
template <int MODE, bool WANT_VAR>
__device__ __forceinline__ void tap(Acc &acc, float4 qc, float4 qg, float qv, float log2h,
                                    float hconst, float kz, float zp, float lp, float nxp,
                                    float nyp, float nzp, float kl, const NormalCoef &nc) {
    float hw;
    if (MODE == kUnit) {
        hw = qg.x > 0.f ? hconst : 0.f;
    } else {
        float t = fmaf(-fabsf(zp - qg.x), kz, log2h);
        t = fmaf(-fabsf(lp - qc.w), kl, t);
        if (MODE != kNormalOff)
            t = add_normal_term<MODE>(t, chord2(nxp, nyp, nzp, qg.y, qg.z, qg.w), nc);
        hw = fast_exp2(t);
    }
    acc.sw += hw;
    acc.sr = fmaf(hw, qc.x, acc.sr);
    acc.sg = fmaf(hw, qc.y, acc.sg);
    acc.sb = fmaf(hw, qc.z, acc.sb);
    if (WANT_VAR) acc.sv = fmaf(hw * hw, qv, acc.sv);
}

template <typename T>
__device__ __forceinline__ void write_out(const AtrousArgs &a, uint32_t o, float r, float g,
                                          float b) {
    if (a.inv_tm) inv_tonemap(r, g, b, a.tm_k);
    sto<T>(a.or_, o, r);
    sto<T>(a.og, o, g);
    sto<T>(a.ob, o, b);
}

template <typename T>
__device__ __forceinline__ void pass_through(const AtrousArgs &a, uint32_t o, const void *r,
                                             const void *g, const void *b) {
    write_out<T>(a, o, ldo<T>(r, o), ldo<T>(g, o), ldo<T>(b, o));
    if (a.var_out) stf(a.var_out, o, 0.f);
}

// ---- 5x5 level, LDS tile ---------------------------------------------------
//
// A workgroup of 256 threads owns TX = 64 columns and TY = 4 * PY rows taken
// on the step lattice: rows ybase + j * STEP, j = 0..TY-1, with ybase = band
// * STEP * TY + phase.  All 25 taps of those pixels then lie in the tile's
// own lattice rows j - 2 .. j + TY + 1 and columns -2 STEP .. TX + 2 STEP,
// so the LDS footprint is (TY + 4) x (TX + 4 STEP) pixels whatever the step.
template <typename T, int STEP, int PY, int MODE, bool WANT_VAR>
__global__ __launch_bounds__(256) void atrous_tile_k(AtrousArgs a) {
    constexpr int TX = 64, TY = 4 * PY, ROWS = TY + 4, COLS = TX + 4 * STEP;
    // The 3x3 variance prefilter needs image rows y-1, y, y+1: inside the
    // tile for STEP 1, three extra staged rows per lattice row otherwise.
    constexpr bool PF_TILE = STEP == 1;
    constexpr bool NEED_V = WANT_VAR || PF_TILE;
    constexpr int PFC = TX + 2;
    __shared__ float4 s_cl[ROWS * COLS];  // r, g, b, L (L = +inf: no tap)
    __shared__ float4 s_gn[ROWS * COLS];  // z, nx, ny, nz (z = 0: no tap)
    __shared__ float s_v[NEED_V ? ROWS * COLS : 1];
    __shared__ float2 s_pf[PF_TILE ? 1 : TY * 3 * PFC];  // (var, 1) or (0, 0)
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TX;
    const int band = blockIdx.y / STEP, phase = blockIdx.y - band * STEP;
    const int ybase = band * STEP * TY + phase;

    for (int i = tid; i < ROWS * COLS; i += 256) {
        const int r = i / COLS, c = i - r * COLS;
        const int gx = x0 - 2 * STEP + c, gy = ybase + (r - 2) * STEP;
        float4 cl = make_float4(0.f, 0.f, 0.f, INFINITY);
        float4 gn = make_float4(0.f, 0.f, 0.f, 0.f);
        float v = 0.f;
        if (gx >= 0 && gx < a.w && gy >= 0 && gy < a.h) {
            const uint32_t o = (uint32_t)gy * (uint32_t)a.pitch + (uint32_t)gx;
            const float zz = ldo<T>(a.z, o);
            if (!empty_px(zz)) {
                const float R = ldo<T>(a.cr, o), G = ldo<T>(a.cg, o),
                            B = ldo<T>(a.cb, o);
                cl = make_float4(R, G, B, luma(R, G, B));
                gn = make_float4(zz, ldo<T>(a.nx, o), ldo<T>(a.ny, o),
                                 ldo<T>(a.nz, o));
                if (NEED_V) v = ldf(a.var, o);
            }
        }
        s_cl[i] = cl;
        s_gn[i] = gn;
        if (NEED_V) s_v[i] = v;
    }
    if (!PF_TILE) {
        for (int i = tid; i < TY * 3 * PFC; i += 256) {
            const int j = i / (3 * PFC), rem = i - j * (3 * PFC);
            const int r3 = rem / PFC, c = rem - r3 * PFC;
            const int gx = x0 - 1 + c, gy = ybase + j * STEP + r3 - 1;
            float2 e = make_float2(0.f, 0.f);
            if (gx >= 0 && gx < a.w && gy >= 0 && gy < a.h) {
                const uint32_t o = (uint32_t)gy * (uint32_t)a.pitch + (uint32_t)gx;
                if (!empty_px(ldo<T>(a.z, o))) e = make_float2(ldf(a.var, o), 1.f);
            }
            s_pf[i] = e;
        }
    }
    __syncthreads();

    const int lx = tid & 63, ly = tid >> 6;
    const int x = x0 + lx;
    if (x >= a.w) return;
#pragma unroll 1
    for (int k = 0; k < PY; ++k) {
        const int j = ly + 4 * k;
        const int y = ybase + j * STEP;
        if (y >= a.h) break;
        const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
        const int ci = (j + 2) * COLS + lx + 2 * STEP;
        const float4 pc = s_cl[ci];
        const float4 pg = s_gn[ci];
        if (pg.x == 0.f) {  // empty pixel
            pass_through<T>(a, o, a.cr, a.cg, a.cb);
            continue;
        }
        // prefiltered variance
        float g;
        if (STEP == 1) {
            float s = 0.f, sw = 0.f;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int qi = ci + dy * COLS + dx;
                    const float kk = s_gn[qi].x > 0.f ? kG3[dx + 1] * kG3[dy + 1] : 0.f;
                    s = fmaf(kk, s_v[qi], s);
                    sw += kk;
                }
            g = s / sw;
        } else {
            float s = 0.f, sw = 0.f;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const float2 e = s_pf[(j * 3 + dy) * PFC + lx + dx];
                    const float kk = e.y * (kG3[dx] * kG3[dy]);
                    s = fmaf(kk, e.x, s);
                    sw += kk;
                }
            g = s / sw;
        }
        float kz[12];
        float kl = 0.f;
        if (MODE != kUnit) {
            kl = luma_scale(a, g, o);
            const float gx = ldo<T>(a.dzdx, o) * (float)STEP;
            const float gy = ldo<T>(a.dzdy, o) * (float)STEP;
#pragma unroll
            for (int b = 0; b <= 2; ++b)
#pragma unroll
                for (int aa = -2; aa <= 2; ++aa) {
                    if (b == 0 && aa <= 0) continue;
                    const float den =
                        fmaf(a.sigma_z, fabsf(fmaf(gx, (float)aa, gy * (float)b)), a.eps_z);
                    kz[kz_index(aa, b)] = kLog2e * fast_rcp(den);
                }
        }
        constexpr float h00 = 0.375f * 0.375f;
        Acc acc;
        acc.sw = h00;
        acc.sr = h00 * pc.x;
        acc.sg = h00 * pc.y;
        acc.sb = h00 * pc.z;
        acc.sv = WANT_VAR ? h00 * h00 * s_v[ci] : 0.f;
#pragma unroll
        for (int b = -2; b <= 2; ++b)
#pragma unroll
            for (int aa = -2; aa <= 2; ++aa) {
                if (aa == 0 && b == 0) continue;
                const int qi = ci + b * COLS + aa * STEP;
                const float qv = WANT_VAR ? s_v[qi] : 0.f;
                tap<MODE, WANT_VAR>(acc, s_cl[qi], s_gn[qi], qv, kLog2H1[aa + 2] + kLog2H1[b + 2],
                                    kH1[aa + 2] * kH1[b + 2], MODE == kUnit ? 0.f : kz[kz_index(aa, b)],
                                    pg.x, pc.w, pg.y, pg.z, pg.w, kl, a.nc);
            }
        const float inv = 1.0f / acc.sw;
        write_out<T>(a, o, acc.sr * inv, acc.sg * inv, acc.sb * inv);
        if (WANT_VAR) stf(a.var_out, o, acc.sv * inv * inv);
    }
}

// ---- 5x5 level, direct loads (any step) -------------------------------------

template <typename T>
__device__ __forceinline__ void load_tap(const AtrousArgs &a, int qx, int qy, float4 &qc,
                                         float4 &qg, float &qv) {
    qc = make_float4(0.f, 0.f, 0.f, INFINITY);
    qg = make_float4(0.f, 0.f, 0.f, 0.f);
    qv = 0.f;
    if (qx < 0 || qx >= a.w || qy < 0 || qy >= a.h) return;
    const uint32_t q = (uint32_t)qy * (uint32_t)a.pitch + (uint32_t)qx;
    const float zz = ldo<T>(a.z, q);
    if (empty_px(zz)) return;
    const float R = ldo<T>(a.cr, q), G = ldo<T>(a.cg, q), B = ldo<T>(a.cb, q);
    qc = make_float4(R, G, B, luma(R, G, B));
    qg = make_float4(zz, ldo<T>(a.nx, q), ldo<T>(a.ny, q), ldo<T>(a.nz, q));
    qv = ldf(a.var, q);
}

template <typename T, int MODE, bool WANT_VAR>
__global__ __launch_bounds__(256) void atrous_direct_k(AtrousArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.w || y >= a.h) return;
    const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    float4 pc, pg;
    float pv;
    load_tap<T>(a, x, y, pc, pg, pv);
    if (pg.x == 0.f) {
        pass_through<T>(a, o, a.cr, a.cg, a.cb);
        return;
    }
    const float g = prefilter_global<T>(a, x, y);
    const float s = (float)a.step;
    float kz[12];
    float kl = 0.f;
    if (MODE != kUnit) {
        kl = luma_scale(a, g, o);
        const float gx = ldo<T>(a.dzdx, o) * s, gy = ldo<T>(a.dzdy, o) * s;
#pragma unroll
        for (int b = 0; b <= 2; ++b)
#pragma unroll
            for (int aa = -2; aa <= 2; ++aa) {
                if (b == 0 && aa <= 0) continue;
                const float den = fmaf(a.sigma_z, fabsf(fmaf(gx, (float)aa, gy * (float)b)), a.eps_z);
                kz[kz_index(aa, b)] = kLog2e * fast_rcp(den);
            }
    }
    constexpr float h00 = 0.375f * 0.375f;
    Acc acc{h00, h00 * pc.x, h00 * pc.y, h00 * pc.z, WANT_VAR ? h00 * h00 * pv : 0.f};
#pragma unroll
    for (int b = -2; b <= 2; ++b)
#pragma unroll
        for (int aa = -2; aa <= 2; ++aa) {
            if (aa == 0 && b == 0) continue;
            float4 qc, qg;
            float qv;
            load_tap<T>(a, x + aa * a.step, y + b * a.step, qc, qg, qv);
            tap<MODE, WANT_VAR>(acc, qc, qg, qv, kLog2H1[aa + 2] + kLog2H1[b + 2],
                                kH1[aa + 2] * kH1[b + 2], MODE == kUnit ? 0.f : kz[kz_index(aa, b)], pg.x,
                                pc.w, pg.y, pg.z, pg.w, kl, a.nc);
        }
    const float inv = 1.0f / acc.sw;
    write_out<T>(a, o, acc.sr * inv, acc.sg * inv, acc.sb * inv);
    if (WANT_VAR) stf(a.var_out, o, acc.sv * inv * inv);
}

// ---- separable level (Section 3.3), direct loads -------------------------------
//
// Horizontal pass: colour only, into the scratch planes (the args' output
// planes).  Vertical pass: reads the scratch planes as colour (cr/cg/cb) and
// var_in for the propagation; g comes from var_in in both.

template <typename T, int MODE, bool VERTICAL, bool WANT_VAR>
__global__ __launch_bounds__(256) void atrous_sep_k(AtrousArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.w || y >= a.h) return;
    const uint32_t o = (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x;
    float4 pc, pg;
    float pv;
    load_tap<T>(a, x, y, pc, pg, pv);
    if (pg.x == 0.f) {
        if (VERTICAL) {
            pass_through<T>(a, o, a.cr, a.cg, a.cb);
        } else {
            sto<T>(a.or_, o, ldo<T>(a.cr, o));
            sto<T>(a.og, o, ldo<T>(a.cg, o));
            sto<T>(a.ob, o, ldo<T>(a.cb, o));
        }
        return;
    }
    const float g = prefilter_global<T>(a, x, y);
    const float s = (float)a.step;
    float kz[2] = {0.f, 0.f};
    float kl = 0.f;
    if (MODE != kUnit) {
        kl = luma_scale(a, g, o);
        const float grad = ld((const T *)(VERTICAL ? a.dzdy : a.dzdx) + o) * s;
#pragma unroll
        for (int i = 1; i <= 2; ++i) {
            const float den = fmaf(a.sigma_z, fabsf(grad * (float)i), a.eps_z);
            kz[i - 1] = kLog2e * fast_rcp(den);
        }
    }
    constexpr float h0 = 0.375f;
    Acc acc{h0, h0 * pc.x, h0 * pc.y, h0 * pc.z, WANT_VAR ? h0 * h0 * pv : 0.f};
#pragma unroll
    for (int t = -2; t <= 2; ++t) {
        if (t == 0) continue;
        float4 qc, qg;
        float qv;
        const int qx = VERTICAL ? x : x + t * a.step, qy = VERTICAL ? y + t * a.step : y;
        load_tap<T>(a, qx, qy, qc, qg, qv);
        tap<MODE, WANT_VAR>(acc, qc, qg, qv, kLog2H1[t + 2], kH1[t + 2],
                            MODE == kUnit ? 0.f : kz[(t < 0 ? -t : t) - 1], pg.x, pc.w, pg.y, pg.z, pg.w,
                            kl, a.nc);
    }
    const float inv = 1.0f / acc.sw;
    if (VERTICAL) {
        write_out<T>(a, o, acc.sr * inv, acc.sg * inv, acc.sb * inv);
        if (WANT_VAR) stf(a.var_out, o, acc.sv * inv * inv);
    } else {
        sto<T>(a.or_, o, acc.sr * inv);
        sto<T>(a.og, o, acc.sg * inv);
        sto<T>(a.ob, o, acc.sb * inv);
    }
}

// ---- launch ---------------------------------------------------------------------

template <typename T, int STEP, int MODE, bool WANT_VAR>
static void launch_tile(const AtrousArgs &a, hipStream_t s) {
    constexpr int PY = 2, TY = 4 * PY;
    const int bands = (a.h + STEP * TY - 1) / (STEP * TY);
    dim3 grid((a.w + 63) / 64, bands * STEP);
    hipLaunchKernelGGL((atrous_tile_k<T, STEP, PY, MODE, WANT_VAR>), grid, dim3(256), 0, s, a);
}

template <typename T, int MODE, bool WANT_VAR>
static void launch_2d(const AtrousArgs &a, hipStream_t s) {
    switch (a.step) {
    case 1: launch_tile<T, 1, MODE, WANT_VAR>(a, s); return;
    case 2: launch_tile<T, 2, MODE, WANT_VAR>(a, s); return;
    case 4: launch_tile<T, 4, MODE, WANT_VAR>(a, s); return;
    case 8: launch_tile<T, 8, MODE, WANT_VAR>(a, s); return;
    case 16: launch_tile<T, 16, MODE, WANT_VAR>(a, s); return;
    default: {
        dim3 grid((a.w + 63) / 64, (a.h + 3) / 4);
        hipLaunchKernelGGL((atrous_direct_k<T, MODE, WANT_VAR>), grid, dim3(256), 0, s, a);
    }
    }
}

template <typename T, int MODE>
static void launch_2d_var(const AtrousArgs &a, hipStream_t s) {
    if (a.var_out) launch_2d<T, MODE, true>(a, s);
    else launch_2d<T, MODE, false>(a, s);
}

template <typename T>
static void dispatch_2d(const AtrousArgs &a, int mode, hipStream_t s) {
    switch (mode) {
    case kUnit: launch_2d_var<T, kUnit>(a, s); return;
    case kNormalOff: launch_2d_var<T, kNormalOff>(a, s); return;
    default: launch_2d_var<T, kNormalLog>(a, s); return;
    }
}

template <typename T, int MODE, bool VERTICAL>
static void launch_sep(const AtrousArgs &a, hipStream_t s) {
    dim3 grid((a.w + 63) / 64, (a.h + 3) / 4);
    if (VERTICAL && a.var_out)
        hipLaunchKernelGGL((atrous_sep_k<T, MODE, VERTICAL, true>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((atrous_sep_k<T, MODE, VERTICAL, false>), grid, dim3(256), 0, s, a);
}

template <typename T, bool VERTICAL>
static void dispatch_sep(const AtrousArgs &a, int mode, hipStream_t s) {
    switch (mode) {
    case kUnit: launch_sep<T, kUnit, VERTICAL>(a, s); return;
    case kNormalOff: launch_sep<T, kNormalOff, VERTICAL>(a, s); return;
    default: launch_sep<T, kNormalLog, VERTICAL>(a, s); return;
    }
}

static int weight_mode(const sv_atrous_params *p) {
    return (p->flags & SV_A_UNIT_WEIGHTS) ? kUnit : normal_mode(p->sigma_n);
}

static int check_atrous(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                        const float *kappa, const sv_rgb *scratch, const sv_rgb *c_out,
                        float *var_out, int32_t step, sv_dims d, sv_dtype t,
                        const sv_atrous_params *p, int *empty) {
    if (!valid_dtype(t)) return SV_EDTYPE;
    int dc = check_dims(d);
    if (dc < 0 || !c_in || !g || !c_out || !p || step < 1) return SV_EINVAL;
    if (!(p->sigma_n >= 0.f)) return SV_EINVAL;
    *empty = dc == 1;
    if (dc == 1) return SV_OK;
    if (!c_in->r || !c_in->g || !c_in->b || !var_in || !g->z || !g->dzdx || !g->dzdy || !g->nx ||
        !g->ny || !g->nz || !c_out->r || !c_out->g || !c_out->b)
        return SV_EINVAL;
    const size_t es = elem_size(t);
    const span ins[] = {plane_span(c_in->r, d, es), plane_span(c_in->g, d, es),
                        plane_span(c_in->b, d, es), plane_span(var_in, d, 4),
                        plane_span(g->z, d, es),    plane_span(g->dzdx, d, es),
                        plane_span(g->dzdy, d, es), plane_span(g->nx, d, es),
                        plane_span(g->ny, d, es),   plane_span(g->nz, d, es),
                        kappa ? plane_span(kappa, d, 4) : span{0, 0}};
    span outs[7];
    int no = 0;
    outs[no++] = plane_span(c_out->r, d, es);
    outs[no++] = plane_span(c_out->g, d, es);
    outs[no++] = plane_span(c_out->b, d, es);
    if (var_out) outs[no++] = plane_span(var_out, d, 4);
    if (scratch) {
        outs[no++] = plane_span(scratch->r, d, es);
        outs[no++] = plane_span(scratch->g, d, es);
        outs[no++] = plane_span(scratch->b, d, es);
    }
    for (int i = 0; i < no; ++i) {
        for (const span &si : ins)
            if (overlaps(outs[i], si)) return SV_EALIAS;
        for (int j = i + 1; j < no; ++j)
            if (overlaps(outs[i], outs[j])) return SV_EALIAS;
    }
    return SV_OK;
}

static AtrousArgs make_args(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                            const float *kappa, const sv_rgb *c_out, float *var_out,
                            int32_t step, sv_dims d, const sv_atrous_params *p) {
    return AtrousArgs{c_in->r, c_in->g, c_in->b, var_in, g->z, g->dzdx, g->dzdy, g->nx, g->ny,
                      g->nz, kappa, c_out->r, c_out->g, c_out->b, var_out, d.w, d.h, d.pitch,
                      step, p->sigma_z, p->sigma_l, p->eps_z, p->eps_l, p->tm_k,
                      make_normal_coef(p->sigma_n), (p->flags & SV_A_INV_TONEMAP) ? 1 : 0};
}

}  // namespace sv

extern "C" int sv_atrous(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                         const float *kappa, const sv_rgb *c_out, float *var_out, int32_t step,
                         sv_dims d, sv_dtype t, const sv_atrous_params *p, sv_stream stream) {
    using namespace sv;
    int empty = 0;
    int rc = check_atrous(c_in, var_in, g, kappa, nullptr, c_out, var_out, step, d, t, p, &empty);
    if (rc != SV_OK || empty) return rc;
    AtrousArgs a = make_args(c_in, var_in, g, kappa, c_out, var_out, step, d, p);
    const int mode = weight_mode(p);
    if (t == SV_F32) dispatch_2d<float>(a, mode, as_stream(stream));
    else dispatch_2d<half_t>(a, mode, as_stream(stream));
    return hip_status(hipGetLastError());
}

extern "C" int sv_atrous_sep(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                             const float *kappa, const sv_rgb *scratch, const sv_rgb *c_out,
                             float *var_out, int32_t step, sv_dims d, sv_dtype t,
                             const sv_atrous_params *p, sv_stream stream) {
    using namespace sv;
    if (!scratch) return SV_EINVAL;
    int empty = 0;
    int rc = check_atrous(c_in, var_in, g, kappa, scratch, c_out, var_out, step, d, t, p, &empty);
    if (rc != SV_OK || empty) return rc;
    if (!scratch->r || !scratch->g || !scratch->b) return SV_EINVAL;
    const int mode = weight_mode(p);
    hipStream_t s = as_stream(stream);
    // horizontal: c_in -> scratch (no variance, no inverse tone map)
    AtrousArgs h = make_args(c_in, var_in, g, kappa, scratch, nullptr, step, d, p);
    h.inv_tm = 0;
    // vertical: scratch -> c_out, variance from var_in
    AtrousArgs v = make_args(scratch, var_in, g, kappa, c_out, var_out, step, d, p);
    if (t == SV_F32) {
        dispatch_sep<float, false>(h, mode, s);
        dispatch_sep<float, true>(v, mode, s);
    } else {
        dispatch_sep<half_t, false>(h, mode, s);
        dispatch_sep<half_t, true>(v, mode, s);
    }
    return hip_status(hipGetLastError());
}
