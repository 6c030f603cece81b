// Edge-avoiding a-trous wavelet levels guided by the variance (Section 2,
// Fig. 1) in 5x5 form, and the separable form of Section 3.3.
//
// Every tap's weight H(a,b) * w_z * w_n * w_l is evaluated as one
// exponential: log2 H - |dz| kz(a,b) - |dL| kl + sigma_n log2 max(0, cos)
// (the normal term as in sv_internal.h),
// with kz(a,b) = log2(e) / (sigma_z |grad z . step (a,b)| + eps_z) (12
// distinct values per pixel, the offsets pairing up as +-(a,b); each one
// reciprocal, see depth_scale) and
// kl = log2(e) / (sigma_l kappa sqrt(g) + eps_l).  A tap outside the image
// or on an empty pixel is staged with luminance +inf and zero colour,
// variance, depth and normal, which drives its exponent to -inf (weight 0)
// without a branch.
#pragma once
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
    // adaptive levels (optional): per-pixel control bytes, this level's
    // index and which of its two launches this is; sr/sg/sb is the level's
    // input colour, which a pixel whose iteration budget is spent keeps
    const uint8_t *ctl;
    int ctl_level, ctl_class;
    const void *sr, *sg, *sb;
};

// Weight modes: every edge weight 1 (plain B3), or the full edge weights
// with the normal term in log form (add_normal_term) or, for large sigma_n,
// as a series (add_normal_series).
enum { kUnit = 0, kWeighted = 1, kWeightedSeries = 2 };

constexpr int kCUs = 256;

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

// Depth scale log2(e) / (sigma_z |d| + eps_z) of an offset whose depth
// difference p's gradient predicts as d, from szl, ezl = sigma_z ln 2,
// eps_z ln 2 (see depth_coefs): one fma and one reciprocal.
__device__ __forceinline__ float depth_scale(float d, float szl, float ezl) {
    return fast_rcp(fmaf(szl, fabsf(d), ezl));
}
__device__ __forceinline__ void depth_coefs(const AtrousArgs &a, float &szl, float &ezl) {
    szl = a.sigma_z * kLn2;
    ezl = a.eps_z * kLn2;
}

// grad z . (a, b) for the tile kernels' offsets: gx, gy are the gradient
// times the (power-of-two) step and a, b in {-2..2}, so both products are
// exact and the fma rounds once.  A term whose offset component is zero is
// left out rather than multiplied by zero.
__device__ __forceinline__ float grad_dot(float gx, float gy, int a, int b) {
    return b == 0 ? gx * (float)a : a == 0 ? gy * (float)b : fmaf(gx, (float)a, gy * (float)b);
}

// Mean s / sw of the 3x3 variance prefilter (sw > 0: the centre counts).
__device__ __forceinline__ float pf_mean(float s, float sw) { return quot(s, sw, fast_rcp(sw)); }

// Luminance scale log2(e) / (sigma_l kappa sqrt(g) + eps_l) from the
// prefiltered variance g >= 0, with the hardware square root and reciprocal
// (about an ulp each; a full-precision divide and square root cost some 25
// instructions per pixel, and g only sets the width of the weight).
__device__ __forceinline__ float lum_scale(float sl_kappa, float g, float eps_l) {
    return kLog2e * fast_rcp(fmaf(sl_kappa, __builtin_amdgcn_sqrtf(g), eps_l));
}

// 3x3 Gaussian of the variance around (x, y) over in-image, non-empty
// pixels, renormalised.  All nine loads are issued before any test.
template <typename T>
__device__ __forceinline__ float prefilter_global(const AtrousArgs &a, int x, int y) {
    float zq[9], vq[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int qx = x + i % 3 - 1, qy = y + i / 3 - 1;
        const bool in = qx >= 0 && qx < a.w && qy >= 0 && qy < a.h;
        const uint32_t q = vofs(in ? (uint32_t)qy * (uint32_t)a.pitch + (uint32_t)qx
                                   : (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x);
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
    return pf_mean(s, sw);
}

__device__ __forceinline__ float luma_scale(const AtrousArgs &a, float g, uint32_t o) {
    const float kap = a.kappa ? ldf(a.kappa, o) : 1.0f;
    return lum_scale(a.sigma_l * kap, g, a.eps_l);
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
        const float s2 = chord2(nxp, nyp, nzp, qg.y, qg.z, qg.w);
        t = MODE == kWeightedSeries ? add_normal_series(t, s2, nc) : add_normal_term(t, s2, nc);
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

// ---- adaptive levels ----------------------------------------------------------
//
// Control byte of pixel p: bits 0-3 the number of levels p takes part in
// (15: all), bit 4 set when p starts one level coarser (its level i uses
// step 2^(i+1)).  A 5x5 level up to kMaxStep2DA runs as one launch that
// picks each pixel's step (kDir2DA); otherwise as two launches over the
// whole image: class 0 at step 2^i writes the pixels without the shift and
// the pixels whose budget is spent (passed through), class 1 at step
// 2^(i+1) the shifted pixels.  Each pixel's output is written by exactly
// one of them.
// Returns 0 when the other launch writes o, 1 to filter it here, 2 to pass
// it through here.
__device__ __forceinline__ int ctl_select(const AtrousArgs &a, uint32_t o) {
    const uint32_t c = a.ctl[o];
    if (a.ctl_level >= (int)(c & 15u)) return a.ctl_class == 0 ? 2 : 0;
    return (int)((c >> 4) & 1u) == a.ctl_class ? 1 : 0;
}

// Whether any of the rows y0 + k * dy, k < rows, at this thread's column x
// holds a pixel that this launch writes: a uniform answer over the
// workgroup (every thread must call it), so that a launch skips the tiles
// of the other class before staging them.
__device__ __forceinline__ bool any_of_class(const AtrousArgs &a, int x, int y0, int dy,
                                             int rows) {
    bool mine = false;
    if (x < a.w)
        for (int k = 0; k < rows; ++k) {
            const int y = y0 + k * dy;
            if (y >= 0 && y < a.h)
                mine |= ctl_select(a, (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x) != 0;
        }
    return __syncthreads_or(mine) != 0;
}

// A pixel outside this level: colour and variance unchanged (the inverse
// tone map still applies on the last level).
template <typename T>
__device__ __forceinline__ void copy_through(const AtrousArgs &a, uint32_t o) {
    write_out<T>(a, o, ldo<T>(a.sr, o), ldo<T>(a.sg, o), ldo<T>(a.sb, o));
    if (a.var_out) stf(a.var_out, o, ldf(a.var, o));
}

// ---- a-trous level, LDS tile -------------------------------------------------
//
// One kernel for the 5x5 level (DIR 0) and the two passes of the separable
// level (DIR 1 horizontal, DIR 2 vertical).  A tile is TX = 64 columns by
// TY = 4 * PY rows taken on the step lattice: rows ybase + j * STEP,
// j = 0..TY-1, with ybase = band * STEP * TY + phase.  The taps of those
// pixels lie in the tile's own lattice rows (HY = 2 above and below, none
// for the horizontal pass) and columns (HX = 2 STEP left and right, none for
// the vertical pass), so the LDS footprint is (TY + 2 HY) x (TX + 2 HX)
// pixels whatever the step, plus the image rows above and below each
// lattice row (and the row itself where the tile holds no variance) for the
// 3x3 variance prefilter, unless the tile holds them all (step 1).
//
// The kernel is persistent: each workgroup walks a strided run of tiles of
// its XCD's contiguous range, and issues the global loads of its next tile
// into registers before computing the current one from LDS, so the memory
// latency of a tile hides behind the arithmetic of the previous one.
// kDir2DA: the 5x5 level of the adaptive blur in one launch, every pixel at
// its own step (the level's, or twice it when its control byte says so):
// the tile holds the halo of the doubled step (four lattice rows and
// columns of the level's step around it).
enum { kDir2D = 0, kDirH = 1, kDirV = 2, kDir2DA = 3 };
// Largest level step run as one adaptive launch: beyond it the doubled halo
// costs more LDS (so occupancy) than the second launch's staging.
constexpr int kMaxStep2DA = 8;

// Staged prefilter entry of a pixel outside the image or without a surface.
constexpr float kNoVar = __builtin_nanf("");

// The tile's variance entry of a pixel outside the image or without a
// surface is -0, which no other entry is: a pixel's own variance is staged
// plus +0, turning -0 into +0 and leaving every other value as it is.  The
// prefilter tells the two kinds apart from this 4-byte entry alone; reading
// the depth out of the 16-byte G-buffer entries instead strides the LDS
// banks four entries at a time and conflicts.  The taps need no test: an
// empty pixel's weight is exactly 0, and 0 * -0 adds nothing.
constexpr uint32_t kNoVarBits = 0x80000000u;
__device__ __forceinline__ bool tile_no_var(float e) { return __float_as_uint(e) == kNoVarBits; }

// Lattice rows per thread of a tile: two, except at the largest steps,
// where the 2 x step-column halo on each side would otherwise hold the
// tile's LDS footprint to two or three resident workgroups per CU (per
// 1080p level, step 16: 53 instead of 74 us; step 8: five workgroups
// instead of three, 53 instead of 55 us).  Step 32, the coarser start of
// the fifth level, takes a wider tile instead (see TileShape).
constexpr int tile_py(int step) { return step >= 8 ? 1 : 2; }

template <int STEP, int PY, int DIR, bool WANT_VAR>
struct TileShape {
    // lattice columns: 64 (one wave per lattice row), or 128 at step 32,
    // where the column halo (2 x 64 pixels) would otherwise be staged for
    // every 64 outputs (two waves per lattice row there: 12 % faster)
    static constexpr int WX = (DIR == kDir2D && STEP == 32) ? 2 : 1;
    static constexpr int TX = 64 * WX, RPP = 4 / WX, TY = RPP * PY;
    static constexpr int HALO = DIR == kDir2DA ? 4 : 2;
    static constexpr int HY = DIR == kDirH ? 0 : HALO, HX = DIR == kDirV ? 0 : HALO * STEP;
    static constexpr int ROWS = TY + 2 * HY, COLS = TX + 2 * HX;
    static constexpr int AMAX = DIR == kDirV ? 0 : 2, BMAX = DIR == kDirH ? 0 : 2;
    static constexpr bool PF_TILE = STEP == 1 && (DIR == kDir2D || DIR == kDir2DA);
    static constexpr bool NEED_V = WANT_VAR || PF_TILE;
    static constexpr int PFC = TX + 2;
    static constexpr int NS = ROWS * COLS, IT = (NS + 255) / 256;
    // prefilter rows staged per lattice row: the image rows above and below
    // it, and the row itself unless the tile already holds its variance
    // (with a column of halo on each side)
    static constexpr bool MID_TILE = !PF_TILE && NEED_V && HX >= 1;
    static constexpr int PFR = PF_TILE ? 0 : MID_TILE ? 2 : 3;
    static constexpr int NP = TY * PFR * PFC, ITP = (NP + 255) / 256;
    // LDS bytes of one workgroup, and the workgroups (one wave per SIMD
    // each) that fit a CU's 160 KiB: the register budget is set to match,
    // so registers never hold occupancy below what LDS allows
    static constexpr int LDS = NS * 32 + (NEED_V ? NS * 4 : 4) + (NP > 0 ? NP * 4 : 4);
    static constexpr int WAVES = 163840 / LDS < 8 ? 163840 / LDS : 8;
};

// Raw values of one tile held in registers between issue and LDS store.
template <int IT, int ITP>
struct TileRegs {
    float z[IT], r[IT], g[IT], b[IT], nx[IT], ny[IT], nz[IT], v[IT];
    bool in[IT];
    float pz[ITP > 0 ? ITP : 1], pv[ITP > 0 ? ITP : 1];
    bool pin[ITP > 0 ? ITP : 1];
};

struct TileOrigin {
    int x0, ybase;
};

template <int STEP, int TY, int TX>
__device__ __forceinline__ TileOrigin tile_origin(int tile, int gxt) {
    const int tyt = tile / gxt;  // band * STEP + phase
    const int band = tyt / STEP, phase = tyt - band * STEP;
    return TileOrigin{(tile - tyt * gxt) * TX, band * STEP * TY + phase};
}

// Issue every global load of a tile (addresses clamped into the image; a
// pixel outside reads pixel (0, 0) and is masked when stored).
template <typename T, class S, class R>
__device__ __forceinline__ void tile_issue(const AtrousArgs &a, TileOrigin t, R &g) {
    constexpr int STEP = S::HX == 0 ? 1 : S::HX / 2;  // only used for HX
#pragma unroll
    for (int it = 0; it < S::IT; ++it) {
        const int i = threadIdx.x + it * 256;
        const int r = i / S::COLS, c = i - r * S::COLS;
        const int gx = t.x0 - S::HX + c;
        const int gy = t.ybase + (r - S::HY) * a.step;
        const bool in = i < S::NS && gx >= 0 && gx < a.w && gy >= 0 && gy < a.h;
        const uint32_t o = vofs(in ? (uint32_t)gy * (uint32_t)a.pitch + (uint32_t)gx : 0u);
        g.in[it] = in;
        g.z[it] = ldo<T>(a.z, o);
        g.r[it] = ldo<T>(a.cr, o);
        g.g[it] = ldo<T>(a.cg, o);
        g.b[it] = ldo<T>(a.cb, o);
        g.nx[it] = ldo<T>(a.nx, o);
        g.ny[it] = ldo<T>(a.ny, o);
        g.nz[it] = ldo<T>(a.nz, o);
        g.v[it] = S::NEED_V ? ldf(a.var, o) : 0.f;
    }
    (void)STEP;
#pragma unroll
    for (int it = 0; it < S::ITP; ++it) {
        const int i = threadIdx.x + it * 256;
        constexpr int PR = S::PFR > 0 ? S::PFR * S::PFC : 1;  // (no rows: no iteration)
        const int j = i / PR, rem = i - j * PR;
        const int rr = rem / S::PFC, c = rem - rr * S::PFC;
        const int dy = S::PFR == 3 ? rr - 1 : 2 * rr - 1;  // image rows -1, (0,) +1
        const int gx = t.x0 - 1 + c, gy = t.ybase + j * a.step + dy;
        const bool in = i < S::NP && gx >= 0 && gx < a.w && gy >= 0 && gy < a.h;
        const uint32_t o = vofs(in ? (uint32_t)gy * (uint32_t)a.pitch + (uint32_t)gx : 0u);
        g.pin[it] = in;
        g.pz[it] = ldo<T>(a.z, o);
        g.pv[it] = ldf(a.var, o);
    }
}

template <class S, class R>
__device__ __forceinline__ void tile_store(const R &g, float4 *s_cl, float4 *s_gn, float *s_v,
                                           float *s_pf) {
#pragma unroll
    for (int it = 0; it < S::IT; ++it) {
        const int i = threadIdx.x + it * 256;
        if (i < S::NS) {
            const bool ok = g.in[it] && !empty_px(g.z[it]);
            s_cl[i] = ok ? make_float4(g.r[it], g.g[it], g.b[it], luma(g.r[it], g.g[it], g.b[it]))
                         : make_float4(0.f, 0.f, 0.f, INFINITY);
            s_gn[i] = ok ? make_float4(g.z[it], g.nx[it], g.ny[it], g.nz[it])
                         : make_float4(0.f, 0.f, 0.f, 0.f);
            if (S::NEED_V) s_v[i] = ok ? g.v[it] + 0.0f : __uint_as_float(kNoVarBits);
        }
    }
#pragma unroll
    for (int it = 0; it < S::ITP; ++it) {
        const int i = threadIdx.x + it * 256;
        if (i < S::NP) s_pf[i] = (g.pin[it] && !empty_px(g.pz[it])) ? g.pv[it] : kNoVar;
    }
}

template <typename T, int STEP, int PY, int MODE, bool WANT_VAR, int DIR>
__device__ __forceinline__ void tile_compute(const AtrousArgs &a, TileOrigin t,
                                             const float4 *s_cl, const float4 *s_gn,
                                             const float *s_v, const float *s_pf) {
    using S = TileShape<STEP, PY, DIR, WANT_VAR>;
    constexpr int COLS = S::COLS, HY = S::HY, HX = S::HX, PFC = S::PFC;
    const int lx = (int)threadIdx.x % S::TX, ly = (int)threadIdx.x / S::TX;
    const int x = t.x0 + lx;
    if (x >= a.w) return;
#pragma unroll 1
    for (int k = 0; k < PY; ++k) {
        const int j = ly + S::RPP * k;
        const int y = t.ybase + j * STEP;
        if (y >= a.h) break;
        const uint32_t o = vofs((uint32_t)y * (uint32_t)a.pitch + (uint32_t)x);
        // the adaptive level in one launch: a pixel whose budget is spent
        // keeps its input, a shifted one takes every tap at twice the step
        int m = 1;
        if (DIR == kDir2DA) {
            const uint32_t c = a.ctl[o];
            if (a.ctl_level >= (int)(c & 15u)) {
                copy_through<T>(a, o);
                continue;
            }
            m = (c & 16u) ? 2 : 1;
        } else if (DIR != kDirH && a.ctl) {  // uniform branch
            const int sel = ctl_select(a, o);
            if (sel != 1) {
                if (sel == 2) copy_through<T>(a, o);
                continue;
            }
        }
        const int ci = (j + HY) * COLS + lx + HX;
        const float4 pc = s_cl[ci];
        const float4 pg = s_gn[ci];
        if (pg.x == 0.f) {  // empty pixel
            if (DIR == kDirH) {
                sto<T>(a.or_, o, ldo<T>(a.cr, o));
                sto<T>(a.og, o, ldo<T>(a.cg, o));
                sto<T>(a.ob, o, ldo<T>(a.cb, o));
            } else {
                pass_through<T>(a, o, a.cr, a.cg, a.cb);
            }
            continue;
        }
        // prefiltered variance
        float g;
        {
            float s = 0.f, sw = 0.f;
            if (S::PF_TILE) {
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) {
                        const float e = s_v[ci + dy * COLS + dx];
                        const float kk = tile_no_var(e) ? 0.f : kG3[dx + 1] * kG3[dy + 1];
                        s = fmaf(kk, e, s);  // 0 * -0 adds nothing
                        sw += kk;
                    }
            } else {
#pragma unroll
                for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        // the lattice row's own entries come from the tile
                        // (-0 there: outside or empty)
                        const int qi = ci + dx - 1;
                        const int pr = S::MID_TILE ? (dy == 0 ? 0 : 1) : dy;
                        const float e = S::MID_TILE && dy == 1
                                            ? (tile_no_var(s_v[qi]) ? kNoVar : s_v[qi])
                                            : s_pf[(j * S::PFR + pr) * PFC + lx + dx];
                        const bool ok = e == e;  // kNoVar: outside or empty
                        const float kk = ok ? kG3[dx] * kG3[dy] : 0.f;
                        s = fmaf(kk, ok ? e : 0.f, s);
                        sw += kk;
                    }
            }
            g = pf_mean(s, sw);
        }
        float kz[12];
        float kl = 0.f;
        if (MODE != kUnit) {
            kl = luma_scale(a, g, o);
            const float gx = DIR == kDirV ? 0.f : ldo<T>(a.dzdx, o) * (float)(STEP * m);
            const float gy = DIR == kDirH ? 0.f : ldo<T>(a.dzdy, o) * (float)(STEP * m);
            float szl, ezl;
            depth_coefs(a, szl, ezl);
#pragma unroll
            for (int b = 0; b <= 2; ++b)
#pragma unroll
                for (int aa = -2; aa <= 2; ++aa) {
                    if (b == 0 && aa <= 0) continue;
                    if ((DIR == kDirH && b != 0) || (DIR == kDirV && aa != 0)) continue;
                    kz[kz_index(aa, b)] = depth_scale(grad_dot(gx, gy, aa, b), szl, ezl);
                }
        }
        constexpr bool FULL = DIR == kDir2D || DIR == kDir2DA;
        constexpr float h0 = FULL ? 0.375f * 0.375f : 0.375f;
        Acc acc;
        acc.sw = h0;
        acc.sr = h0 * pc.x;
        acc.sg = h0 * pc.y;
        acc.sb = h0 * pc.z;
        acc.sv = WANT_VAR ? h0 * h0 * s_v[ci] : 0.f;
        // taps at lattice offsets (aa, b) times m: a shifted pixel of the
        // adaptive level (m = 2) takes the same instructions with a runtime
        // stride, so that a wave mixing both kinds does not run both
        const int rs = (DIR == kDir2DA ? m : 1) * COLS, cs = (DIR == kDir2DA ? m : 1) * STEP;
#pragma unroll
        for (int b = -S::BMAX; b <= S::BMAX; ++b)
#pragma unroll
            for (int aa = -S::AMAX; aa <= S::AMAX; ++aa) {
                if (aa == 0 && b == 0) continue;
                const int qi = ci + b * rs + aa * cs;
                const float qv = WANT_VAR ? s_v[qi] : 0.f;
                const float log2h = FULL ? kLog2H1[aa + 2] + kLog2H1[b + 2]
                                         : kLog2H1[(DIR == kDirH ? aa : b) + 2];
                const float hc = FULL ? kH1[aa + 2] * kH1[b + 2] : kH1[(DIR == kDirH ? aa : b) + 2];
                tap<MODE, WANT_VAR>(acc, s_cl[qi], s_gn[qi], qv, log2h, hc,
                                    MODE == kUnit ? 0.f : kz[kz_index(aa, b)], pg.x, pc.w, pg.y,
                                    pg.z, pg.w, kl, a.nc);
            }
        const float inv = fast_rcp(acc.sw);
        if (DIR == kDirH) {
            sto<T>(a.or_, o, quot(acc.sr, acc.sw, inv));
            sto<T>(a.og, o, quot(acc.sg, acc.sw, inv));
            sto<T>(a.ob, o, quot(acc.sb, acc.sw, inv));
        } else {
            write_out<T>(a, o, quot(acc.sr, acc.sw, inv), quot(acc.sg, acc.sw, inv),
                     quot(acc.sb, acc.sw, inv));
            if (WANT_VAR) stf(a.var_out, o, acc.sv * inv * inv);
        }
    }
}

template <typename T, int STEP, int PY, int MODE, bool WANT_VAR, int DIR, bool PERSIST>
__global__ __launch_bounds__(256) __attribute__((
    amdgpu_waves_per_eu(TileShape<STEP, PY, DIR, WANT_VAR>::WAVES))) void atrous_tile_k(AtrousArgs a, int tiles, int per_xcd) {
    using S = TileShape<STEP, PY, DIR, WANT_VAR>;
    __shared__ float4 s_cl[S::NS];  // r, g, b, L (L = +inf: no tap)
    __shared__ float4 s_gn[S::NS];  // z, nx, ny, nz (z = 0: no tap)
    __shared__ float s_v[S::NEED_V ? S::NS : 1];
    __shared__ float s_pf[S::NP > 0 ? S::NP : 1];  // var, or kNoVar
    const int gxt = (a.w + S::TX - 1) / S::TX;
    // this workgroup's run of tiles: its XCD's range, strided by the number
    // of workgroups on that XCD
    const int xcd = (int)blockIdx.x % kXCD, slot = (int)blockIdx.x / kXCD;
    const int nslot = (int)gridDim.x / kXCD;
    const int first = xcd * per_xcd, last = min(tiles, first + per_xcd);
    int t = first + slot;
    if (t >= last) return;
    TileRegs<S::IT, S::ITP> regs;
    if (!PERSIST) {  // one tile per workgroup: no prefetch registers live
        const TileOrigin o = tile_origin<STEP, S::TY, S::TX>(t, gxt);
        // adaptive levels: a tile without a pixel of this launch's class
        // is not staged at all (uniform branch)
        if ((DIR == kDir2D || DIR == kDirV) && a.ctl &&
            !any_of_class(a, o.x0 + (int)threadIdx.x % S::TX,
                          o.ybase + (int)threadIdx.x / S::TX * STEP, S::RPP * STEP, PY))
            return;
        tile_issue<T, S>(a, o, regs);
        tile_store<S>(regs, s_cl, s_gn, s_v, s_pf);
        __syncthreads();
        tile_compute<T, STEP, PY, MODE, WANT_VAR, DIR>(a, o, s_cl, s_gn, s_v, s_pf);
        return;
    }
    tile_issue<T, S>(a, tile_origin<STEP, S::TY, S::TX>(t, gxt), regs);
    tile_store<S>(regs, s_cl, s_gn, s_v, s_pf);
    __syncthreads();
    for (;;) {
        const int tn = t + nslot;
        if (tn < last) tile_issue<T, S>(a, tile_origin<STEP, S::TY, S::TX>(tn, gxt), regs);
        tile_compute<T, STEP, PY, MODE, WANT_VAR, DIR>(a, tile_origin<STEP, S::TY, S::TX>(t, gxt),
                                                       s_cl, s_gn, s_v, s_pf);
        if (tn >= last) break;
        __syncthreads();
        tile_store<S>(regs, s_cl, s_gn, s_v, s_pf);
        __syncthreads();
        t = tn;
    }
}

// Batched form: the tiles of many streams (each its own AtrousArgs), one
// tile per workgroup; every tile is staged and computed exactly as above.
template <typename T, int STEP, int PY, int MODE, bool WANT_VAR, int DIR>
__global__ __launch_bounds__(256) __attribute__((
    amdgpu_waves_per_eu(TileShape<STEP, PY, DIR, WANT_VAR>::WAVES))) void atrous_batch_k(const AtrousArgs *args, const int *prefix,
                                                      int n, int total) {
    using S = TileShape<STEP, PY, DIR, WANT_VAR>;
    __shared__ float4 s_cl[S::NS];
    __shared__ float4 s_gn[S::NS];
    __shared__ float s_v[S::NEED_V ? S::NS : 1];
    __shared__ float s_pf[S::NP > 0 ? S::NP : 1];
    int s = 0;
    const int lt = batch_tile(prefix, n, total, s);
    if (lt < 0) return;
    const AtrousArgs a = args[s];  // a copy: the kernel's stores cannot alias it
    const int gxt = (a.w + S::TX - 1) / S::TX;
    const TileOrigin o = tile_origin<STEP, S::TY, S::TX>(lt, gxt);
    if ((DIR == kDir2D || DIR == kDirV) && a.ctl &&
        !any_of_class(a, o.x0 + (int)threadIdx.x % S::TX, o.ybase + (int)threadIdx.x / S::TX * STEP,
                      S::RPP * STEP, PY))
        return;
    TileRegs<S::IT, S::ITP> regs;
    tile_issue<T, S>(a, o, regs);
    tile_store<S>(regs, s_cl, s_gn, s_v, s_pf);
    __syncthreads();
    tile_compute<T, STEP, PY, MODE, WANT_VAR, DIR>(a, o, s_cl, s_gn, s_v, s_pf);
}

template <typename T, int STEP, int PY, int MODE, bool WANT_VAR, int DIR>
void atrous_batch_launch(const void *args, const int *prefix, int n, int total, hipStream_t s) {
    hipLaunchKernelGGL((atrous_batch_k<T, STEP, PY, MODE, WANT_VAR, DIR>), dim3(xcd_grid(total)),
                       dim3(256), 0, s, (const AtrousArgs *)args, prefix, n, total);
}

// ---- 5x5 level, direct loads (any step) -------------------------------------

template <typename T>
__device__ __forceinline__ void load_tap(const AtrousArgs &a, int qx, int qy, float4 &qc,
                                         float4 &qg, float &qv) {
    qc = make_float4(0.f, 0.f, 0.f, INFINITY);
    qg = make_float4(0.f, 0.f, 0.f, 0.f);
    qv = 0.f;
    if (qx < 0 || qx >= a.w || qy < 0 || qy >= a.h) return;
    const uint32_t q = vofs((uint32_t)qy * (uint32_t)a.pitch + (uint32_t)qx);
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
    const uint32_t o = vofs((uint32_t)y * (uint32_t)a.pitch + (uint32_t)x);
    if (a.ctl) {
        const int sel = ctl_select(a, o);
        if (sel != 1) {
            if (sel == 2) copy_through<T>(a, o);
            return;
        }
    }
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
        // any step here: the offsets step (a, b) are integers, but their
        // products with the gradient need not be exact (see grad_offset)
        const float gx = ldo<T>(a.dzdx, o), gy = ldo<T>(a.dzdy, o);
        float szl, ezl;
        depth_coefs(a, szl, ezl);
#pragma unroll
        for (int b = 0; b <= 2; ++b)
#pragma unroll
            for (int aa = -2; aa <= 2; ++aa) {
                if (b == 0 && aa <= 0) continue;
                kz[kz_index(aa, b)] =
                    depth_scale(grad_offset(gx, gy, s * (float)aa, s * (float)b), szl, ezl);
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
    const float inv = fast_rcp(acc.sw);
    write_out<T>(a, o, quot(acc.sr, acc.sw, inv), quot(acc.sg, acc.sw, inv),
                     quot(acc.sb, acc.sw, inv));
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
    const uint32_t o = vofs((uint32_t)y * (uint32_t)a.pitch + (uint32_t)x);
    if (VERTICAL && a.ctl) {
        const int sel = ctl_select(a, o);
        if (sel != 1) {
            if (sel == 2) copy_through<T>(a, o);
            return;
        }
    }
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
        const float grad = ld((const T *)(VERTICAL ? a.dzdy : a.dzdx) + o);
        float szl, ezl;
        depth_coefs(a, szl, ezl);
#pragma unroll
        for (int i = 1; i <= 2; ++i) kz[i - 1] = depth_scale(grad * (s * (float)i), szl, ezl);
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
    const float inv = fast_rcp(acc.sw);
    if (VERTICAL) {
        write_out<T>(a, o, quot(acc.sr, acc.sw, inv), quot(acc.sg, acc.sw, inv),
                     quot(acc.sb, acc.sw, inv));
        if (WANT_VAR) stf(a.var_out, o, acc.sv * inv * inv);
    } else {
        sto<T>(a.or_, o, quot(acc.sr, acc.sw, inv));
        sto<T>(a.og, o, quot(acc.sg, acc.sw, inv));
        sto<T>(a.ob, o, quot(acc.sb, acc.sw, inv));
    }
}

// ---- separable level, both passes fused -------------------------------------
//
// One wave owns 64 columns and walks hv_rows(STEP) + 4 lattice rows of one step
// phase (image rows ph + j * STEP).  Each row is staged once in LDS for the
// horizontal pass, its loads issued two rows ahead; the horizontal results
// of the last five rows live in a register ring (slot = row mod 5, static
// after unrolling by ten), which is exactly the vertical pass's 5-tap
// window for the row two behind.  (A 256-thread tile form with both passes
// in LDS, one or two lattice rows per thread and a persistent prefetching
// variant all measured 5-30 % slower than this walker.)  The
// horizontal result is rounded to the storage type as the scratch planes
// of the two-pass form would round it, and every weight, sum and order is
// that of the two passes, so the output is bitwise theirs.  The level
// reads the G-buffer and colour once and writes only its outputs.
// Output rows per wave: 16 at the small steps; 6 from step 8, whose wider
// halo makes a wave's rows costlier, so that more, shorter waves hide their
// latency better (measured at 1080p: 53 instead of 58 us per level at steps
// 8 and 16, but 55-58 instead of 48-50 us at steps 1-4).
constexpr int hv_rows(int step) { return step >= 8 ? 6 : 16; }

template <int STEP, int OUT_ = hv_rows(STEP)>
struct HvShape {
    static constexpr int TX = 64, HX = 2 * STEP, COLS = TX + 2 * HX, PFC = TX + 2;
    static constexpr int IT = (COLS + 63) / 64, ITP = (3 * PFC + 63) / 64;
    static constexpr int OUT = OUT_, ROWS = OUT + 4;
    static_assert(ROWS % 10 == 0, "rows per tile must fill the five-slot ring and the two load buffers");
};

template <int STEP>
struct HvRow {  // one lattice row's loads, held between issue and LDS store
    float r[HvShape<STEP>::IT], g[HvShape<STEP>::IT], b[HvShape<STEP>::IT];
    float z[HvShape<STEP>::IT], nx[HvShape<STEP>::IT], ny[HvShape<STEP>::IT],
        nz[HvShape<STEP>::IT];
    // in-image flags as 0/1 in VGPRs: held over two rows, lane masks would
    // take two scalar registers each and spill
    uint32_t in[HvShape<STEP>::IT];
    float pz[HvShape<STEP>::ITP], pv[HvShape<STEP>::ITP];
    uint32_t pin[HvShape<STEP>::ITP];
    float dzdx, dzdy, kap;  // this lane's pixel
};

template <typename T>
__device__ __forceinline__ float round_to(float v) {
    return (float)(T)v;
}

template <typename T, int STEP>
__device__ __forceinline__ void hv_issue(const AtrousArgs &a, int x0, int y, HvRow<STEP> &q) {
    using S = HvShape<STEP>;
    const int lx = threadIdx.x;
    const bool yin = y >= 0 && y < a.h;
#pragma unroll
    for (int it = 0; it < S::IT; ++it) {
        const int i = lx + it * 64;
        const int gx = x0 - S::HX + i;
        const bool in = i < S::COLS && yin && gx >= 0 && gx < a.w;
        const uint32_t o = vofs(in ? (uint32_t)y * (uint32_t)a.pitch + (uint32_t)gx : 0u);
        q.in[it] = vofs(in ? 1u : 0u);
        q.z[it] = ldo<T>(a.z, o);
        q.r[it] = ldo<T>(a.cr, o);
        q.g[it] = ldo<T>(a.cg, o);
        q.b[it] = ldo<T>(a.cb, o);
        q.nx[it] = ldo<T>(a.nx, o);
        q.ny[it] = ldo<T>(a.ny, o);
        q.nz[it] = ldo<T>(a.nz, o);
    }
#pragma unroll
    for (int it = 0; it < S::ITP; ++it) {
        const int i = lx + it * 64;
        const int rr = i / S::PFC, c = i - rr * S::PFC;
        const int gx = x0 - 1 + c, gy = y + rr - 1;
        const bool in = i < 3 * S::PFC && gx >= 0 && gx < a.w && gy >= 0 && gy < a.h;
        const uint32_t o = vofs(in ? (uint32_t)gy * (uint32_t)a.pitch + (uint32_t)gx : 0u);
        q.pin[it] = vofs(in ? 1u : 0u);
        q.pz[it] = ldo<T>(a.z, o);
        q.pv[it] = ldf(a.var, o);
    }
    const int x = x0 + lx;
    const uint32_t o = vofs((yin && x < a.w) ? (uint32_t)y * (uint32_t)a.pitch + (uint32_t)x : 0u);
    q.dzdx = ldo<T>(a.dzdx, o);
    q.dzdy = ldo<T>(a.dzdy, o);
    q.kap = a.kappa ? ldf(a.kappa, o) : 1.0f;
}

template <int STEP>
__device__ __forceinline__ void hv_store(const HvRow<STEP> &q, float4 *s_cl, float4 *s_gn,
                                         float2 *s_pf) {
    using S = HvShape<STEP>;
    const int lx = threadIdx.x;
#pragma unroll
    for (int it = 0; it < S::IT; ++it) {
        const int i = lx + it * 64;
        if (i < S::COLS) {
            const bool ok = q.in[it] != 0u && !empty_px(q.z[it]);
            s_cl[i] = ok ? make_float4(q.r[it], q.g[it], q.b[it], luma(q.r[it], q.g[it], q.b[it]))
                         : make_float4(0.f, 0.f, 0.f, INFINITY);
            s_gn[i] = ok ? make_float4(q.z[it], q.nx[it], q.ny[it], q.nz[it])
                         : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
#pragma unroll
    for (int it = 0; it < S::ITP; ++it) {
        const int i = lx + it * 64;
        if (i < 3 * S::PFC)
            s_pf[i] = (q.pin[it] != 0u && !empty_px(q.pz[it])) ? make_float2(q.pv[it], 1.f)
                                                         : make_float2(0.f, 0.f);
    }
}

// One slot of the ring: a row's horizontal result at this lane's column
// and what the vertical pass needs of that pixel.
struct HvSlot {
    float4 c;   // r, g, b (rounded to the storage type), L (+inf: not a tap)
    float4 gn;  // z (0: not a tap), normal
    float v;    // input variance (0 when not a tap)
    float g;    // prefiltered variance
    float dzdy, kap;
};

template <typename T, int STEP, int OUT, int MODE, int SLOT>
__device__ __forceinline__ void hv_row(const AtrousArgs &ah, const AtrousArgs &av, int x0, int ph,
                                       int j0, int ro, HvSlot (&ring)[5], float4 *s_cl,
                                       float4 *s_gn, float2 *s_pf, HvRow<STEP> &q) {
    using S = HvShape<STEP, OUT>;
    // packed: MODE & 1 = weights, MODE & 2 = variance, MODE & 4 = series normal term
    constexpr bool WANT_VAR = (MODE & 2) != 0;
    constexpr int WM = (MODE & 1) ? ((MODE & 4) ? kWeightedSeries : kWeighted) : kUnit;
    const int lx = threadIdx.x, x = x0 + lx;
    const int r = ro + SLOT;  // row index within the tile
    const int y = ph + (j0 - 2 + r) * STEP;
    // stage this row (its loads were issued two rows ago), then start
    // loading the row after next into the same registers
    __syncthreads();
    hv_store<STEP>(q, s_cl, s_gn, s_pf);
    __syncthreads();
    const float dzdx = q.dzdx, dzdy = q.dzdy, kap = q.kap;
    if (r + 2 < S::ROWS) hv_issue<T, STEP>(ah, x0, ph + (j0 + r) * STEP, q);
    // ---- horizontal pass at (x, y) ----
    HvSlot &cur = ring[SLOT % 5];
    const int ci = lx + S::HX;
    const float4 pc = s_cl[ci], pg = s_gn[ci];
    cur.gn = pg;
    cur.v = s_pf[S::PFC + lx + 1].x;
    cur.dzdy = dzdy;
    cur.kap = kap;
    {
        float s = 0.f, sw = 0.f;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const float2 e = s_pf[dy * S::PFC + lx + dx];
                const float kk = e.y * (kG3[dx] * kG3[dy]);
                s = fmaf(kk, e.x, s);
                sw += kk;
            }
        cur.g = pf_mean(s, sw);
    }
    if (pg.x == 0.f) {
        // not a tap; an empty pixel inside the image passes its colour on
        cur.c = make_float4(pc.x, pc.y, pc.z, INFINITY);
        if (y >= 0 && y < ah.h && x < ah.w) {
            const uint32_t o = vofs((uint32_t)y * (uint32_t)ah.pitch + (uint32_t)x);
            cur.c.x = ldo<T>(ah.cr, o);
            cur.c.y = ldo<T>(ah.cg, o);
            cur.c.z = ldo<T>(ah.cb, o);
        }
    } else {
        float kz[2] = {0.f, 0.f};
        float kl = 0.f;
        if (WM != kUnit) {
            kl = lum_scale(ah.sigma_l * kap, cur.g, ah.eps_l);
            const float gx = dzdx * (float)STEP;
            float szl, ezl;
            depth_coefs(ah, szl, ezl);
#pragma unroll
            for (int aa = 1; aa <= 2; ++aa)
                kz[aa - 1] = depth_scale(grad_dot(gx, 0.f, aa, 0), szl, ezl);
        }
        constexpr float h0 = 0.375f;
        Acc acc;
        acc.sw = h0;
        acc.sr = h0 * pc.x;
        acc.sg = h0 * pc.y;
        acc.sb = h0 * pc.z;
        acc.sv = 0.f;
#pragma unroll
        for (int aa = -2; aa <= 2; ++aa) {
            if (aa == 0) continue;
            const int qi = ci + aa * STEP;
            tap<WM, false>(acc, s_cl[qi], s_gn[qi], 0.f, kLog2H1[aa + 2], kH1[aa + 2],
                           WM == kUnit ? 0.f : kz[(aa < 0 ? -aa : aa) - 1], pg.x, pc.w, pg.y, pg.z,
                           pg.w, kl, ah.nc);
        }
        const float inv = fast_rcp(acc.sw);
        const float hr = round_to<T>(quot(acc.sr, acc.sw, inv)),
                    hg = round_to<T>(quot(acc.sg, acc.sw, inv)),
                    hb = round_to<T>(quot(acc.sb, acc.sw, inv));
        cur.c = make_float4(hr, hg, hb, luma(hr, hg, hb));
    }
    // ---- vertical pass for the row two behind ----
    if (r < 4) return;
    constexpr int CS = (SLOT + 3) % 5;  // centre: row r - 2 (slot (r - 2) mod 5)
    const HvSlot &cen = ring[CS];
    const int yc = ph + (j0 - 4 + r) * STEP;
    if (x >= av.w || yc >= av.h) return;
    const uint32_t o = vofs((uint32_t)yc * (uint32_t)av.pitch + (uint32_t)x);
    if (av.ctl) {
        const int sel = ctl_select(av, o);
        if (sel != 1) {
            if (sel == 2) copy_through<T>(av, o);
            return;
        }
    }
    if (cen.gn.x == 0.f) {  // empty pixel: pass through
        write_out<T>(av, o, cen.c.x, cen.c.y, cen.c.z);
        if (av.var_out) stf(av.var_out, o, 0.f);
        return;
    }
    float kz[2] = {0.f, 0.f};
    float kl = 0.f;
    if (WM != kUnit) {
        kl = lum_scale(av.sigma_l * cen.kap, cen.g, av.eps_l);
        const float gy = cen.dzdy * (float)STEP;
        float szl, ezl;
        depth_coefs(av, szl, ezl);
#pragma unroll
        for (int b = 1; b <= 2; ++b) kz[b - 1] = depth_scale(grad_dot(0.f, gy, 0, b), szl, ezl);
    }
    constexpr float h0 = 0.375f;
    Acc acc;
    acc.sw = h0;
    acc.sr = h0 * cen.c.x;
    acc.sg = h0 * cen.c.y;
    acc.sb = h0 * cen.c.z;
    acc.sv = WANT_VAR ? h0 * h0 * cen.v : 0.f;
#pragma unroll
    for (int b = -2; b <= 2; ++b) {
        if (b == 0) continue;
        const HvSlot &qs = ring[(SLOT + 3 + b) % 5];
        tap<WM, WANT_VAR>(acc, qs.c, qs.gn, qs.v, kLog2H1[b + 2], kH1[b + 2],
                          WM == kUnit ? 0.f : kz[(b < 0 ? -b : b) - 1], cen.gn.x, cen.c.w,
                          cen.gn.y, cen.gn.z, cen.gn.w, kl, av.nc);
    }
    const float inv = fast_rcp(acc.sw);
    write_out<T>(av, o, quot(acc.sr, acc.sw, inv), quot(acc.sg, acc.sw, inv),
                 quot(acc.sb, acc.sw, inv));
    if (WANT_VAR) stf(av.var_out, o, acc.sv * inv * inv);
}

// Arguments of the fused level: those of its vertical pass (outputs,
// variance output, inverse tone map, adaptive control).  The horizontal
// pass reads the same input colour, variance and G-buffer from them and
// no output field, so one struct serves both passes (two copies overflow
// the kernel's scalar registers, and the spilled arguments cost VALU
// reloads in every row).
typedef AtrousArgs HvArgs;

inline int hv_tiles(const AtrousArgs &a, int rows) {
    return ((a.w + 63) / 64) * a.step * ((((a.h + a.step - 1) / a.step) + rows - 1) / rows);
}

// Tile t: 64 columns x hv_rows(STEP) lattice rows of one phase (columns fastest,
// then phases, then bands of rows).  MODE: bit 0 = edge weights on,
// bit 1 = variance output, bit 2 = the normal term as a series.
template <typename T, int STEP, int OUT, int MODE>
__device__ __forceinline__ void hv_tile(const HvArgs &a, int t, float4 *s_cl, float4 *s_gn,
                                        float2 *s_pf) {
    using S = HvShape<STEP, OUT>;
    const int gxt = (a.w + 63) / 64;
    const int cx = t % gxt, rest = t / gxt;
    const int ph = rest % STEP, band = rest / STEP;
    const int x0 = cx * 64, j0 = band * S::OUT;
    // adaptive levels: a tile without a pixel of this launch's class is
    // skipped (uniform branch)
    if (a.ctl && !any_of_class(a, x0 + (int)threadIdx.x, ph + j0 * STEP, STEP, S::OUT))
        return;
    HvSlot ring[5];
    HvRow<STEP> q0, q1;  // even and odd rows' loads, two rows in flight
    hv_issue<T, STEP>(a, x0, ph + (j0 - 2) * STEP, q0);
    hv_issue<T, STEP>(a, x0, ph + (j0 - 1) * STEP, q1);
    // ten rows per iteration: each ring slot and each load buffer a fixed
    // register set
#pragma unroll 1
    for (int ro = 0; ro < S::ROWS; ro += 10) {
        hv_row<T, STEP, OUT, MODE, 0>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q0);
        hv_row<T, STEP, OUT, MODE, 1>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q1);
        hv_row<T, STEP, OUT, MODE, 2>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q0);
        hv_row<T, STEP, OUT, MODE, 3>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q1);
        hv_row<T, STEP, OUT, MODE, 4>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q0);
        hv_row<T, STEP, OUT, MODE, 5>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q1);
        hv_row<T, STEP, OUT, MODE, 6>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q0);
        hv_row<T, STEP, OUT, MODE, 7>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q1);
        hv_row<T, STEP, OUT, MODE, 8>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q0);
        hv_row<T, STEP, OUT, MODE, 9>(a, a, x0, ph, j0, ro, ring, s_cl, s_gn, s_pf, q1);
    }
}

template <typename T, int STEP, int OUT, int MODE>
__global__ __launch_bounds__(64) void atrous_hv_k(HvArgs a, int tiles) {
    using S = HvShape<STEP, OUT>;
    __shared__ float4 s_cl[S::COLS];
    __shared__ float4 s_gn[S::COLS];
    __shared__ float2 s_pf[3 * S::PFC];
    const int t = xcd_tile(tiles);
    if (t < 0) return;
    hv_tile<T, STEP, OUT, MODE>(a, t, s_cl, s_gn, s_pf);
}

template <typename T, int STEP, int OUT, int MODE>
__global__ __launch_bounds__(64) void atrous_hv_batch_k(const HvArgs *args, const int *prefix,
                                                        int n, int total) {
    using S = HvShape<STEP, OUT>;
    __shared__ float4 s_cl[S::COLS];
    __shared__ float4 s_gn[S::COLS];
    __shared__ float2 s_pf[3 * S::PFC];
    int s = 0;
    const int lt = batch_tile(prefix, n, total, s);
    if (lt < 0) return;
    const HvArgs a = args[s];
    hv_tile<T, STEP, OUT, MODE>(a, lt, s_cl, s_gn, s_pf);
}

template <typename T, int STEP, int OUT, int MODE>
void hv_batch_launch(const void *args, const int *prefix, int n, int total, hipStream_t s) {
    hipLaunchKernelGGL((atrous_hv_batch_k<T, STEP, OUT, MODE>), dim3(xcd_grid(total)), dim3(64),
                       0, s, (const HvArgs *)args, prefix, n, total);
}

template <typename T, int STEP, int OUT, int MODE>
void launch_hv_mode(const HvArgs &a, hipStream_t s) {
    const int tiles = hv_tiles(a, OUT);
    if (record_pass(&hv_batch_launch<T, STEP, OUT, MODE>, a, tiles)) return;
    hipLaunchKernelGGL((atrous_hv_k<T, STEP, OUT, MODE>), dim3(xcd_grid(tiles)), dim3(64), 0, s,
                       a, tiles);
}

template <typename T, int STEP, int OUT>
void launch_hv_rows(const HvArgs &a, int mode, hipStream_t s) {
    switch (mode) {
    case 0: launch_hv_mode<T, STEP, OUT, 0>(a, s); return;
    case 1: launch_hv_mode<T, STEP, OUT, 1>(a, s); return;
    case 2: launch_hv_mode<T, STEP, OUT, 2>(a, s); return;
    case 3: launch_hv_mode<T, STEP, OUT, 3>(a, s); return;
    case 5: launch_hv_mode<T, STEP, OUT, 5>(a, s); return;
    default: launch_hv_mode<T, STEP, OUT, 7>(a, s); return;
    }
}

template <typename T, int STEP>
void launch_hv_step(const HvArgs &a, int mode, int rows, hipStream_t s) {
    if ((rows == 0 ? hv_rows(STEP) : rows) == 6) launch_hv_rows<T, STEP, 6>(a, mode, s);
    else launch_hv_rows<T, STEP, 16>(a, mode, s);
}

// Fused separable level; false when the step has no fused form (then the
// two passes run through a scratch buffer).  rows: output rows per wave,
// 6 or 16 (0: hv_rows(step)).
template <typename T>
bool launch_hv(const HvArgs &a, bool unit, int rows, hipStream_t s) {
    const int mode = (unit ? 0 : (a.nc.series ? 5 : 1)) | (a.var_out ? 2 : 0);
    switch (a.step) {
    case 1: launch_hv_step<T, 1>(a, mode, rows, s); return true;
    case 2: launch_hv_step<T, 2>(a, mode, rows, s); return true;
    case 4: launch_hv_step<T, 4>(a, mode, rows, s); return true;
    case 8: launch_hv_step<T, 8>(a, mode, rows, s); return true;
    case 16: launch_hv_step<T, 16>(a, mode, rows, s); return true;
    case 32: launch_hv_step<T, 32>(a, mode, rows, s); return true;
    default: return false;
    }
}

// ---- launch ---------------------------------------------------------------------

// Launch-time tile configuration (autotuned by the caller, or the defaults).
// rows: lattice rows per thread of the 5x5 level's tile, 1 or 2 (0: tile_py).
struct TileCfg {
    bool persistent;
    int blocks_per_cu;
    int rows;
};

template <typename T, int STEP, int PY, int MODE, bool WANT_VAR, int DIR>
void launch_tile_py(const AtrousArgs &a, TileCfg cfg, hipStream_t s) {
    using S = TileShape<STEP, PY, DIR, WANT_VAR>;
    constexpr int TY = S::TY;
    const int bands = (a.h + STEP * TY - 1) / (STEP * TY);
    const int tiles = ((a.w + S::TX - 1) / S::TX) * bands * STEP;
    const int per_xcd = (tiles + kXCD - 1) / kXCD;
    if (record_pass(&atrous_batch_launch<T, STEP, PY, MODE, WANT_VAR, DIR>, a, tiles)) return;
    // the adaptive level's wider tile leaves no registers for a prefetched
    // next tile: it always runs one tile per workgroup
    if constexpr (DIR != kDir2DA) {
        if (cfg.persistent) {
            const int slots = min(per_xcd, kCUs / kXCD * max(1, cfg.blocks_per_cu));
            hipLaunchKernelGGL((atrous_tile_k<T, STEP, PY, MODE, WANT_VAR, DIR, true>),
                               dim3(slots * kXCD), dim3(256), 0, s, a, tiles, per_xcd);
            return;
        }
    }
    hipLaunchKernelGGL((atrous_tile_k<T, STEP, PY, MODE, WANT_VAR, DIR, false>),
                       dim3(per_xcd * kXCD), dim3(256), 0, s, a, tiles, per_xcd);
}

// The tile height: the caller's choice for 5x5 levels up to step 16; at
// step 32 (the adaptive level's coarser start) the 128-column tile with two
// rows per thread (78 KB of LDS, as many workgroups per CU as the 64-column
// one-row tile); tile_py otherwise.
template <typename T, int STEP, int MODE, bool WANT_VAR, int DIR>
void launch_tile(const AtrousArgs &a, TileCfg cfg, hipStream_t s) {
    if constexpr (DIR == kDir2DA) {  // two rows per thread (measured best at every step)
        launch_tile_py<T, STEP, 2, MODE, WANT_VAR, DIR>(a, cfg, s);
    } else if constexpr (DIR == kDir2D && STEP == 32) {  // the 128-column tile, two rows
        launch_tile_py<T, STEP, 2, MODE, WANT_VAR, DIR>(a, cfg, s);
    } else {
        const int py = (DIR == kDir2D && STEP <= 16 && cfg.rows > 0) ? cfg.rows : tile_py(STEP);
        if (py == 1) launch_tile_py<T, STEP, 1, MODE, WANT_VAR, DIR>(a, cfg, s);
        else launch_tile_py<T, STEP, (STEP <= 16 ? 2 : 1), MODE, WANT_VAR, DIR>(a, cfg, s);
    }
}

template <typename T, int MODE, bool WANT_VAR, int DIR>
void launch_steps(const AtrousArgs &a, TileCfg cfg, hipStream_t s) {
    if constexpr (DIR == kDir2DA) {  // steps up to kMaxStep2DA
        switch (a.step) {
        case 1: launch_tile<T, 1, MODE, WANT_VAR, DIR>(a, cfg, s); return;
        case 2: launch_tile<T, 2, MODE, WANT_VAR, DIR>(a, cfg, s); return;
        case 4: launch_tile<T, 4, MODE, WANT_VAR, DIR>(a, cfg, s); return;
        case 8:
            if constexpr (kMaxStep2DA >= 8) launch_tile<T, 8, MODE, WANT_VAR, DIR>(a, cfg, s);
            return;
        default: return;
        }
    } else {
        switch (a.step) {
        case 1: launch_tile<T, 1, MODE, WANT_VAR, DIR>(a, cfg, s); return;
        case 2: launch_tile<T, 2, MODE, WANT_VAR, DIR>(a, cfg, s); return;
        case 4: launch_tile<T, 4, MODE, WANT_VAR, DIR>(a, cfg, s); return;
        case 8: launch_tile<T, 8, MODE, WANT_VAR, DIR>(a, cfg, s); return;
        case 16: launch_tile<T, 16, MODE, WANT_VAR, DIR>(a, cfg, s); return;
        case 32: launch_tile<T, 32, MODE, WANT_VAR, DIR>(a, cfg, s); return;
        default: {  // other steps: direct loads (not available batched)
            if (record_pass<AtrousArgs>(nullptr, a, 0)) return;
            dim3 grid((a.w + 63) / 64, (a.h + 3) / 4);
            if (DIR == kDir2D)
                hipLaunchKernelGGL((atrous_direct_k<T, MODE, WANT_VAR>), grid, dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((atrous_sep_k<T, MODE, DIR == kDirV, WANT_VAR>), grid,
                                   dim3(256), 0, s, a);
        }
        }
    }
}

// One pass (5x5 level, or one half of a separable level) for storage type T.
template <typename T, int DIR>
void launch_pass(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s) {
    const bool wv = a.var_out != nullptr && DIR != kDirH;
    if (unit) {
        if (wv) launch_steps<T, kUnit, true, DIR>(a, cfg, s);
        else launch_steps<T, kUnit, false, DIR>(a, cfg, s);
    } else {
        if (a.nc.series) {
            if (wv) launch_steps<T, kWeightedSeries, true, DIR>(a, cfg, s);
            else launch_steps<T, kWeightedSeries, false, DIR>(a, cfg, s);
        } else {
            if (wv) launch_steps<T, kWeighted, true, DIR>(a, cfg, s);
            else launch_steps<T, kWeighted, false, DIR>(a, cfg, s);
        }
    }
}

// Entry points of the per-(type, direction) compilation units.
void launch_pass_f32_2d(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s);
void launch_pass_f32_h(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s);
void launch_pass_f32_v(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s);
void launch_pass_f16_2d(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s);
void launch_pass_f16_h(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s);
void launch_pass_f16_v(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s);
void launch_pass_f32_2da(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s);
void launch_pass_f16_2da(const AtrousArgs &a, bool unit, TileCfg cfg, hipStream_t s);
bool launch_hv_f32(const HvArgs &a, bool unit, int rows, hipStream_t s);
bool launch_hv_f16(const HvArgs &a, bool unit, int rows, hipStream_t s);

}  // namespace sv
