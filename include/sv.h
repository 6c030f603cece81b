/*
 * sv.h - C ABI of the MI355X (gfx950) SVGF-style denoiser.
 *
 * The calls follow the denoiser of "Hybrid-Rendering Techniques in GPU"
 * (Granja & Pereira, 2021): Reinhard tone map before denoising and its
 * inverse after (Section 3.4); a temporal filter with backward reprojection,
 * variance colour clamping of the history and accumulation of colour and
 * luminance moments (Sections 2, 3 step 4, 3.1); a variance estimate
 * (Section 2); and the edge-avoiding a-trous wavelet filter guided by that
 * variance, in 5x5 form (Section 2, Fig. 1) and in separable form
 * (Section 3.3).  The paper names these operations without formulas; the
 * formulas implemented are those of spatiotemporal variance-guided
 * filtering, which Section 2 cites, with the readings stated per call.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Images are planes (structure of arrays), row-major.  Every plane of a
 *    call has the same width w, height h and row pitch (in ELEMENTS of the
 *    plane's own type, pitch >= w).  Pixel (x, y) of plane P is P[y*pitch+x].
 *  - Colour planes and G-buffer planes have the call's storage type
 *    (SV_F32: float, SV_F16: IEEE binary16).  Moments (m1, m2), variance,
 *    kappa and alpha maps are always float; history lengths and object ids
 *    are always uint8_t.  All arithmetic is binary32.
 *  - Every pointer is a DEVICE pointer to memory the caller owns and keeps
 *    alive until the work on the stream has finished.  The library never
 *    allocates, frees or retains them and keeps no state between calls.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default
 *    stream) and the call returns without synchronising.
 *  - Arguments are checked on the host before any HIP call; on failure
 *    nothing is enqueued and a status below is returned.  w == 0 or h == 0
 *    is a valid empty call that enqueues nothing.  Limits: w, h <= 32768,
 *    pitch * h <= 2^29 (every byte offset into a plane then fits in 32
 *    bits); larger sizes return SV_EINVAL.
 *  - A pixel is EMPTY (no surface) when its depth z is not > 0 or not
 *    finite.  Empty pixels pass their colour through, get zero moments,
 *    variance and history length, and are never used as neighbours.
 *  - Stencil calls (clamp, temporal, variance, a-trous) read neighbours:
 *    their outputs must not overlap any input plane (SV_EALIAS).
 *  - Results are deterministic: a fixed summation order per pixel.  The
 *    atomics the library uses decide no value: the variance pass appends
 *    short-history pixels to its list with one atomic add per workgroup
 *    (the list's order changes, each pixel's estimate does not), and the
 *    temporal gradient takes the lowest colliding stratum with an atomic
 *    minimum.
 *  - Luminance is L(c) = 0.2126 r + 0.7152 g + 0.0722 b (Rec. 709).
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ----------------------------------------------------- */
enum {
    SV_OK = 0,
    SV_EINVAL = 1,      /* null required pointer, bad size, pitch, step, param */
    SV_EALIAS = 2,      /* an output overlaps an input of a stencil call */
    SV_EDTYPE = 3,      /* unknown storage type */
    SV_EHIP = 4,        /* the HIP runtime reported an error on launch */
    SV_EUNSUPPORTED = 5, /* valid but not implemented combination */
    SV_ETOOBIG = 6       /* larger than the fixed workspace of sv_variance_noalloc */
};

typedef void *sv_stream; /* a hipStream_t */

typedef struct {
    int32_t w, h;  /* image size in pixels */
    int32_t pitch; /* row pitch in elements, >= w */
} sv_dims;

typedef enum { SV_F32 = 0, SV_F16 = 1 } sv_dtype;

/* Three colour planes.  Inputs are only read through these pointers. */
typedef struct {
    void *r, *g, *b;
} sv_rgb;

/* G-buffer of one frame (Section 3 step 2): view depth z (> 0 for a
 * surface), its screen gradients dz/dx and dz/dy in depth units per pixel,
 * unit normal (nx, ny, nz), and an optional object id (may be NULL). */
typedef struct {
    const void *z, *dzdx, *dzdy, *nx, *ny, *nz;
    const uint8_t *id;
} sv_gbuf;

/* ---- Reinhard tone map (Section 3.4) ----------------------------------- */
typedef enum {
    SV_TM_LUMA = 0,    /* forward c/(1 + k L(c)); inverse c/(1 - k L(c)) */
    SV_TM_CHANNEL = 1, /* forward c/(1 + k c) per channel; inverse c/(1 - k c) */
    SV_TM_PAPER = 2    /* inverse only: the listing's c (1 + L(c)) weight */
} sv_tm_mode;

typedef struct {
    float k;      /* luminance multiplier (lumaMultiplier), default 1 */
    float weight; /* reinhardToneMappingWeight, SV_TM_PAPER only */
    int32_t mode; /* sv_tm_mode */
} sv_tm_params;

/* Pointwise tone map (inverse = 0) or its inverse (inverse = 1) of `in`
 * into `out`; in place (out == in) is allowed.  The forward map divides the
 * radiance by 1 + k L(c) as the paper's listing does.  Its exact inverse
 * c' / (1 - k L(c')) is the default "remove" step (the denominator is
 * floored at 2^-20); the listing's own c' (1 + L(c')) w, which is not an
 * inverse, is available as SV_TM_PAPER.  Returns SV_EINVAL for null planes
 * or p == NULL, SV_EUNSUPPORTED for SV_TM_PAPER forward. */
int sv_tonemap(const sv_rgb *in, const sv_rgb *out, sv_dims d, sv_dtype t,
               int inverse, const sv_tm_params *p, sv_stream stream);

/* ---- variance colour clamp (Sections 2, 3.1) -------------------------- */

/* History rectification by variance colour clamping.  For each pixel the
 * mean mu and the population standard deviation sigma (two-pass) of `cur`
 * over its 3x3 neighbourhood (pixels inside the image and, if z != NULL,
 * not empty) are computed per channel, and `hist` is clamped to
 * [mu - gamma sigma, mu + gamma sigma] into `out`.  gamma <= 0 copies.
 * `z` (storage type, may be NULL) marks empty pixels.  `out` may equal
 * `hist` but must not overlap `cur`. */
int sv_clamp(const sv_rgb *hist, const sv_rgb *cur, const sv_rgb *out,
             const void *z, sv_dims d, sv_dtype t, float gamma,
             sv_stream stream);

/* History rectification by variance colour clipping, the alternative that
 * Section 3.1 tested beside the clamp.  Same box as sv_clamp (centre mu,
 * half-widths gamma sigma per channel); a history colour h outside it is
 * moved toward mu along the segment from mu onto the box's surface:
 * mu + t (h - mu) with t the smallest gamma sigma_c / |h_c - mu_c| over the
 * channels outside the box (a channel with zero spread and a nonzero
 * deviation gives mu).  A colour inside the box, an empty centre pixel and
 * gamma <= 0 copy.  Box statistics and the segment are evaluated in
 * binary64.  Arguments, aliasing rules and errors as sv_clamp. */
int sv_clip(const sv_rgb *hist, const sv_rgb *cur, const sv_rgb *out,
            const void *z, sv_dims d, sv_dtype t, float gamma,
            sv_stream stream);

/* ---- temporal filter (Section 2; Section 3 step 4; Section 3.1) -------- */
enum {
    SV_T_CLAMP = 1,     /* clamp the reprojected history (gamma > 0) */
    SV_T_USE_ID = 2,    /* object ids of the taps must match */
    SV_T_TONEMAP_IN = 4, /* forward tone map (LUMA, tm_k) the current colour */
    SV_T_CLIP = 8        /* clip the reprojected history (gamma > 0) as sv_clip
                            does; not together with SV_T_CLAMP */
};

typedef struct {
    sv_rgb cur;              /* current 1-spp colour */
    sv_gbuf g;               /* current G-buffer (dz/dx, dz/dy unused) */
    const void *mvx, *mvy;   /* backward motion in pixels: p was at p + mv */
    sv_gbuf prev;            /* previous frame's z, normal, id */
    sv_rgb hist;             /* colour history (previous output) */
    const float *hist_m1;    /* luminance moment history E[L] */
    const float *hist_m2c;   /* central moment history E[L^2] - E[L]^2 */
    const uint8_t *hist_n;   /* history length, 0 = none */
    sv_rgb out;              /* accumulated colour */
    float *out_m1, *out_m2c; /* accumulated moments (m2c central) */
    uint8_t *out_n;          /* new history length */
    const float *alpha_map;  /* optional per-pixel colour alpha (NULL) */
    /* Learned mode (optional): with `mlp` set, the per-pixel network of
     * sv_mlp_forward runs inside the step on the features sv_mlp_features
     * would write (needs g.dzdx, g.dzdy and albedo) and its alpha replaces
     * the colour blend factor (alpha_map is ignored); its kappa is written
     * to kappa_out and its alpha to alpha_out when given (binary32 planes).
     * Bitwise the same as sv_mlp_features + sv_mlp_forward + sv_temporal
     * with that alpha as alpha_map. */
    const struct sv_mlp_s *mlp;
    sv_rgb albedo;
    float *kappa_out, *alpha_out;
    /* Variance estimate, first part (optional): with `var` set, var =
     * max(0, m2c) is written where the new history length is >= var_min_hist
     * (0 for empty pixels), and the pixels with a shorter history are
     * listed in `var_work` (an sv_variance workspace); sv_variance with
     * SV_V_LISTED then does the rest.  Bitwise the same as sv_variance
     * alone. */
    float *var;
    void *var_work;
    int32_t var_min_hist;
} sv_temporal_io;

typedef struct {
    float alpha;     /* colour blend weight, default 0.2 */
    float alpha_m;   /* moment blend weight, default 0.2 */
    float gamma;     /* clamp box half-width in sigmas, default 1 */
    float tau_z;     /* relative depth tolerance, default 0.1 */
    float tau_n;     /* normal cosine threshold, default 0.9 */
    float tm_k;      /* tone-map multiplier for SV_T_TONEMAP_IN, default 1 */
    int32_t max_hist;/* history length cap, 1..255, default 255 */
    int32_t flags;   /* SV_T_* */
} sv_temporal_params;

/* One temporal step, fused.  The luminance moments are the exponential
 * moving averages of L and L^2 that the method accumulates; the second one
 * is kept as the central moment m2c = E[L^2] - E[L]^2 (the same
 * information, free of the cancellation E[L^2] - E[L]^2 suffers in
 * binary32).  Steps: (1) the current colour c, tone mapped if
 * SV_T_TONEMAP_IN; (2) backward reprojection: with x0 = x + floor(mvx),
 * fx = mvx - floor(mvx) (likewise y) the four history pixels around
 * p + mv are bilinear taps; a tap is usable if it is inside the image, its
 * history length is >= 1, |prev.z - z| <= tau_z z, prev.n . n >= tau_n
 * (and ids match under SV_T_USE_ID) - these tests are evaluated in binary32
 * as written, the cosine as fma(nz,nz', fma(ny,ny', nx*nx')); the usable
 * taps' bilinear weights are renormalised and the history length is the
 * largest among usable taps of positive weight; no usable tap (or |mv| not
 * finite or >= 2^20) discards the history; (3) with SV_T_CLAMP the
 * reprojected colour is clamped to the 3x3 mean +- gamma sigma of c, with
 * SV_T_CLIP clipped into that box as sv_clip does (both: SV_EINVAL);
 * (4) with n = min(n_hist + 1, max_hist), a = max(alpha, 1/n),
 * am = max(alpha_m, 1/n): out = (1-a) hist + a c, m1 = (1-am) m1_hist +
 * am L(c), m2c = (1-am) (m2c_hist + am (L(c) - m1_hist)^2), which is the
 * central form of the EMA (1-am) E[L^2] + am L^2; the reprojected m2c is
 * the bilinear mixture's central moment (taps' m2c plus the spread of
 * their m1).  A discarded history gives out = c, m1 = L, m2c = 0, n = 1.  alpha_map, if given, replaces alpha
 * per pixel.  Outputs must not overlap any input (SV_EALIAS).  Required:
 * cur, g.z, g.n*, mvx, mvy, prev.z, prev.n*, hist, hist_m1, hist_m2c,
 * hist_n, out, out_m1, out_m2c, out_n; ids when SV_T_USE_ID. */
int sv_temporal(const sv_temporal_io *io, sv_dims d, sv_dtype t,
                const sv_temporal_params *p, sv_stream stream);

/* ---- variance estimate (Section 2) ------------------------------------ */
typedef struct {
    float sigma_z;    /* depth weight scale, default 1 */
    float sigma_n;    /* normal weight exponent, default 128 */
    float eps_z;      /* depth weight epsilon, default 1e-10 */
    int32_t min_hist; /* history length for the temporal estimate, default 4 */
    int32_t radius;   /* spatial window radius, 0..7, default 3 */
    int32_t flags;    /* SV_V_* */
} sv_variance_params;

/* The long-history variance and the list of short-history pixels were
 * already written into var and work by sv_temporal (its var outputs, same
 * min_hist): only the spatial estimate of the listed pixels remains. */
#define SV_V_LISTED 1

/* Two passes: every pixel with n >= min_hist gets the temporal estimate and
 * the others are listed in `work`; a second pass spreads the listed pixels
 * over the whole GPU for the spatial estimate (they are few, about 1% in
 * steady motion, but clustered at disocclusions).
 * var = max(0, m2c) where n >= min_hist (m2c = E[L^2] - E[L]^2 as
 * sv_temporal writes it).  Where 1 <= n < min_hist the moments are averaged
 * over the (2 radius + 1)^2 window (inside the image, not empty) with
 * weight 1 at the centre and
 * exp(-|z(p)-z(q)| / (sigma_z |dzdx(p) dx + dzdy(p) dy| + eps_z))
 * * max(0, cos(n(p), n(q)))^sigma_n elsewhere (cosine of unit normals taken
 * as 1 - |n(p) - n(q)|^2 / 2), and var = weighted mean of m2c + weighted
 * spread of m1 about its weighted mean (floored at 0), the variance of the
 * mixture.  n == 0 or an empty pixel gives 0.  `var` must not overlap the
 * inputs. */
int sv_variance(const float *m1, const float *m2c, const uint8_t *n,
                const sv_gbuf *g, float *var, void *work, sv_dims d, sv_dtype t,
                const sv_variance_params *p, sv_stream stream);

/* Size in bytes of the `work` buffer sv_variance needs for dims d (0 for
 * invalid dims): eight lines of counters and a list of the short-history
 * pixels.  The caller allocates it on the device and ZEROES it before its
 * first use.  The counters are never reset: each listing pass (sv_variance,
 * or sv_temporal with var_work) appends after what the last sv_variance
 * read, and each sv_variance leaves them consistent for the next call, so
 * one buffer sized for the largest dims serves any number of calls of any
 * size, in order on one stream (calls that may run concurrently need one
 * buffer each).  A list sv_temporal wrote must be read by sv_variance with
 * SV_V_LISTED before the next listing pass.  It must not overlap any input
 * or `var`. */
size_t sv_variance_work_bytes(sv_dims d);

/* sv_variance without the `work` argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, rules and
 * results (bitwise) as sv_variance, minus `work`.  The workspace is a
 * fixed 32 MiB array in the library's device memory, one per GPU, held
 * until the process ends: calls whose sv_variance_work_bytes(d) exceeds
 * 32 MiB (33,554,432 bytes; 3840x2160 needs 33,178,624) return SV_ETOOBIG
 * without touching the GPU.  The first call on a device looks up that
 * device's copy of the array (with the device current).  Each call clears
 * the array's counters on `stream` before use; it calls no allocator.
 * Every call on one GPU uses the same array, so calls that may overlap on
 * one GPU (other streams, other threads) race: order them on one stream.
 * SV_V_LISTED is rejected (SV_EINVAL): a list sv_temporal wrote lives in
 * the caller's workspace.  SV_EHIP if the array's address cannot be had. */
int sv_variance_noalloc(const float *m1, const float *m2c, const uint8_t *n,
                        const sv_gbuf *g, float *var, sv_dims d, sv_dtype t,
                        const sv_variance_params *p, sv_stream stream);

/* ---- edge-avoiding a-trous level (Section 2, Fig. 1; Section 3.3) ------ */
enum {
    SV_A_UNIT_WEIGHTS = 1, /* every edge-stopping weight 1 (plain B3) */
    SV_A_INV_TONEMAP = 2   /* exact inverse LUMA tone map (tm_k) on output */
};

typedef struct {
    float sigma_z; /* default 1 */
    float sigma_n; /* default 128 */
    float sigma_l; /* default 4 */
    float eps_z;   /* default 1e-10 */
    float eps_l;   /* default 1e-10 */
    float tm_k;    /* tone-map multiplier for SV_A_INV_TONEMAP, default 1 */
    int32_t flags; /* SV_A_* */
    /* Launch shape of the LDS-tiled kernels (results do not depend on it):
     * persistent: -1 library default (one tile per workgroup), 0 one tile
     * per workgroup, 1 each
     * workgroup loops over tiles and prefetches the next one;
     * blocks_per_cu: workgroups per CU of a persistent launch (0 default);
     * tile_rows: the LDS tile's height.  5x5 levels: lattice rows per
     * thread, 1 or 2 (a tile of 64 x 4 tile_rows lattice rows); fused
     * separable levels: output rows per wave, 6 or 16.  0 = library default
     * (5x5: 2 up to step 4, 1 above; separable: 16 up to step 4, 6 above);
     * other values are SV_EINVAL. */
    int32_t persistent;
    int32_t blocks_per_cu;
    int32_t tile_rows;
} sv_atrous_params;

/* One level with hole spacing `step` (>= 1; 1, 2, 4, 8, 16 for the five
 * levels).  g(p) is the 3x3 Gaussian (1/4, 1/2, 1/4)^2 of var_in over
 * in-image, non-empty pixels, renormalised.  Over taps q = p + step (a, b),
 * a, b in -2..2, inside the image and not empty, with the B3-spline weights
 * H = h(a) h(b), h = (1, 4, 6, 4, 1)/16, and edge weights (1 at q = p)
 *   w = exp(-|z(p)-z(q)| / (sigma_z |dzdx(p) step a + dzdy(p) step b| + eps_z))
 *     * max(0, 1 - |n(p) - n(q)|^2 / 2)^sigma_n
 *     * exp(-|L(c(p)) - L(c(q))| / (sigma_l kappa(p) sqrt(g(p)) + eps_l)),
 * the output is c' = sum H w c(q) / sum H w and
 * var' = sum (H w)^2 var_in(q) / (sum H w)^2.  kappa may be NULL (1);
 * var_out may be NULL (not written, e.g. on the last level).  Outputs must
 * not overlap inputs. */
int sv_atrous(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
              const float *kappa, const sv_rgb *c_out, float *var_out,
              int32_t step, sv_dims d, sv_dtype t, const sv_atrous_params *p,
              sv_stream stream);

/* Separable level (Section 3.3): the 5x5 kernel split into a horizontal
 * pass of 5 taps (a, 0) and a vertical pass of 5 taps (0, b), 10 neighbour
 * visits instead of 25.  Both passes use g from var_in.  The horizontal
 * pass filters colour only; the vertical pass filters its result
 * (luminance taken from it, the result rounded to the storage type) and
 * alone updates the variance:
 * var' = sum (h(b) w)^2 var_in(q) / (sum h(b) w)^2.  Weights as sv_atrous
 * with the offset (step a, 0) or (0, step b).
 * With `scratch` (caller-owned planes of the storage type, same dims; must
 * not overlap inputs or outputs) the horizontal result is written there
 * and read back by a second kernel.  With scratch NULL both passes run in
 * one kernel and the horizontal result never leaves the chip (steps 1, 2,
 * 4, 8, 16, 32; other steps return SV_EUNSUPPORTED); the outputs are bitwise
 * those of the two-kernel form. */
int sv_atrous_sep(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                  const float *kappa, const sv_rgb *scratch,
                  const sv_rgb *c_out, float *var_out, int32_t step,
                  sv_dims d, sv_dtype t, const sv_atrous_params *p,
                  sv_stream stream);

/* ---- blur adapted to scene features (Sections 3.2, 3.5) ---------------- */

/* Per-pixel control byte of the adaptive levels: bits 0-3 the number of
 * levels the pixel takes part in (15: every level), bit 4 set when it
 * starts one level coarser, so that its level i uses step 2^(i+1) and its
 * first level equals the usual second one while the count stays the same
 * (Section 3.2).  Bits 5-7 must be 0. */
#define SV_CTL_LEVELS_MASK 15
#define SV_CTL_SHIFT 16

typedef struct {
    float rough_shift;  /* shift when roughness > this (0.2) */
    float angle_shift;  /* ... or when the shadow angle > this (6.0) */
    float rough_none;   /* roughness <= this: it_none levels (0.0) */
    float rough_one;    /* otherwise roughness <= this: it_one levels (0.05) */
    int32_t it_none, it_one, it_rest; /* 0, 1 and 15 (every level), 0..15 */
    int32_t flags;      /* SV_BR_SHIFT | SV_BR_TABLE */
} sv_blur_rule;

enum {
    SV_BR_SHIFT = 1, /* the coarser start of Section 3.2 */
    SV_BR_TABLE = 2  /* the roughness -> iteration count table of Section 3.5 */
};

/* Control bytes from per-pixel roughness and shadow angle (binary32
 * planes; either may be NULL when no rule uses it).  With SV_BR_SHIFT the
 * shift bit is (roughness > rough_shift) or (angle > angle_shift); with
 * SV_BR_TABLE the level count is it_none, it_one or it_rest by the
 * comparisons roughness <= rough_none, roughness <= rough_one in that
 * order, else 15.  Comparisons are binary32, as written (a NaN compares
 * false).  SV_EINVAL for a count outside 0..15, SV_BR_TABLE without
 * roughness, SV_BR_SHIFT with neither plane, or `ctl` overlapping them. */
int sv_blur_control(const float *roughness, const float *shadow_angle,
                    uint8_t *ctl, sv_dims d, const sv_blur_rule *r,
                    sv_stream stream);

/* One adaptive a-trous level `level` (0, 1, ...): pixel p with control
 * byte c is filtered at step 2^(level + shift(c)) exactly as sv_atrous
 * (separable = 0) or sv_atrous_sep (separable = 1) filters it, when
 * level < levels(c); otherwise its colour and variance pass through
 * unchanged (the inverse tone map of SV_A_INV_TONEMAP still applies).  A
 * shifted separable pixel takes the vertical pass of the horizontal result
 * at its own step.  A 5x5 level at step 2^level <= 8 is one launch, each
 * pixel taking its taps at its own step (p->persistent and tile_rows do
 * not apply there: tiles of 64 x 8 lattice rows, one per workgroup);
 * otherwise, and for separable levels, two launches over the image, one
 * per step, each pixel written by one.  `scratch`: as sv_atrous_sep,
 * separable only (NULL selects the fused form, steps up to 32, so levels
 * 0..4; SV_EUNSUPPORTED above).  `ctl` (one byte per pixel, pitch d.pitch) must not overlap the
 * outputs.  Other arguments and errors as sv_atrous; level outside 0..12
 * is SV_EINVAL. */
int sv_atrous_adaptive(const sv_rgb *c_in, const float *var_in,
                       const sv_gbuf *g, const float *kappa,
                       const uint8_t *ctl, const sv_rgb *scratch,
                       const sv_rgb *c_out, float *var_out, int32_t level,
                       int32_t separable, sv_dims d, sv_dtype t,
                       const sv_atrous_params *p, sv_stream stream);

/* ---- learned blend factor and edge scale ------------------------------
 *
 * Not in the paper, which blends with one fixed alpha and filters with one
 * fixed sigma_l (Section 2).  A per-pixel network predicts both:
 *
 *   x (14 features) -> 32 -> ReLU -> 32 -> ReLU -> (o1, o2)
 *   alpha = 0.05 + 0.95 sigmoid(o1)      (colour blend factor, sv_temporal
 *                                          alpha_map; the 1/n floor still
 *                                          applies)
 *   kappa = 2^(2 tanh(o2))               (sigma_l scale, sv_atrous kappa)
 *
 * Features, from the temporal step's own intermediates: luminance of the
 * current (tone-mapped) colour; luminance of the reprojected, clamped
 * history (0 without history); its reprojected central second moment (0
 * without history); the population variance of the current luminance over
 * the in-image, non-empty 3x3 neighbourhood; new history length / 255;
 * dz/dx; dz/dy; the normal (3); motion length (0 where the motion is
 * discarded); albedo (3).  Empty pixels have all-zero raw features.  Each
 * is standardised as (x - mu) * inv_s in binary32 and stored as bfloat16
 * (round to nearest even): one row of 16 values per pixel (the last two
 * zero), row index y * w + x, no pitch.
 *
 * Parameters, flat binary32 vector of SV_MLP_PARAMS in this order: W1
 * (32 x 14, row-major [out][in]), b1 (32), W2 (32 x 32), b2 (32), W3 (2 x 32),
 * b3 (2).  Matrix products take their operands as bfloat16 (weights from
 * the bfloat16 mirror `wq` of the flat vector, activations and, in the
 * backward pass, the incoming gradients rounded to nearest even) and
 * accumulate in binary32; biases are binary32. */
#define SV_MLP_IN 14
#define SV_MLP_HIDDEN 32
#define SV_MLP_PARAMS 1602

typedef struct sv_mlp_s {
    const float *params;    /* SV_MLP_PARAMS binary32 (biases read here) */
    const uint16_t *wq;     /* SV_MLP_PARAMS bfloat16 mirror (matrices read here) */
    const float *mu;        /* 14 feature means */
    const float *inv_s;     /* 14 inverse feature scales */
} sv_mlp;

/* Feature rows for sv_mlp_forward / sv_mlp_backward.  `io` supplies the
 * current frame, G-buffer (dzdx, dzdy required), motion, previous G-buffer
 * and history exactly as for sv_temporal with the same `p`; its outputs
 * and alpha_map are ignored.  `feat` receives w*h rows of 16 bfloat16
 * (32 bytes each, 16-byte aligned).  `hist_out` (optional, binary32 planes
 * with the call's pitch) receives the clamped reprojected history colour,
 * 0 where there is no history: the blend's other operand, needed by
 * sv_mlp_alpha_grad. */
int sv_mlp_features(const sv_temporal_io *io, const sv_rgb *albedo, const sv_mlp *w,
                    void *feat, const sv_rgb *hist_out, sv_dims d, sv_dtype t,
                    const sv_temporal_params *p, sv_stream stream);

/* Network forward over the w*h feature rows: alpha and kappa as binary32
 * planes with the pitch of d (either may be NULL). */
int sv_mlp_forward(const sv_mlp *w, const void *feat, float *alpha, float *kappa,
                   sv_dims d, sv_stream stream);

/* Gradient of L = sum over pixels of (d_alpha * alpha + d_kappa * kappa)
 * (binary32 planes with the pitch of d: dL/dalpha and dL/dkappa per pixel)
 * with respect to every parameter, times `scale`, written to `grad`
 * (SV_MLP_PARAMS binary32, flat order).  The forward pass is recomputed.
 * `work`: device buffer of sv_mlp_backward_work_bytes(d) bytes (per-wave
 * partial sums, reduced in a fixed order, so the result is deterministic). */
int sv_mlp_backward(const sv_mlp *w, const void *feat, const float *d_alpha,
                    const float *d_kappa, float scale, float *grad, void *work,
                    sv_dims d, sv_stream stream);
size_t sv_mlp_backward_work_bytes(sv_dims d);

typedef struct {
    float lr, beta1, beta2, eps; /* defaults 1e-3, 0.9, 0.999, 1e-8 */
} sv_adam_params;

/* One Adam step over n binary32 parameters (t counts from 1): m, v and the
 * master `params` are updated in place, and `wq` (optional) receives the
 * bfloat16 mirror of the new parameters. */
int sv_adam(float *params, uint16_t *wq, float *m, float *v, const float *grad, int32_t n,
            int32_t t, const sv_adam_params *p, sv_stream stream);

/* Per pixel, (2/3) sum_c (c_t - y) / (y^2 + 0.01) (cur - hist): with c_t
 * the temporal output, dL/dalpha of the per-pixel RelMSE term
 * (1/3) sum_c (c_t - y)^2 / (y^2 + 0.01) with the history held fixed
 * (c_t = (1 - a) hist + a cur, a = max(alpha, 1/n)); with c_t a later
 * colour (the chain's final output) the same local derivative weighted by
 * that colour's residual.  Zero where 1/n wins or the pixel is empty.
 * c_t: storage type; cur: the current colour, tone mapped here if
 * tm_k > 0; hist: sv_mlp_features' hist_out; y: target colour (binary32,
 * in the space of c_t); n: the new history length. */
int sv_mlp_alpha_grad(const sv_rgb *c_t, const sv_rgb *cur, const sv_rgb *hist,
                      const sv_rgb *y, const float *alpha, const uint8_t *n, const void *z,
                      float tm_k, float *d_alpha, sv_dims d, sv_dtype t, sv_stream stream);

/* Adds to d_kappa, per pixel, (2/3) sum_c r_c / (y_c^2 + 0.01) dc'_c/dkappa:
 * the local derivative of one 5x5 a-trous level's colour output c' with
 * respect to kappa(p), the level input held fixed,
 * dc'/dkappa = sum H (dw/dkappa) (c(q) - c') / sum H w (only the luminance
 * weight depends on kappa), times the residual r = c' - y of the level's
 * own output, or r = ref - y when `ref` (binary32 planes, optional) is
 * given - e.g. the chain's final output, so that every level's local
 * derivative is weighted by the error that reaches the end.  Arguments as
 * sv_atrous (no outputs; p's flags other than the sigmas and epsilons are
 * ignored); y is binary32. */
int sv_atrous_kappa_grad(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                         const float *kappa, const sv_rgb *y, const sv_rgb *ref,
                         float *d_kappa, int32_t step, sv_dims d, sv_dtype t,
                         const sv_atrous_params *p, sv_stream stream);

/* ---- temporal gradient (A-SVGF, related work of Section 2) ------------- */

/* The answer to temporal lag that the paper names: surface samples of the
 * previous frame are carried forward and traced again in the current frame
 * with their old random numbers, and the change of their shading raises
 * the temporal blend factor.  Readings (the paper gives no formulas):
 *  1. one sample per 3x3 stratum of the previous frame, pixel
 *     q = (3 sx + k % 3, 3 sy + k / 3), k = pick[sy * CW + sx] (0..8; a k
 *     above 8 or a q outside the image gives none); CW = ceil(w / 3),
 *     CH = ceil(h / 3);
 *  2. it lands on p = floor(q + fmv(q) + 1/2) (binary32 additions) if p is
 *     inside the image, has a surface, and |z(p) - fz(q)| <= tau_z z(p);
 *  3. in the 3x3 cell of p the lowest stratum index wins;
 *  4. sample: delta = L(reshade(q)) - L(prev(q)), norm = the larger of the
 *     two luminances;
 *  5. (delta, norm, present) are filtered alike by `levels` 5x5 B3 a-trous
 *     passes over the cells (cell steps 1, 2, 4, ...) with the depth weight
 *     exp(-|z_c - z_d| / (sigma_z |grad z . o| + 1e-10)) between the cells'
 *     centre pixels (3 c + 1, clamped; o the offset in pixels);
 *  6. lambda = min(1, |delta| / norm) of the filtered sums (0 where nothing
 *     reached the cell), and every pixel of the cell gets
 *     alpha_map = alpha + lambda (1 - alpha) - for sv_temporal's alpha_map.
 * prev, reshade, fmvx/fmvy (forward motion of the previous frame's pixels),
 * fz (view depth of the moved point) and g->z, g->dzdx, g->dzdy have the
 * storage type and dims d; pick is CH x CW bytes, contiguous; alpha_map is
 * a binary32 plane of dims d; lambda (optional) CH x CW binary32,
 * contiguous; work: sv_grad_work_bytes(d) bytes of device memory, any
 * contents, 16-byte aligned (SV_EINVAL otherwise).  Outputs and work must
 * not overlap inputs (SV_EALIAS). */
typedef struct {
    float alpha;    /* blend factor where nothing changed (0.2) */
    float tau_z;    /* depth test of the landing pixel (0.1) */
    float sigma_z;  /* depth edge weight of the reconstruction (1) */
    int32_t levels; /* reconstruction levels, 0..8 (3) */
} sv_grad_params;

size_t sv_grad_work_bytes(sv_dims d);

int sv_temporal_gradient(const sv_rgb *prev, const sv_rgb *reshade,
                         const void *fmvx, const void *fmvy, const void *fz,
                         const uint8_t *pick, const sv_gbuf *g,
                         float *alpha_map, float *lambda, void *work,
                         sv_dims d, sv_dtype t, const sv_grad_params *p,
                         sv_stream stream);

/* ---- composition of the channels (Section 3, step 7) ------------------ */

/* The paper denoises shadows and indirect specular light as separate
 * channels and blends them with the noise-free (rasterised) direct
 * lighting.  Reading of that blend: out = direct * shadow + spec per colour
 * channel (shadow: the denoised visibility, spec: the denoised indirect
 * specular radiance), evaluated as one binary32 fma and rounded to the
 * storage type.  shadow NULL means 1, spec NULL means 0.  Every plane has
 * the storage type; an output plane may be the same plane as the same
 * channel of an input, but no other overlap is allowed (SV_EALIAS). */
int sv_compose(const sv_rgb *direct, const sv_rgb *shadow, const sv_rgb *spec,
               const sv_rgb *out, sv_dims d, sv_dtype t, sv_stream stream);

/* ---- one frame of the whole filter (Section 3, steps 4 and 5) --------- */

/* Caller-owned buffers of one denoiser instance; every plane has the
 * call's dims, colour planes the storage type.  The library keeps nothing:
 * the history lives here between calls. */
typedef struct {
    sv_rgb hist[2];          /* colour history, double-buffered */
    float *m1[2], *m2c[2];   /* moment history (m2c central), double-buffered */
    uint8_t *n[2];           /* history length, double-buffered (0 = none) */
    sv_rgb temporal;         /* temporal output (scratch) */
    float *var;              /* variance estimate (scratch) */
    void *var_work;          /* sv_variance workspace (zeroed once) */
    sv_rgb level[2];         /* a-trous colour ping-pong (scratch) */
    float *level_var[2];     /* a-trous variance ping-pong (scratch) */
    sv_rgb scratch;          /* separable horizontal result (separable levels at
                                steps above 16 only; may be empty otherwise) */
    sv_rgb out;              /* final output of the frame */
    int32_t cur;             /* 0 or 1: which history buffers are current;
                                each call flips it */
    float *kappa;            /* learned mode: the network's kappa (scratch) */
} sv_denoiser;

typedef struct {
    sv_rgb cur;              /* current 1-spp colour */
    sv_gbuf g;               /* current G-buffer (all planes) */
    const void *mvx, *mvy;   /* backward motion in pixels */
    sv_gbuf prev;            /* previous frame's z, normal, id */
    const float *alpha_map;  /* optional per-pixel colour alpha (NULL) */
    const float *kappa;      /* optional per-pixel sigma_l scale (NULL) */
    /* learned mode (optional): the network runs inside the temporal step
     * and its alpha and kappa replace alpha_map and kappa; needs
     * g.dzdx, g.dzdy, albedo and the state's kappa plane */
    const sv_mlp *mlp;
    sv_rgb albedo;
    /* optional control bytes (sv_blur_control): the levels run as
     * sv_atrous_adaptive; separable levels at step 32 (level 4 shifted)
     * need the state's scratch planes */
    const uint8_t *blur_ctl;
} sv_frame_in;

typedef struct {
    sv_temporal_params temporal; /* SV_T_TONEMAP_IN also inverts at the end */
    sv_variance_params variance;
    sv_atrous_params atrous;     /* SV_A_INV_TONEMAP is set by the driver */
    int32_t levels;              /* a-trous levels, steps 1, 2, 4, ...; 0..10 */
    int32_t separable;           /* 1: sv_atrous_sep levels */
    int32_t feedback;            /* colour history: 0 level-0 output,
                                    1 temporal output */
    /* per-level launch shape overriding atrous.persistent / blocks_per_cu /
     * tile_rows when >= 0 / > 0 / > 0 (set by an autotuner; results do not
     * depend on it) */
    int32_t level_persistent[10];
    int32_t level_blocks_per_cu[10];
    int32_t level_tile_rows[10];
} sv_frame_params;

/* Enqueues one frame: sv_temporal (history -> temporal), sv_variance,
 * `levels` a-trous levels with steps 2^i (the inverse LUMA tone map fused
 * into the last one when the temporal step tone maps), the colour history
 * of the next frame being the level-0 output (feedback 0) or the temporal
 * output (feedback 1); then flips st->cur.  The result is in st->out.
 * Exactly the kernels of the individual calls, in the same order, so the
 * output is bitwise that of calling them one by one. */
int sv_denoise_frame(const sv_frame_in *in, sv_denoiser *st, sv_dims d,
                     sv_dtype t, const sv_frame_params *p, sv_stream stream);

/* ---- batched streams: many independent denoisers, one launch per pass ---
 *
 * Not in the paper.  A plan over n streams (1..64) of any sizes, each with
 * its own caller-owned sv_denoiser buffers, all with the same storage type
 * and sv_frame_params (1..5 levels; one level only with feedback = 1).
 * Each sv_batch_frame does for every stream exactly what sv_denoise_frame
 * does (the same kernels' tile code, so each stream's results are bitwise
 * those of sv_denoise_frame), but every pass runs once for all streams: one
 * launch over the tiles of all of them (one workgroup per tile), the passes
 * of a frame captured on the first call as a HIP graph and replayed
 * afterwards.
 *
 * The plan is the one object of the library that allocates (a device
 * buffer of the streams' per-pass arguments, pinned staging for it, two
 * events, a capture stream and the graph); sv_batch_destroy frees them.
 * The plan keeps the `states` pointers: those structures must outlive it.
 * Frames of one plan must be issued in order on one stream. */
typedef struct sv_batch sv_batch;

int sv_batch_create(const sv_dims *dims, sv_denoiser *const *states, int32_t n,
                    sv_dtype t, const sv_frame_params *p, sv_batch **out);

/* As sv_batch_create with its own sv_frame_params per stream (params[i] for
 * stream i): e.g. the channels of one frame (Section 3: shadows, indirect
 * specular) filtered with different settings in one launch per pass.  The
 * streams must run the same kernels pass by pass - the same level count,
 * form (2D / separable), rectification and id test, and the learned or
 * adaptive inputs on all or none; the tone map, the sigmas, the blend
 * factors and the thresholds may differ.  A mismatch is found on the first
 * sv_batch_frame, which then returns SV_EINVAL. */
int sv_batch_create_each(const sv_dims *dims, sv_denoiser *const *states,
                         int32_t n, sv_dtype t, const sv_frame_params *params,
                         sv_batch **out);

/* One frame of every stream: in[i] are stream i's inputs (as for
 * sv_denoise_frame).  Flips every state's `cur`. */
int sv_batch_frame(sv_batch *b, const sv_frame_in *in, sv_stream stream);

/* Passes (launches) per frame once the first frame has run, else 0; -1 for
 * a NULL plan. */
int sv_batch_passes(const sv_batch *b);

/* How later sv_batch_frame calls launch the passes: 0 (default) replays
 * the frame's HIP graph, 1 launches the same batched passes one by one on
 * the caller's stream (no graph; with large streams each launch already
 * fills the GPU, and the graph's kernel nodes measured slower there).
 * Results are bitwise the same either way.  SV_EINVAL for a NULL plan or a
 * value other than 0 or 1. */
int sv_batch_set_direct(sv_batch *b, int32_t direct);

void sv_batch_destroy(sv_batch *b);

/* ---- misc --------------------------------------------------------------- */

/* ABI self-check for bindings: writes sizeof of sv_dims, sv_rgb, sv_gbuf,
 * sv_tm_params, sv_temporal_io, sv_temporal_params, sv_variance_params,
 * sv_atrous_params, sv_denoiser, sv_frame_in, sv_frame_params, sv_mlp,
 * sv_adam_params, sv_blur_rule and sv_grad_params (in that order, at most n
 * of them) and returns how many
 * there are; SV_EINVAL for sizes == NULL or n < 0. */
int sv_struct_sizes(size_t *sizes, int32_t n);

/* Static string for a status code (never NULL). */
const char *sv_status_str(int status);

/* ABI version: increases when a signature or a struct changes. */
int sv_version(void);

/* The hipError_t of the last SV_EHIP returned on this thread (0 if none). */
int sv_last_hip_error(void);

/* Device-to-device copy of `bytes` (a multiple of 16, pointers 16-byte
 * aligned) by a plain streaming kernel: the bandwidth probe that the
 * roofline figures are compared with. */
int sv_probe_copy(void *dst, const void *src, size_t bytes, sv_stream stream);

/* Issue-rate probe: `blocks` workgroups of 256 lanes, each lane running
 * eight independent chains of `iters` links, a link being one fma
 * (kind 0), or exp2 and a multiply (1), or an add, log2 and a multiply
 * (2), or the same with rcp (3) or sqrt (4).  Kind 0's fma is a form
 * that issues at the full rate (a wave64 instruction in about two cycles on
 * MI355X); timed against it, the other kinds give the issue cost of those
 * instructions in full-rate slots, which prices the a-trous level's
 * arithmetic in the roofline.  `out`: device buffer of
 * blocks * 256 floats (one result per lane, written).  SV_EINVAL for a
 * kind outside 0..4, iters outside 1..2^20, blocks outside 1..65536 or a
 * null `out`. */
int sv_probe_issue(int32_t kind, int32_t iters, float *out, int32_t blocks, sv_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */
