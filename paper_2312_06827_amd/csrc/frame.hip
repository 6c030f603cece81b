// Per-frame driver: the sequence of library calls of one denoiser frame,
// enqueued from native code (one host call per frame).
#include "sv_internal.h"

extern "C" int sv_denoise_frame(const sv_frame_in *in, sv_denoiser *st, sv_dims d, sv_dtype t,
                                const sv_frame_params *p, sv_stream stream) {
    using namespace sv;
    if (!in || !st || !p) return SV_EINVAL;
    if (p->levels < 0 || p->levels > 10 || (st->cur != 0 && st->cur != 1)) return SV_EINVAL;
    if (check_dims(d) == 1) return SV_OK;
    const int k = st->cur, k1 = 1 - k;
    // with no level the colour history is the temporal output in any case
    const bool fb_temporal = p->feedback == 1 || p->levels == 0;
    const bool tm = (p->temporal.flags & SV_T_TONEMAP_IN) != 0;

    const bool learn = in->mlp != nullptr;
    if (learn && !st->kappa) return SV_EINVAL;
    // temporal: history k -> (temporal output | hist k1), moments k -> k1
    sv_temporal_io io{};
    io.cur = in->cur;
    io.g = in->g;
    io.mvx = in->mvx;
    io.mvy = in->mvy;
    io.prev = in->prev;
    io.hist = st->hist[k];
    io.hist_m1 = st->m1[k];
    io.hist_m2c = st->m2c[k];
    io.hist_n = st->n[k];
    io.out = fb_temporal ? st->hist[k1] : st->temporal;
    io.out_m1 = st->m1[k1];
    io.out_m2c = st->m2c[k1];
    io.out_n = st->n[k1];
    io.alpha_map = in->alpha_map;
    if (learn) {
        io.mlp = in->mlp;
        io.albedo = in->albedo;
        io.kappa_out = st->kappa;
    }
    const float *kappa = learn ? st->kappa : in->kappa;
    // the variance's pointwise part and its list come out of the temporal step
    io.var = st->var;
    io.var_work = st->var_work;
    io.var_min_hist = p->variance.min_hist;
    int rc = sv_temporal(&io, d, t, &p->temporal, stream);
    if (rc != SV_OK) return rc;
    sv_variance_params vp = p->variance;
    vp.flags |= SV_V_LISTED;
    rc = sv_variance(st->m1[k1], st->m2c[k1], st->n[k1], &in->g, st->var, st->var_work, d, t, &vp,
                     stream);
    if (rc != SV_OK) return rc;

    sv_rgb c = io.out;
    const float *v = st->var;
    const int L = p->levels;
    for (int i = 0; i < L; ++i) {
        const bool last = i == L - 1;
        const bool level0_is_hist = i == 0 && !fb_temporal;
        sv_atrous_params ap = p->atrous;
        ap.flags &= ~SV_A_INV_TONEMAP;
        if (p->level_persistent[i] >= 0) ap.persistent = p->level_persistent[i];
        if (p->level_blocks_per_cu[i] > 0) ap.blocks_per_cu = p->level_blocks_per_cu[i];
        if (p->level_tile_rows[i] > 0) ap.tile_rows = p->level_tile_rows[i];
        if (tm && last && !level0_is_hist) ap.flags |= SV_A_INV_TONEMAP;
        const sv_rgb dst = level0_is_hist ? st->hist[k1] : (last ? st->out : st->level[i & 1]);
        float *dst_var = last ? nullptr : st->level_var[i & 1];
        if (in->blur_ctl) {
            // adaptive levels: launches at steps 2^i and 2^(i+1); separable
            // ones fused while both steps have the fused form
            const bool fused = (2 << i) <= 32;
            const sv_rgb *scr = p->separable && !fused ? &st->scratch : nullptr;
            rc = sv_atrous_adaptive(&c, v, &in->g, kappa, in->blur_ctl, scr, &dst, dst_var, i,
                                    p->separable, d, t, &ap, stream);
        } else {
            // separable levels: the fused form (no scratch) where the step has one
            const bool fused = (1 << i) <= 32;
            rc = p->separable
                     ? sv_atrous_sep(&c, v, &in->g, kappa, fused ? nullptr : &st->scratch, &dst,
                                     dst_var, 1 << i, d, t, &ap, stream)
                     : sv_atrous(&c, v, &in->g, kappa, &dst, dst_var, 1 << i, d, t, &ap, stream);
        }
        if (rc != SV_OK) return rc;
        c = dst;
        v = dst_var;
    }
    // levels 0, or one level whose output is also the (tone-mapped) history:
    // the inverse tone map (or a copy) still has to reach st->out
    if (L == 0 || (L == 1 && !fb_temporal)) {
        sv_tm_params tp{p->temporal.tm_k, 1.0f, SV_TM_LUMA};
        if (tm) {
            rc = sv_tonemap(&c, &st->out, d, t, 1, &tp, stream);
        } else {
            const size_t es = elem_size(t);
            const size_t row = (size_t)d.w * es, pitch = (size_t)d.pitch * es;
            void *dst[3] = {st->out.r, st->out.g, st->out.b};
            const void *src[3] = {c.r, c.g, c.b};
            for (int ch = 0; ch < 3 && rc == SV_OK; ++ch)
                rc = hip_status(hipMemcpy2DAsync(dst[ch], pitch, src[ch], pitch, row, d.h,
                                                 hipMemcpyDeviceToDevice, as_stream(stream)));
        }
        if (rc != SV_OK) return rc;
    }
    st->cur = k1;
    return SV_OK;
}
