// Edge-avoiding a-trous entry points (Section 2, Fig. 1; Section 3.3): checks
// and dispatch to the per-type, per-direction pass launchers.
#include "atrous_impl.h"

namespace sv {

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

static TileCfg tile_cfg(const sv_atrous_params *p, int dir) {
    // default: one tile per workgroup, which measured fastest (or within
    // noise of the persistent forms) for every level at 1080p; callers pick
    // the persistent form and the tile height through the params (the
    // autotuner does)
    TileCfg c{false, 4, 0};
    if (p->persistent > 0) c.persistent = true;
    if (p->blocks_per_cu > 0) c.blocks_per_cu = p->blocks_per_cu;
    if (dir == kDir2D) c.rows = p->tile_rows;
    return c;
}

// tile_rows: 5x5 levels 0, 1 or 2; fused separable levels 0, 6 or 16
static bool valid_rows(const sv_atrous_params *p, bool separable) {
    const int r = p->tile_rows;
    return separable ? (r == 0 || r == 6 || r == 16) : (r == 0 || r == 1 || r == 2);
}

static void run_pass(const AtrousArgs &a, sv_dtype t, int dir, bool unit, TileCfg cfg,
                     hipStream_t s) {
    if (t == SV_F32) {
        if (dir == kDir2D) launch_pass_f32_2d(a, unit, cfg, s);
        else if (dir == kDir2DA) launch_pass_f32_2da(a, unit, cfg, s);
        else if (dir == kDirH) launch_pass_f32_h(a, unit, cfg, s);
        else launch_pass_f32_v(a, unit, cfg, s);
    } else {
        if (dir == kDir2D) launch_pass_f16_2d(a, unit, cfg, s);
        else if (dir == kDir2DA) launch_pass_f16_2da(a, unit, cfg, s);
        else if (dir == kDirH) launch_pass_f16_h(a, unit, cfg, s);
        else launch_pass_f16_v(a, unit, cfg, s);
    }
}

static AtrousArgs make_args(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                            const float *kappa, const sv_rgb *c_out, float *var_out,
                            int32_t step, sv_dims d, const sv_atrous_params *p) {
    return AtrousArgs{c_in->r, c_in->g, c_in->b, var_in, g->z, g->dzdx, g->dzdy, g->nx, g->ny,
                      g->nz, kappa, c_out->r, c_out->g, c_out->b, var_out, d.w, d.h, d.pitch,
                      step, p->sigma_z, p->sigma_l, p->eps_z, p->eps_l, p->tm_k,
                      make_normal_coef(p->sigma_n), (p->flags & SV_A_INV_TONEMAP) ? 1 : 0,
                      nullptr, 0, 0, c_in->r, c_in->g, c_in->b};
}

}  // namespace sv

extern "C" int sv_atrous(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                         const float *kappa, const sv_rgb *c_out, float *var_out, int32_t step,
                         sv_dims d, sv_dtype t, const sv_atrous_params *p, sv_stream stream) {
    using namespace sv;
    int empty = 0;
    if (p && !valid_rows(p, false)) return SV_EINVAL;
    int rc = check_atrous(c_in, var_in, g, kappa, nullptr, c_out, var_out, step, d, t, p, &empty);
    if (rc != SV_OK || empty) return rc;
    AtrousArgs a = make_args(c_in, var_in, g, kappa, c_out, var_out, step, d, p);
    const bool unit = (p->flags & SV_A_UNIT_WEIGHTS) != 0;
    TileCfg cfg = tile_cfg(p, kDir2D);
    run_pass(a, t, kDir2D, unit, cfg, as_stream(stream));
    return hip_status(hipGetLastError());
}

extern "C" int sv_atrous_sep(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                             const float *kappa, const sv_rgb *scratch, const sv_rgb *c_out,
                             float *var_out, int32_t step, sv_dims d, sv_dtype t,
                             const sv_atrous_params *p, sv_stream stream) {
    using namespace sv;
    int empty = 0;
    if (scratch && (!scratch->r || !scratch->g || !scratch->b)) return SV_EINVAL;
    if (p && !valid_rows(p, true)) return SV_EINVAL;
    int rc = check_atrous(c_in, var_in, g, kappa, scratch, c_out, var_out, step, d, t, p, &empty);
    if (rc != SV_OK || empty) return rc;
    const bool unit = (p->flags & SV_A_UNIT_WEIGHTS) != 0;
    hipStream_t s = as_stream(stream);
    if (!scratch) {  // both passes in one kernel, the horizontal result kept on chip
        const HvArgs a = make_args(c_in, var_in, g, kappa, c_out, var_out, step, d, p);
        const bool ok = t == SV_F32 ? launch_hv_f32(a, unit, p->tile_rows, s)
                                    : launch_hv_f16(a, unit, p->tile_rows, s);
        if (!ok) return SV_EUNSUPPORTED;
        return hip_status(hipGetLastError());
    }
    // horizontal: c_in -> scratch (no variance, no inverse tone map)
    AtrousArgs h = make_args(c_in, var_in, g, kappa, scratch, nullptr, step, d, p);
    h.inv_tm = 0;
    // vertical: scratch -> c_out, variance from var_in
    AtrousArgs v = make_args(scratch, var_in, g, kappa, c_out, var_out, step, d, p);
    run_pass(h, t, kDirH, unit, tile_cfg(p, kDirH), s);
    run_pass(v, t, kDirV, unit, tile_cfg(p, kDirV), s);
    return hip_status(hipGetLastError());
}

extern "C" int sv_atrous_adaptive(const sv_rgb *c_in, const float *var_in, const sv_gbuf *g,
                                  const float *kappa, const uint8_t *ctl, const sv_rgb *scratch,
                                  const sv_rgb *c_out, float *var_out, int32_t level,
                                  int32_t separable, sv_dims d, sv_dtype t,
                                  const sv_atrous_params *p, sv_stream stream) {
    using namespace sv;
    if (level < 0 || level > 12 || (separable != 0 && separable != 1)) return SV_EINVAL;
    if (!separable && scratch) return SV_EINVAL;
    if (scratch && (!scratch->r || !scratch->g || !scratch->b)) return SV_EINVAL;
    if (p && !valid_rows(p, separable != 0)) return SV_EINVAL;
    int empty = 0;
    int rc = check_atrous(c_in, var_in, g, kappa, scratch, c_out, var_out, 1 << level, d, t, p,
                          &empty);
    if (rc != SV_OK || empty) return rc;
    if (!ctl) return SV_EINVAL;
    {
        const span cs = plane_span(ctl, d, 1);
        const span outs[] = {plane_span(c_out->r, d, elem_size(t)),
                             plane_span(c_out->g, d, elem_size(t)),
                             plane_span(c_out->b, d, elem_size(t)),
                             var_out ? plane_span(var_out, d, 4) : span{0, 0},
                             scratch ? plane_span(scratch->r, d, elem_size(t)) : span{0, 0},
                             scratch ? plane_span(scratch->g, d, elem_size(t)) : span{0, 0},
                             scratch ? plane_span(scratch->b, d, elem_size(t)) : span{0, 0}};
        for (const span &so : outs)
            if (overlaps(so, cs)) return SV_EALIAS;
    }
    // separable launches at steps above 32 need the two-pass form
    if (separable && !scratch && level + 1 > 5) return SV_EUNSUPPORTED;
    const bool unit = (p->flags & SV_A_UNIT_WEIGHTS) != 0;
    hipStream_t s = as_stream(stream);
    if (!separable && (1 << level) <= kMaxStep2DA) {  // one launch, each pixel at its step
        AtrousArgs a = make_args(c_in, var_in, g, kappa, c_out, var_out, 1 << level, d, p);
        a.ctl = ctl;
        a.ctl_level = level;
        run_pass(a, t, kDir2DA, unit, tile_cfg(p, kDir2D), s);
        return hip_status(hipGetLastError());
    }
    for (int cls = 0; cls < 2; ++cls) {
        const int step = 1 << (level + cls);
        if (!separable) {
            AtrousArgs a = make_args(c_in, var_in, g, kappa, c_out, var_out, step, d, p);
            a.ctl = ctl;
            a.ctl_level = level;
            a.ctl_class = cls;
            run_pass(a, t, kDir2D, unit, tile_cfg(p, kDir2D), s);
        } else if (!scratch) {
            HvArgs a = make_args(c_in, var_in, g, kappa, c_out, var_out, step, d, p);
            a.ctl = ctl;
            a.ctl_level = level;
            a.ctl_class = cls;
            const bool ok = t == SV_F32 ? launch_hv_f32(a, unit, p->tile_rows, s)
                                        : launch_hv_f16(a, unit, p->tile_rows, s);
            if (!ok) return SV_EUNSUPPORTED;
        } else {
            // the horizontal pass covers every pixel at this launch's step;
            // only the vertical pass's writes are selected
            AtrousArgs h = make_args(c_in, var_in, g, kappa, scratch, nullptr, step, d, p);
            h.inv_tm = 0;
            AtrousArgs v = make_args(scratch, var_in, g, kappa, c_out, var_out, step, d, p);
            v.sr = c_in->r;
            v.sg = c_in->g;
            v.sb = c_in->b;
            v.ctl = ctl;
            v.ctl_level = level;
            v.ctl_class = cls;
            run_pass(h, t, kDirH, unit, tile_cfg(p, kDirH), s);
            run_pass(v, t, kDirV, unit, tile_cfg(p, kDirV), s);
        }
    }
    return hip_status(hipGetLastError());
}
