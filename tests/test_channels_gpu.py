"""The paper's two-channel pipeline (Section 3): shadow and indirect
specular channels denoised with their own settings in one batch plan, then
composed with the direct light.  Against the FP64 oracle (each channel's
chain with its own parameters and control bytes, then the composition),
and bitwise against the channels run one by one.

Tolerance of the shadow channel.  A one-sample visibility is 0 or 1, so
its variance vanishes away from the penumbrae, and the luminance edge
weight exp(-|dL| / (sigma_l sqrt(g) + eps_l)) becomes a near step function
of the luminance difference at scales far below what binary32 resolves
(eps_l = 1e-10).  The kernels keep flat regions exactly flat (grey-exact
luminance, correctly rounded weighted means), which holds every stage to
1e-5 from the same inputs (test_shadow_channel_stages_from_the_oracle_state,
measured 2e-6).  A chain that feeds each side its own output back as the
next frame's history is another matter: beside the penumbrae an ulp of
difference in the history can switch a neighbour's weight on or off, and
through four levels and over frames, lit pixels move by up to 3e-5 of
their value and near-black ones (visibility ~1e-5) by a few percent of
theirs, at most 1e-5 of the plane's scale (measured).  The chained shadow
output (and the composite it enters) is therefore held to 1e-4 of
max(|value|, plane RMS); the separable level's variance on such input,
which differs by up to 4x where it is 1e-6 of its plane's RMS, is measured
against that RMS at 1e-5.  The
specular channel, whose variance does not vanish, is held to 1e-5 of
every value in its chain."""

from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_06827_amd import lib as L
from paper_2312_06827_amd.pipeline import (SHADOW, SPECULAR, ChannelDenoiser, Denoiser,
                                           FrameInputs)
from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
from tests._util import frac_over, rel_err, say, worst
from tests.test_parity_gpu import dev, empty_like_dev, host

pytestmark = pytest.mark.gpu
TOL32 = 1e-5
FLOOR_BINARY = 1.0  # chained zero-variance visibility: errors measured against the plane RMS
TOL_CHAIN = 1e-4  # ... and held to 1e-4 of max(|value|, RMS) (see above)
OVER_CHAIN = 2e-3  # the fraction of chained shadow values past 1e-5 of that (measured 6.3e-4)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_compose(dtype):
    H, W = 37, 70
    r = np.random.default_rng(1200)
    d, s, p = (r.uniform(0, 1, (3, H, W)), r.uniform(0, 1, (3, H, W)), r.uniform(0, 2, (3, H, W)))
    if dtype == torch.float16:
        d, s, p = (O.quantize_half(a) for a in (d, s, p))
    P = W + 6
    dd, sd, pd = dev(d, P, dtype), dev(s, P, dtype), dev(p, P, dtype)
    for shadow, spec in [(True, True), (True, False), (False, True), (False, False)]:
        say(f"compose {dtype} shadow={shadow} spec={spec}")
        out = empty_like_dev((3, H, W), P, dtype)
        L.sv_compose(dd, sd if shadow else None, pd if spec else None, out)
        ref = O.compose(d, s if shadow else None, p if spec else None,
                        half_out=dtype == torch.float16)
        tol = TOL32 if dtype == torch.float32 else 2e-3
        assert rel_err(host(out), ref) <= tol
    # in place: the output is the direct light's planes
    L.sv_compose(dd, sd, pd, dd)
    assert rel_err(host(dd), O.compose(d, s, p, half_out=dtype == torch.float16)) <= (
        TOL32 if dtype == torch.float32 else 2e-3)


def _channel_frames(W=320, H=180, frames=6):
    cfg = replace(with_size(CONFIGS["hd_motion"], W, H, frames), channels=True)
    return list(sequence(cfg))


@pytest.mark.parametrize("adaptive", [True, False])
def test_channel_pipeline_matches_oracle(adaptive):
    frames = _channel_frames()
    H, W = frames[0]["z"].shape
    den = ChannelDenoiser(H, W, adaptive=adaptive)
    ps = O.OracleParams(clamp=True, use_id=True, levels=4)
    pr = O.OracleParams(clamp=True, tonemap=True, use_id=True, levels=4)
    ss, sp = O.new_state(H, W), O.new_state(H, W)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    try:
        for f, fr in enumerate(frames):
            say(f"channels adaptive={adaptive} frame {f}")
            out = den.frame(FrameInputs.from_numpy(fr), t(fr["shadow"]), t(fr["spec"]),
                            t(fr["direct"]), roughness=t(fr["roughness"]),
                            shadow_angle=t(fr["shadow_angle"]))
            fs, fp = dict(fr), dict(fr)
            fs["rgb"], fp["rgb"] = fr["shadow"], fr["spec"]
            cs = O.blur_control(None, fr["shadow_angle"], table=False) if adaptive else None
            cp = O.blur_control(fr["roughness"]) if adaptive else None
            os_, ss, _ = O.run_frame(fs, ss, ps, ctl=cs)
            op, sp, _ = O.run_frame(fp, sp, pr, ctl=cp)
            ref = O.compose(fr["direct"], os_, op)
            e = (rel_err(host(den.batch.streams[0].out), os_, floor=FLOOR_BINARY),
                 rel_err(host(den.batch.streams[1].out), op),
                 rel_err(host(out), ref, floor=FLOOR_BINARY))
            # the strict bar's misses are counted, as decision flips are
            over = frac_over(host(den.batch.streams[0].out), os_, TOL32, floor=FLOOR_BINARY)
            say(f"  shadow {e[0]:.2e} specular {e[1]:.2e} composite {e[2]:.2e}; shadow values"
                f" beyond 1e-5: {over:.2e} of them; worst shadow "
                f"{worst(host(den.batch.streams[0].out), os_, floor=FLOOR_BINARY)}")
            assert e[0] <= TOL_CHAIN and e[1] <= TOL32 and e[2] <= TOL_CHAIN, (f, e)
            assert over <= OVER_CHAIN, (f, over)
    finally:
        den.close()


def test_shadow_channel_stages_from_the_oracle_state():
    """Every stage of the shadow channel, frame after frame, from the same
    inputs as the oracle's (its history, temporal output, variance and level
    inputs, rounded to binary32): the temporal step, the variance estimate
    and the four levels, each within 1e-5 of the oracle, with identical
    history lengths."""
    frames = _channel_frames()
    H, W = frames[0]["z"].shape
    ps = O.OracleParams(clamp=True, use_id=True, levels=4)
    st = O.new_state(H, W)
    f32 = lambda a: np.asarray(a, np.float32)
    for f, fr in enumerate(frames):
        fs = dict(fr)
        fs["rgb"] = fr["shadow"]
        _, st_next, inter = O.run_frame(fs, st, ps)
        g = L.GBuf(dev(fr["z"]), dev(fr["dzdx"]), dev(fr["dzdy"]), dev(fr["n"]),
                   dev(fr["id"], dtype=torch.uint8))
        prev = L.GBuf(dev(fr["prev_z"]), None, None, dev(fr["prev_n"]),
                      dev(fr["prev_id"], dtype=torch.uint8))
        out, om1, om2 = empty_like_dev((3, H, W)), empty_like_dev((H, W)), empty_like_dev((H, W))
        on = empty_like_dev((H, W), dtype=torch.uint8)
        L.sv_temporal(dev(fs["rgb"]), g, dev(fr["mv"]), prev, dev(f32(st["rgb"])),
                      dev(f32(st["m1"])), dev(f32(st["m2"] - st["m1"] ** 2)),
                      dev(st["n"], dtype=torch.uint8), out, om1, om2, on, SHADOW.temporal())
        t = inter["temporal"]
        e = {"temporal": rel_err(host(out), t["rgb"]), "m1": rel_err(host(om1), t["m1"])}
        np.testing.assert_array_equal(host(on), t["n"])
        m1, m2c = f32(t["m1"]), f32(np.maximum(t["m2c"], 0.0))
        var = empty_like_dev((H, W))
        L.sv_variance(dev(m1), dev(m2c), dev(t["n"], dtype=torch.uint8), g, var,
                      SHADOW.variance(), L.variance_workspace(var))
        e["variance"] = rel_err(host(var), O.variance(
            m1, m2c.astype(np.float64) + m1.astype(np.float64) ** 2, t["n"], fr["z"],
            fr["dzdx"], fr["dzdy"], fr["n"]))
        c, v = f32(t["rgb"]), f32(inter["var"])
        for i in range(4):
            last = i == 3
            rc, rv = O.atrous(c, v, fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], 1 << i,
                              want_var=not last)
            co = empty_like_dev((3, H, W))
            vo = None if last else empty_like_dev((H, W))
            L.sv_atrous(dev(c), dev(v), g, co, vo, 1 << i, SHADOW.atrous())
            e[f"level{i}"] = rel_err(host(co), rc)
            if not last:
                e[f"var{i}"] = rel_err(host(vo), rv)
                c, v = f32(rc), f32(rv)
        say(f"shadow stages frame {f}: " + " ".join(f"{k} {x:.1e}" for k, x in e.items()))
        assert max(e.values()) <= TOL32, (f, e)
        st = st_next


def test_channel_batch_equals_channels_alone():
    frames = _channel_frames(W=200, H=120, frames=4)
    H, W = frames[0]["z"].shape
    den = ChannelDenoiser(H, W)
    alone = [Denoiser(H, W, SHADOW), Denoiser(H, W, SPECULAR)]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    try:
        for f, fr in enumerate(frames):
            say(f"channel batch vs alone frame {f}")
            geo = FrameInputs.from_numpy(fr)
            out = den.frame(geo, t(fr["shadow"]), t(fr["spec"]), t(fr["direct"]),
                            roughness=t(fr["roughness"]), shadow_angle=t(fr["shadow_angle"]))
            outs = []
            for k, (d, key) in enumerate(zip(alone, ("shadow", "spec"))):
                inp = replace(geo, rgb=t(fr[key]), blur_ctl=den.ctl[k])
                outs.append(d.frame(inp))
            direct = t(fr["direct"])
            ref = torch.empty_like(direct)
            L.sv_compose(direct, outs[0], outs[1], ref)
            torch.cuda.synchronize()
            assert torch.equal(den.batch.streams[0].out, outs[0])
            assert torch.equal(den.batch.streams[1].out, outs[1])
            assert torch.equal(out, ref)
        # temporal, variance x2, one launch per adaptive level (steps 1 to 8)
        assert den.batch.passes() == 2 + 4
    finally:
        den.close()


@pytest.mark.parametrize("sep", [False, True])
def test_levels_on_binary_visibility(sep):
    """Grey 0/1 visibility with zero variance almost everywhere: the
    luminance edge weight divides by a nearly vanishing scale there, so the
    luminance differences must be exact for grey colours (the level is
    still within 1e-5 of the oracle, colour and variance)."""
    fr = _channel_frames(W=200, H=120, frames=1)[0]
    z, dzdx, dzdy, n = fr["z"], fr["dzdx"], fr["dzdy"], fr["n"]
    vis = fr["shadow"].astype(np.float32)
    # the variance a first frame gives such a signal: the spatial estimate
    var = O.variance(vis[0], vis[0] ** 2, np.ones(z.shape, np.int32), z, dzdx, dzdy, n)
    var = var.astype(np.float32)
    c, v = vis, var
    g = L.GBuf(dev(z), dev(dzdx), dev(dzdy), dev(n))
    for i in range(4):
        step = 1 << i
        say(f"binary visibility sep={sep} step={step} zero-var {(v == 0).mean():.2f}")
        out, vo = empty_like_dev((3,) + z.shape), empty_like_dev(z.shape)
        if sep:
            L.sv_atrous_sep(dev(c), dev(v), g, None, out, vo, step, L.AtrousParams())
            rc, rv, _ = O.atrous_sep(c, v, z, dzdx, dzdy, n, step)
        else:
            L.sv_atrous(dev(c), dev(v), g, out, vo, step, L.AtrousParams())
            rc, rv = O.atrous(c, v, z, dzdx, dzdy, n, step)
        ec = rel_err(host(out), rc)
        # the separable level's variance where it nearly vanishes is measured
        # against the plane's own scale (see above)
        ev = rel_err(host(vo), rv, floor=1.0 if sep else 1e-3)
        say(f"  colour {ec:.2e} {worst(host(out), rc)}  var {ev:.2e} {worst(host(vo), rv)}")
        assert ec <= TOL32 and ev <= TOL32
        # the next level's input: this level's device output
        c, v = host(out).astype(np.float32), host(vo).astype(np.float32)


def test_channel_pipeline_with_temporal_gradient():
    """The shadow channel's blend factor from the temporal gradient: the
    batched channels against the oracle chain fed the oracle's gradient."""
    from oracle import gradient as OG
    frames = _channel_frames(W=200, H=120, frames=5)
    H, W = frames[0]["z"].shape
    den = ChannelDenoiser(H, W, adaptive=False)
    ps = O.OracleParams(clamp=True, use_id=True, levels=4)
    pr = O.OracleParams(clamp=True, tonemap=True, use_id=True, levels=4)
    ss, sp = O.new_state(H, W), O.new_state(H, W)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    try:
        for f, fr in enumerate(frames):
            grad, am = None, None
            if f > 0:
                pv = frames[f - 1]
                re = np.broadcast_to(fr["shadow_reshade"][None], (3, H, W)).copy()
                grad = {"prev": t(pv["shadow"]), "reshade": t(re), "fmv": t(fr["fmv"]),
                        "fz": t(fr["fz"]), "pick": t(fr["grad_pick"])}
                am, _ = OG.temporal_gradient(pv["shadow"], re, fr["fmv"], fr["fz"],
                                             fr["grad_pick"], fr["z"], fr["dzdx"], fr["dzdy"])
            say(f"channels with gradient frame {f}")
            out = den.frame(FrameInputs.from_numpy(fr), t(fr["shadow"]), t(fr["spec"]),
                            t(fr["direct"]), gradient=grad)
            fs, fp = dict(fr), dict(fr)
            fs["rgb"], fp["rgb"] = fr["shadow"], fr["spec"]
            os_, ss, _ = O.run_frame(fs, ss, ps, alpha_map=am)
            op, sp, _ = O.run_frame(fp, sp, pr)
            if am is not None:
                np.testing.assert_allclose(host(den.grad_alpha), am, atol=1e-5, rtol=0)
            e = (rel_err(host(den.batch.streams[0].out), os_, floor=FLOOR_BINARY),
                 rel_err(host(den.batch.streams[1].out), op))
            say(f"  shadow {e[0]:.2e} specular {e[1]:.2e}")
            assert e[0] <= TOL_CHAIN and e[1] <= TOL32, (f, e)
    finally:
        den.close()
