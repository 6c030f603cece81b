"""The library at its size limits, against the FP64 oracle element by
element: the largest plane the calls accept (pitch * h = 2^29 elements, so
binary32 byte offsets reach 2^31 and the last rows sit at the top of a
2 GiB allocation) and the widest image (w = 32768, the largest x that the
variance pass's short-history list encodes).  Covered: the 2D a-trous
level at steps 1 and 16, the fused separable level, the temporal step and
the variance estimate.  The row padding holds NaN, so a read past the end
of a row would reach the outputs."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_06827_amd import lib as L
from paper_2312_06827_amd.scene import CONFIGS, render_frame, with_size
from tests._util import random_gbuf, rel_err, say

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
LIMIT = 1 << 29                       # largest pitch * h (elements)
TALL = (32768, 64, LIMIT // 32768)    # (H, W, pitch): pitch * h == 2^29
WIDE = (4, 32768, 32768)


def padded(a, pitch, dtype=torch.float32):
    """numpy (.., H, W) -> device view (.., H, W) of a (.., H, pitch)
    allocation whose padding is NaN (0 for integer planes)."""
    a = np.ascontiguousarray(a)
    full = torch.full(a.shape[:-1] + (pitch,), float("nan") if dtype.is_floating_point else 0,
                      dtype=dtype, device="cuda")
    view = full[..., : a.shape[-1]]
    view.copy_(torch.from_numpy(a).to(dtype).cuda())
    return view


def out_plane(shape, pitch, dtype=torch.float32):
    full = torch.full(shape[:-1] + (pitch,), float("nan") if dtype.is_floating_point else 0,
                      dtype=dtype, device="cuda")
    return full[..., : shape[-1]]


def host(t):
    torch.cuda.synchronize()
    return t.detach().to(torch.float64).cpu().numpy() if t.dtype.is_floating_point \
        else t.detach().cpu().numpy()


def gbuf(z, dzdx, dzdy, n, pitch):
    return L.GBuf(padded(z, pitch), padded(dzdx, pitch), padded(dzdy, pitch), padded(n, pitch))


def _atrous_inputs(H, W, seed):
    r = np.random.default_rng(seed)
    z, dzdx, dzdy, n = random_gbuf(r, H, W)
    z = z.copy()
    z[r.random((H, W)) < 0.02] = 0.0  # a few empty pixels
    c = r.exponential(0.5, (3, H, W)).astype(np.float32)
    var = r.uniform(0.001, 0.05, (H, W)).astype(np.float32)
    return c, var, z, dzdx, dzdy, n


@pytest.fixture(autouse=True)
def _release():
    yield
    torch.cuda.empty_cache()


@pytest.mark.parametrize("H,W,P", [TALL, WIDE])
def test_atrous_at_the_limits(H, W, P):
    assert P * H <= LIMIT
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 1000 + W)
    g = gbuf(z, dzdx, dzdy, n, P)
    ci, vi = padded(c, P), padded(var, P)
    for step in (1, 16):
        say(f"atrous {H}x{W} pitch {P} step {step}")
        out, vo = out_plane((3, H, W), P), out_plane((H, W), P)
        L.sv_atrous(ci, vi, g, out, vo, step, L.AtrousParams())
        rc, rv = O.atrous(c, var, z, dzdx, dzdy, n, step, want_var=True)
        assert rel_err(host(out), rc) <= TOL32
        assert rel_err(host(vo), rv) <= TOL32
    step = 16
    say(f"atrous_sep (fused) {H}x{W} pitch {P} step {step}")
    out, vo = out_plane((3, H, W), P), out_plane((H, W), P)
    L.sv_atrous_sep(ci, vi, g, None, out, vo, step, L.AtrousParams())
    rc, rv, _ = O.atrous_sep(c, var, z, dzdx, dzdy, n, step, want_var=True)
    assert rel_err(host(out), rc) <= TOL32
    assert rel_err(host(vo), rv) <= TOL32


@pytest.mark.parametrize("H,W,P", [TALL, WIDE])
def test_temporal_and_variance_at_the_limits(H, W, P):
    fr = render_frame(with_size(CONFIGS["hd_motion"], W, H, 4), 3)
    r = np.random.default_rng(2000 + W)
    hist = (np.roll(fr["clean"], 1, axis=-1) * r.uniform(0.7, 1.3, (3, H, W))).astype(np.float32)
    m1 = (hist.mean(0) * r.uniform(0.9, 1.1, (H, W))).astype(np.float32)
    m2c = (m1 * m1 * r.uniform(0.0, 1.0, (H, W))).astype(np.float32)
    hn = r.integers(0, 6, (H, W)).astype(np.uint8)  # many short histories
    st = {"rgb": hist, "m1": m1, "m2c": m2c,
          "m2": m2c.astype(np.float64) + m1.astype(np.float64) ** 2, "n": hn}
    p = O.OracleParams(clamp=True, tonemap=True, gamma=1.0)
    ref = O.temporal(fr, st, p)
    say(f"temporal {H}x{W} pitch {P}")
    g = gbuf(fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], P)
    prev = L.GBuf(padded(fr["prev_z"], P), None, None, padded(fr["prev_n"], P))
    out = out_plane((3, H, W), P)
    om1, om2 = out_plane((H, W), P), out_plane((H, W), P)
    on = out_plane((H, W), P, torch.uint8)
    L.sv_temporal(padded(fr["rgb"], P), g, padded(fr["mv"], P), prev, padded(hist, P),
                  padded(m1, P), padded(m2c, P), padded(hn, P, torch.uint8), out, om1, om2, on,
                  L.TemporalParams(clamp=True, tonemap=True, gamma=1.0))
    np.testing.assert_array_equal(host(on), ref["n"])
    assert rel_err(host(out), ref["rgb"]) <= TOL32
    assert rel_err(host(om1), ref["m1"]) <= TOL32
    assert rel_err(host(om2), ref["m2c"]) <= TOL32
    del out, om1, om2, on
    # the variance estimate at the same size, both sides from the same
    # binary32 moments (the oracle's), with many short histories listed (x up
    # to 32767 or y up to 32767)
    m1v = ref["m1"].astype(np.float32)
    m2cv = np.maximum(ref["m2c"], 0.0).astype(np.float32)
    nv = ref["n"].astype(np.uint8)
    say(f"variance {H}x{W} pitch {P}")
    var = out_plane((H, W), P)
    work = L.variance_workspace(var)
    L.sv_variance(padded(m1v, P), padded(m2cv, P), padded(nv, P, torch.uint8), g, var,
                  L.VarianceParams(), work)
    m2raw = m2cv.astype(np.float64) + m1v.astype(np.float64) ** 2
    rv = O.variance(m1v, m2raw, nv, fr["z"], fr["dzdx"], fr["dzdy"], fr["n"])
    assert (nv[fr["z"] > 0] < 4).sum() > 1000  # the spatial estimate is exercised
    assert rel_err(host(var), rv) <= TOL32


@pytest.mark.parametrize("H,W,P", [TALL, WIDE])
def test_atrous_half_at_the_limits(H, W, P):
    """Binary16 storage (byte offsets up to 2^30) against the oracle with
    binary16 rounding at the same storage points, bar 2e-3."""
    r = np.random.default_rng(3000 + W)
    z, dzdx, dzdy, n = (a.astype(np.float16) for a in random_gbuf(r, H, W))
    c = r.exponential(0.5, (3, H, W)).astype(np.float16)
    var = r.uniform(0.001, 0.05, (H, W)).astype(np.float32)
    h = torch.float16
    g = L.GBuf(padded(z, P, h), padded(dzdx, P, h), padded(dzdy, P, h), padded(n, P, h))
    ci, vi = padded(c, P, h), padded(var, P)
    for step, sep in ((1, False), (16, False), (16, True)):
        say(f"atrous f16 {H}x{W} pitch {P} step {step} sep={sep}")
        out, vo = out_plane((3, H, W), P, h), out_plane((H, W), P)
        if sep:
            L.sv_atrous_sep(ci, vi, g, None, out, vo, step, L.AtrousParams())
            rc, rv, _ = O.atrous_sep(c, var, z, dzdx, dzdy, n, step, half_out=True)
        else:
            L.sv_atrous(ci, vi, g, out, vo, step, L.AtrousParams())
            rc, rv = O.atrous(c, var, z, dzdx, dzdy, n, step, half_out=True)
        assert rel_err(host(out), rc) <= 2e-3
        assert rel_err(host(vo), rv) <= 2e-3


def test_batch_of_the_tallest_and_widest_streams():
    """A batch plan whose streams are the tallest and the widest image: each
    stream equals, bitwise, the same stream run alone (the batched passes
    index tiles through prefix sums over the streams)."""
    from paper_2312_06827_amd.pipeline import MOTION, BatchDenoiser, Denoiser, FrameInputs
    sizes = [(TALL[0], TALL[1]), (WIDE[0], WIDE[1])]
    cfgs = [with_size(CONFIGS["hd_motion"], w, h, 2) for (h, w) in sizes]
    batch = BatchDenoiser(sizes, MOTION)
    singles = [Denoiser(h, w, MOTION) for (h, w) in sizes]
    try:
        for f in range(2):
            say(f"batch of the limit shapes, frame {f}")
            inputs = [FrameInputs.from_numpy(render_frame(c, f)) for c in cfgs]
            outs = batch.frame(inputs)
            refs = [d.frame(inp) for d, inp in zip(singles, inputs)]
            torch.cuda.synchronize()
            for i in range(len(sizes)):
                assert torch.equal(outs[i], refs[i]), (f, i)
    finally:
        batch.close()


@pytest.mark.parametrize("H,W,P", [(32768, 8, LIMIT // 32768), WIDE])
def test_temporal_gradient_at_the_limits(H, W, P):
    """The gradient's strata, cells and normalized convolution at the
    limits (the tall case keeps to 8 columns: the oracle is Python)."""
    from oracle import gradient as OG
    r = np.random.default_rng(4000 + W)
    q = lambda a: a.astype(np.float32).astype(np.float64)
    prev = q(r.uniform(0, 2, (3, H, W)))
    re = q(np.where(r.random((3, H, W)) < 0.7, prev, r.uniform(0, 2, (3, H, W))))
    fmv = q(r.normal(0, 2.5, (2, H, W)))
    z = q(r.uniform(4, 6, (H, W)))
    z[r.random((H, W)) < 0.03] = 0.0
    fz = q(z * np.where(r.random((H, W)) < 0.1, 1.5, 1.0))
    dzdx, dzdy = q(r.normal(0, 0.05, (H, W))), q(r.normal(0, 0.05, (H, W)))
    pick = r.integers(0, 10, OG.cells_of(H, W)).astype(np.uint8)
    say(f"temporal gradient {H}x{W} pitch {P}")
    g = L.GBuf(padded(z, P), padded(dzdx, P), padded(dzdy, P), padded(np.zeros((3, H, W)), P))
    am = out_plane((H, W), P)
    lam = torch.full(OG.cells_of(H, W), float("nan"), device="cuda")
    L.sv_temporal_gradient(padded(prev, P), padded(re, P), padded(fmv, P), padded(fz, P),
                           torch.from_numpy(pick).cuda(), g, am, L.gradient_workspace(am),
                           alpha=0.2, levels=3, lam=lam)
    ram, rlam = OG.temporal_gradient(prev, re, fmv, fz, pick, z, dzdx, dzdy)
    np.testing.assert_allclose(host(lam), rlam, atol=1e-5, rtol=0)
    np.testing.assert_allclose(host(am), ram, atol=1e-5, rtol=0)


@pytest.mark.parametrize("H,W,P", [TALL, WIDE])
def test_adaptive_levels_at_the_limits(H, W, P):
    """Control bytes from roughness (bitwise) and the first two adaptive
    levels, 2D and fused separable, at the limits."""
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 5000 + W)
    rough = np.random.default_rng(5000).uniform(0.0, 0.4, (H, W)).astype(np.float32)
    rough[:, ::7] = 0.0  # some pixels with no blur at all
    ctl = out_plane((H, W), P, torch.uint8)
    L.sv_blur_control(padded(rough, P), None, ctl, L.BlurRule())
    rctl = O.blur_control(rough)
    np.testing.assert_array_equal(host(ctl), rctl)
    g = gbuf(z, dzdx, dzdy, n, P)
    for sep in (False, True):
        ci, vi = c, var
        for level in (0, 1):
            say(f"adaptive {H}x{W} pitch {P} level {level} sep={sep}")
            out, vo = out_plane((3, H, W), P), out_plane((H, W), P)
            L.sv_atrous_adaptive(padded(ci, P), padded(vi, P), g, ctl, None, out, vo, level, sep,
                                 L.AtrousParams())
            rc, rv = O.atrous_adaptive(ci, vi, z, dzdx, dzdy, n, rctl, level, separable=sep)[:2]
            assert rel_err(host(out), rc) <= TOL32
            assert rel_err(host(vo), rv) <= TOL32
            ci, vi = rc.astype(np.float32), rv.astype(np.float32)
