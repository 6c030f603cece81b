"""Parity of every library call, through the C ABI, with the FP64 oracle on
identical seeded inputs (binary32 storage): element by element, maximum
relative error 1e-5 (per plane, denominators floored at 1e-3 of the
plane's RMS).  History lengths are compared exactly.  Sizes span several
64x8 tiles with ragged tails, down to 1x1, and planes with a row pitch
larger than the width."""

from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_06827_amd import lib as L
from paper_2312_06827_amd.scene import CONFIGS, render_frame, with_size
from tests._util import guard, guard_value, list_consumed, rel_err, random_gbuf, say, worst

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
SIZES = [(1, 1), (3, 5), (37, 70), (67, 131)]  # (H, W)


def dev(a, pitch=None, dtype=torch.float32):
    """numpy (.., H, W) -> device tensor view with row pitch `pitch`.  The
    padding past the width holds NaN (0xA5 in byte planes): a read past a
    row's end would carry it into the result."""
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a).to(dtype)
    if pitch is None or pitch == a.shape[-1]:
        return t.cuda()
    full = torch.full(a.shape[:-1] + (pitch,), guard_value(dtype), dtype=dtype)
    full[..., : a.shape[-1]] = t
    return full.cuda()[..., : a.shape[-1]]


def empty_like_dev(shape, pitch=None, dtype=torch.float32):
    """Output planes, NaN-filled (0xA5 in byte planes).  With a pitch past
    the width the padding is a guard band: the test's end checks that no
    call wrote into it."""
    W = shape[-1]
    p = W if pitch is None else pitch
    t = torch.full(shape[:-1] + (p,), guard_value(dtype), dtype=dtype, device="cuda")
    if p > W:
        guard(t, W)
    return t[..., :W]


def host(t):
    torch.cuda.synchronize()
    return t.detach().to(torch.float64).cpu().numpy() if t.dtype.is_floating_point \
        else t.detach().cpu().numpy()


def gbuf_dev(z, dzdx, dzdy, n, pitch=None, ids=None):
    return L.GBuf(dev(z, pitch), dev(dzdx, pitch), dev(dzdy, pitch), dev(n, pitch),
                  None if ids is None else dev(ids, pitch, torch.uint8))


def scene_frame(H, W, frame=3, seed=2):
    cfg = replace(with_size(CONFIGS["hd_motion"], W, H, frame + 1), seed=seed)
    return render_frame(cfg, frame)


# ---- tone map -----------------------------------------------------------------

@pytest.mark.parametrize("H,W", SIZES)
def test_tonemap(H, W):
    r = np.random.default_rng(100 + H)
    c = r.exponential(1.0, (3, H, W)).astype(np.float32) * 3
    for mode, name in [(L.SV_TM_LUMA, "luma"), (L.SV_TM_CHANNEL, "channel")]:
        for inverse in (False, True):
            src = c if not inverse else O.tonemap(c, mode=name).astype(np.float32)
            say(f"tonemap {H}x{W} mode={name} inverse={inverse}")
            out = empty_like_dev((3, H, W), pitch=W + 3)
            L.sv_tonemap(dev(src, W + 3), out, inverse=inverse, mode=mode, k=1.0)
            ref = O.tonemap(src, inverse=inverse, mode=name)
            assert rel_err(host(out), ref) <= TOL32
    src = O.tonemap(c).astype(np.float32)
    out = empty_like_dev((3, H, W))
    L.sv_tonemap(dev(src), out, inverse=True, mode=L.SV_TM_PAPER, weight=0.7)
    assert rel_err(host(out), O.tonemap(src, inverse=True, mode="paper", weight=0.7)) <= TOL32


def test_tonemap_in_place():
    c = np.random.default_rng(1).exponential(1.0, (3, 40, 50)).astype(np.float32)
    t = dev(c)
    L.sv_tonemap(t, t)
    assert rel_err(host(t), O.tonemap(c)) <= TOL32


# ---- clamp --------------------------------------------------------------------------

@pytest.mark.parametrize("H,W", SIZES)
@pytest.mark.parametrize("gamma", [0.0, 1.0, 2.5])
def test_clamp(H, W, gamma):
    r = np.random.default_rng(200 + H + int(gamma * 10))
    cur = r.uniform(0, 1, (3, H, W)).astype(np.float32)
    hist = r.uniform(-0.5, 1.5, (3, H, W)).astype(np.float32)
    z = r.uniform(1, 2, (H, W)).astype(np.float32)
    z[r.random((H, W)) < 0.1] = 0.0  # empty pixels
    say(f"clamp {H}x{W} gamma={gamma}")
    out = empty_like_dev((3, H, W), pitch=W + 1)
    L.sv_clamp(dev(hist, W + 1), dev(cur, W + 1), out, gamma, z=dev(z, W + 1))
    ref = O.clamp(hist, cur, gamma, z=z)
    assert rel_err(host(out), ref) <= TOL32


@pytest.mark.parametrize("H,W", SIZES)
@pytest.mark.parametrize("gamma", [0.0, 1.0, 2.5])
def test_clip(H, W, gamma):
    r = np.random.default_rng(300 + H + int(gamma * 10))
    cur = r.uniform(0, 1, (3, H, W)).astype(np.float32)
    hist = r.uniform(-0.5, 1.5, (3, H, W)).astype(np.float32)
    # flat patches (zero spread in every channel) send the history to mu;
    # a patch flat in one channel only collapses t to 0 wherever that
    # channel deviates
    if H >= 8 and W >= 8:
        cur[:, 1:6, 1:6] = 0.25
        cur[1, 1:6, -6:-1] = 0.5
    z = r.uniform(1, 2, (H, W)).astype(np.float32)
    z[r.random((H, W)) < 0.1] = 0.0  # empty pixels
    say(f"clip {H}x{W} gamma={gamma}")
    out = empty_like_dev((3, H, W), pitch=W + 1)
    L.sv_clip(dev(hist, W + 1), dev(cur, W + 1), out, gamma, z=dev(z, W + 1))
    ref = O.clip(hist, cur, gamma, z=z)
    assert rel_err(host(out), ref) <= TOL32
    if gamma > 0 and H >= 8 and W >= 8:
        inner = host(out)[:, 2:5, 2:5]
        live = z[2:5, 2:5] > 0
        np.testing.assert_array_equal(inner[:, live], 0.25)


# ---- temporal ---------------------------------------------------------------------

def _temporal_case(H, W, seed):
    fr = scene_frame(H, W, frame=3, seed=seed)
    r = np.random.default_rng(seed)
    # a synthetic history: shifted clean image plus noise, random moments,
    # lengths 0..12 (some taps have no history)
    hist = (np.roll(fr["clean"], 1, axis=-1) * r.uniform(0.7, 1.3, (3, H, W))).astype(np.float32)
    L0 = hist.mean(0)
    m1 = (L0 * r.uniform(0.9, 1.1, (H, W))).astype(np.float32)
    m2c = (m1 * m1 * r.uniform(0.0, 1.0, (H, W))).astype(np.float32)
    hn = r.integers(0, 13, (H, W)).astype(np.uint8)
    # the oracle keeps the raw second moment E[L^2] = m2c + m1^2
    state = {"rgb": hist, "m1": m1, "m2c": m2c,
             "m2": m2c.astype(np.float64) + m1.astype(np.float64) ** 2, "n": hn}
    return fr, state


@pytest.mark.parametrize("H,W", [(3, 5), (37, 70), (67, 131)])
@pytest.mark.parametrize("clamp,tonemap,use_id", [
    (False, False, False), (True, False, False), (False, True, False), (True, True, True)])
def test_temporal(H, W, clamp, tonemap, use_id):
    fr, st = _temporal_case(H, W, 7 + H)
    if H > 10:  # a few empty pixels
        fr = dict(fr)
        fr["z"] = fr["z"].copy()
        fr["z"][5, 7] = 0.0
        fr["z"][-1, -1] = np.inf
    p = O.OracleParams(clamp=clamp, tonemap=tonemap, use_id=use_id, gamma=1.0)
    ref = O.temporal(fr, st, p)
    P = W + 5
    say(f"temporal {H}x{W} clamp={clamp} tm={tonemap} id={use_id}")
    g = gbuf_dev(fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], P, fr["id"])
    prev = L.GBuf(dev(fr["prev_z"], P), None, None, dev(fr["prev_n"], P),
                  dev(fr["prev_id"], P, torch.uint8))
    out = empty_like_dev((3, H, W), P)
    om1, om2 = empty_like_dev((H, W), P), empty_like_dev((H, W), P)
    on = empty_like_dev((H, W), P, torch.uint8)
    tp = L.TemporalParams(clamp=clamp, tonemap=tonemap, use_id=use_id, gamma=1.0)
    L.sv_temporal(dev(fr["rgb"], P), g, dev(fr["mv"], P), prev, dev(st["rgb"], P),
                  dev(st["m1"], P), dev(st["m2c"], P), dev(st["n"], P, torch.uint8),
                  out, om1, om2, on, tp)
    np.testing.assert_array_equal(host(on), ref["n"])
    assert rel_err(host(out), ref["rgb"]) <= TOL32
    assert rel_err(host(om1), ref["m1"]) <= TOL32
    assert rel_err(host(om2), ref["m2c"]) <= TOL32


@pytest.mark.parametrize("H,W", [(3, 5), (67, 131)])
@pytest.mark.parametrize("tonemap,use_id", [(False, False), (True, True)])
def test_temporal_clip(H, W, tonemap, use_id):
    fr, st = _temporal_case(H, W, 11 + H)
    p = O.OracleParams(clip=True, tonemap=tonemap, use_id=use_id, gamma=1.0)
    ref = O.temporal(fr, st, p)
    P = W + 3
    say(f"temporal clip {H}x{W} tm={tonemap} id={use_id}")
    g = gbuf_dev(fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], P, fr["id"])
    prev = L.GBuf(dev(fr["prev_z"], P), None, None, dev(fr["prev_n"], P),
                  dev(fr["prev_id"], P, torch.uint8))
    out = empty_like_dev((3, H, W), P)
    om1, om2 = empty_like_dev((H, W), P), empty_like_dev((H, W), P)
    on = empty_like_dev((H, W), P, torch.uint8)
    tp = L.TemporalParams(clip=True, tonemap=tonemap, use_id=use_id, gamma=1.0)
    L.sv_temporal(dev(fr["rgb"], P), g, dev(fr["mv"], P), prev, dev(st["rgb"], P),
                  dev(st["m1"], P), dev(st["m2c"], P), dev(st["n"], P, torch.uint8),
                  out, om1, om2, on, tp)
    np.testing.assert_array_equal(host(on), ref["n"])
    assert rel_err(host(out), ref["rgb"]) <= TOL32
    assert rel_err(host(om1), ref["m1"]) <= TOL32
    # clamp and clip together are refused
    with pytest.raises(RuntimeError):
        L.sv_temporal(dev(fr["rgb"], P), g, dev(fr["mv"], P), prev, dev(st["rgb"], P),
                      dev(st["m1"], P), dev(st["m2c"], P), dev(st["n"], P, torch.uint8),
                      out, om1, om2, on, L.TemporalParams(clip=True, clamp=True, gamma=1.0))


def test_temporal_alpha_map_and_discarded_motion():
    H, W = 40, 72
    fr, st = _temporal_case(H, W, 31)
    fr = dict(fr)
    fr["mv"] = fr["mv"].copy()
    fr["mv"][0, 3, 3] = np.nan
    fr["mv"][1, 4, 4] = 2.0e6
    am = np.random.default_rng(3).uniform(0.05, 1.0, (H, W)).astype(np.float32)
    p = O.OracleParams(clamp=True, tonemap=True)
    ref = O.temporal(fr, st, p, alpha_map=am)
    say("temporal alpha_map")
    g = gbuf_dev(fr["z"], fr["dzdx"], fr["dzdy"], fr["n"])
    prev = L.GBuf(dev(fr["prev_z"]), None, None, dev(fr["prev_n"]))
    out, om1, om2 = empty_like_dev((3, H, W)), empty_like_dev((H, W)), empty_like_dev((H, W))
    on = empty_like_dev((H, W), dtype=torch.uint8)
    L.sv_temporal(dev(fr["rgb"]), g, dev(fr["mv"]), prev, dev(st["rgb"]), dev(st["m1"]),
                  dev(st["m2c"]), dev(st["n"], dtype=torch.uint8), out, om1, om2, on,
                  L.TemporalParams(clamp=True, tonemap=True), alpha_map=dev(am))
    np.testing.assert_array_equal(host(on), ref["n"])
    assert host(on)[3, 3] == 1 and host(on)[4, 4] == 1
    assert rel_err(host(out), ref["rgb"]) <= TOL32


@pytest.mark.parametrize("mvx,mvy", [(42.999966, -1.551829e-05), (-3.0e-07, 5.999998),
                                     (-0.4999999, -0.25)])
def test_temporal_small_negative_motion(mvx, mvy):
    """Motion just below an integer, or just above one from below zero: one
    bilinear factor is tiny.  Histories are withheld (n = 0) so that only
    the taps with tiny factors remain usable, and their weights alone form
    the history: each tiny factor must be exact (for -1/2 < mv < 0, 1 - f
    with f = 1 + mv rounded in binary32 is not)."""
    H, W = 16, 96
    r = np.random.default_rng(77)
    cur = r.uniform(0.05, 1.0, (3, H, W)).astype(np.float32)
    z = np.full((H, W), 5.0, np.float32)
    n = np.zeros((3, H, W), np.float32)
    n[1] = 1.0
    mv = np.empty((2, H, W), np.float32)
    mv[0], mv[1] = np.float32(mvx), np.float32(mvy)
    fr = {"rgb": cur, "z": z, "n": n, "id": None, "mv": mv, "prev_z": z.copy(),
          "prev_n": n.copy(), "prev_id": None}
    hist = r.uniform(0.05, 1.0, (3, H, W)).astype(np.float32)
    m1 = hist.mean(0).astype(np.float32)
    m2c = (0.1 * m1 * m1).astype(np.float32)
    cols, rows = np.meshgrid(np.arange(W), np.arange(H))
    hn = np.where((cols % 2 == 1) & (rows % 2 == 0), 0, 3).astype(np.uint8)
    st = {"rgb": hist, "m1": m1, "m2c": m2c,
          "m2": m2c.astype(np.float64) + m1.astype(np.float64) ** 2, "n": hn}
    ref = O.temporal(fr, st, O.OracleParams())
    say(f"temporal tiny bilinear factor mv=({mvx}, {mvy})")
    g = L.GBuf(dev(z), None, None, dev(n))
    prev = L.GBuf(dev(z), None, None, dev(n))
    out, om1, om2 = empty_like_dev((3, H, W)), empty_like_dev((H, W)), empty_like_dev((H, W))
    on = empty_like_dev((H, W), dtype=torch.uint8)
    L.sv_temporal(dev(cur), g, dev(mv), prev, dev(hist), dev(m1), dev(m2c),
                  dev(hn, dtype=torch.uint8), out, om1, om2, on, L.TemporalParams())
    np.testing.assert_array_equal(host(on), ref["n"])
    assert (ref["n"] > 1).sum() > H * W // 4  # histories were used
    assert rel_err(host(out), ref["rgb"]) <= TOL32
    assert rel_err(host(om1), ref["m1"]) <= TOL32
    assert rel_err(host(om2), ref["m2c"]) <= TOL32


# ---- variance ------------------------------------------------------------------------

@pytest.mark.parametrize("H,W", SIZES)
def test_variance(H, W):
    r = np.random.default_rng(300 + H)
    z, dzdx, dzdy, n = random_gbuf(r, H, W)
    if H > 10:
        z[r.random((H, W)) < 0.05] = 0.0
    m1 = r.uniform(0.1, 1.0, (H, W)).astype(np.float32)
    m2c = (m1 * m1 * r.uniform(0.0, 1.0, (H, W))).astype(np.float32)
    m2 = m2c.astype(np.float64) + m1.astype(np.float64) ** 2  # raw moment for the oracle
    hn = r.integers(0, 7, (H, W)).astype(np.uint8)
    for sigma_n in (128.0, 16.0, 0.0):
        say(f"variance {H}x{W} sigma_n={sigma_n}")
        out = empty_like_dev((H, W), W + 2)
        work = L.variance_workspace(out)
        L.sv_variance(dev(m1, W + 2), dev(m2c, W + 2), dev(hn, W + 2, torch.uint8),
                      gbuf_dev(z, dzdx, dzdy, n, W + 2), out, L.VarianceParams(sigma_n=sigma_n),
                      work)
        L.sv_variance(dev(m1, W + 2), dev(m2c, W + 2), dev(hn, W + 2, torch.uint8),
                      gbuf_dev(z, dzdx, dzdy, n, W + 2), out, L.VarianceParams(sigma_n=sigma_n),
                      work)  # a second call continues from the first one's counters
        assert list_consumed(work)
        ref = O.variance(m1, m2, hn, z, dzdx, dzdy, n, sigma_n=sigma_n)
        assert rel_err(host(out), ref) <= TOL32


def test_variance_workspace_across_sizes():
    """One workspace, sized for the largest frame, serves calls of any
    smaller size in any order: the list of one call never leaks into the
    next, also when the smaller image has fewer than eight tiles (sublists
    that no tile of the call reaches)."""
    big, small = (37, 300), (4, 64)
    r = np.random.default_rng(311)
    cases = {}
    for H, W in (big, small):
        z, dzdx, dzdy, n = random_gbuf(r, H, W)
        m1 = r.uniform(0.1, 1.0, (H, W)).astype(np.float32)
        m2c = (m1 * m1 * r.uniform(0.0, 1.0, (H, W))).astype(np.float32)
        hn = r.integers(0, 7, (H, W)).astype(np.uint8)
        ref = O.variance(m1, m2c.astype(np.float64) + m1.astype(np.float64) ** 2, hn, z, dzdx,
                         dzdy, n)
        cases[(H, W)] = (m1, m2c, hn, gbuf_dev(z, dzdx, dzdy, n), ref)
    work = L.variance_workspace(empty_like_dev(big))
    for H, W in (big, small, small, big, small):
        m1, m2c, hn, g, ref = cases[(H, W)]
        say(f"variance {H}x{W} on a workspace for {big}")
        out = empty_like_dev((H, W))
        L.sv_variance(dev(m1), dev(m2c), dev(hn, None, torch.uint8), g, out, L.VarianceParams(),
                      work)
        assert list_consumed(work)
        assert rel_err(host(out), ref) <= TOL32


# ---- a-trous ----------------------------------------------------------------------------

def _atrous_inputs(H, W, seed, holes=False, scene=True):
    r = np.random.default_rng(seed)
    if scene and H >= 8 and W >= 8:
        fr = scene_frame(H, W, frame=2, seed=seed)
        z, dzdx, dzdy, n = fr["z"], fr["dzdx"], fr["dzdy"], fr["n"]
        c = O.tonemap(fr["rgb"]).astype(np.float32)
    else:
        z, dzdx, dzdy, n = random_gbuf(r, H, W)
        c = r.exponential(0.5, (3, H, W)).astype(np.float32)
    z = z.copy()
    if holes:
        z[r.random((H, W)) < 0.03] = 0.0
    var = (r.uniform(0.001, 0.05, (H, W))).astype(np.float32)
    return c, var, z, dzdx, dzdy, n


@pytest.mark.parametrize("H,W,step", [(h, w, s) for (h, w) in SIZES + [(130, 200)]
                                      for s in (1, 2, 3, 4, 8, 16, 32)] +
                         # several column tiles at the large steps (at step 32 the
                         # tile is 16 lattice columns of 8-column groups), ragged
                         [(70, 1100, 16), (70, 1100, 32), (37, 4100, 32)])
def test_atrous(H, W, step):
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 400 + step + H, holes=(step == 2))
    P = W + 7
    g = gbuf_dev(z, dzdx, dzdy, n, P)
    for unit, want_var, inv in [(False, True, False), (False, False, True), (True, True, False)]:
        say(f"atrous {H}x{W} step={step} unit={unit} var={want_var} inv={inv}")
        out = empty_like_dev((3, H, W), P)
        vo = empty_like_dev((H, W), P) if want_var else None
        L.sv_atrous(dev(c, P), dev(var, P), g, out, vo, step,
                    L.AtrousParams(unit_weights=unit, inv_tonemap=inv))
        rc, rv = O.atrous(c, var, z, dzdx, dzdy, n, step, unit_weights=unit, inv_tonemap=inv,
                          want_var=want_var)
        assert rel_err(host(out), rc) <= TOL32
        if want_var:
            assert rel_err(host(vo), rv) <= TOL32


@pytest.mark.parametrize("step", [1, 2])
def test_atrous_signed_zero_variance(step):
    """Live pixels of variance -0 and +0 beside empty ones.  The tile marks
    an empty neighbour's variance entry as -0 and stages a live pixel's
    plus +0, so a live pixel of variance -0 still counts in the 3x3
    prefilter (at steps 1 and 2 the prefilter's middle row comes from the
    tile) and the output matches the oracle's, which takes -0 as 0."""
    H, W = 70, 130
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 470 + step, holes=True)
    u = np.random.default_rng(471 + step).random((H, W))
    var[u < 0.2] = -0.0
    var[(u >= 0.2) & (u < 0.3)] = 0.0
    assert np.signbit(var).sum() > 0.1 * H * W and np.sum(z == 0) > 0
    g = gbuf_dev(z, dzdx, dzdy, n)
    out, vo = empty_like_dev((3, H, W)), empty_like_dev((H, W))
    say(f"atrous signed-zero variance {H}x{W} step={step}")
    L.sv_atrous(dev(c), dev(var), g, out, vo, step, L.AtrousParams())
    rc, rv = O.atrous(c, var, z, dzdx, dzdy, n, step)
    assert rel_err(host(out), rc) <= TOL32
    assert rel_err(host(vo), rv) <= TOL32


@pytest.mark.parametrize("step", [1, 3, 4, 16])
def test_atrous_kappa_and_params(step):
    """sigma_n from 64 up takes the normal term as a series (no logarithm),
    below 64 in log form: both, at tile steps and a direct-load step."""
    H, W = 90, 150
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 500 + step)
    kappa = np.random.default_rng(5).uniform(0.25, 4.0, (H, W)).astype(np.float32)
    g = gbuf_dev(z, dzdx, dzdy, n)
    errs = {}
    for sz, sn, sl, kap in [(1.0, 128.0, 4.0, None), (1.0, 128.0, 4.0, kappa),
                            (2.0, 0.0, 1.0, kappa), (0.5, 32.0, 8.0, kappa),
                            (1.0, 64.0, 4.0, None), (1.0, 1.0, 4.0, None)]:
        out, vo = empty_like_dev((3, H, W)), empty_like_dev((H, W))
        L.sv_atrous(dev(c), dev(var), g, out, vo, step,
                    L.AtrousParams(sigma_z=sz, sigma_n=sn, sigma_l=sl),
                    kappa=None if kap is None else dev(kap))
        rc, rv = O.atrous(c, var, z, dzdx, dzdy, n, step, kappa=kap, sigma_z=sz, sigma_n=sn,
                          sigma_l=sl)
        key = f"sz={sz} sn={sn} sl={sl} kappa={kap is not None}"
        errs[key] = (rel_err(host(out), rc), rel_err(host(vo), rv))
        say(f"atrous params step={step} {key}: {errs[key][0]:.2e} {errs[key][1]:.2e} "
            f"worst {worst(host(out), rc)}")
    assert max(max(e) for e in errs.values()) <= TOL32, errs


@pytest.mark.parametrize("H,W", SIZES + [(130, 200)])
@pytest.mark.parametrize("step", [1, 2, 4, 8, 16, 5])
def test_atrous_sep(H, W, step):
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 600 + step + H, holes=(step == 4))
    P = W + 2
    g = gbuf_dev(z, dzdx, dzdy, n, P)
    for unit, want_var, inv in [(False, True, False), (False, False, True), (True, True, False)]:
        say(f"atrous_sep {H}x{W} step={step} unit={unit} var={want_var} inv={inv}")
        out, sh = empty_like_dev((3, H, W), P), empty_like_dev((3, H, W), P)
        vo = empty_like_dev((H, W), P) if want_var else None
        L.sv_atrous_sep(dev(c, P), dev(var, P), g, sh, out, vo, step,
                        L.AtrousParams(unit_weights=unit, inv_tonemap=inv))
        rc, rv, rsh = O.atrous_sep(c, var, z, dzdx, dzdy, n, step, unit_weights=unit,
                                   inv_tonemap=inv, want_var=want_var)
        assert rel_err(host(sh), rsh) <= TOL32
        assert rel_err(host(out), rc) <= TOL32
        if want_var:
            assert rel_err(host(vo), rv) <= TOL32


@pytest.mark.parametrize("sep", [False, True])
def test_atrous_launch_shape_does_not_change_results(sep):
    """Every launch shape the autotuner chooses from (persistent or not, any
    workgroups per CU, either tile height; for the separable level the
    two-pass form and both band heights of the fused one): bitwise
    identical output."""
    from paper_2312_06827_amd.autotune import CANDIDATES, SEP_CANDIDATES
    H, W = 300, 450
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 700)
    g = gbuf_dev(z, dzdx, dzdy, n)
    cd, vd = dev(c), dev(var)
    cands = [(per, bpc, 0, True) for per, bpc, _ in CANDIDATES[:6]] + \
        [(per, bpc, rows, False) for per, bpc, rows in SEP_CANDIDATES] if sep else \
        [(per, bpc, rows, False) for per, bpc, rows in CANDIDATES]
    for step in (1, 2, 8, 16):
        ref = None
        for per, bpc, rows, two_pass in cands:
            say(f"launch shape sep={sep} step={step} persistent={per} bpc={bpc} rows={rows}"
                f" two_pass={two_pass}")
            out, vo, sh = empty_like_dev((3, H, W)), empty_like_dev((H, W)), empty_like_dev((3, H, W))
            p = L.AtrousParams(persistent=per, blocks_per_cu=bpc, tile_rows=rows)
            if sep:
                L.sv_atrous_sep(cd, vd, g, sh if two_pass else None, out, vo, step, p)
            else:
                L.sv_atrous(cd, vd, g, out, vo, step, p)
            got = (host(out), host(vo))
            if ref is None:
                ref = got
                rc, rv = (O.atrous_sep if sep else O.atrous)(c, var, z, dzdx, dzdy, n, step)[:2]
                assert rel_err(got[0], rc) <= TOL32 and rel_err(got[1], rv) <= TOL32
            else:
                np.testing.assert_array_equal(got[0], ref[0])
                np.testing.assert_array_equal(got[1], ref[1])


@pytest.mark.parametrize("H,W", [(1, 1), (3, 70), (67, 131), (130, 200)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_atrous_sep_fused_equals_two_pass(H, W, dtype):
    """The single-kernel separable level (no scratch) gives bitwise the
    two-kernel result (the horizontal result rounded to the storage type
    on chip exactly as the scratch planes round it)."""
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 800 + H, holes=True)
    P = W + 5
    dv = lambda a: dev(a, P, dtype)
    g = L.GBuf(dv(z), dv(dzdx), dv(dzdy), dv(n))
    kappa = np.random.default_rng(H).uniform(0.5, 2.0, (H, W)).astype(np.float32)
    for step in (1, 2, 4, 8, 16, 32):
        for unit, want_var, inv, kap, sn in [(False, True, False, None, 128.0),
                                             (False, False, True, kappa, 128.0),
                                             (True, True, False, None, 128.0),
                                             (False, True, False, kappa, 128.0),
                                             (False, True, False, None, 16.0)]:
            say(f"sep fused {H}x{W} {dtype} step={step} unit={unit} var={want_var} inv={inv} "
                f"kappa={kap is not None} sigma_n={sn}")
            p = L.AtrousParams(unit_weights=unit, inv_tonemap=inv, sigma_n=sn)
            kd = None if kap is None else dev(kap, P)
            res = []
            for fused in (False, True):
                out = empty_like_dev((3, H, W), P, dtype)
                sh = empty_like_dev((3, H, W), P, dtype)
                vo = empty_like_dev((H, W), P) if want_var else None
                L.sv_atrous_sep(dv(c), dev(var, P), g, None if fused else sh, out, vo, step, p,
                                kappa=kd)
                res.append((host(out), None if vo is None else host(vo)))
            np.testing.assert_array_equal(res[1][0], res[0][0])
            if want_var:
                np.testing.assert_array_equal(res[1][1], res[0][1])


@pytest.mark.parametrize("H,W", [(37, 70), (130, 200)])
def test_temporal_variance_listing_equals_variance_pass(H, W):
    """sv_temporal writing the variance's pointwise part and its list, then
    sv_variance(listed), gives bitwise what sv_temporal then sv_variance
    give; twice in a row on one workspace (the second listing starts after
    what the first reading pass consumed)."""
    fr, st = _temporal_case(H, W, 57 + H)
    g = gbuf_dev(fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], None, fr["id"])
    prev = L.GBuf(dev(fr["prev_z"]), None, None, dev(fr["prev_n"]), dev(fr["prev_id"], None, torch.uint8))
    tp = L.TemporalParams(clamp=True, tonemap=True, use_id=True)
    res = []
    shared = L.variance_workspace(empty_like_dev((H, W)))
    for fused in (False, True, True):
        out = empty_like_dev((3, H, W))
        om1, om2 = empty_like_dev((H, W)), empty_like_dev((H, W))
        on = empty_like_dev((H, W), dtype=torch.uint8)
        var = empty_like_dev((H, W))
        work = shared if fused else L.variance_workspace(var)
        say(f"temporal + variance listing {H}x{W} fused={fused}")
        L.sv_temporal(dev(fr["rgb"]), g, dev(fr["mv"]), prev, dev(st["rgb"]), dev(st["m1"]),
                      dev(st["m2c"]), dev(st["n"], None, torch.uint8), out, om1, om2, on, tp,
                      var=var if fused else None, var_work=work if fused else None)
        L.sv_variance(om1, om2, on, g, var, L.VarianceParams(listed=fused), work)
        res.append((host(out), host(var)))
        assert list_consumed(work)
    for r in res[1:]:
        np.testing.assert_array_equal(r[0], res[0][0])
        np.testing.assert_array_equal(r[1], res[0][1])


def test_temporal_variance_listing_across_sizes():
    """The listing path (sv_temporal's list read by sv_variance with
    SV_V_LISTED) on one workspace sized for the largest frame, with frames
    of two sizes in turn, the smaller one under eight tiles: each frame's
    variance equals, bitwise, the two-pass variance on a fresh workspace."""
    big, small = (130, 200), (4, 64)
    tp = L.TemporalParams(clamp=True, tonemap=True, use_id=True)
    cases = {}
    for H, W in (big, small):
        fr, st = _temporal_case(H, W, 91 + H)
        g = gbuf_dev(fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], None, fr["id"])
        prev = L.GBuf(dev(fr["prev_z"]), None, None, dev(fr["prev_n"]),
                      dev(fr["prev_id"], None, torch.uint8))
        cases[(H, W)] = (fr, st, g, prev)

    def run(H, W, work, fused):
        fr, st, g, prev = cases[(H, W)]
        out = empty_like_dev((3, H, W))
        om1, om2 = empty_like_dev((H, W)), empty_like_dev((H, W))
        on = empty_like_dev((H, W), dtype=torch.uint8)
        var = empty_like_dev((H, W))
        if work is None:
            work = L.variance_workspace(var)
        L.sv_temporal(dev(fr["rgb"]), g, dev(fr["mv"]), prev, dev(st["rgb"]), dev(st["m1"]),
                      dev(st["m2c"]), dev(st["n"], None, torch.uint8), out, om1, om2, on, tp,
                      var=var if fused else None, var_work=work if fused else None)
        L.sv_variance(om1, om2, on, g, var, L.VarianceParams(listed=fused), work)
        assert list_consumed(work)
        return host(var)

    ref = {hw: run(*hw, None, False) for hw in (big, small)}
    shared = L.variance_workspace(empty_like_dev(big))
    for hw in (big, small, small, big, small):
        say(f"temporal listing {hw} on a workspace for {big}")
        np.testing.assert_array_equal(run(*hw, shared, True), ref[hw])
