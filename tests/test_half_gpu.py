"""Binary16 storage form: colour, G-buffer and motion planes stored as
binary16, moments and variance as binary32, all arithmetic in binary32.

Two kinds of check:

* exact: with inputs representable in binary16, a call on binary16 planes
  computes what the binary32 call computes and rounds it to binary16 (RNE)
  at the store; moments, variance and history lengths are bitwise equal;
* parity: against the FP64 oracle run with binary16 rounding at the same
  storage points (inputs, every stored colour, the separable pass's
  scratch), maximum relative error 2e-3 with the same per-plane floor as
  the binary32 tests.  Errors against the unrounded oracle and against the
  binary32 device path are printed, not gated.
"""

from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_06827_amd import lib as L
from paper_2312_06827_amd.pipeline import MOTION, MOTION_SEP, Denoiser, FrameInputs
from paper_2312_06827_amd.scene import CONFIGS, render_frame, sequence, with_size
from tests._util import rel_err, say, worst

pytestmark = pytest.mark.gpu

TOL16 = 2e-3


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().to(torch.float64).cpu().numpy() if t.dtype.is_floating_point \
        else t.detach().cpu().numpy()


def h16(t):
    """binary32 device tensor rounded to binary16 (RNE), as float64 numpy."""
    return host(t.to(torch.float16))


def half_frame(H, W, frame=3, seed=3):
    cfg = replace(with_size(CONFIGS["uhd_half"], W, H, frame + 1), seed=seed)
    return render_frame(cfg, frame)


def gbuf(fr, dtype, prev=False):
    if prev:
        return L.GBuf(dev(fr["prev_z"], dtype), None, None, dev(fr["prev_n"], dtype),
                      dev(fr["prev_id"], torch.uint8))
    return L.GBuf(dev(fr["z"], dtype), dev(fr["dzdx"], dtype), dev(fr["dzdy"], dtype),
                  dev(fr["n"], dtype), dev(fr["id"], torch.uint8))


def _atrous_case(H, W, seed):
    fr = half_frame(H, W, seed=seed)
    assert fr["z"].dtype == np.float16
    c = O.tonemap(fr["rgb"]).astype(np.float16)  # representable in binary16
    var = np.random.default_rng(seed).uniform(0.001, 0.05, (H, W)).astype(np.float32)
    return fr, c, var


# ---- exact: binary16 storage = binary32 arithmetic + rounding at the store --------

@pytest.mark.parametrize("sep", [False, True])
@pytest.mark.parametrize("step", [1, 2, 16])
def test_atrous_half_is_rounded_f32(sep, step):
    H, W = 70, 133
    fr, c, var = _atrous_case(H, W, 40 + step)
    say(f"atrous f16 vs rounded f32: sep={sep} step={step}")
    res = {}
    for dt in (torch.float32, torch.float16):
        out = torch.empty((3, H, W), dtype=dt, device="cuda")
        sh = torch.empty((3, H, W), dtype=dt, device="cuda")
        vo = torch.empty((H, W), dtype=torch.float32, device="cuda")
        if sep:
            L.sv_atrous_sep(dev(c, dt), dev(var, torch.float32), gbuf(fr, dt), sh, out, vo,
                            step, L.AtrousParams())
        else:
            L.sv_atrous(dev(c, dt), dev(var, torch.float32), gbuf(fr, dt), out, vo, step,
                        L.AtrousParams())
        res[dt] = (out, vo, sh)
    o32, v32, s32 = res[torch.float32]
    o16, v16, s16 = res[torch.float16]
    if sep:
        # the vertical pass reads the rounded scratch, so only the scratch
        # itself is compared; the two instantiations of the horizontal pass
        # are compiled separately and a few binary32 results differ in the
        # last bit, which can move a rounding by one binary16 ulp
        a, b = host(s16), h16(s32)
        diff = a != b
        ulp16 = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(b), 2.0 ** -14))) - 10)
        assert diff.mean() <= 1e-3
        assert np.all(np.abs(a - b)[diff] <= ulp16[diff])
    else:
        np.testing.assert_array_equal(host(o16), h16(o32))
        np.testing.assert_array_equal(host(v16), host(v32))


def test_temporal_half_is_rounded_f32():
    H, W = 67, 131
    fr = half_frame(H, W, seed=9)
    r = np.random.default_rng(9)
    hist = (fr["clean"].astype(np.float32) * r.uniform(0.7, 1.3, (3, H, W))).astype(np.float16)
    m1 = (hist.astype(np.float32).mean(0) * r.uniform(0.9, 1.1, (H, W))).astype(np.float32)
    m2c = (m1 * m1 * r.uniform(0.0, 1.0, (H, W))).astype(np.float32)
    hn = r.integers(0, 13, (H, W)).astype(np.uint8)
    say("temporal f16 vs rounded f32")
    res = {}
    for dt in (torch.float32, torch.float16):
        out = torch.empty((3, H, W), dtype=dt, device="cuda")
        om1 = torch.empty((H, W), dtype=torch.float32, device="cuda")
        om2 = torch.empty_like(om1)
        on = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        L.sv_temporal(dev(fr["rgb"], dt), gbuf(fr, dt), dev(fr["mv"], dt), gbuf(fr, dt, True),
                      dev(hist, dt), dev(m1, torch.float32), dev(m2c, torch.float32),
                      dev(hn, torch.uint8), out, om1, om2, on,
                      L.TemporalParams(clamp=True, tonemap=True, use_id=True))
        res[dt] = (out, om1, om2, on)
    a, b = res[torch.float32], res[torch.float16]
    np.testing.assert_array_equal(host(b[0]), h16(a[0]))
    for i in (1, 2, 3):
        np.testing.assert_array_equal(host(b[i]), host(a[i]))


# ---- parity with the binary16-rounding oracle -------------------------------------

@pytest.mark.parametrize("H,W", [(5, 7), (70, 133)])
@pytest.mark.parametrize("step", [1, 4, 16])
def test_atrous_half_parity(H, W, step):
    fr, c, var = _atrous_case(H, W, 60 + step + H)
    g = gbuf(fr, torch.float16)
    for sep in (False, True):
        say(f"atrous f16 parity {H}x{W} step={step} sep={sep}")
        out = torch.empty((3, H, W), dtype=torch.float16, device="cuda")
        sh = torch.empty_like(out)
        vo = torch.empty((H, W), dtype=torch.float32, device="cuda")
        args = (fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], step)
        if sep:
            L.sv_atrous_sep(dev(c, torch.float16), dev(var, torch.float32), g, sh, out, vo, step,
                            L.AtrousParams())
            rc, rv, rsh = O.atrous_sep(c, var, *args, half_out=True)
            assert rel_err(host(sh), rsh) <= TOL16
        else:
            L.sv_atrous(dev(c, torch.float16), dev(var, torch.float32), g, out, vo, step,
                        L.AtrousParams())
            rc, rv = O.atrous(c, var, *args, half_out=True)
        e = (rel_err(host(out), rc), rel_err(host(vo), rv))
        say(f"  rel err colour {e[0]:.2e} var {e[1]:.2e}")
        assert max(e) <= TOL16, (e, worst(host(out), rc))


def _elementwise_rel(gpu, ora, floor=1e-3):
    g = np.asarray(gpu, np.float64).reshape(-1, *gpu.shape[-2:])
    o = np.asarray(ora, np.float64).reshape(-1, *ora.shape[-2:])
    out = []
    for gp, op in zip(g, o):
        den = np.maximum(np.abs(op), floor * np.sqrt(np.mean(op * op)))
        out.append(np.abs(gp - op) / np.where(den > 0, den, 1.0))
    return np.stack(out)


def _run_half_sequence(cfg, sep, frames=None, tail=None):
    """tail: None gates the maximum at TOL16; (q, cap) gates the q-quantile
    of the output's element errors at TOL16 and their maximum at cap."""
    filt = MOTION_SEP if sep else MOTION
    ofilt = O.OracleParams(clamp=True, tonemap=True, use_id=True, separable=sep, half=True)
    oraw = replace(ofilt, half=False)
    d16 = Denoiser(cfg.height, cfg.width, filt, dtype=torch.float16)
    d32 = Denoiser(cfg.height, cfg.width, filt, dtype=torch.float32)
    st, st_raw = O.new_state(cfg.height, cfg.width), O.new_state(cfg.height, cfg.width)
    fails = []
    for f, fr in enumerate(sequence(cfg, 0, frames)):
        o16 = d16.frame(FrameInputs.from_numpy(fr))
        fr32 = {k: (v.astype(np.float32) if v.dtype == np.float16 else v) for k, v in fr.items()}
        o32 = d32.frame(FrameInputs.from_numpy(fr32))
        ref, st, ex = O.run_frame(fr, st, ofilt)
        raw, st_raw, _ = O.run_frame(fr, st_raw, oraw)
        inter = d16.intermediates()
        np.testing.assert_array_equal(host(inter["n"]), ex["temporal"]["n"])
        g16 = host(o16)
        errs = {
            "out": rel_err(g16, ref),
            "temporal": rel_err(host(inter["t_rgb"]), ex["temporal"]["rgb"]),
            "m1": rel_err(host(inter["m1"]), ex["temporal"]["m1"]),
            "var": rel_err(host(inter["var"]), ex["var"]),
        }
        d_raw = np.abs(g16 - raw) / np.maximum(np.abs(raw), 1e-3 * np.sqrt(np.mean(raw ** 2)))
        d_f32 = np.abs(g16 - host(o32)) / np.maximum(np.abs(raw), 1e-3 * np.sqrt(np.mean(raw ** 2)))
        if errs["out"] > TOL16 * 0.8:
            wo = worst(g16, ref)
            say(f"    worst out (plane, y, x, device, oracle): {wo}; oracle luminance there "
                f"{O.luma(ref)[wo[1], wo[2]]:.3f}, history length {int(ex['temporal']['n'][wo[1], wo[2]])}")
        say(f"  frame {f}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items())
            + f" | vs unrounded oracle p50 {np.median(d_raw):.1e} p99 {np.quantile(d_raw, 0.99):.1e}"
            f" max {d_raw.max():.1e} | vs f32 device p99 {np.quantile(d_f32, 0.99):.1e}"
            f" max {d_f32.max():.1e}")
        if tail is not None:
            q, cap = tail
            eo = _elementwise_rel(g16, ref)
            qv = float(np.quantile(eo, q))
            say(f"    output error quantile {q}: {qv:.2e}, max {eo.max():.2e} "
                f"({int((eo > TOL16).sum())} of {eo.size} elements above {TOL16})")
            if qv > TOL16 or eo.max() > cap:
                fails.append((f, "out-tail", qv, float(eo.max())))
            errs.pop("out")
        fails += [(f, k, v) for k, v in errs.items() if v > TOL16]
    assert not fails, fails


@pytest.mark.parametrize("sep", [False, True])
def test_half_sequence_reduced(sep):
    cfg = with_size(CONFIGS["uhd_half"], 480, 270, 10)
    say(f"f16 sequence 480x270 motion, separable={sep}, 10 frames")
    _run_half_sequence(cfg, sep)


def _ulp16(x):
    """One binary16 ulp at |x| (subnormal spacing below 2^-14)."""
    return 2.0 ** (np.floor(np.log2(np.maximum(np.abs(x), 2.0 ** -14))) - 10)


def _flips(dev16, ora16):
    """Storage-rounding flips: elements where the device's binary16 value
    and the oracle's differ.  From shared inputs each must be one binary16
    ulp, where the binary32 result and the FP64 one fall on either side of a
    rounding midpoint.  Returns (count, all of them one ulp)."""
    diff = dev16 != ora16
    one = np.abs(dev16 - ora16)[diff] <= _ulp16(ora16)[diff]
    return int(diff.sum()), bool(np.all(one))


@pytest.mark.timeout(900)
def test_half_4k_stages_and_chain():
    """3840x2160, binary16 storage, six frames of the moving sequence (the
    temporal variance of the history takes over at n >= 4).

    Gated, per frame, every stage from shared inputs at the 2e-3 maximum:
    the temporal step from the oracle's own history (as the device stores
    it: binary16 colour, binary32 moments), the variance from the device's
    temporal moments, and each of the five levels from the device's own
    previous level.  Each stage's binary16 outputs may differ from the
    oracle's only by single-ulp storage-rounding flips, which are counted.

    Reported, not gated: the chained run (each side feeding back its own
    history), whose flips compound through the levels and frames: its
    maximum error, the elements above 2e-3 and the elements that differ at
    all; and on the last frame its error against the unrounded oracle and
    the binary32 device path."""
    cfg = CONFIGS["uhd_half"]
    F = 6
    H, W = cfg.height, cfg.width
    ofilt = O.OracleParams(clamp=True, tonemap=True, use_id=True, half=True)
    oraw = replace(ofilt, half=False)
    f16, f32t = torch.float16, torch.float32
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    d16 = Denoiser(H, W, MOTION, dtype=f16)
    d32 = Denoiser(H, W, MOTION, dtype=f32t)
    st, st_raw = O.new_state(H, W), O.new_state(H, W)
    tp, vp = MOTION.temporal(), MOTION.variance()
    fails = []
    for f, fr in enumerate(sequence(cfg, 0, F)):
        say(f"4K binary16 frame {f}: stages")
        g, prev = gbuf(fr, f16), gbuf(fr, f16, prev=True)
        # -- temporal, from the oracle's history as the device stores it
        m1s, m2cs = f32(st["m1"]), f32(st["m2"] - st["m1"] ** 2)
        st_s = {"rgb": st["rgb"], "m1": m1s, "m2": m2cs + m1s ** 2, "n": st["n"]}
        t = O.temporal(fr, st_s, ofilt)
        out = torch.empty((3, H, W), dtype=f16, device="cuda")
        om1 = torch.empty((H, W), dtype=f32t, device="cuda")
        om2 = torch.empty_like(om1)
        on = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        L.sv_temporal(dev(fr["rgb"], f16), g, dev(fr["mv"], f16), prev, dev(st["rgb"], f16),
                      dev(m1s, f32t), dev(m2cs, f32t), dev(st["n"], torch.uint8),
                      out, om1, om2, on, tp)
        np.testing.assert_array_equal(host(on), t["n"])
        hm1, hm2c, t_rgb = host(om1), host(om2), host(out)
        e = {"temporal": rel_err(t_rgb, t["rgb"]), "m1": rel_err(hm1, t["m1"]),
             "m2": rel_err(hm2c + hm1 ** 2, t["m2"])}
        flips = {"temporal": _flips(t_rgb, t["rgb"])}
        # -- variance, from the device's moments
        var = torch.empty((H, W), dtype=f32t, device="cuda")
        L.sv_variance(om1, om2, on, g, var, vp, L.variance_workspace(var))
        rv = O.variance(hm1, hm2c + hm1 ** 2, host(on), fr["z"], fr["dzdx"], fr["dzdy"], fr["n"])
        e["var"] = rel_err(host(var), rv)
        # -- the five levels, each from the device's previous one
        c, v = out, var
        for i in range(5):
            last = i == 4
            co = torch.empty((3, H, W), dtype=f16, device="cuda")
            vo = None if last else torch.empty((H, W), dtype=f32t, device="cuda")
            L.sv_atrous(c, v, g, co, vo, 1 << i, MOTION.atrous(inv_tonemap=last))
            rc, rvo = O.atrous(host(c), host(v), fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], 1 << i,
                               inv_tonemap=last, half_out=True, want_var=not last)
            hc = host(co)
            e[f"level{i}"] = rel_err(hc, rc)
            flips[f"level{i}"] = _flips(hc, rc)
            if not last:
                e[f"var{i}"] = rel_err(host(vo), rvo)
            c, v = co, vo
        say("  " + " ".join(f"{k}={x:.2e}" for k, x in e.items()))
        say("  storage-rounding flips (count, all one ulp): "
            + " ".join(f"{k}={x}" for k, x in flips.items()))
        fails += [(f, k, x) for k, x in e.items() if x > TOL16]
        fails += [(f, k, "flip of more than one ulp") for k, x in flips.items() if not x[1]]
        # -- the chained run, reported
        o16 = host(d16.frame(FrameInputs.from_numpy(fr)))
        ref, st, ex = O.run_frame(fr, st, ofilt)
        np.testing.assert_array_equal(host(d16.intermediates()["n"]), ex["temporal"]["n"])
        eo = _elementwise_rel(o16, ref)
        say(f"  chained output: max rel err {eo.max():.2e}, {int((eo > TOL16).sum())} of "
            f"{eo.size} elements above {TOL16}, {int((o16 != ref).sum())} differ at all; "
            f"history lengths equal")
        rr, st_raw, _ = O.run_frame(fr, st_raw, oraw)
        fr32 = {k: (x.astype(np.float32) if x.dtype == np.float16 else x) for k, x in fr.items()}
        o32 = d32.frame(FrameInputs.from_numpy(fr32))
        if f == F - 1:
            o32 = host(o32)
            er = _elementwise_rel(o16, rr)
            e32 = _elementwise_rel(o16, o32)
            say(f"  vs the unrounded oracle: p50 {np.median(er):.1e} p99 {np.quantile(er, 0.99):.1e}"
                f" max {er.max():.1e}; vs the binary32 device path: p50 {np.median(e32):.1e}"
                f" p99 {np.quantile(e32, 0.99):.1e} max {e32.max():.1e}")
    assert not fails, fails
