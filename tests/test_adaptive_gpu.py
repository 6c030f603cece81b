"""Blur adapted to scene features (Sections 3.2, 3.5) on the device against
the FP64 oracle: the control bytes bit for bit, each adaptive level (2D,
separable fused and two-pass) and whole frames of the driver within 1e-5
(binary32 storage)."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_06827_amd import lib as L
from paper_2312_06827_amd.pipeline import MOTION, MOTION_SEP, Denoiser, FrameInputs
from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
from tests._util import rel_err, say
from tests.test_parity_gpu import _atrous_inputs, dev, empty_like_dev, gbuf_dev, host

pytestmark = pytest.mark.gpu
TOL32 = 1e-5


def _ctl(r, H, W, budget_max=15):
    """Random control bytes: every budget 0..budget_max, shift on half."""
    b = r.integers(0, budget_max + 1, (H, W))
    b[r.random((H, W)) < 0.4] = 15
    s = (r.random((H, W)) < 0.5).astype(np.int64) * 16
    return (b | s).astype(np.uint8)


def test_blur_control_bit_exact():
    H, W = 45, 70
    r = np.random.default_rng(800)
    f32 = np.float32
    rough = r.uniform(-0.1, 0.5, (H, W)).astype(f32)
    ang = r.uniform(0.0, 12.0, (H, W)).astype(f32)
    # the thresholds themselves and their neighbours, and a NaN
    edge = [0.0, 0.05, 0.2]
    for i, v in enumerate(edge):
        rough[i, :3] = [np.nextafter(f32(v), f32(-1)), f32(v), np.nextafter(f32(v), f32(1))]
    ang[0, :3] = [np.nextafter(f32(6), f32(0)), f32(6), np.nextafter(f32(6), f32(9))]
    rough[5, 5] = np.nan
    P = W + 9
    for rule in [L.BlurRule(), L.BlurRule(shift=False), L.BlurRule(table=False),
                 L.BlurRule(rough_shift=0.1, it_rest=4)]:
        for use_angle in (False, True):
            say(f"blur control {rule} angle={use_angle}")
            ctl = empty_like_dev((H, W), P, torch.uint8)
            L.sv_blur_control(dev(rough, P), dev(ang, P) if use_angle else None, ctl, rule)
            ref = O.blur_control(rough, ang if use_angle else None, rule.rough_shift,
                                 rule.angle_shift, rule.rough_none, rule.rough_one,
                                 rule.it_none, rule.it_one, rule.it_rest, rule.shift, rule.table)
            np.testing.assert_array_equal(host(ctl), ref)


@pytest.mark.parametrize("H,W,level", [(5, 7, l) for l in range(5)] +
                         [(67, 131, l) for l in range(5)] +
                         [(130, 200, l) for l in range(5)] +
                         # several column tiles of the step-32 class (16 lattice
                         # columns of 8-column groups each), ragged at both ends
                         [(70, 1100, 3), (70, 1100, 4)])
def test_adaptive_level_2d(H, W, level):
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 900 + level + H, holes=(level == 1))
    ctl = _ctl(np.random.default_rng(901 + level), H, W)
    P = W + 5
    g = gbuf_dev(z, dzdx, dzdy, n, P)
    for want_var, inv in [(True, False), (False, True)]:
        say(f"adaptive 2d {H}x{W} level={level} var={want_var} inv={inv}")
        out = empty_like_dev((3, H, W), P)
        vo = empty_like_dev((H, W), P) if want_var else None
        L.sv_atrous_adaptive(dev(c, P), dev(var, P), g, dev(ctl, P, torch.uint8), None, out, vo,
                             level, False, L.AtrousParams(inv_tonemap=inv))
        rc, rv = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, ctl, level, inv_tonemap=inv,
                                   want_var=want_var)
        assert rel_err(host(out), rc) <= TOL32
        if want_var:
            assert rel_err(host(vo), rv) <= TOL32


@pytest.mark.parametrize("H,W", [(5, 7), (67, 131), (130, 200)])
@pytest.mark.parametrize("level", [0, 2, 3, 4])
def test_adaptive_level_separable(H, W, level):
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 950 + level + H, holes=(level == 2))
    ctl = _ctl(np.random.default_rng(951 + level), H, W)
    P = W + 3
    g = gbuf_dev(z, dzdx, dzdy, n, P)
    rc, rv = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, ctl, level, separable=True)
    for fused in (True, False):
        say(f"adaptive separable {H}x{W} level={level} fused={fused}")
        out, vo = empty_like_dev((3, H, W), P), empty_like_dev((H, W), P)
        scratch = None if fused else empty_like_dev((3, H, W), P)
        args = (dev(c, P), dev(var, P), g, dev(ctl, P, torch.uint8), scratch, out, vo, level,
                True, L.AtrousParams())
        L.sv_atrous_adaptive(*args)
        assert rel_err(host(out), rc) <= TOL32
        assert rel_err(host(vo), rv) <= TOL32


def test_adaptive_uniform_controls_equal_the_plain_levels():
    """Every pixel unshifted with a full budget: bitwise the plain level;
    every pixel shifted: bitwise the plain level at twice the step."""
    H, W = 96, 160
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 990)
    g = gbuf_dev(z, dzdx, dzdy, n)
    cd, vd = dev(c), dev(var)
    for level in (0, 3):
        for shift in (0, 16):
            ctl = torch.full((H, W), 15 | shift, dtype=torch.uint8, device="cuda")
            step = 1 << (level + (1 if shift else 0))
            for sep in (False, True):
                say(f"adaptive uniform level={level} shift={shift} sep={sep}")
                a, av = empty_like_dev((3, H, W)), empty_like_dev((H, W))
                b, bv = empty_like_dev((3, H, W)), empty_like_dev((H, W))
                L.sv_atrous_adaptive(cd, vd, g, ctl, None, a, av, level, sep, L.AtrousParams())
                if sep:
                    L.sv_atrous_sep(cd, vd, g, None, b, bv, step, L.AtrousParams())
                else:
                    L.sv_atrous(cd, vd, g, b, bv, step, L.AtrousParams())
                torch.cuda.synchronize()
                assert torch.equal(a, b) and torch.equal(av, bv)


@pytest.mark.parametrize("sep", [False, True])
def test_driver_with_adaptive_levels(sep):
    """The native frame driver with control bytes from the scene's roughness
    (Sections 3.2 and 3.5 rules) against the oracle chain, frame by frame."""
    cfg = with_size(CONFIGS["hd_motion"], 320, 180, 6)
    filt = MOTION_SEP if sep else MOTION
    ofilt = O.OracleParams(clamp=True, tonemap=True, use_id=True, separable=sep)
    den = Denoiser(cfg.height, cfg.width, filt)
    st = O.new_state(cfg.height, cfg.width)
    rule = L.BlurRule()
    worst_all = 0.0
    for f, fr in enumerate(sequence(cfg)):
        say(f"adaptive driver sep={sep} frame {f}")
        inp = FrameInputs.from_numpy(fr)
        inp.blur_ctl = torch.empty((cfg.height, cfg.width), dtype=torch.uint8, device="cuda")
        L.sv_blur_control(torch.from_numpy(fr["roughness"]).cuda(), None, inp.blur_ctl, rule)
        ctl = O.blur_control(fr["roughness"])
        np.testing.assert_array_equal(host(inp.blur_ctl), ctl)
        out = den.frame(inp)
        ref, st, _ = O.run_frame(fr, st, ofilt, ctl=ctl)
        e = rel_err(host(out), ref)
        worst_all = max(worst_all, e)
        assert e <= TOL32, (f, e)
    say(f"  worst {worst_all:.2e}")
    # every band of the roughness table is present in the scene
    assert set(np.unique(ctl & 15)) >= {0, 1, 15} and (ctl >> 4).any()


def test_adaptive_separable_beyond_the_fused_steps():
    """Level 5 shifted is step 64: only the two-pass form has it."""
    H, W = 40, 70
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 990)
    g = gbuf_dev(z, dzdx, dzdy, n)
    ctl = dev(np.full((H, W), 31, np.uint8), None, torch.uint8)
    out, vo = empty_like_dev((3, H, W)), empty_like_dev((H, W))
    with pytest.raises(L.SVError):
        L.sv_atrous_adaptive(dev(c), dev(var), g, ctl, None, out, vo, 5, True, L.AtrousParams())
    L.sv_atrous_adaptive(dev(c), dev(var), g, ctl, empty_like_dev((3, H, W)), out, vo, 5, True,
                         L.AtrousParams())
    rc, rv = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, np.full((H, W), 31, np.uint8), 5,
                               separable=True)
    assert rel_err(host(out), rc) <= TOL32


@pytest.mark.parametrize("sep", [False, True])
def test_adaptive_level_binary16(sep):
    """Binary16 storage: against the oracle rounding its stored colours to
    binary16 (within 2e-3)."""
    H, W = 67, 131
    c, var, z, dzdx, dzdy, n = _atrous_inputs(H, W, 970 + int(sep))
    q = lambda a: O.quantize_half(a)
    c, z, dzdx, dzdy, n = q(c), q(z), q(dzdx), q(dzdy), q(n)
    ctl = _ctl(np.random.default_rng(971), H, W)
    h16 = lambda a: dev(a, None, torch.float16)
    g = L.GBuf(h16(z), h16(dzdx), h16(dzdy), h16(n))
    for level in (0, 2):
        say(f"adaptive binary16 sep={sep} level={level}")
        out, vo = empty_like_dev((3, H, W), None, torch.float16), empty_like_dev((H, W))
        L.sv_atrous_adaptive(h16(c), dev(var), g, dev(ctl, None, torch.uint8), None, out, vo,
                             level, sep, L.AtrousParams())
        rc, rv = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, ctl, level, separable=sep,
                                   half_out=True)
        assert rel_err(host(out), rc) <= 2e-3
        assert rel_err(host(vo), rv) <= 2e-3
