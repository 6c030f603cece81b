"""Degenerate frames through the frame driver against the oracle chain,
frame after frame: no surface anywhere (depth 0, or not finite), motion
that is unusable everywhere, a constant image, and images of one or two
pixels.  Outputs, temporal intermediates and variance within 1e-5 (the
variance, which is zero but for rounding residues in some of these cases,
measured in its own units: the mean squared luminance), history lengths
exact; the closed forms each case has are checked as well."""

from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle as O
from paper_2312_06827_amd.pipeline import MOTION, MOTION_SEP, PLAIN, Denoiser, FrameInputs
from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
from tests._util import make_hostile, rel_err, say

pytestmark = pytest.mark.gpu
TOL32 = 1e-5

FILTERS = {
    "plain": (PLAIN, O.OracleParams()),
    "motion": (MOTION, O.OracleParams(clamp=True, tonemap=True, use_id=True)),
    "motion_sep": (MOTION_SEP, O.OracleParams(clamp=True, tonemap=True, use_id=True,
                                              separable=True)),
}


def host(t):
    torch.cuda.synchronize()
    return t.detach().to(torch.float64).cpu().numpy() if t.dtype.is_floating_point \
        else t.detach().cpu().numpy()


def _frames(H, W, n=3):
    return list(sequence(with_size(CONFIGS["hd_motion"], W, H, n)))


def _run(frames, filt, ofilt):
    H, W = frames[0]["z"].shape
    den = Denoiser(H, W, filt)
    st = O.new_state(H, W)
    outs = []
    for f, fr in enumerate(frames):
        out = den.frame(FrameInputs.from_numpy(fr))
        ref, st, ex = O.run_frame(fr, st, ofilt)
        inter = den.intermediates()
        np.testing.assert_array_equal(host(inter["n"]), ex["temporal"]["n"])
        # a variance plane that is zero but for rounding residues (a constant
        # image, one pixel) is measured in its own units: differences below
        # 1e-12 of the mean squared luminance (binary32's resolution of a
        # square) are zero
        lsq = float(np.mean(ex["temporal"]["m1"] ** 2))
        errs = {"out": rel_err(host(out), ref),
                "temporal": rel_err(host(inter["t_rgb"]), ex["temporal"]["rgb"]),
                "m1": rel_err(host(inter["m1"]), ex["temporal"]["m1"]),
                "var": rel_err(host(inter["var"]), ex["var"], abs_floor=1e-7 * lsq)}
        say(f"  frame {f}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        assert max(errs.values()) <= TOL32, (f, errs)
        outs.append((host(out), host(inter["n"]), host(inter["var"])))
    return outs


@pytest.mark.parametrize("name", list(FILTERS))
@pytest.mark.parametrize("depth", [0.0, np.inf, np.nan])
def test_no_surface_anywhere(name, depth):
    """Every pixel empty: colour passes through unchanged (the tone map and
    its inverse fused in the chain return it), history lengths and
    variance are zero."""
    frames = _frames(37, 70)
    for fr in frames:
        fr["z"] = np.full_like(fr["z"], depth)
        fr["prev_z"] = np.full_like(fr["prev_z"], depth)
    say(f"no surface ({depth}), {name}")
    for (out, n, var), fr in zip(_run(frames, *FILTERS[name]), frames):
        assert np.all(n == 0) and np.all(var == 0.0)
        assert rel_err(out, fr["rgb"]) <= TOL32


@pytest.mark.parametrize("name", list(FILTERS))
def test_motion_unusable_everywhere(name):
    """Motion that is not finite or beyond 2^20 pixels: no history is ever
    taken, every pixel's history length is 1 and its variance the spatial
    estimate's."""
    frames = _frames(37, 70)
    for i, fr in enumerate(frames):
        fr["mv"] = np.full_like(fr["mv"], np.nan if i % 2 else 3.0e6)
    say(f"unusable motion, {name}")
    for _, n, _ in _run(frames, *FILTERS[name]):
        live = frames[0]["z"] > 0
        assert np.all(n[live] == 1)


@pytest.mark.parametrize("name", list(FILTERS))
def test_constant_image(name):
    """A constant colour over a moving scene is a fixed point of the whole
    chain: every output pixel equals it, up to the binary32 roundings of
    the chain (tone map, blend, five weighted means and the inverse tone
    map per frame, fed back over frames: within 5e-6 of the value, about
    40 ulps)."""
    frames = _frames(37, 70, 4)
    k = np.array([0.3, 0.55, 0.8], np.float32)[:, None, None]
    for fr in frames:
        fr["rgb"] = np.broadcast_to(k, fr["rgb"].shape).copy()
    say(f"constant image, {name}")
    for (out, _, _), fr in zip(_run(frames, *FILTERS[name]), frames):
        assert (np.abs(out - k) / k).max() <= 5e-6


@pytest.mark.parametrize("name", list(FILTERS))
@pytest.mark.parametrize("H,W", [(37, 70), (67, 131)])
def test_hostile_mixed_inputs(name, H, W):
    """Every kind of unusable input scattered over the frame, so that live
    and unusable pixels meet inside tiles and at their edges: empty pixels
    of every kind in the current and the previous depth (0, -0, negative,
    NaN, infinite), motion that is not finite or beyond 2^20 pixels, motion
    that leaves the image, and taps straddling its border.  Each frame
    through the frame driver against the oracle chain, to the same bars."""
    r = np.random.default_rng(4242 + H + len(name))
    frames = [make_hostile(fr, r) for fr in _frames(H, W, 3)]
    say(f"hostile mixed inputs {H}x{W}, {name}")
    _run(frames, *FILTERS[name])


@pytest.mark.parametrize("H,W", [(1, 1), (1, 2), (2, 1), (1, 70), (37, 1)])
def test_tiny_images(H, W):
    """Images of a single row, column or pixel (every stencil clipped to
    the image, every tile ragged)."""
    cfg = with_size(CONFIGS["hd_motion"], max(W, 8), max(H, 8), 3)
    frames = []
    for fr in sequence(cfg):
        fr = {k: (v[..., :H, :W].copy() if isinstance(v, np.ndarray) and v.ndim >= 2 else v)
              for k, v in fr.items()}
        frames.append(fr)
    for name in ("motion", "motion_sep"):
        say(f"tiny image {H}x{W}, {name}")
        _run(frames, *FILTERS[name])
