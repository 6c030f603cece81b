"""Batched streams: every stream of a sv_batch plan equals, bitwise, the
same stream run alone through sv_denoise_frame (the same tile code; only
the launch differs), frame after frame of graph replays with other GPU
work in between.  Sizes are uneven and ragged."""

from dataclasses import replace

import numpy as np
import pytest
import torch

from paper_2312_06827_amd.pipeline import MOTION, MOTION_SEP, BatchDenoiser, Denoiser, FrameInputs
from paper_2312_06827_amd.scene import batched_configs, render_frame, with_size
from tests._util import make_hostile, say

pytestmark = pytest.mark.gpu

SIZES = [(60, 100), (130, 257), (64, 64), (37, 45), (9, 200)]  # (H, W)


def _streams(half, frames):
    base = batched_configs(len(SIZES), frames, half=half)
    return [with_size(c, w, h, frames) for c, (h, w) in zip(base, SIZES)]


@pytest.mark.parametrize("half,sep,levels,feedback,rows,graph", [
    (False, False, 5, "atrous0", 0, True), (True, False, 5, "atrous0", 0, True),
    (True, True, 5, "atrous0", 0, True), (False, True, 3, "temporal", 0, True),
    (False, False, 1, "temporal", 0, True), (True, False, 5, "atrous0", 1, True),
    (False, True, 5, "atrous0", 6, True), (False, False, 5, "atrous0", 0, False),
    (True, True, 5, "atrous0", 0, False)])
def test_batch_equals_single_streams(half, sep, levels, feedback, rows, graph):
    """rows: tile height of every level (0: the library default), as the
    autotuner passes it, in the batched launches and the single ones.
    graph: the plan's passes replayed as a HIP graph, or launched one by
    one."""
    dt = torch.float16 if half else torch.float32
    cfg = replace(MOTION_SEP if sep else MOTION, levels=levels, feedback=feedback)
    frames = 5
    scfg = _streams(half, frames)
    tiles = [(0, 0, rows)] * levels if rows else None
    say(f"batch: {len(SIZES)} streams half={half} sep={sep} levels={levels} feedback={feedback}"
        f" rows={rows} graph={graph}")
    batch = BatchDenoiser(SIZES, cfg, dt, tiles=tiles, graph=graph)
    singles = [Denoiser(h, w, cfg, dt, tiles=tiles) for (h, w) in SIZES]
    try:
        for f in range(frames):
            inputs = [FrameInputs.from_numpy(render_frame(c, f)) for c in scfg]
            outs = batch.frame(inputs)
            # other work on the GPU between two replays: the single streams
            refs = [d.frame(inp) for d, inp in zip(singles, inputs)]
            torch.cuda.synchronize()
            for i, (b, d) in enumerate(zip(batch.streams, singles)):
                assert b.k == d.k
                assert torch.equal(outs[i], refs[i]), (f, i)
                for name, tb, td in [("m1", b.m1[b.k], d.m1[d.k]), ("m2c", b.m2c[b.k], d.m2c[d.k]),
                                     ("n", b.n[b.k], d.n[d.k]), ("hist", b.c_hist[b.k], d.c_hist[d.k]),
                                     ("var", b.var, d.var)]:
                    assert torch.equal(tb, td), (f, i, name)
            say(f"  frame {f}: {len(SIZES)} streams bitwise equal; {batch.passes()} launches per frame")
        assert batch.passes() == 2 + levels  # temporal, variance, one per level (separable fused)
    finally:
        batch.close()


@pytest.mark.parametrize("half,sep", [(False, False), (True, True)])
def test_batch_hostile_inputs_equal_single_streams(half, sep):
    """Every kind of unusable depth and motion scattered over every stream
    (the single-stream path is held to the oracle on such frames by the
    degenerate-frame tests): each batched stream still equals, bitwise, the
    stream run alone."""
    dt = torch.float16 if half else torch.float32
    cfg = MOTION_SEP if sep else MOTION
    frames = 3
    scfg = _streams(half, frames)
    r = np.random.default_rng(77 + int(half) + 2 * int(sep))
    say(f"batch hostile inputs: {len(SIZES)} streams half={half} sep={sep}")
    batch = BatchDenoiser(SIZES, cfg, dt)
    singles = [Denoiser(h, w, cfg, dt) for (h, w) in SIZES]
    try:
        for f in range(frames):
            inputs = [FrameInputs.from_numpy(make_hostile(render_frame(c, f), r)) for c in scfg]
            outs = batch.frame(inputs)
            refs = [d.frame(inp) for d, inp in zip(singles, inputs)]
            torch.cuda.synchronize()
            for i, (b, d) in enumerate(zip(batch.streams, singles)):
                assert torch.equal(outs[i], refs[i]), (f, i)
                assert torch.equal(b.n[b.k], d.n[d.k]), (f, i)
                assert torch.equal(b.var, d.var), (f, i)
            say(f"  frame {f}: bitwise equal")
    finally:
        batch.close()


@pytest.mark.parametrize("half,sep", [(False, False), (True, False), (False, True), (True, True)])
def test_batch_streams_match_the_oracle(half, sep):
    """Every stream of a batch plan against the FP64 oracle run on that
    stream alone, frame after frame: 1e-5 with binary32 storage, 2e-3 with
    binary16 storage (against the oracle that rounds to binary16 at the
    same storage points); history lengths exactly."""
    import oracle as O
    from tests._util import rel_err
    dt = torch.float16 if half else torch.float32
    tol = 2e-3 if half else 1e-5
    cfg = MOTION_SEP if sep else MOTION
    ofilt = O.OracleParams(clamp=True, tonemap=True, use_id=True, separable=sep, half=half)
    frames = 5
    scfg = _streams(half, frames)
    say(f"batch vs oracle: {len(SIZES)} streams half={half} sep={sep}")
    batch = BatchDenoiser(SIZES, cfg, dt)
    states = [O.new_state(h, w) for (h, w) in SIZES]
    try:
        for f in range(frames):
            frs = [render_frame(c, f) for c in scfg]
            outs = batch.frame([FrameInputs.from_numpy(fr) for fr in frs])
            torch.cuda.synchronize()
            errs = []
            for i, (fr, b) in enumerate(zip(frs, batch.streams)):
                ref, states[i], ex = O.run_frame(fr, states[i], ofilt)
                np.testing.assert_array_equal(b.n[b.k].cpu().numpy(), ex["temporal"]["n"])
                e = rel_err(outs[i].double().cpu().numpy(), ref)
                errs.append(e)
                assert e <= tol, (f, i, SIZES[i], e)
            say(f"  frame {f}: max rel err per stream " + " ".join(f"{e:.1e}" for e in errs))
    finally:
        batch.close()


def test_batch_sixteen_uneven_streams_first_frames():
    """The sixteen-stream workload (640x360 .. 2560x1440, binary16), two
    frames, against single-stream runs."""
    scfg = batched_configs(16, 2, half=True)
    sizes = [(c.height, c.width) for c in scfg]
    say(f"batch of 16 streams, {sum(h * w for h, w in sizes) / 1e6:.1f} Mpix")
    batch = BatchDenoiser(sizes, MOTION, torch.float16)
    singles = [Denoiser(h, w, MOTION, torch.float16) for (h, w) in sizes]
    try:
        for f in range(2):
            inputs = [FrameInputs.from_numpy(render_frame(c, f)) for c in scfg]
            outs = batch.frame(inputs)
            refs = [d.frame(inp) for d, inp in zip(singles, inputs)]
            torch.cuda.synchronize()
            for i in range(16):
                assert torch.equal(outs[i], refs[i]), (f, i)
            say(f"  frame {f}: 16 streams bitwise equal")
    finally:
        batch.close()


def test_batch_learned_streams():
    """Batched streams with the network inside the temporal step equal the
    single streams bitwise."""
    from oracle import mlp as M
    from paper_2312_06827_amd import lib as L
    w = M.init_weights(7)
    w.w3 = np.random.default_rng(7).normal(0, 0.5, w.w3.shape)
    mlp = L.MLP(w.flat(), np.zeros(14), np.ones(14))
    scfg = _streams(False, 3)
    batch = BatchDenoiser(SIZES, MOTION, torch.float32, mlp=mlp)
    singles = [Denoiser(h, w_, MOTION, torch.float32, mlp=mlp) for (h, w_) in SIZES]
    say("batch of learned streams")
    try:
        for f in range(3):
            inputs = [FrameInputs.from_numpy(render_frame(c, f)) for c in scfg]
            outs = batch.frame(inputs)
            refs = [d.frame(inp) for d, inp in zip(singles, inputs)]
            torch.cuda.synchronize()
            for i in range(len(SIZES)):
                assert torch.equal(outs[i], refs[i]), (f, i)
                assert torch.equal(batch.streams[i].kappa, singles[i].kappa), (f, i)
    finally:
        batch.close()


@pytest.mark.parametrize("sep", [False, True])
def test_batch_with_adaptive_levels_and_per_stream_settings(sep):
    """Adaptive levels (control bytes from each stream's roughness) and
    per-stream settings (tone map on some streams, clipping on none): the
    plan still equals the streams run alone, bitwise."""
    from paper_2312_06827_amd import lib as L
    cfgs = [replace(MOTION_SEP if sep else MOTION, tonemap=(i % 2 == 0)) for i in range(len(SIZES))]
    frames = 3
    scfg = _streams(False, frames)
    rule = L.BlurRule()
    say(f"batch adaptive sep={sep}")
    batch = BatchDenoiser(SIZES, cfgs)
    singles = [Denoiser(h, w, c) for (h, w), c in zip(SIZES, cfgs)]
    ctl = [torch.empty((h, w), dtype=torch.uint8, device="cuda") for (h, w) in SIZES]
    try:
        for f in range(frames):
            frs = [render_frame(c, f) for c in scfg]
            inputs = []
            for i, fr in enumerate(frs):
                inp = FrameInputs.from_numpy(fr)
                L.sv_blur_control(torch.from_numpy(fr["roughness"]).cuda(), None, ctl[i], rule)
                inp.blur_ctl = ctl[i]
                inputs.append(inp)
            outs = batch.frame(inputs)
            refs = [d.frame(inp) for d, inp in zip(singles, inputs)]
            torch.cuda.synchronize()
            for i in range(len(SIZES)):
                assert torch.equal(outs[i], refs[i]), (f, i)
            say(f"  frame {f}: bitwise equal; {batch.passes()} launches per frame")
        # the 5x5 adaptive levels at steps 1 to 8 are one launch each, the one
        # at step 16 and the separable ones two (one per step class)
        assert batch.passes() == 2 + (2 * 5 if sep else 4 + 2)
    finally:
        batch.close()
