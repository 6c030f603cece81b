"""Checkpoint and resume of a stream's state, and a frame whose every
history tap is unusable ("disocclusion storm").

A stream run for six frames equals, bitwise, the same stream run for three
frames, saved, loaded into a new denoiser and run for the last three.  A
frame whose motion sends every pixel off the previous image restarts every
history at one sample and equals that frame on a denoiser with no history
at all."""

from dataclasses import replace

import numpy as np
import pytest
import torch

from paper_2312_06827_amd.pipeline import MOTION, MOTION_SEP, Denoiser, FrameInputs
from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
from tests._util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,sep,feedback", [
    (torch.float32, False, "atrous0"), (torch.float16, False, "atrous0"),
    (torch.float32, True, "temporal")])
def test_resume_from_a_saved_state_is_bitwise(tmp_path, dtype, sep, feedback):
    half = dtype == torch.float16
    cfg = replace(with_size(CONFIGS["hd_motion"], 200, 120, 6), half=half)
    filt = replace(MOTION_SEP if sep else MOTION, feedback=feedback)
    frames = [FrameInputs.from_numpy(fr) for fr in sequence(cfg)]
    say(f"checkpoint {dtype} sep={sep} feedback={feedback}")
    full = Denoiser(cfg.height, cfg.width, filt, dtype)
    ref = [full.frame(fr).clone() for fr in frames]
    first = Denoiser(cfg.height, cfg.width, filt, dtype)
    for fr in frames[:3]:
        first.frame(fr)
    path = str(tmp_path / "state.npz")
    first.save_state(path)
    resumed = Denoiser(cfg.height, cfg.width, filt, dtype)
    resumed.load_state(path)
    assert resumed.k == first.k and resumed.frames == first.frames
    for i, fr in enumerate(frames[3:], start=3):
        out = resumed.frame(fr)
        torch.cuda.synchronize()
        assert torch.equal(out, ref[i]), i
    # a state of another size is refused
    other = Denoiser(cfg.height, cfg.width + 8, filt, dtype)
    with pytest.raises(ValueError):
        other.load_state(path)


def test_disocclusion_storm_restarts_every_history():
    cfg = with_size(CONFIGS["hd_motion"], 160, 96, 5)
    frames = list(sequence(cfg))
    den = Denoiser(cfg.height, cfg.width, MOTION)
    for fr in frames[:4]:
        den.frame(FrameInputs.from_numpy(fr))
    storm = dict(frames[4])
    r = np.random.default_rng(7)
    # every backward motion vector leaves the previous image
    storm["mv"] = (np.sign(r.uniform(-1, 1, storm["mv"].shape)) * 1e4).astype(storm["mv"].dtype)
    say("disocclusion storm")
    out = den.frame(FrameInputs.from_numpy(storm)).clone()
    n = den.state()["n"].cpu().numpy()
    live = np.isfinite(storm["z"]) & (storm["z"] > 0)
    assert np.all(n[live] == 1), np.unique(n[live])
    fresh = Denoiser(cfg.height, cfg.width, MOTION)
    out_fresh = fresh.frame(FrameInputs.from_numpy(storm))
    torch.cuda.synchronize()
    assert torch.equal(out, out_fresh)
