"""The autotuner on the device: every level gets a shape from its
candidate set, the choice is cached by device, size, type, form and level,
a cached choice is returned without timing, and a frame run with the
tuned shapes equals one with the library defaults bitwise."""

import json

import pytest
import torch

from paper_2312_06827_amd import autotune as A
from paper_2312_06827_amd.pipeline import MOTION, MOTION_SEP, Denoiser, FrameInputs
from paper_2312_06827_amd.scene import CONFIGS, render_frame, with_size
from tests._util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("separable,dtype", [(False, torch.float32), (True, torch.float32),
                                             (False, torch.float16)])
def test_tiles_for_choose_from_the_candidates_and_cache(tmp_path, monkeypatch, separable, dtype):
    H, W = 96, 200
    cache = str(tmp_path / "tune.json")
    say(f"autotune {H}x{W} separable={separable} {dtype}")
    shapes = A.tiles_for(H, W, dtype, separable=separable, cache=cache)
    allowed = set(A.SEP_CANDIDATES if separable else A.CANDIDATES)
    assert len(shapes) == 5 and all(tuple(s) in allowed for s in shapes), shapes
    with open(cache) as f:
        table = json.load(f)
    dev = torch.cuda.get_device_name()
    for i, s in enumerate(shapes):
        assert table[A._key(dev, W, H, dtype, separable, i)] == list(s)

    # a cached choice comes back without timing anything
    def no_tuning(*args, **kwargs):
        raise AssertionError("tuned again although every level is cached")

    monkeypatch.setattr(A, "tune", no_tuning)
    assert A.tiles_for(H, W, dtype, separable=separable, cache=cache) == [tuple(s) for s in shapes]


@pytest.mark.parametrize("separable", [False, True])
def test_tuned_shapes_leave_the_frame_unchanged(tmp_path, separable):
    cfg = with_size(CONFIGS["hd_motion"], 256, 144, 3)
    shapes = A.tiles_for(cfg.height, cfg.width, separable=separable, cache=str(tmp_path / "t.json"))
    filt = MOTION_SEP if separable else MOTION
    say(f"tuned frame separable={separable} shapes={shapes}")
    a = Denoiser(cfg.height, cfg.width, filt, tiles=shapes)
    b = Denoiser(cfg.height, cfg.width, filt)
    for f in range(cfg.frames):
        inp = FrameInputs.from_numpy(render_frame(cfg, f))
        oa, ob = a.frame(inp).clone(), b.frame(inp).clone()
        torch.cuda.synchronize()
        assert torch.equal(oa, ob), f
