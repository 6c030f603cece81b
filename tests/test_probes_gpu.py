"""The library's measurement probes on the device: the copy probe copies,
and the issue-rate probe's chains give finite results and issue costs in a
plausible range (between half a slot and eight slots of an FMA)."""

import pytest
import torch

from paper_2312_06827_amd import lib as L
from tests._util import say

pytestmark = pytest.mark.gpu


def test_copy_probe_copies():
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    L.sv_probe_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)


def test_issue_probe():
    import bench
    out = torch.full((64 * 256,), float("nan"), device="cuda")
    for kind in range(5):
        L.sv_probe_issue(out, kind, 16)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all(), kind
    # the benchmark's own sizing: each timed chain runs 0.5-2.5 ms, far
    # above the launch overhead that would otherwise set the ratios
    costs = bench.issue_costs(torch)
    say(f"issue costs in FMA slots: {costs}")
    for k, c in costs.items():
        assert 0.5 <= c <= 8.0, (k, c)
