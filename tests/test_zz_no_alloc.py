"""The allocation-free variance entry point (sv_variance_noalloc) against
sv_variance with a caller workspace: bitwise the same on two calls in a
row, the second on a smaller frame (the fixed workspace keeps what the
first call left there)."""

import numpy as np
import pytest
import torch

from paper_2312_06827_amd import lib as L
from tests._util import random_gbuf, say

pytestmark = pytest.mark.gpu


def _case(H, W, seed):
    r = np.random.default_rng(seed)
    z, dzdx, dzdy, n = random_gbuf(r, H, W)
    z = z.copy()
    z[r.random((H, W)) < 0.02] = 0.0  # pixels without a surface
    m1 = r.uniform(0.05, 1.0, (H, W)).astype(np.float32)
    m2c = (m1 * m1 * r.uniform(0.0, 0.5, (H, W))).astype(np.float32)
    hn = r.integers(0, 9, (H, W)).astype(np.uint8)  # short and long histories
    d = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda()
    g = L.GBuf(d(z), d(dzdx), d(dzdy), d(n))
    return d(m1), d(m2c), d(hn, torch.uint8), g


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_variance_noalloc_equals_variance(dtype):
    vp = L.VarianceParams()
    for k, (H, W) in enumerate([(270, 480), (37, 70)]):
        m1, m2c, hn, g = _case(H, W, 10 + k)
        if dtype == torch.float16:
            g = L.GBuf(g.z.half(), g.dzdx.half(), g.dzdy.half(), g.n.half())
        say(f"variance noalloc {H}x{W} {dtype}, call {k + 1}")
        ref = torch.full((H, W), float("nan"), device="cuda")
        L.sv_variance(m1, m2c, hn, g, ref, vp, L.variance_workspace(ref))
        got = torch.full((H, W), float("nan"), device="cuda")
        L.sv_variance_noalloc(m1, m2c, hn, g, got, vp)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), (H, W, dtype)
        # short histories took the spatial branch on both sides
        assert int(((hn > 0) & (hn < 4)).sum()) > 0
