"""The temporal gradient (A-SVGF) on the device against the FP64 oracle:
the blend-factor map and the per-cell lambda within 1e-5 (absolute; both
lie in [0, 1]), on the scene's moving shadows and on random inputs with
every edge case of the projection (NaN and far motion, picks above 8,
depth mismatches, colliding samples)."""

from dataclasses import replace

import numpy as np
import pytest
import torch

from oracle import gradient as OG
from paper_2312_06827_amd import lib as L
from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
from tests._util import say
from tests.test_parity_gpu import dev, empty_like_dev, host

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _run(prev, re, fmv, fz, pick, z, dzdx, dzdy, dtype=torch.float32, levels=3, alpha=0.2,
         pitch=None):
    H, W = z.shape
    P = pitch or W
    dv = lambda a: dev(a, P, dtype)
    g = L.GBuf(dv(z), dv(dzdx), dv(dzdy), dv(np.zeros((3, H, W))))
    am = empty_like_dev((H, W), P)
    lam = torch.full(OG.cells_of(H, W), float("nan"), device="cuda")
    work = L.gradient_workspace(am)
    L.sv_temporal_gradient(dv(prev), dv(re), dv(fmv), dv(fz),
                           torch.from_numpy(np.ascontiguousarray(pick)).cuda(), g, am, work,
                           alpha=alpha, levels=levels, lam=lam)
    return host(am), host(lam)


def test_gradient_on_moving_shadows():
    cfg = replace(with_size(CONFIGS["hd_motion"], 200, 120, 4), channels=True)
    frames = list(sequence(cfg))
    for f in (1, 2, 3):
        fr, pv = frames[f], frames[f - 1]
        re = np.broadcast_to(fr["shadow_reshade"][None], (3,) + fr["z"].shape)
        args = (pv["shadow"], re, fr["fmv"], fr["fz"], fr["grad_pick"], fr["z"], fr["dzdx"],
                fr["dzdy"])
        am, lam = _run(*args)
        ram, rlam = OG.temporal_gradient(*args)
        say(f"gradient frame {f}: lambda>0 on {(rlam > 0).mean():.3f} of the cells, "
            f"max |d lambda| {np.abs(lam - rlam).max():.2e}")
        assert (rlam > 0).any()
        np.testing.assert_allclose(lam, rlam, atol=TOL, rtol=0)
        np.testing.assert_allclose(am, ram, atol=TOL, rtol=0)


@pytest.mark.parametrize("H,W", [(7, 11), (40, 70), (64, 131)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_gradient_random_inputs(H, W, dtype):
    r = np.random.default_rng(H * 1000 + W)
    q = (lambda a: a.astype(np.float16).astype(np.float64)) if dtype == torch.float16 \
        else (lambda a: a.astype(np.float32).astype(np.float64))
    prev = q(r.uniform(0, 2, (3, H, W)))
    re = q(np.where(r.random((3, H, W)) < 0.7, prev, r.uniform(0, 2, (3, H, W))))
    fmv = q(r.normal(0, 2.5, (2, H, W)))
    fmv[0][r.random((H, W)) < 0.02] = np.nan
    fmv[1][r.random((H, W)) < 0.02] = 500.0
    z = q(r.uniform(4, 6, (H, W)))
    z[r.random((H, W)) < 0.03] = 0.0  # empty pixels
    fz = q(z * np.where(r.random((H, W)) < 0.1, 1.5, 1.0))
    dzdx, dzdy = q(r.normal(0, 0.05, (H, W))), q(r.normal(0, 0.05, (H, W)))
    pick = r.integers(0, 10, OG.cells_of(H, W)).astype(np.uint8)  # 9: no sample
    for levels in (0, 3):
        say(f"gradient random {H}x{W} {dtype} levels={levels}")
        am, lam = _run(prev, re, fmv, fz, pick, z, dzdx, dzdy, dtype, levels, pitch=W + 3)
        ram, rlam = OG.temporal_gradient(prev, re, fmv, fz, pick, z, dzdx, dzdy, levels=levels)
        np.testing.assert_allclose(lam, rlam, atol=TOL, rtol=0)
        np.testing.assert_allclose(am, ram, atol=TOL, rtol=0)


@pytest.mark.parametrize("levels", [1, 2, 4, 5, 6])
def test_gradient_levels_across_tiles(levels):
    """Every cascade depth on a grid of cells several tiles wide and high
    (134 x 67 cells, ragged at both edges), the steps reaching past a
    tile's width at depth 6."""
    H, W = 200, 401
    r = np.random.default_rng(4000 + levels)
    q = lambda a: a.astype(np.float32).astype(np.float64)
    prev = q(r.uniform(0, 2, (3, H, W)))
    re = q(np.where(r.random((3, H, W)) < 0.6, prev, r.uniform(0, 2, (3, H, W))))
    fmv = q(r.normal(0, 2.0, (2, H, W)))
    z = q(r.uniform(4, 6, (H, W)))
    z[r.random((H, W)) < 0.02] = 0.0
    fz = q(z * np.where(r.random((H, W)) < 0.05, 1.5, 1.0))
    dzdx, dzdy = q(r.normal(0, 0.05, (H, W))), q(r.normal(0, 0.05, (H, W)))
    pick = r.integers(0, 10, OG.cells_of(H, W)).astype(np.uint8)
    say(f"gradient {H}x{W} levels={levels}")
    am, lam = _run(prev, re, fmv, fz, pick, z, dzdx, dzdy, levels=levels, pitch=W + 7)
    ram, rlam = OG.temporal_gradient(prev, re, fmv, fz, pick, z, dzdx, dzdy, levels=levels)
    np.testing.assert_allclose(lam, rlam, atol=TOL, rtol=0)
    np.testing.assert_allclose(am, ram, atol=TOL, rtol=0)


def test_gradient_without_change_keeps_alpha():
    H, W = 33, 50
    r = np.random.default_rng(9)
    prev = r.uniform(0, 1, (3, H, W))
    z = np.full((H, W), 5.0)
    zero = np.zeros((H, W))
    pick = r.integers(0, 9, OG.cells_of(H, W)).astype(np.uint8)
    am, lam = _run(prev, prev, np.zeros((2, H, W)), z, pick, z, zero, zero, alpha=0.3)
    assert np.all(lam == 0.0)
    np.testing.assert_array_equal(am, np.float32(0.3))


def test_gradient_with_tiny_weights():
    """A cell without a sample between two that lie far across depth edges
    (weights about e^-733, far below binary32's range, in the ratio 3:1):
    its lambda is the ratio of their weighted means, as the oracle forms
    it, not 0 from weights that underflowed."""
    H, W = 3, 9
    g = 1e-3
    den = abs(np.float32(g) * 3.0) + 1e-10
    z = np.full((H, W), 5.0)
    z[1, 1] = 5.0 + 733.0 * den
    z[1, 7] = 5.0 + 733.0 * den + np.log(3.0) * den
    z = z.astype(np.float32).astype(np.float64)
    dzdx = np.zeros((H, W))
    dzdx[1, 4] = g
    dzdx = dzdx.astype(np.float32).astype(np.float64)
    dzdy = np.zeros((H, W))
    prev = np.full((3, H, W), 0.5)
    re = np.full((3, H, W), 0.5)
    prev[:, 1, 1], re[:, 1, 1] = 0.7, 1.0   # delta 0.3, norm 1
    prev[:, 1, 7], re[:, 1, 7] = 2.0, 1.5   # delta -0.5, norm 2
    pick = np.array([[4, 9, 4]], np.uint8)  # the middle stratum has no sample
    fmv = np.zeros((2, H, W))
    for levels in (1, 3):
        am, lam = _run(prev, re, fmv, z, pick, z, dzdx, dzdy, levels=levels)
        ram, rlam = OG.temporal_gradient(prev, re, fmv, z, pick, z, dzdx, dzdy, levels=levels)
        say(f"tiny weights, levels {levels}: lambda {lam.ravel()} oracle {rlam.ravel()}")
        assert rlam[0, 1] > 0.05
        np.testing.assert_allclose(lam, rlam, atol=TOL, rtol=0)
        np.testing.assert_allclose(am, ram, atol=TOL, rtol=0)
