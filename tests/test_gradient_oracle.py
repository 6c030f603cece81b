"""Pins of the temporal-gradient oracle (oracle/gradient.py) against closed
forms, brute force and a library routine (CPU only)."""

import numpy as np
import pytest
from scipy.ndimage import correlate

from oracle import gradient as G


def _frame(H, W, seed=0):
    r = np.random.default_rng(seed)
    prev = r.uniform(0.1, 1.0, (3, H, W))
    z = np.full((H, W), 5.0)
    dz = np.zeros((H, W))
    pick = r.integers(0, 9, G.cells_of(H, W)).astype(np.uint8)
    return prev, z, dz, pick


def test_no_change_gives_no_gradient():
    H, W = 20, 26
    prev, z, dz, pick = _frame(H, W)
    fmv = np.zeros((2, H, W))
    am, lam = G.temporal_gradient(prev, prev, fmv, z, pick, z, dz, dz, alpha=0.2)
    assert np.all(lam == 0.0)
    np.testing.assert_array_equal(am, 0.2)


@pytest.mark.parametrize("scale,expect", [(2.0, 0.5), (0.0, 1.0), (0.5, 0.5)])
def test_uniform_relative_change_gives_its_ratio(scale, expect):
    # every sample changes by the same factor, so |delta| / norm is the
    # same ratio everywhere and the normalized convolution keeps it
    H, W = 21, 24
    prev, z, dz, pick = _frame(H, W, 1)
    fmv = np.zeros((2, H, W))
    am, lam = G.temporal_gradient(prev, scale * prev, fmv, z, pick, z, dz, dz, alpha=0.2)
    np.testing.assert_allclose(lam, expect, rtol=1e-13)
    np.testing.assert_allclose(am, (1 - expect) * 0.2 + expect, rtol=1e-13)


def test_projection_shift_conflict_and_depth_test():
    H, W = 9, 12  # 3 x 4 cells
    prev, z, dz, pick = _frame(H, W, 2)
    pick[:] = 4  # the centre pixel of each stratum
    fmv = np.zeros((2, H, W))
    fmv[0] += 3.0  # one cell to the right
    d, n, present, src = G.gradient_samples(prev, prev, fmv, z, pick, z)
    CW = 4
    exp = -np.ones((3, 4), np.int64)
    for sy in range(3):
        for sx in range(3):  # the last column's samples leave the image
            exp[sy, sx + 1] = sy * CW + sx
    np.testing.assert_array_equal(src, exp)
    # two strata onto one cell: the lower index wins
    fmv2 = np.zeros((2, H, W))
    fmv2[0, 1, 4] = -3.0  # stratum (0, 1) moves onto cell (0, 0)
    _, _, _, src2 = G.gradient_samples(prev, prev, fmv2, z, pick, z)
    assert src2[0, 0] == 0 and src2[0, 1] == -1
    fmv3 = np.zeros((2, H, W))
    fmv3[0, 1, 1] = 3.0  # stratum (0, 0) moves onto cell (0, 1): index 0 beats 1
    _, _, _, src3 = G.gradient_samples(prev, prev, fmv3, z, pick, z)
    assert src3[0, 1] == 0 and src3[0, 0] == -1
    # rounding to the nearest pixel: +1.49 stays in the cell, +1.5 crosses
    fmv4 = np.zeros((2, H, W))
    fmv4[0, 1, 1] = 1.49
    _, _, _, s4 = G.gradient_samples(prev, prev, fmv4, z, pick, z)
    assert s4[0, 0] == 0
    fmv4[0, 1, 1] = 1.5
    _, _, _, s4 = G.gradient_samples(prev, prev, fmv4, z, pick, z)
    # cell (0, 0) is left empty; cell (0, 1) keeps stratum 0 over its own stratum 1
    assert s4[0, 0] == -1 and s4[0, 1] == 0
    # a moved depth that disagrees with the current one drops the sample
    fz = z.copy()
    fz[1, 1] = 10.0
    _, _, pr, _ = G.gradient_samples(prev, prev, np.zeros((2, H, W)), fz, pick, z)
    assert pr[0, 0] == 0 and pr.sum() == 11
    # a pick outside the image gives no sample (W = 11: the last stratum is two wide)
    H2, W2 = 9, 11
    prev2, z2, _, pick2 = _frame(H2, W2, 3)
    pick2[:] = 2  # third column of each stratum
    _, _, pr2, _ = G.gradient_samples(prev2, prev2, np.zeros((2, H2, W2)), z2, pick2, z2)
    assert pr2[:, 3].sum() == 0 and pr2[:, :3].sum() == 9


def test_samples_are_the_luminance_difference_and_maximum():
    H, W = 6, 6
    prev, z, dz, pick = _frame(H, W, 4)
    re = np.random.default_rng(5).uniform(0.1, 1.0, (3, H, W))
    pick[:] = np.array([[0, 8], [4, 2]], np.uint8)
    d, n, present, src = G.gradient_samples(prev, re, np.zeros((2, H, W)), z, pick, z)
    L = lambda c: 0.2126 * c[0] + 0.7152 * c[1] + 0.0722 * c[2]
    for (cy, cx), k in np.ndenumerate(pick):
        qy, qx = 3 * cy + k // 3, 3 * cx + k % 3
        assert d[cy, cx] == pytest.approx(L(re[:, qy, qx]) - L(prev[:, qy, qx]), rel=1e-14)
        assert n[cy, cx] == pytest.approx(max(L(re[:, qy, qx]), L(prev[:, qy, qx])), rel=1e-14)


def test_reconstruction_on_flat_depth_is_the_normalized_b3_cascade():
    # constant depth makes every edge weight 1: the cascade is the
    # correlation with the dilated B3 kernels (scipy), divided at the end
    r = np.random.default_rng(6)
    CH, CW = 11, 14
    H, W = 3 * CH, 3 * CW
    z = np.full((H, W), 4.0)
    dz = np.zeros((H, W))
    present = (r.random((CH, CW)) < 0.6).astype(np.float64)
    delta = r.uniform(-1, 1, (CH, CW)) * present
    norm = r.uniform(0.5, 2, (CH, CW)) * present
    lam = G.reconstruct(delta, norm, present, z, dz, dz, levels=3)
    h = np.array([1, 4, 6, 4, 1]) / 16.0
    a = [delta, norm, present]
    for lvl in range(3):
        s = 1 << lvl
        k1 = np.zeros(4 * s + 1)
        k1[::s] = h
        a = [correlate(x, np.outer(k1, k1), mode="constant") for x in a]
    ref = np.where(a[2] > 0, np.minimum(1, np.abs(a[0] / a[2]) / (a[1] / a[2])), 0)
    np.testing.assert_allclose(lam, ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("seed,H,W", [(11, 31, 40), (12, 27, 35)])
def test_reconstruction_equals_plain_sums_at_ordinary_weights(seed, H, W):
    """Random depth with a non-trivial gradient field and ragged cells: the
    log-domain form of the oracle gives the quotients of the plain binary64
    normalized convolution, sum_j w_j x_j / sum_j w_j p_j cascaded over the
    levels, with the depth weight of each cell's centre pixel and its own
    gradient.  Written out here tap by tap."""
    r = np.random.default_rng(seed)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    z = 5.0 + 0.04 * xs - 0.03 * ys + 0.3 * np.sin(0.2 * xs) * np.cos(0.15 * ys) \
        + r.normal(0, 0.02, (H, W))
    dzdx = 0.04 + 0.06 * np.cos(0.2 * xs) * np.cos(0.15 * ys)
    dzdy = -0.03 - 0.045 * np.sin(0.2 * xs) * np.sin(0.15 * ys)
    CH, CW = G.cells_of(H, W)
    present = (r.random((CH, CW)) < 0.5).astype(np.float64)
    delta = r.uniform(-1, 1, (CH, CW)) * present
    norm = r.uniform(0.5, 2, (CH, CW)) * present
    levels = 3
    lam = G.reconstruct(delta, norm, present, z, dzdx, dzdy, levels=levels)
    h = np.array([1, 4, 6, 4, 1]) / 16.0
    cy = np.minimum(3 * np.arange(CH) + 1, H - 1)
    cx = np.minimum(3 * np.arange(CW) + 1, W - 1)
    X = [delta * present, norm * present, present.copy()]
    for lvl in range(levels):
        s = 1 << lvl
        Y = [np.zeros((CH, CW)) for _ in X]
        for i in range(CH):
            for j in range(CW):
                zc, gx, gy = z[cy[i], cx[j]], dzdx[cy[i], cx[j]], dzdy[cy[i], cx[j]]
                for b in range(-2, 3):
                    for a in range(-2, 3):
                        ii, jj = i + b * s, j + a * s
                        if not (0 <= ii < CH and 0 <= jj < CW):
                            continue
                        den = abs(gx * 3.0 * a * s + gy * 3.0 * b * s) + 1e-10
                        w = h[a + 2] * h[b + 2] * np.exp(-abs(zc - z[cy[ii], cx[jj]]) / den)
                        for k in range(3):
                            Y[k][i, j] += w * X[k][ii, jj]
        X = Y
    ok = (X[2] > 0) & (X[1] > 0)
    ref = np.where(ok, np.minimum(1.0, np.abs(X[0] / np.where(ok, X[2], 1))
                                  / np.where(ok, X[1] / np.where(ok, X[2], 1), 1)), 0.0)
    np.testing.assert_allclose(lam, ref, rtol=1e-12, atol=1e-15)
    # every reached cell's filtered indicator is an ordinary number (not the
    # underflow case of the test below), and most lambdas are fractions
    assert X[2][X[2] > 0].min() > 1e-100
    assert np.count_nonzero((ref > 0) & (ref < 1)) > CH * CW // 2


def test_depth_edges_keep_gradients_apart():
    # two depth planes far apart: a gradient on one side does not leak
    CH, CW = 6, 10
    H, W = 3 * CH, 3 * CW
    z = np.full((H, W), 4.0)
    z[:, W // 2:] = 40.0
    dz = np.zeros((H, W))
    present = np.ones((CH, CW))
    delta = np.zeros((CH, CW))
    delta[:, :CW // 2] = 1.0
    norm = np.ones((CH, CW))
    lam = G.reconstruct(delta, norm, present, z, dz, dz, levels=3)
    np.testing.assert_allclose(lam[:, :CW // 2], 1.0, rtol=1e-12)
    np.testing.assert_allclose(lam[:, CW // 2:], 0.0, atol=1e-12)


def test_reconstruction_keeps_the_ratio_of_tiny_weights():
    """A cell without a sample between two cells far across depth edges:
    their weights are about e^-733 (1e-318, subnormal in binary64) and in the
    ratio 3:1 by construction, so the cell's means are the 3:1 averages of
    theirs and lambda has a closed form, which summing the tiny weights in
    plain binary64 would lose."""
    H, W = 3, 9  # one row of three cells, centre pixels x = 1, 4, 7
    g = 1e-3
    den = 1.0 * abs(g * 3.0) + 1e-10
    z = np.full((H, W), 5.0)
    z[1, 1] = 5.0 + 733.0 * den
    z[1, 7] = 5.0 + 733.0 * den + np.log(3.0) * den
    dzdx = np.zeros((H, W))
    dzdx[1, 4] = g
    dzdy = np.zeros((H, W))
    delta = np.array([[0.3, 0.0, -0.5]])
    norm = np.array([[1.0, 0.0, 2.0]])
    present = np.array([[1.0, 0.0, 1.0]])
    lam = G.reconstruct(delta, norm, present, z, dzdx, dzdy, levels=1)
    d_hat = (3 * 0.3 + 1 * -0.5) / 4
    n_hat = (3 * 1.0 + 1 * 2.0) / 4
    assert abs(lam[0, 1] - abs(d_hat) / n_hat) < 1e-12
