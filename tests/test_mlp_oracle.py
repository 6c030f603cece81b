"""Pins of the learned component's oracle (oracle/mlp.py) against values
that do not come from it: finite differences, closed forms, brute force
and library routines."""

import numpy as np
import pytest
import torch

import oracle as O
from oracle import mlp as M
from tests._util import random_gbuf


def _weights(seed=0, scale=0.5):
    r = np.random.default_rng(seed)
    w = M.init_weights(seed)
    w.w3 = r.normal(0, scale, w.w3.shape)
    w.b1 = r.normal(0, 0.1, w.b1.shape)
    w.b2 = r.normal(0, 0.1, w.b2.shape)
    w.b3 = r.normal(0, 0.3, w.b3.shape)
    return w


def test_bf16_matches_torch_rne():
    r = np.random.default_rng(1)
    x = np.concatenate([r.normal(0, 10, 5000), r.uniform(-1e-3, 1e-3, 500),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 65504.0, 1e-40]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16(x), ref)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert M.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0
    assert M.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6


def test_zero_weights_give_closed_form_heads():
    w = M.init_weights(3)
    w.w1[:] = 0.0
    w.w2[:] = 0.0
    w.w3[:] = 0.0
    w.b3 = np.array([0.7, -0.4])
    x = np.random.default_rng(2).normal(size=(M.N_IN, 50))
    for q in (False, True):
        fw = M.forward(w, x, bf16_ops=q)
        b = M.f32(w.b3) if q else w.b3
        np.testing.assert_allclose(fw["alpha"], 0.05 + 0.95 / (1 + np.exp(-b[0])), rtol=1e-15)
        np.testing.assert_allclose(fw["kappa"], 2.0 ** (2 * np.tanh(b[1])), rtol=1e-15)


def test_backward_matches_finite_differences():
    w = _weights(4)
    x = np.random.default_rng(5).normal(size=(M.N_IN, 40))
    g_o = np.random.default_rng(6).normal(size=(2, 40))
    fw = M.forward(w, x, bf16_ops=False)
    grad = M.backward(w, fw, g_o, bf16_ops=False)
    flat = w.flat()
    h = 1e-6

    def loss(v):
        ww = M.Weights.from_flat(v, w.mu, w.inv_s)
        return float((g_o * M.forward(ww, x, bf16_ops=False)["o"]).sum())

    idx = np.random.default_rng(7).choice(flat.size, 120, replace=False)
    idx = np.concatenate([idx, [0, M.N_PARAMS - 1, M.N_PARAMS - 2]])
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        fd = (loss(flat + e) - loss(flat - e)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_head_grads_match_finite_differences():
    w = _weights(8)
    x = np.random.default_rng(9).normal(size=(M.N_IN, 30))
    da = np.random.default_rng(10).normal(size=30)
    dk = np.random.default_rng(11).normal(size=30)
    fw = M.forward(w, x, bf16_ops=False)
    g = M.head_grads(fw, da, dk)
    h = 1e-6
    for k in range(2):
        wp, wm = M.Weights.from_flat(w.flat(), w.mu, w.inv_s), M.Weights.from_flat(w.flat(), w.mu, w.inv_s)
        wp.b3 = w.b3.copy()
        wm.b3 = w.b3.copy()
        wp.b3[k] += h
        wm.b3[k] -= h
        fp, fm = M.forward(wp, x, bf16_ops=False), M.forward(wm, x, bf16_ops=False)
        fd = ((fp["alpha"] - fm["alpha"]) * da + (fp["kappa"] - fm["kappa"]) * dk) / (2 * h)
        np.testing.assert_allclose(g[k], fd, rtol=1e-6, atol=1e-9)


def test_adam_closed_forms():
    p = M.AdamParams(lr=1e-3)
    g = np.array([2.0, -3.0, 1e-3])
    w0 = np.array([1.0, 1.0, 1.0])
    w, m, v = w0, np.zeros(3), np.zeros(3)
    # with a constant gradient every bias-corrected step is lr * g / (|g| + eps)
    for t in range(1, 6):
        w, m, v = M.adam(w, m, v, g, t, p)
        np.testing.assert_allclose(w, w0 - t * p.lr * g / (np.abs(g) + p.eps), rtol=1e-12)


def test_box_luma_variance_brute_force():
    r = np.random.default_rng(12)
    L = r.uniform(0, 2, (9, 11))
    z = r.uniform(1, 2, (9, 11))
    z[r.random((9, 11)) < 0.2] = 0.0
    got = M.box_luma_variance(L, z)
    for y in range(9):
        for x in range(11):
            vals = [L[j, i] for j in range(y - 1, y + 2) for i in range(x - 1, x + 2)
                    if 0 <= j < 9 and 0 <= i < 11 and z[j, i] > 0]
            want = np.var(vals) if vals else 0.0
            assert abs(got[y, x] - want) <= 1e-12


def test_alpha_grad_matches_finite_differences_of_blend():
    r = np.random.default_rng(13)
    H, W = 6, 7
    cur = r.uniform(0.1, 1, (3, H, W))
    hist = r.uniform(0.1, 1, (3, H, W))
    y = r.uniform(0.1, 1, (3, H, W))
    z = np.ones((H, W))
    n_h = r.integers(0, 9, (H, W))
    valid = np.ones((H, W), np.int32)
    am = r.uniform(0.05, 1, (H, W))
    n_new = np.minimum(n_h + 1, 255)

    def loss(a):
        c = O.blend(cur, z, hist, np.zeros((H, W)), np.zeros((H, W)), n_h, valid, alpha_map=a)["rgb"]
        return (((c - y) ** 2) * M.relmse_weight(y)).mean(0)

    c_t = O.blend(cur, z, hist, np.zeros((H, W)), np.zeros((H, W)), n_h, valid, alpha_map=am)["rgb"]
    g = M.alpha_grad(c_t, cur, hist, y, am, n_new)
    h = 1e-7
    fd = (loss(am + h) - loss(am - h)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-9)


@pytest.mark.parametrize("step", [1, 2])
def test_kappa_derivative_matches_finite_differences_of_atrous(step):
    """Against the C oracle's a-trous level (an independent implementation
    of the forward filter)."""
    r = np.random.default_rng(20 + step)
    H, W = 12, 14
    z, dzdx, dzdy, n = random_gbuf(r, H, W)
    c = r.uniform(0.05, 1.0, (3, H, W))
    var = r.uniform(0.001, 0.05, (H, W))
    kappa = r.uniform(0.5, 2.0, (H, W))
    d = M.atrous_kappa_derivative(c, var, z, dzdx, dzdy, n, kappa, step)
    h = 1e-6
    for (y, x) in [(0, 0), (5, 6), (11, 13), (3, 9)]:
        kp, km = kappa.copy(), kappa.copy()
        kp[y, x] += h
        km[y, x] -= h
        op = O.atrous(c, var, z, dzdx, dzdy, n, step, kappa=kp)[0]
        om = O.atrous(c, var, z, dzdx, dzdy, n, step, kappa=km)[0]
        fd = (op[:, y, x] - om[:, y, x]) / (2 * h)
        np.testing.assert_allclose(d[:, y, x], fd, rtol=1e-5, atol=1e-10)


def test_features_of_a_static_sequence():
    """Static camera, history of n frames: every pixel valid, history
    luminance = luminance of the clamped history, n/255 feature exact, and
    the G-buffer features are the inputs themselves."""
    from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
    cfg = with_size(CONFIGS["small_static"], 40, 30, 4)
    p = O.OracleParams(clamp=True, tonemap=True)
    st = O.new_state(30, 40)
    for f, fr in enumerate(sequence(cfg)):
        ft = M.features(fr, st, p)
        x = ft["x"]
        np.testing.assert_array_equal(x[4], np.minimum(f + 1, 255) / 255.0)
        np.testing.assert_array_equal(x[5], fr["dzdx"].astype(np.float64))
        np.testing.assert_array_equal(x[7:10], fr["n"].astype(np.float64))
        np.testing.assert_array_equal(x[10], 0.0)
        np.testing.assert_array_equal(x[11:14], fr["albedo"].astype(np.float64))
        np.testing.assert_allclose(x[0], O.luma(O.tonemap(fr["rgb"])), rtol=1e-15)
        if f == 0:
            assert not ft["valid"].any()
            np.testing.assert_array_equal(x[1], 0.0)
        else:
            assert ft["valid"].all()
            np.testing.assert_allclose(x[1], O.luma(ft["hist"]), rtol=1e-15)
        _, st, _ = O.run_frame(fr, st, p)


def _gbuf_with_holes(r, H, W, holes):
    """random_gbuf with some pixels without a surface (sky: z = inf, and
    z = 0), as the level treats them (R15)."""
    z, dzdx, dzdy, n = random_gbuf(r, H, W)
    z = z.astype(np.float64)
    for k, (y, x) in enumerate(holes):
        z[y, x] = np.inf if k % 2 == 0 else 0.0
    return z, dzdx, dzdy, n


@pytest.mark.parametrize("step", [1, 2])
def test_kappa_derivative_next_to_empty_pixels(step):
    """The level's variance prefilter skips empty neighbours (their
    variance is no sample of p's surface); the derivative must be that of
    the level as the C oracle runs it, so finite differences through it
    pin the prefilter beside sky pixels too."""
    r = np.random.default_rng(40 + step)
    H, W = 11, 13
    holes = [(4, 5), (4, 6), (0, 12), (9, 2)]
    z, dzdx, dzdy, n = _gbuf_with_holes(r, H, W, holes)
    c = r.uniform(0.05, 1.0, (3, H, W))
    # the empty pixels' variance is large, so a prefilter that averaged it
    # in would move the derivative well past the tolerance
    var = np.where(np.isfinite(z) & (z > 0), r.uniform(0.001, 0.05, (H, W)), 3.0)
    kappa = r.uniform(0.5, 2.0, (H, W))
    d = M.atrous_kappa_derivative(c, var, z, dzdx, dzdy, n, kappa, step)
    h = 1e-6
    for (y, x) in [(3, 5), (5, 6), (4, 7), (1, 11), (8, 2), (4, 5), (0, 12)]:
        kp, km = kappa.copy(), kappa.copy()
        kp[y, x] += h
        km[y, x] -= h
        op = O.atrous(c, var, z, dzdx, dzdy, n, step, kappa=kp)[0]
        om = O.atrous(c, var, z, dzdx, dzdy, n, step, kappa=km)[0]
        fd = (op[:, y, x] - om[:, y, x]) / (2 * h)
        np.testing.assert_allclose(d[:, y, x], fd, rtol=1e-5, atol=1e-10)
    # an empty pixel passes its input through: no dependence on kappa
    for (y, x) in holes:
        assert np.all(d[:, y, x] == 0.0)


@pytest.mark.parametrize("step", [1, 4])
def test_kappa_grad_level_matches_finite_differences_of_level_relmse(step):
    """dL/dkappa(p) of one level, L the level output's RelMSE summed over
    pixels (mean over channels), against central differences of L through
    the C oracle's level with kappa moved at p alone.  kappa(p) scales p's
    own luminance width only, so the other pixels must not move at all."""
    r = np.random.default_rng(60 + step)
    H, W = 12, 15
    z, dzdx, dzdy, n = _gbuf_with_holes(r, H, W, [(6, 7), (2, 2)])
    c = r.uniform(0.05, 1.0, (3, H, W))
    var = r.uniform(0.001, 0.05, (H, W))
    kappa = r.uniform(0.5, 2.0, (H, W))
    y_ref = r.uniform(0.05, 1.0, (3, H, W))
    out = O.atrous(c, var, z, dzdx, dzdy, n, step, kappa=kappa)[0]
    d = M.atrous_kappa_derivative(c, var, z, dzdx, dzdy, n, kappa, step)
    g = M.kappa_grad_level(out, y_ref, d)

    def loss(o):
        return float((((o - y_ref) ** 2) * M.relmse_weight(y_ref)).mean(0).sum())

    h = 1e-6
    for (py, px) in [(0, 0), (5, 7), (6, 8), (11, 14), (3, 10), (6, 7)]:
        kp, km = kappa.copy(), kappa.copy()
        kp[py, px] += h
        km[py, px] -= h
        op = O.atrous(c, var, z, dzdx, dzdy, n, step, kappa=kp)[0]
        om = O.atrous(c, var, z, dzdx, dzdy, n, step, kappa=km)[0]
        mask = np.ones((H, W), bool)
        mask[py, px] = False
        np.testing.assert_array_equal(op[:, mask], out[:, mask])
        np.testing.assert_array_equal(om[:, mask], out[:, mask])
        fd = (loss(op) - loss(om)) / (2 * h)
        assert abs(g[py, px] - fd) <= 1e-5 * max(abs(fd), 1e-6), (py, px, g[py, px], fd)


def test_features_of_a_moving_sequence():
    """Rows 2 (reprojected central moment) and 10 (motion length) where the
    camera and three spheres move, with motion planted that the temporal
    step discards (not finite, or 2^20 pixels and more): row 2 equals
    m2 - m1^2 of the bilinear mixture worked out here pixel by pixel from
    the history, row 10 the length of the kept motion and 0 elsewhere."""
    import math
    from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
    cfg = with_size(CONFIGS["hd_motion"], 48, 30, 4)
    p = O.OracleParams(clamp=True, tonemap=True, use_id=True)
    H, W = 30, 48
    st = O.new_state(H, W)
    planted = {(3, 4): (np.nan, 0.5), (5, 6): (0.25, 2.0 ** 20), (7, 8): (-2.0 ** 21, 0.0),
               (9, 10): (0.0, np.inf), (11, 12): (2.0 ** 20 - 1, -3.0)}
    f32 = np.float32
    nonzero_moment = moving = 0
    for f, fr in enumerate(sequence(cfg)):
        fr = dict(fr)
        mv = fr["mv"].astype(np.float64)
        for (y, x), v in planted.items():
            mv[:, y, x] = v
        fr["mv"] = mv
        x_ft = M.features(fr, st, p)["x"]
        for yy in range(H):
            for xx in range(W):
                mx, my = mv[0, yy, xx], mv[1, yy, xx]
                kept = math.isfinite(mx) and math.isfinite(my) and abs(mx) < 2 ** 20 and abs(my) < 2 ** 20
                want = math.hypot(mx, my) if kept else 0.0
                assert abs(x_ft[10, yy, xx] - want) <= 1e-15 * max(1.0, want), (f, yy, xx)
                if want > 0.5:
                    moving += 1
                # bilinear mixture of the history's raw moments over the usable taps
                if not kept:
                    assert x_ft[2, yy, xx] == 0.0
                    continue
                x0, y0 = xx + math.floor(mx), yy + math.floor(my)
                fx, fy = mx - math.floor(mx), my - math.floor(my)
                sw = s1 = s2 = 0.0
                for t in range(4):
                    tx, ty = x0 + (t & 1), y0 + (t >> 1)
                    bw = (fx if t & 1 else 1 - fx) * (fy if t >> 1 else 1 - fy)
                    if bw <= 0 or not (0 <= tx < W and 0 <= ty < H) or st["n"][ty, tx] < 1:
                        continue
                    zc = f32(fr["z"][yy, xx])
                    if not abs(f32(f32(fr["prev_z"][ty, tx]) - zc)) <= f32(f32(p.tau_z) * zc):
                        continue
                    a, b = fr["prev_n"][:, ty, tx].astype(f32), fr["n"][:, yy, xx].astype(f32)
                    # binary32 dot in the decision's order, each fma as an
                    # exact binary64 product and sum rounded to binary32
                    dn = f32(a[0] * b[0])
                    dn = f32(float(a[1]) * float(b[1]) + float(dn))
                    dn = f32(float(a[2]) * float(b[2]) + float(dn))
                    if not dn >= f32(p.tau_n):
                        continue
                    if fr["id"][yy, xx] != fr["prev_id"][ty, tx]:
                        continue
                    sw += bw
                    s1 += bw * st["m1"][ty, tx]
                    s2 += bw * st["m2"][ty, tx]
                want2 = max(s2 / sw - (s1 / sw) ** 2, 0.0) if sw > 0 else 0.0
                assert abs(x_ft[2, yy, xx] - want2) <= 1e-12 * max(1e-3, want2), (f, yy, xx)
                if want2 > 1e-4:
                    nonzero_moment += 1
        _, st, _ = O.run_frame(fr, st, p)
    assert moving > 1000 and nonzero_moment > 1000, (moving, nonzero_moment)


def test_per_pixel_pass_of_the_flip_bounds_equals_the_oracle():
    """tests/_mlp_bounds.pixel_pass (the per-pixel model the GPU tests use
    to bound bfloat16 rounding flips) reproduces the oracle's batched
    forward and backward exactly when nothing is overridden, and a flip
    moves one value by one bfloat16 ulp."""
    from tests import _mlp_bounds as B
    w = _weights(31)
    r = np.random.default_rng(32)
    xs = M.bf16(r.normal(0, 1.2, (M.N_IN, 25)))
    da, dk = M.f32(r.normal(0, 1, 25)), M.f32(r.normal(0, 1, 25))
    fw = M.forward(w, xs, bf16_ops=True)
    ref = M.backward(w, fw, M.head_grads(fw, da, dk), bf16_ops=True)
    tot = np.zeros(M.N_PARAMS)
    for p in range(25):
        al, ka, c, _ = B.pixel_pass(w, xs[:, p], da[p], dk[p])
        assert al == fw["alpha"][p] and ka == fw["kappa"][p]
        tot += c
    np.testing.assert_allclose(tot, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    v = np.array([1.0 + 2 ** -8, 3.0 * (1 + 2 ** -9 + 2 ** -20)])
    alt = B.other_rounding(v)
    assert np.all(alt != M.bf16(v)) and np.all(np.abs(alt - v) < 2 * np.abs(M.bf16(v) - v) + 2 ** -6 * np.abs(v))
    assert B.near_midpoint(np.array([1.0 + 2 ** -8]))[0] and not B.near_midpoint(np.array([1.0]))[0]
    # a sum whose terms are 2^12 times larger may be off by far more of its ulps
    v = np.array([1.0 + 2 ** -8 + 2 ** -16])
    assert not B.near_midpoint(v)[0] and B.near_midpoint(v, 4096.0)[0]
