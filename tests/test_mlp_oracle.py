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
