"""Parity of the learned component's kernels with its FP64 oracle
(oracle/mlp.py), and the gain of a network trained by them.

Tolerances.  The device rounds matrix operands to bfloat16 exactly as the
oracle's precision model does, but its binary32 sums run in another order;
a value within a few binary32 ulps of a bfloat16 rounding midpoint can
therefore round the other way (one bfloat16 ulp of one activation or
gradient).  The forward and backward tests hold the median error at the
binary32 level and every element within the summed effect of the flips
that could reach it (tests/_mlp_bounds.py: each candidate value rounded
the other way, the pixel run again) plus binary32 rounding slack; the
flips are counted.
"""

import numpy as np
import pytest
import torch

import oracle as O
from oracle import mlp as M
from paper_2312_06827_amd import lib as L
from paper_2312_06827_amd.scene import CONFIGS, render_frame, sequence, with_size
from tests import _mlp_bounds as B
from tests._util import rel_err, say

pytestmark = pytest.mark.gpu


def host(t):
    torch.cuda.synchronize()
    return t.detach().to(torch.float64).cpu().numpy() if t.dtype.is_floating_point \
        else t.detach().cpu().numpy()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _weights(seed):
    r = np.random.default_rng(seed)
    w = M.init_weights(seed)
    w.w3 = r.normal(0, 0.6, w.w3.shape)
    w.b1 = r.normal(0, 0.2, w.b1.shape)
    w.b2 = r.normal(0, 0.2, w.b2.shape)
    w.b3 = r.normal(0, 0.3, w.b3.shape)
    w.mu = r.normal(0, 0.5, M.N_IN)
    w.inv_s = r.uniform(0.5, 2.0, M.N_IN)
    # binary32 master values
    for k in ("w1", "b1", "w2", "b2", "w3", "b3", "mu", "inv_s"):
        setattr(w, k, M.f32(getattr(w, k)))
    return w


def _device_mlp(w):
    return L.MLP(w.flat(), w.mu, w.inv_s)


def _rows(xs):
    """(14, N) bf16-representable values -> device feature rows (N, 16)."""
    N = xs.shape[1]
    rows = np.zeros((N, 16), np.float32)
    rows[:, :14] = xs.T
    t = torch.from_numpy(rows).to(torch.bfloat16)
    assert np.array_equal(t.to(torch.float64).numpy()[:, :14], xs.T)
    return t.view(torch.int16).cuda()


@pytest.mark.parametrize("H,W", [(1, 1), (5, 7), (33, 61), (64, 64)])
def test_forward_parity(H, W):
    w = _weights(10 + H)
    xs = M.bf16(np.random.default_rng(H).normal(0, 1.2, (14, H * W)))
    mlp = _device_mlp(w)
    P = W + 3
    a = torch.full((H, P), float("nan"), device="cuda")[:, :W]
    k = torch.full((H, P), float("nan"), device="cuda")[:, :W]
    say(f"mlp forward {H}x{W}")
    L.sv_mlp_forward(mlp, _rows(xs), a, k, a)
    fw = M.forward(w, xs, bf16_ops=True)
    ea = np.abs(host(a).ravel() - fw["alpha"])
    ek = np.abs(host(k).ravel() - fw["kappa"]) / fw["kappa"]
    zero = np.zeros(H * W)
    ba, bk, _, _, _, nflip = B.flip_bounds(w, xs, zero, zero, forward_only=True)
    say(f"  alpha err median {np.median(ea):.1e} max {ea.max():.1e}; "
        f"kappa rel err median {np.median(ek):.1e} max {ek.max():.1e}; "
        f"{nflip} flip candidates, {int((ea > 1e-6).sum())} alphas off by more than 1e-6")
    assert np.median(ea) <= 1e-6 and np.median(ek) <= 1e-6
    # binary32 heads: 1e-6 beside the flips
    assert np.all(ea <= ba + 1e-6), np.argmax(ea - ba)
    assert np.all(ek <= bk + 1e-6), np.argmax(ek - bk)


@pytest.mark.parametrize("N", [40, 1000, 4096 + 17])
def test_backward_parity(N):
    w = _weights(20 + N)
    r = np.random.default_rng(N)
    xs = M.bf16(r.normal(0, 1.2, (14, N)))
    da = r.normal(0, 1.0, N)
    dk = r.normal(0, 1.0, N)
    H, W = 1, N
    mlp = _device_mlp(w)
    grad = torch.empty(L.SV_MLP_PARAMS, device="cuda")
    like = torch.empty((H, W), device="cuda")
    work = L.mlp_workspace(like)
    say(f"mlp backward N={N}")
    L.sv_mlp_backward(mlp, _rows(xs), dev(da[None]), dev(dk[None]), grad, work, like, scale=0.5)
    fw = M.forward(w, xs, bf16_ops=True)
    g_o = M.head_grads(fw, M.f32(da), M.f32(dk))
    ref = 0.5 * M.backward(w, fw, g_o, bf16_ops=True)
    got = host(grad)
    _, _, bg, asum, _, nflip = B.flip_bounds(w, xs, M.f32(da), M.f32(dk))
    # binary32 sums over the pixels in the device's order: 2^-16 of the sum
    # of the magnitudes summed (far above the about 200 additions on the
    # longest path times 2^-24)
    allow = 0.5 * (bg + 2.0 ** -16 * asum)
    err = np.abs(got - ref)
    off = 0
    for name, n in [("W1", 448), ("b1", 32), ("W2", 1024), ("b2", 32), ("W3", 64), ("b3", 2)]:
        g, o = got[off:off + n], ref[off:off + n]
        e = np.abs(g - o).max() / max(np.abs(o).max(), 1e-30)
        say(f"  {name}: max err / max |grad| = {e:.1e}; max err / allowed = "
            f"{(err[off:off + n] / np.maximum(allow[off:off + n], 1e-30)).max():.2f}")
        off += n
    say(f"  {nflip} flip candidates over {N} pixels")
    assert np.all(err <= allow), (int(np.argmax(err - allow)), float((err - allow).max()))
    # a second call with the same inputs is bitwise identical (fixed order)
    g2 = torch.empty_like(grad)
    L.sv_mlp_backward(mlp, _rows(xs), dev(da[None]), dev(dk[None]), g2, work, like, scale=0.5)
    assert torch.equal(grad, g2)


def test_adam_parity():
    r = np.random.default_rng(3)
    p0 = M.f32(r.normal(0, 1, L.SV_MLP_PARAMS))
    mlp = L.MLP(p0, np.zeros(14), np.ones(14))
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t in range(1, 4):
        g = M.f32(r.normal(0, 1, L.SV_MLP_PARAMS))
        L.sv_adam(mlp, dev(g), lr=1e-2)
        p, m, v = M.adam(p, m, v, g, t, M.AdamParams(lr=1e-2))
    assert rel_err(host(mlp.params)[None], p[None]) <= 1e-5
    mirror = mlp.wq.view(torch.bfloat16).to(torch.float64).cpu().numpy()
    np.testing.assert_array_equal(mirror, M.bf16(host(mlp.params)))


def _history_state(H, W, seed, frames=4):
    """Oracle state after a few frames of a motion sequence, and the next frame."""
    cfg = with_size(CONFIGS["hd_motion"], W, H, frames + 1)
    from dataclasses import replace
    cfg = replace(cfg, seed=seed)
    p = O.OracleParams(clamp=True, tonemap=True, use_id=True)
    st = O.new_state(H, W)
    frs = list(sequence(cfg))
    for fr in frs[:frames]:
        _, st, _ = O.run_frame(fr, st, p)
    return frs[frames], st, p


@pytest.mark.parametrize("H,W", [(37, 70), (90, 160)])
def test_features_parity(H, W):
    fr, st, p = _history_state(H, W, 77 + H)
    fr = dict(fr)
    fr["z"] = fr["z"].copy()
    fr["z"][3, 4] = 0.0  # an empty pixel
    w = _weights(5)
    mlp = _device_mlp(w)
    feat = L.feature_rows(H, W)
    hist_out = torch.empty((3, H, W), device="cuda")
    g = L.GBuf(dev(fr["z"]), dev(fr["dzdx"]), dev(fr["dzdy"]), dev(fr["n"]),
               dev(fr["id"], torch.uint8))
    prev = L.GBuf(dev(fr["prev_z"]), None, None, dev(fr["prev_n"]), dev(fr["prev_id"], torch.uint8))
    m2c = (st["m2"] - st["m1"] ** 2).astype(np.float32)
    say(f"mlp features {H}x{W}")
    L.sv_mlp_features(dev(fr["rgb"]), g, dev(fr["mv"]), prev, dev(st["rgb"]), dev(st["m1"]),
                      dev(m2c), dev(st["n"], torch.uint8), dev(fr["albedo"]), mlp, feat,
                      L.TemporalParams(clamp=True, tonemap=True, use_id=True),
                      hist_out=hist_out)
    # the oracle gets the same (binary32) history the device read
    st32 = dict(st)
    st32["m1"] = st["m1"].astype(np.float32).astype(np.float64)
    st32["m2"] = m2c.astype(np.float64) + st32["m1"] ** 2
    st32["rgb"] = st["rgb"].astype(np.float32).astype(np.float64)
    ft = M.features(fr, st32, p)
    ref = M.standardise(ft["x"], w).T.reshape(H * W, 14)
    got = feat.view(torch.bfloat16).to(torch.float64).cpu().numpy()
    assert np.all(got[:, 14:] == 0)
    got = got[:, :14]
    ulp = np.maximum(np.abs(ref), 1e-30) * 2.0 ** -7  # one bf16 ulp (upper bound)
    bad = np.abs(got - ref) > ulp
    say(f"  features differing by more than one bf16 ulp: {int(bad.sum())} of {bad.size}; "
        f"differing at all: {int((got != ref).sum())}")
    assert not bad.any(), np.argwhere(bad)[:5]
    assert (got != ref).mean() <= 2e-3
    assert rel_err(host(hist_out), ft["hist"]) <= 1e-5


def test_alpha_grad_parity():
    H, W = 40, 72
    fr, st, p = _history_state(H, W, 91)
    r = np.random.default_rng(4)
    alpha = r.uniform(0.05, 1.0, (H, W)).astype(np.float32)
    ft = M.features(fr, st, p)
    t = O.temporal(fr, st, p, alpha_map=alpha)
    y = O.tonemap(fr["clean"])
    # the oracle takes the binary32 values the device reads
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    ct, hist, y32 = f32(t["rgb"]), f32(ft["hist"]), f32(y)
    ref = M.alpha_grad(ct, ft["cur"], hist, y32, alpha, t["n"])
    out = torch.empty((H, W), device="cuda")
    say("mlp alpha grad")
    L.sv_mlp_alpha_grad(dev(ct), dev(fr["rgb"]), dev(hist), dev(y32), dev(alpha),
                        dev(t["n"], torch.uint8), dev(fr["z"]), out, tm_k=1.0)
    e = rel_err(host(out), ref)
    say(f"  rel err max {e:.1e}")
    assert e <= 1e-5


@pytest.mark.parametrize("step", [1, 4])
def test_kappa_grad_parity(step):
    H, W = 48, 80
    fr = dict(render_frame(with_size(CONFIGS["hd_motion"], W, H, 3), 2))
    # pixels without a surface: skipped by the level's variance prefilter
    z = fr["z"].copy()
    for k, (y0, x0) in enumerate([(10, 11), (10, 12), (30, 40), (0, 79), (47, 0)]):
        z[y0, x0] = np.inf if k % 2 == 0 else 0.0
    fr["z"] = z
    r = np.random.default_rng(step)
    c = O.tonemap(fr["rgb"]).astype(np.float32)
    var = r.uniform(0.001, 0.05, (H, W)).astype(np.float32)
    kappa = r.uniform(0.5, 2.0, (H, W)).astype(np.float32)
    y = O.tonemap(fr["clean"]).astype(np.float32)
    deriv = M.atrous_kappa_derivative(c, var, fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], kappa, step)
    outc = O.atrous(c, var, fr["z"], fr["dzdx"], fr["dzdy"], fr["n"], step, kappa=kappa)[0]
    other = (y * r.uniform(0.8, 1.2, y.shape)).astype(np.float32)  # another residual source
    g = L.GBuf(dev(fr["z"]), dev(fr["dzdx"]), dev(fr["dzdy"]), dev(fr["n"]))
    for use_ref in (False, True):
        src = other if use_ref else outc
        ref = M.kappa_grad_level(src, y, deriv)
        say(f"kappa grad step={step} ref={use_ref}")
        # from zero: the gradient itself, at the binary32 bar
        dk = torch.zeros((H, W), device="cuda")
        L.sv_atrous_kappa_grad(dev(c), dev(var), g, dev(kappa), dev(y), dk, step,
                               L.AtrousParams(), ref=dev(other) if use_ref else None)
        e = rel_err(host(dk), ref)
        say(f"  rel err max {e:.1e}")
        assert e <= 1e-5
        # onto 0.25: the call accumulates (one binary32 addition)
        acc = torch.full((H, W), 0.25, device="cuda")
        L.sv_atrous_kappa_grad(dev(c), dev(var), g, dev(kappa), dev(y), acc, step,
                               L.AtrousParams(), ref=dev(other) if use_ref else None)
        want = (torch.full((H, W), 0.25, device="cuda") + dk)
        assert torch.equal(acc, want)


def test_training_beats_plain_filter():
    """A network trained from scratch by the library's kernels lowers the
    RelMSE-to-clean of the filter on held-out sequences."""
    from paper_2312_06827_amd import learn
    # sequences long enough for the history length to pass 1/alpha: below
    # that the blend factor is max(alpha, 1/n) and alpha gets no gradient
    cfg = learn.TrainConfig(width=256, height=144, frames=24, sequences=16, warm=2,
                            lr=3e-3, stat_frames=24)
    say("training 16 sequences of 24 frames at 256x144")
    net = learn.train(cfg, log=say)
    plain = learn.evaluate([5900, 5901], 256, 144, 30, None, first=10)
    learned = learn.evaluate([5900, 5901], 256, 144, 30, net, first=10)
    say(f"held-out RelMSE: plain {plain:.5f}, learned {learned:.5f}")
    assert np.isfinite(learned)
    assert learned < plain


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_learned_temporal_equals_separate_path(dtype):
    """The network inside sv_temporal gives bitwise what sv_mlp_features +
    sv_mlp_forward + sv_temporal(alpha_map) give, alpha and kappa included."""
    H, W = 90, 160
    fr, st, p = _history_state(H, W, 123)
    w = _weights(31)
    mlp = _device_mlp(w)
    d = lambda a, dt=dtype: dev(a, dt)
    g = L.GBuf(d(fr["z"]), d(fr["dzdx"]), d(fr["dzdy"]), d(fr["n"]), dev(fr["id"], torch.uint8))
    prev = L.GBuf(d(fr["prev_z"]), None, None, d(fr["prev_n"]), dev(fr["prev_id"], torch.uint8))
    m2c = (st["m2"] - st["m1"] ** 2).astype(np.float32)
    hist = (d(st["rgb"]), dev(st["m1"]), dev(m2c), dev(st["n"], torch.uint8))
    tp = L.TemporalParams(clamp=True, tonemap=True, use_id=True)
    alb = d(fr["albedo"])
    say(f"learned temporal, {dtype}")
    # separate kernels
    feat = L.feature_rows(H, W)
    L.sv_mlp_features(d(fr["rgb"]), g, d(fr["mv"]), prev, *hist, alb, mlp, feat, tp)
    a1 = torch.empty((H, W), device="cuda")
    k1 = torch.empty((H, W), device="cuda")
    L.sv_mlp_forward(mlp, feat, a1, k1, a1)
    outs = []
    for fused in (False, True):
        out = torch.empty((3, H, W), dtype=dtype, device="cuda")
        om1, om2 = torch.empty((H, W), device="cuda"), torch.empty((H, W), device="cuda")
        on = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        a2, k2 = torch.empty((H, W), device="cuda"), torch.empty((H, W), device="cuda")
        if fused:
            L.sv_temporal(d(fr["rgb"]), g, d(fr["mv"]), prev, *hist, out, om1, om2, on, tp,
                          mlp=mlp, albedo=alb, kappa_out=k2, alpha_out=a2)
        else:
            L.sv_temporal(d(fr["rgb"]), g, d(fr["mv"]), prev, *hist, out, om1, om2, on, tp,
                          alpha_map=a1)
            a2, k2 = a1, k1
        outs.append([host(t) for t in (out, om1, om2, on, a2, k2)])
    for name, x, y in zip(("rgb", "m1", "m2c", "n", "alpha", "kappa"), *outs):
        np.testing.assert_array_equal(x, y, err_msg=name)


def test_learned_driver_matches_learned_calls():
    """Denoiser(mlp=...) through the native driver equals its call-by-call
    path and the separate-kernel learned chain, bitwise, over a sequence."""
    from paper_2312_06827_amd import learn
    from paper_2312_06827_amd.pipeline import MOTION, Denoiser, FrameInputs
    cfg = with_size(CONFIGS["hd_motion"], 200, 120, 5)
    w = _weights(41)
    mlp = _device_mlp(w)
    a = Denoiser(cfg.height, cfg.width, MOTION, mlp=mlp)
    b = Denoiser(cfg.height, cfg.width, MOTION, mlp=mlp)
    c = learn.LearnedDenoiser(cfg.height, cfg.width, mlp, MOTION)

    class _Null:
        def __call__(self, name):
            import contextlib
            return contextlib.nullcontext()

    say("learned native driver vs calls vs separate kernels")
    for fr in sequence(cfg):
        inp = FrameInputs.from_numpy(fr)
        oa = a.frame(inp).clone()
        ob = b.frame(inp, timer=_Null()).clone()
        oc = c.frame(inp, inp.albedo).clone()
        assert torch.equal(oa, ob)
        assert torch.equal(oa, oc)
