"""FP64 oracle of the learned blend / edge-scale predictor.

TEST INFRASTRUCTURE ONLY: the plain reference that the device MLP kernels
are checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.

The paper has no learned component.  It filters with a fixed temporal
blend factor and a fixed luminance edge sigma (Section 2).  This module
defines a per-pixel network that predicts both per pixel:

    x  (14 features) -> 32 -> ReLU -> 32 -> ReLU -> 2 -> (alpha, kappa)

where alpha in [0.05, 1] replaces the colour blend factor of the temporal
step and kappa in [1/4, 4] scales sigma_l in every a-trous level.

Features, per pixel, computed from the temporal step's own intermediates:
 0  luminance of the current (tone-mapped) colour
 1  luminance of the reprojected, clamped history colour (0 without history)
 2  reprojected central second moment of the luminance (0 without history)
 3  population variance of the current luminance over the in-image,
    non-empty 3x3 neighbourhood
 4  the new history length / 255
 5, 6  depth gradients dz/dx, dz/dy
 7, 8, 9  normal
 10  motion length |mv| (0 where the motion is discarded: not finite, or
     a component of 2^20 pixels or more)
 11, 12, 13  albedo
Empty pixels (z <= 0 or non-finite) have all-zero raw features.  Each
feature is standardised with a fixed (mean, 1/scale) pair stored with the
weights.

Precision model of the device (``bf16=True``): matrix-product operands
(weights, standardised features, hidden activations, and in the backward
pass the incoming gradients) are rounded to bfloat16 (round to nearest
even); sums and biases are binary32, so each layer's pre-activation is
rounded to binary32.  ``bf16=False`` is plain FP64, used for finite-
difference checks of the backward pass.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

from . import clamp as _clamp
from . import luma, reproject, tonemap

N_IN, N_HID, N_OUT = 14, 32, 2
ALPHA_MIN = 0.05
KAPPA_LOG2_RANGE = 2.0  # kappa = 2^(2 tanh(o2))


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) via binary32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


@dataclass
class Weights:
    """FP32 master weights, row-major [out, in], plus the standardisation."""
    w1: np.ndarray  # (32, 14)
    b1: np.ndarray  # (32,)
    w2: np.ndarray  # (32, 32)
    b2: np.ndarray
    w3: np.ndarray  # (2, 32)
    b3: np.ndarray  # (2,)
    mu: np.ndarray  # (14,)
    inv_s: np.ndarray  # (14,)

    def flat(self):
        return np.concatenate([self.w1.ravel(), self.b1, self.w2.ravel(), self.b2,
                               self.w3.ravel(), self.b3])

    @staticmethod
    def from_flat(v, mu, inv_s):
        v = np.asarray(v, dtype=np.float64)
        o = 0

        def take(shape):
            nonlocal o
            k = int(np.prod(shape))
            a = v[o:o + k].reshape(shape)
            o += k
            return a
        w = Weights(take((N_HID, N_IN)), take((N_HID,)), take((N_HID, N_HID)), take((N_HID,)),
                    take((N_OUT, N_HID)), take((N_OUT,)), np.asarray(mu, np.float64),
                    np.asarray(inv_s, np.float64))
        assert o == v.size
        return w


N_PARAMS = N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + N_OUT * N_HID + N_OUT  # 1602


def init_weights(seed: int, mu=None, inv_s=None) -> Weights:
    """He-normal hidden layers; output layer zero (alpha = 0.05 + 0.95 / 2,
    kappa = 1 at the start)."""
    r = np.random.default_rng(seed)
    f = lambda a: a.astype(np.float32).astype(np.float64)
    return Weights(
        f(r.normal(0, np.sqrt(2 / N_IN), (N_HID, N_IN))), np.zeros(N_HID),
        f(r.normal(0, np.sqrt(2 / N_HID), (N_HID, N_HID))), np.zeros(N_HID),
        np.zeros((N_OUT, N_HID)), np.zeros(N_OUT),
        np.zeros(N_IN) if mu is None else np.asarray(mu, np.float64),
        np.ones(N_IN) if inv_s is None else np.asarray(inv_s, np.float64))


# ---- features ---------------------------------------------------------------

def _empty(z):
    z = np.asarray(z, dtype=np.float64)
    return ~(np.isfinite(z) & (z > 0))


def box_luma_variance(L, z):
    """Population variance of L over each pixel's in-image, non-empty 3x3
    neighbourhood (0 where that set is empty)."""
    L = np.asarray(L, dtype=np.float64)
    ok = ~_empty(z)
    H, W = L.shape
    s1, s2, cnt = np.zeros((H, W)), np.zeros((H, W)), np.zeros((H, W))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ys0, ys1 = max(0, dy), H + min(0, dy)
            xs0, xs1 = max(0, dx), W + min(0, dx)
            src = (slice(ys0, ys1), slice(xs0, xs1))
            dst = (slice(ys0 - dy, ys1 - dy), slice(xs0 - dx, xs1 - dx))
            m = ok[src]
            s1[dst] += np.where(m, L[src], 0.0)
            s2[dst] += np.where(m, L[src] ** 2, 0.0)
            cnt[dst] += m
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = s1 / cnt
        v = s2 / cnt - mean * mean
    return np.where(cnt > 0, np.maximum(v, 0.0), 0.0)


def features(frame: Dict[str, np.ndarray], state: Dict[str, np.ndarray], p) -> Dict[str, np.ndarray]:
    """Raw features (14, H, W) of one frame, plus the clamped reprojected
    history colour (the blend's other operand) and the tone-mapped current
    colour.  `p` is an oracle.OracleParams."""
    cur = tonemap(frame["rgb"], k=p.tm_k) if p.tonemap else np.asarray(frame["rgb"], np.float64)
    z = np.asarray(frame["z"], np.float64)
    r = reproject(frame["z"], frame["n"], frame["mv"], frame["prev_z"], frame["prev_n"],
                  state["rgb"], state["m1"], state["m2"], state["n"], p.tau_z, p.tau_n,
                  frame.get("id"), frame.get("prev_id"), p.use_id)
    valid = r["valid"] != 0
    hist = _clamp(r["rgb"], cur, p.gamma, z=z) if p.clamp else r["rgb"]
    hist = np.where(valid[None], hist, 0.0)
    empty = _empty(z)
    Lc = luma(cur)
    mv = np.asarray(frame["mv"], np.float64)
    n_new = np.where(valid, np.minimum(r["n"] + 1, p.max_hist), 1)
    # motion that is not finite or not below 2^20 pixels is discarded
    with np.errstate(invalid="ignore"):
        mv_ok = np.isfinite(mv).all(0) & (np.abs(mv) < 2.0 ** 20).all(0)
    x = np.stack([
        Lc,
        np.where(valid, luma(hist), 0.0),
        np.where(valid, np.maximum(r["m2"] - r["m1"] ** 2, 0.0), 0.0),
        box_luma_variance(Lc, z),
        n_new / 255.0,
        np.asarray(frame["dzdx"], np.float64),
        np.asarray(frame["dzdy"], np.float64),
        *np.asarray(frame["n"], np.float64),
        np.where(mv_ok, np.sqrt(np.where(mv_ok, mv[0] ** 2 + mv[1] ** 2, 0.0)), 0.0),
        *np.asarray(frame["albedo"], np.float64),
    ])
    x = np.where(empty[None], 0.0, x)
    return {"x": x, "hist": hist, "cur": cur, "valid": valid, "n_new": n_new}


def standardise(x, w: Weights, bf16_out=True):
    """(14, N) raw -> (14, N) standardised, bf16-rounded as the device's
    matrix operand (binary32 arithmetic in the device's order)."""
    x = np.asarray(x, np.float64).reshape(N_IN, -1)
    if not bf16_out:
        return (x - w.mu[:, None]) * w.inv_s[:, None]
    mu, s = f32(w.mu)[:, None], f32(w.inv_s)[:, None]
    return bf16(f32(f32(f32(x) - mu) * s))


# ---- network ----------------------------------------------------------------

def _q(a, on):
    return bf16(a) if on else a


def _r32(a, on):
    return f32(a) if on else a


def forward(w: Weights, xs, bf16_ops=True):
    """xs: standardised features (14, N).  Returns dict with the heads
    (alpha, kappa), raw outputs o (2, N) and the activations the backward
    pass needs."""
    q = lambda a: _q(a, bf16_ops)
    r = lambda a: _r32(a, bf16_ops)
    x = q(xs)
    a1 = r(q(w.w1) @ x + w.b1[:, None])
    h1 = np.maximum(a1, 0.0)
    a2 = r(q(w.w2) @ q(h1) + w.b2[:, None])
    h2 = np.maximum(a2, 0.0)
    o = r(q(w.w3) @ q(h2) + w.b3[:, None])
    sig = 1.0 / (1.0 + np.exp(-o[0]))
    th = np.tanh(o[1])
    alpha = ALPHA_MIN + (1.0 - ALPHA_MIN) * sig
    kappa = np.exp2(KAPPA_LOG2_RANGE * th)
    return {"alpha": alpha, "kappa": kappa, "o": o, "a1": a1, "h1": h1, "a2": a2, "h2": h2,
            "x": x, "sig": sig, "tanh": th}


def head_grads(fw, d_alpha, d_kappa):
    """dL/do (2, N) from dL/dalpha and dL/dkappa (binary32 on the device)."""
    g0 = d_alpha * (1.0 - ALPHA_MIN) * fw["sig"] * (1.0 - fw["sig"])
    g1 = d_kappa * fw["kappa"] * np.log(2.0) * KAPPA_LOG2_RANGE * (1.0 - fw["tanh"] ** 2)
    return np.stack([g0, g1])


def backward(w: Weights, fw, g_o, bf16_ops=True):
    """Gradients of sum_pixels(g_o . o) with respect to every parameter, in
    the flat order of Weights.flat()."""
    q = lambda a: _q(a, bf16_ops)
    r = lambda a: _r32(a, bf16_ops)
    go = r(g_o)
    dw3 = q(go) @ q(fw["h2"]).T
    db3 = go.sum(1)
    gh2 = r(q(w.w3).T @ q(go)) * (fw["a2"] > 0)
    dw2 = q(gh2) @ q(fw["h1"]).T
    db2 = gh2.sum(1)
    gh1 = r(q(w.w2).T @ q(gh2)) * (fw["a1"] > 0)
    dw1 = q(gh1) @ fw["x"].T
    db1 = gh1.sum(1)
    return np.concatenate([dw1.ravel(), db1, dw2.ravel(), db2, dw3.ravel(), db3])


@dataclass
class AdamParams:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


def adam(master, m, v, g, t, p: AdamParams = AdamParams()):
    """One Adam step (t counts from 1).  Returns new (master, m, v)."""
    m = p.beta1 * m + (1 - p.beta1) * g
    v = p.beta2 * v + (1 - p.beta2) * g * g
    mh = m / (1 - p.beta1 ** t)
    vh = v / (1 - p.beta2 ** t)
    return master - p.lr * mh / (np.sqrt(vh) + p.eps), m, v


# ---- truncated loss gradients ----------------------------------------------

def relmse_weight(y):
    """RelMSE of x against target y: mean over pixels and channels of
    (x - y)^2 / (y^2 + 0.01).  This is d/dx of one element's term / 2."""
    y = np.asarray(y, np.float64)
    return 1.0 / (y * y + 0.01)


def alpha_grad(c_t, cur, hist, y, alpha_map, n_new):
    """dL/dalpha per pixel for L = sum over pixels of the per-pixel RelMSE
    term (mean over the three channels) of the temporal output c_t against
    y, holding the history fixed: c_t = (1 - a) hist + a cur with
    a = max(alpha, 1/n); zero where 1/n wins."""
    c_t, cur, hist, y = (np.asarray(a, np.float64) for a in (c_t, cur, hist, y))
    g = (2.0 / 3.0) * ((c_t - y) * relmse_weight(y) * (cur - hist)).sum(0)
    return np.where(np.asarray(alpha_map) >= 1.0 / np.asarray(n_new, np.float64), g, 0.0)


def atrous_kappa_derivative(c, var, z, dzdx, dzdy, n, kappa, step, sigma_z=1.0,
                            sigma_n=128.0, sigma_l=4.0, eps_z=1e-10, eps_l=1e-10):
    """d c'(p) / d kappa(p) of one 5x5 a-trous level (3, H, W), with the
    level input held fixed.  Only the luminance weight depends on kappa:
    w_l = exp(-|dL| / (sigma_l kappa sqrt(g) + eps_l)), so
    d w_l / d kappa = w_l |dL| sigma_l sqrt(g) / (sigma_l kappa sqrt(g) + eps_l)^2,
    and c' = sum H w c / sum H w gives
    d c' / d kappa = sum H (dw/dkappa) (c_q - c') / sum H w."""
    c = np.asarray(c, np.float64)
    var, z, dzdx, dzdy, n, kappa = (np.asarray(a, np.float64) for a in (var, z, dzdx, dzdy, n, kappa))
    H, W = z.shape
    h1 = np.array([1, 4, 6, 4, 1]) / 16.0
    k3 = np.array([0.25, 0.5, 0.25])
    ok = ~_empty(z)
    # 3x3 Gaussian of var over the in-image, non-empty taps, renormalised
    # (the level's own prefilter: an empty pixel is no neighbour)
    okf = ok.astype(np.float64)
    num, den = np.zeros((H, W)), np.zeros((H, W))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            vv, mm = _shift(np.where(ok, var, 0.0), dx, dy), _shift(okf, dx, dy)
            num += k3[dy + 1] * k3[dx + 1] * vv
            den += k3[dy + 1] * k3[dx + 1] * mm
    with np.errstate(invalid="ignore", divide="ignore"):
        g = np.where(ok, num / den, 0.0)
    L = luma(c)
    dl = sigma_l * kappa * np.sqrt(g) + eps_l
    sw, sc = np.zeros((H, W)), np.zeros((3, H, W))
    sd, sdc = np.zeros((H, W)), np.zeros((3, H, W))
    for b in range(-2, 3):
        for a in range(-2, 3):
            hh = h1[a + 2] * h1[b + 2]
            if a == 0 and b == 0:
                w, d = np.ones((H, W)), np.zeros((H, W))
                cq = c
            else:
                inside = _shift(np.ones((H, W)), a * step, b * step) > 0
                zq = _shift(z, a * step, b * step)
                okq = _shift(ok.astype(np.float64), a * step, b * step) > 0
                nq = np.stack([_shift(n[i], a * step, b * step) for i in range(3)])
                cq = np.stack([_shift(c[i], a * step, b * step) for i in range(3)])
                Lq = luma(cq)
                dz = sigma_z * np.abs(dzdx * step * a + dzdy * step * b) + eps_z
                wz = np.exp(-np.abs(z - zq) / dz)
                chord = ((n - nq) ** 2).sum(0)
                wn = np.maximum(0.0, 1.0 - 0.5 * chord) ** sigma_n
                adl = np.abs(L - Lq)
                wl = np.exp(-adl / dl)
                w = np.where(inside & okq, wz * wn * wl, 0.0)
                d = np.where(inside & okq, w * adl * sigma_l * np.sqrt(g) / (dl * dl), 0.0)
            sw += hh * w
            sc += hh * w * cq
            sd += hh * d
            sdc += hh * d * cq
    out = sc / sw
    deriv = (sdc - out * sd) / sw
    return np.where(ok[None], deriv, 0.0)


def _shift(a, dx, dy):
    """b[y, x] = a[y + dy, x + dx], 0 outside the image."""
    H, W = a.shape
    b = np.zeros_like(a)
    ys0, ys1 = max(0, -dy), min(H, H - dy)
    xs0, xs1 = max(0, -dx), min(W, W - dx)
    if ys0 < ys1 and xs0 < xs1:
        b[ys0:ys1, xs0:xs1] = a[ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
    return b


def kappa_grad_level(out_level, y, deriv):
    """dL/dkappa contribution of one level: the per-pixel RelMSE term (mean
    over channels) of the level's output against y, times d out / d kappa."""
    out_level, y, deriv = (np.asarray(a, np.float64) for a in (out_level, y, deriv))
    return (2.0 / 3.0) * ((out_level - y) * relmse_weight(y) * deriv).sum(0)
