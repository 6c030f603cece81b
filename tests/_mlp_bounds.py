"""Error bounds for the learned component's device kernels against the
oracle's precision model (oracle/mlp.py): which roundings to bfloat16 can
go the other way on the device, and what that does to each output.

The device rounds the same quantities to bfloat16 as the oracle (hidden
activations, the head gradients, the back-propagated hidden gradients),
but forms them in binary32 in another order (matrix-core sums, binary32
heads).  Where a value lies within a few binary32 ulps of a bfloat16
rounding midpoint the two sides can round it to the two neighbours: a
flip of one bfloat16 ulp.  A flip candidate is such a value; its effect
is worked out by running the pixel again with that one value rounded the
other way.  The parity tests allow, per output, the sum of the effects of
its candidates plus a binary32 summation slack, and nothing else.
"""

from __future__ import annotations

import numpy as np

from oracle import mlp as M

# distance to a bfloat16 midpoint, in binary32 ulps, within which the two
# sides' binary32 values may round apart
MIDPOINT_ULPS = 64


def _f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def near_midpoint(v, scale=None, k=MIDPOINT_ULPS):
    """True where binary32 v lies within k binary32 ulps of `scale` (the
    magnitude its rounding error is relative to: |v| for a product, the sum
    of the terms' magnitudes for a sum) of a bfloat16 rounding midpoint."""
    v = np.asarray(v, np.float64)
    b = np.ascontiguousarray(v.astype(np.float32)).view(np.uint32).astype(np.uint64)
    lo = (b >> 16) << 16
    to = lambda u: np.ascontiguousarray(u.astype(np.uint32)).view(np.float32).astype(np.float64)
    mid = 0.5 * (to(lo) + to(lo + (1 << 16)))
    scale = np.abs(v) if scale is None else np.maximum(np.asarray(scale, np.float64), np.abs(v))
    return (np.abs(v - mid) <= k * 2.0 ** -24 * scale) & (v != 0)


def other_rounding(v):
    """The bfloat16 neighbour of binary32 v that round-to-nearest-even does
    not pick."""
    b = np.asarray(np.asarray(v, np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    lo = (b >> 16) << 16
    hi = lo + (1 << 16)
    to = lambda u: np.asarray(u.astype(np.uint32)).view(np.float32).astype(np.float64)
    q = M.bf16(v)
    return np.where(q == to(lo), to(hi), to(lo))


def pixel_pass(w: M.Weights, x, da, dk, over=None):
    """Forward and backward of one pixel in the oracle's precision model.
    x: 14 standardised bfloat16 features; da, dk: binary32 loss gradients
    of alpha and kappa.  over: {(name, index): value} replaces the
    bfloat16-rounded value of h1, h2, go, gh2 or gh1 at index, or (for
    "m1", "m2") the ReLU's decision a > 0 of a pre-activation whose sign
    the binary32 sums could take the other way.  Returns (alpha, kappa,
    contribution to the 1602 parameter gradients, and the pre-rounding
    values {name: vector}, with "a1", "a2" and their magnitude scales
    "s1", "s2")."""
    over = over or {}
    q = M.bf16

    def rq(name, v):
        r = q(v)
        for (n, i), val in over.items():
            if n == name:
                r = r.copy()
                r[i] = val
        return r

    def mask(name, a):
        m = a > 0
        for (n, i), val in over.items():
            if n == name:
                m = m.copy()
                m[i] = val
        return m

    w1, w2, w3 = q(w.w1), q(w.w2), q(w.w3)
    a1 = _f32(w1 @ x + w.b1)
    m1 = mask("m1", a1)
    h1 = np.where(m1, np.maximum(a1, 0.0), 0.0)
    h1q = rq("h1", h1)
    a2 = _f32(w2 @ h1q + w.b2)
    m2 = mask("m2", a2)
    h2 = np.where(m2, np.maximum(a2, 0.0), 0.0)
    h2q = rq("h2", h2)
    o = _f32(w3 @ h2q + w.b3)
    sig = 1.0 / (1.0 + np.exp(-o[0]))
    th = np.tanh(o[1])
    alpha = M.ALPHA_MIN + (1.0 - M.ALPHA_MIN) * sig
    kappa = np.exp2(M.KAPPA_LOG2_RANGE * th)
    go = _f32(np.array([da * (1.0 - M.ALPHA_MIN) * sig * (1.0 - sig),
                        dk * kappa * np.log(2.0) * M.KAPPA_LOG2_RANGE * (1.0 - th * th)]))
    goq = rq("go", go)
    gh2 = _f32(w3.T @ goq) * m2
    gh2q = rq("gh2", gh2)
    gh1 = _f32(w2.T @ gh2q) * m1
    gh1q = rq("gh1", gh1)
    contrib = np.concatenate([np.outer(gh1q, x).ravel(), gh1, np.outer(gh2q, h1q).ravel(), gh2,
                              np.outer(goq, h2q).ravel(), go])
    # magnitudes the binary32 sums' rounding errors scale with
    s1 = np.abs(w1) @ np.abs(x) + np.abs(w.b1)
    s2 = np.abs(w2) @ np.abs(h1q) + np.abs(w.b2)
    sg2 = np.abs(w3.T) @ np.abs(goq)
    sg1 = np.abs(w2.T) @ np.abs(gh2q)
    # the head gradients come through the heads from o, whose binary32 sum
    # may be off by its own rounding (relative to the magnitude so): the
    # heads' slopes are at most 1 in o (sigmoid') and 4 ln 2 (2^(2 tanh))
    so = np.abs(w3) @ np.abs(h2q) + np.abs(w.b3)
    sgo = np.abs(go) * (1.0 + 4.0 * so)
    return alpha, kappa, contrib, {"h1": h1, "h2": h2, "go": go, "gh2": gh2, "gh1": gh1,
                                   "a1": a1, "a2": a2, "s1": s1, "s2": s2,
                                   "scale": {"h1": s1, "h2": s2, "go": sgo, "gh2": sg2,
                                             "gh1": sg1}}


def near_zero(a, scale, k=MIDPOINT_ULPS):
    """True where a sum a of terms of total magnitude `scale` lies within k
    binary32 ulps of that magnitude of zero, so that another summation
    order can give it the other sign (or zero)."""
    return np.abs(a) <= k * 2.0 ** -23 * scale


def flip_bounds(w: M.Weights, xs, da, dk, forward_only=False):
    """Per pixel (columns of xs): the summed effect of every flip candidate
    on alpha, on kappa (relative) and on the 1602 gradient contributions.
    Returns (bound_alpha (N,), bound_kappa (N,), bound_grad (1602,),
    abs_sum (1602,) = sum over pixels of |contribution|, contributions'
    sum (1602,), number of candidates)."""
    N = xs.shape[1]
    ba, bk = np.zeros(N), np.zeros(N)
    bg, asum, total = np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS)
    count = 0
    names = ("h1", "h2") if forward_only else ("h1", "h2", "go", "gh2", "gh1")
    for p in range(N):
        al, ka, c, pre = pixel_pass(w, xs[:, p], da[p], dk[p])
        asum += np.abs(c)
        total += c
        flips = []
        for name in names:
            v = pre[name]
            flips += [{(name, int(i)): other_rounding(v[i:i + 1])[0]}
                      for i in np.nonzero(near_midpoint(v, pre["scale"][name]))[0]]
        for mname, aname, sname in (("m1", "a1", "s1"), ("m2", "a2", "s2")):
            a = pre[aname]
            flips += [{(mname, int(i)): not bool(a[i] > 0)}
                      for i in np.nonzero(near_zero(a, pre[sname]))[0]]
        for ov in flips:
            al2, ka2, c2, _ = pixel_pass(w, xs[:, p], da[p], dk[p], ov)
            ba[p] += abs(al2 - al)
            bk[p] += abs(ka2 - ka) / ka
            bg += np.abs(c2 - c)
            count += 1
    return ba, bk, bg, asum, total, count
