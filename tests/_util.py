"""Shared test helpers: the parity metric and seeded synthetic call inputs."""

import sys

import numpy as np


def say(msg):
    """Progress line, flushed, so a GPU run names its case before it runs."""
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(gpu, ora, floor=1e-3, abs_floor=0.0):
    """Largest relative error |g - o| / max(|o|, floor * RMS(o), abs_floor),
    taken per plane (leading axes are planes) and maximised.  abs_floor
    states the plane's scale where the oracle's plane alone cannot (a
    variance that is zero but for rounding residues)."""
    g = np.asarray(gpu, dtype=np.float64)
    o = np.asarray(ora, dtype=np.float64)
    assert g.shape == o.shape, (g.shape, o.shape)
    if o.ndim == 2:
        g, o = g[None], o[None]
    g = g.reshape(-1, *o.shape[-2:])
    o = o.reshape(-1, *o.shape[-2:])
    worst = 0.0
    for gp, op in zip(g, o):
        rms = np.sqrt(np.mean(op * op))
        den = np.maximum(np.maximum(np.abs(op), floor * rms), abs_floor)
        den = np.where(den > 0, den, 1.0)
        e = np.abs(gp - op) / den
        if not np.all(np.isfinite(e)):
            return float("inf")
        worst = max(worst, float(e.max()))
    return worst


def random_gbuf(r, H, W, z_range=(4.0, 6.0)):
    """A smooth random surface with its analytic gradients and normals."""
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    kx, ky, ph = r.uniform(0.02, 0.1), r.uniform(0.02, 0.1), r.uniform(0, 6.28)
    z = z_range[0] + (z_range[1] - z_range[0]) * 0.5 * (1 + np.sin(kx * xs + ph) * np.cos(ky * ys))
    amp = 0.5 * (z_range[1] - z_range[0])
    dzdx = amp * kx * np.cos(kx * xs + ph) * np.cos(ky * ys)
    dzdy = -amp * ky * np.sin(kx * xs + ph) * np.sin(ky * ys)
    n = np.stack([-dzdx, np.ones_like(z), -dzdy])
    n /= np.linalg.norm(n, axis=0)
    f = lambda a: a.astype(np.float32)
    return f(z), f(dzdx), f(dzdy), f(n)


def frac_over(gpu, ora, tol, floor=1e-3, abs_floor=0.0):
    """Fraction of the elements whose relative error (as rel_err() takes
    it) exceeds tol."""
    g = np.asarray(gpu, dtype=np.float64)
    o = np.asarray(ora, dtype=np.float64)
    if o.ndim == 2:
        g, o = g[None], o[None]
    over = total = 0
    for gp, op in zip(g.reshape(-1, *o.shape[-2:]), o.reshape(-1, *o.shape[-2:])):
        rms = np.sqrt(np.mean(op * op))
        den = np.maximum(np.maximum(np.abs(op), floor * rms), abs_floor)
        den = np.where(den > 0, den, 1.0)
        over += int(np.count_nonzero(np.abs(gp - op) / den > tol))
        total += gp.size
    return over / max(total, 1)


def worst(gpu, ora, floor=1e-3, abs_floor=0.0):
    """Where the relative error of rel_err() peaks: (plane, y, x, gpu, oracle)."""
    g = np.asarray(gpu, dtype=np.float64)
    o = np.asarray(ora, dtype=np.float64)
    if o.ndim == 2:
        g, o = g[None], o[None]
    best = (0.0, None)
    for k, (gp, op) in enumerate(zip(g, o)):
        rms = np.sqrt(np.mean(op * op))
        den = np.maximum(np.maximum(np.abs(op), floor * rms), abs_floor)
        den = np.where(den > 0, den, 1.0)
        e = np.abs(gp - op) / den
        i = np.unravel_index(int(np.argmax(e)), e.shape)
        if e[i] > best[0]:
            best = (float(e[i]), (k,) + tuple(int(v) for v in i) + (float(gp[i]), float(op[i])))
    return best[1]


# ---- guard bands of pitched output planes --------------------------------------
#
# Output planes with a row pitch larger than the width are registered here
# with their padding filled (NaN, or 0xA5 in byte planes); after every test
# the padding must be unchanged: a kernel that writes past a row's end fails
# the test that ran it.

GUARDED = []


def guard_value(dtype):
    return float("nan") if dtype.is_floating_point else 0xA5


def guard(full, width):
    """Register the full pitched tensor whose columns >= width are padding."""
    GUARDED.append((full, width))


def check_guards():
    if not GUARDED:
        return
    import torch
    torch.cuda.synchronize()
    bad = []
    for full, width in GUARDED:
        pad = full[..., width:]
        ok = bool(torch.isnan(pad).all()) if pad.dtype.is_floating_point \
            else bool((pad == 0xA5).all())
        if not ok:
            bad.append((tuple(full.shape), width, str(full.dtype)))
    GUARDED.clear()
    assert not bad, f"writes into the row padding of pitched outputs: {bad}"


def list_consumed(work):
    """Whether the variance workspace's short-history list has been read:
    each of the eight counter lines (32 words) holds its append count in
    word 0 and, once the reading pass has run, the same value in word 2."""
    c = work[:256].view(8, 32).cpu()
    return bool((c[:, 0] == c[:, 2]).all())


def make_hostile(fr, r):
    """Scatter every kind of unusable input over one frame (in place, in the
    frame's own dtype; binary16 overflows to infinity): empty pixels of
    every kind in the current and previous depth (0, -0, negative, NaN,
    infinite), motion that is not finite or beyond 2^20 pixels, motion that
    leaves the image, and taps straddling its border."""
    H, W = fr["z"].shape
    bad_z = np.array([0.0, -0.0, -1.0, np.nan, np.inf])
    bad_mv = np.array([1e7, -1e7, np.nan, np.inf, 1048575.5, -1048576.0, 3.0 * 1048576.0])
    ys, xs = np.mgrid[0:H, 0:W]
    with np.errstate(over="ignore", invalid="ignore"):
        for key in ("z", "prev_z"):
            z = fr[key].copy()
            pick = r.random((H, W)) < 0.12
            z[pick] = bad_z[r.integers(0, len(bad_z), pick.sum())]
            fr[key] = z
        mv = fr["mv"].copy()
        u = r.random((H, W))
        hard = u < 0.08
        mv[0][hard] = bad_mv[r.integers(0, len(bad_mv), hard.sum())]
        mv[1][hard] = bad_mv[r.integers(0, len(bad_mv), hard.sum())]
        off = (u >= 0.08) & (u < 0.16)  # well off the image
        mv[0][off] = (r.random(off.sum()) - 0.5) * 4.0 * (W + 2)
        mv[1][off] = (r.random(off.sum()) - 0.5) * 4.0 * (H + 2)
        edge = (u >= 0.16) & (u < 0.2)  # taps straddling x = -1 and y = H - 1
        mv[0][edge] = -xs[edge] - 0.5
        mv[1][edge] = H - 1 - ys[edge] + 0.25
        fr["mv"] = mv
    return fr
