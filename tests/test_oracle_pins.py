"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms, library routines (scipy.ndimage.correlate, numpy statistics,
numpy's binary16 conversion), invariants and hand-derived worked examples.

Each test is built so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a wrong normaliser) fails it.
"""

import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
B3 = np.array([1, 4, 6, 4, 1], dtype=np.float64) / 16.0
LUMA_W = np.array([0.2126, 0.7152, 0.0722])


def rng(seed):
    return np.random.default_rng(seed)


def dilated_b3(step):
    k = np.zeros(4 * step + 1)
    k[::step] = B3
    return k


def kernel2d(step):
    k = dilated_b3(step)
    return np.outer(k, k)  # [row = b (y), col = a (x)]


def corr(img, k):
    return ndimage.correlate(img, k, mode="constant", cval=0.0)


def flat_gbuf(H, W, z=5.0):
    """Constant depth with zero gradient and one shared normal: every depth
    and normal weight is exactly 1."""
    n = np.zeros((3, H, W))
    n[1] = 1.0
    return np.full((H, W), z), np.zeros((H, W)), np.zeros((H, W)), n


def equal_luma_rgb(r, H, W, L0=0.5):
    """Colours that differ in chroma but share luminance L0 (luminance
    weight exactly 1)."""
    red = r.uniform(0.0, 1.0, (H, W))
    blue = r.uniform(0.0, 1.0, (H, W))
    green = (L0 - LUMA_W[0] * red - LUMA_W[2] * blue) / LUMA_W[1]
    return np.stack([red, green, blue])


# ---- tone map (Section 3.4) ------------------------------------------------

def test_tonemap_grey_is_c_over_1_plus_kc():
    c = np.linspace(0.0, 20.0, 41)
    grey = np.stack([c, c, c])[:, None, :]
    for k in (1.0, 2.0, 0.5):
        out = O.tonemap(grey, k=k)
        np.testing.assert_allclose(out[0, 0], c / (1.0 + k * c), rtol=1e-15, atol=0)


def test_tonemap_primaries_pin_luma_weights():
    eye = np.eye(3)[:, :, None, None] * np.ones((1, 1, 1, 1))  # three images
    for ch, w in enumerate(LUMA_W):
        out = O.tonemap(eye[ch])
        expect = np.zeros(3)
        expect[ch] = 1.0 / (1.0 + w)
        np.testing.assert_allclose(out[:, 0, 0], expect, rtol=1e-15, atol=0)


def test_tonemap_exact_inverse_round_trip():
    c = rng(1).exponential(1.0, (3, 17, 9)) * 5.0
    for k in (1.0, 0.3):
        back = O.tonemap(O.tonemap(c, k=k), inverse=True, k=k)
        np.testing.assert_allclose(back, c, rtol=1e-13, atol=1e-15)
    back = O.tonemap(O.tonemap(c, mode="channel"), inverse=True, mode="channel")
    np.testing.assert_allclose(back, c, rtol=1e-13, atol=1e-15)


def test_tonemap_paper_inverse_is_not_an_inverse():
    # The listing "removes" the tone map with c' (1 + L(c')) w.  For grey c
    # (L = c) and k = w = 1 that returns c (1 + 2c) / (1 + c)^2.
    with open(os.path.join(GOLDEN, "tonemap_paper_inverse.json")) as f:
        gold = json.load(f)
    for row in gold["cases"]:
        c = row["L"]
        grey = np.full((3, 1, 1), c)
        back = O.tonemap(O.tonemap(grey), inverse=True, mode="paper", weight=1.0)
        assert back[0, 0, 0] / c == pytest.approx(row["ratio"], rel=1e-12)


# ---- binary16 storage ---------------------------------------------------------

def test_quantize_half_matches_numpy_float16():
    r = rng(2)
    x = np.concatenate([
        r.normal(0, 1, 5000), r.normal(0, 1e-5, 2000), r.normal(0, 3e4, 2000),
        # exact ties between neighbouring binary16 values
        (np.arange(1024, 2048) + 0.5) / 1024.0, -(np.arange(1024, 2048) + 0.5) / 512.0,
        [65504.0, 65519.9, 65520.0, 1e6, -1e6, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26, 0.0],
    ])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    got = O.quantize_half(x)
    np.testing.assert_array_equal(got, ref)


# ---- reprojection (Section 2) -------------------------------------------------

def _static_prev(H, W, z=5.0):
    z_, dzdx, dzdy, n = flat_gbuf(H, W, z)
    return z_, n


def test_reproject_integer_motion_is_a_shift():
    H, W = 13, 21
    r = rng(3)
    z, n = _static_prev(H, W)
    hist = r.uniform(0, 1, (3, H, W))
    m1, m2 = r.uniform(0, 1, (H, W)), r.uniform(0, 1, (H, W))
    hn = np.full((H, W), 7, np.int32)
    mv = np.zeros((2, H, W))
    mv[0], mv[1] = 3.0, -2.0
    out = O.reproject(z, n, mv, z, n, hist, m1, m2, hn)
    ys, xs = np.mgrid[0:H, 0:W]
    inside = (xs + 3 < W) & (ys - 2 >= 0)
    assert np.array_equal(out["valid"].astype(bool), inside)
    src_y, src_x = ys[inside] - 2, xs[inside] + 3
    np.testing.assert_array_equal(out["rgb"][:, inside], hist[:, src_y, src_x])
    np.testing.assert_array_equal(out["m1"][inside], m1[src_y, src_x])
    np.testing.assert_array_equal(out["m2"][inside], m2[src_y, src_x])
    assert np.all(out["n"][inside] == 7)


def test_reproject_bilinear_is_exact_on_affine_history():
    H, W = 11, 16
    z, n = _static_prev(H, W)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    hist = np.stack([1.0 + 0.3 * xs - 0.2 * ys, 2.0 - 0.1 * xs + 0.7 * ys, 0.5 + 0.05 * xs])
    hn = np.full((H, W), 5, np.int32)
    for mvx, mvy in [(0.25, 0.6), (-1.75, 2.125), (-0.5, -0.375)]:
        mv = np.stack([np.full((H, W), mvx), np.full((H, W), mvy)])
        out = O.reproject(z, n, mv, z, n, hist, hist[0], hist[1], hn)
        x0 = xs + np.floor(mvx)
        y0 = ys + np.floor(mvy)
        inside = (x0 >= 0) & (x0 + 1 < W) & (y0 >= 0) & (y0 + 1 < H)
        expect = np.stack([1.0 + 0.3 * (xs + mvx) - 0.2 * (ys + mvy),
                           2.0 - 0.1 * (xs + mvx) + 0.7 * (ys + mvy),
                           0.5 + 0.05 * (xs + mvx)])
        np.testing.assert_allclose(out["rgb"][:, inside], expect[:, inside], rtol=0, atol=1e-13)


@pytest.mark.parametrize("kill", ["depth", "normal", "id", "nohist", "outside"])
def test_reproject_drops_inconsistent_tap_and_renormalises(kill):
    H, W = 6, 6
    z, n = _static_prev(H, W, z=10.0)
    pz, pn = z.copy(), n.copy()
    hist = np.zeros((3, H, W))
    vals = {(2, 2): 1.0, (3, 2): 2.0, (2, 3): 4.0, (3, 3): 8.0}  # (x, y) -> value
    for (x, y), v in vals.items():
        hist[:, y, x] = v
    hn = np.full((H, W), 3, np.int32)
    ids = np.zeros((H, W), np.uint8)
    pid = ids.copy()
    use_id = False
    if kill == "depth":
        pz[3, 3] = 10.0 * 1.2  # 20% off, beyond the 10% tolerance
    elif kill == "normal":
        pn[:, 3, 3] = [1.0, 0.0, 0.0]  # perpendicular
    elif kill == "id":
        pid[3, 3] = 4
        use_id = True
    elif kill == "nohist":
        hn[3, 3] = 0
    mv = np.zeros((2, H, W))
    mv[:, 2, 2] = 0.5  # p = (2, 2) reads the four taps with weight 1/4 each
    if kill == "outside":
        # p = (5, 5) at the corner: only its own tap is inside
        mv[:, 5, 5] = 0.5
        hist[:, 5, 5] = 3.0
        out = O.reproject(z, n, mv, pz, pn, hist, hist[0], hist[1], hn)
        assert out["valid"][5, 5] == 1
        assert out["rgb"][0, 5, 5] == pytest.approx(3.0, rel=1e-15)
        return
    out = O.reproject(z, n, mv, pz, pn, hist, hist[0], hist[1], hn, id=ids,
                      prev_id=pid, use_id=use_id)
    assert out["valid"][2, 2] == 1
    assert out["rgb"][0, 2, 2] == pytest.approx((1.0 + 2.0 + 4.0) / 3.0, rel=1e-15)


def test_reproject_history_length_from_positive_weight_taps_only():
    H, W = 5, 5
    z, n = _static_prev(H, W)
    hist = np.ones((3, H, W))
    hn = np.zeros((H, W), np.int32)
    hn[1, 1], hn[1, 2], hn[2, 1], hn[2, 2] = 3, 9, 5, 7  # [y, x]
    mv = np.zeros((2, H, W))
    mv[1, 1, 1] = 0.5  # fx = 0: the x0+1 column has zero weight
    out = O.reproject(z, n, mv, z, n, hist, hist[0], hist[1], hn)
    assert out["n"][1, 1] == 5  # max over (1,1)->3 and (1,2)->5 [x, y]


def test_reproject_tolerances_are_inclusive_in_binary32():
    H, W = 1, 2
    z = np.full((H, W), 10.0)
    n = np.zeros((3, H, W))
    n[1] = 1.0
    hist = np.ones((3, H, W))
    hn = np.ones((H, W), np.int32)
    mv = np.zeros((2, H, W))
    pz = z.copy()
    pz[0, 0] = 11.25  # |dz| = 1.25 = 0.125 * 10 exactly
    out = O.reproject(z, n, mv, pz, n, hist, hist[0], hist[1], hn, tau_z=0.125)
    assert out["valid"][0, 0] == 1
    pz[0, 0] = float(np.nextafter(np.float32(11.25), np.float32(20)))
    out = O.reproject(z, n, mv, pz, n, hist, hist[0], hist[1], hn, tau_z=0.125)
    assert out["valid"][0, 0] == 0
    pn = n.copy()
    pn[:, 0, 1] = [0.0, 0.5, 0.0]  # cosine 0.5 against threshold 0.5
    out = O.reproject(z, n, mv, z, pn, hist, hist[0], hist[1], hn, tau_n=0.5)
    assert out["valid"][0, 1] == 1
    pn[:, 0, 1] = [0.0, float(np.nextafter(np.float32(0.5), np.float32(0))), 0.0]
    out = O.reproject(z, n, mv, z, pn, hist, hist[0], hist[1], hn, tau_n=0.5)
    assert out["valid"][0, 1] == 0


# ---- variance colour clamp (Sections 2, 3.1) --------------------------------

def _box_stats(c, x, y):
    H, W = c.shape
    win = c[max(0, y - 1):y + 2, max(0, x - 1):x + 2]
    return win.mean(), win.std(ddof=0)


@pytest.mark.parametrize("gamma", [1.0, 2.5])
def test_clamp_box_is_mean_and_population_std(gamma):
    H, W = 7, 10
    cur = rng(4).uniform(0, 2, (3, H, W))
    for sign in (1.0, -1.0):
        hist = np.full((3, H, W), sign * 1e9)
        out = O.clamp(hist, cur, gamma)
        for ch in range(3):
            for y in range(H):
                for x in range(W):
                    mu, sd = _box_stats(cur[ch], x, y)
                    assert out[ch, y, x] == pytest.approx(mu + sign * gamma * sd, rel=1e-13, abs=1e-14)


def test_clamp_idempotent_identity_and_constant():
    H, W = 9, 8
    r = rng(5)
    cur = r.uniform(0, 1, (3, H, W))
    hist = r.uniform(-1, 2, (3, H, W))
    once = O.clamp(hist, cur, 1.0)
    np.testing.assert_array_equal(O.clamp(once, cur, 1.0), once)
    np.testing.assert_array_equal(O.clamp(hist, cur, 1e12), hist)
    np.testing.assert_array_equal(O.clamp(hist, cur, 0.0), hist)
    const = np.full((3, H, W), 0.375)
    np.testing.assert_array_equal(O.clamp(hist, const, 1.0), const)
    # a history at the box centre stays
    mu = np.stack([corr(cur[c], np.ones((3, 3))) / corr(np.ones((H, W)), np.ones((3, 3)))
                   for c in range(3)])
    np.testing.assert_allclose(O.clamp(mu, cur, 1.0), mu, rtol=1e-15)


# ---- variance colour clipping (Section 3.1) ------------------------------------

def _box(cur, x, y, gamma):
    st = [_box_stats(cur[ch], x, y) for ch in range(3)]
    return np.array([m for m, _ in st]), gamma * np.array([sd for _, sd in st])


def test_clip_is_the_last_point_of_the_segment_inside_the_box():
    # Brute force: bisection over t in [0, 1] for the largest t with
    # mu + t (h - mu) inside the box, against the oracle's closed form.
    H, W = 6, 7
    r = rng(40)
    cur = r.uniform(0, 1, (3, H, W))
    hist = r.uniform(-1, 2, (3, H, W))
    for gamma in (0.5, 1.0, 2.0):
        out = O.clip(hist, cur, gamma)
        for y in range(H):
            for x in range(W):
                mu, half = _box(cur, x, y, gamma)
                d = hist[:, y, x] - mu
                inside = lambda t: np.all(np.abs(t * d) <= half * (1 + 1e-15))
                lo, hi = 0.0, 1.0
                if inside(1.0):
                    lo = 1.0
                else:
                    for _ in range(80):
                        m = 0.5 * (lo + hi)
                        lo, hi = (m, hi) if inside(m) else (lo, m)
                np.testing.assert_allclose(out[:, y, x], mu + lo * d, rtol=1e-12, atol=1e-14)


def test_clip_keeps_the_hue_and_lands_on_the_box():
    H, W = 8, 9
    r = rng(41)
    cur = r.uniform(0, 1, (3, H, W))
    hist = r.uniform(-2, 3, (3, H, W))
    out = O.clip(hist, cur, 1.0)
    for y in range(H):
        for x in range(W):
            mu, half = _box(cur, x, y, 1.0)
            d, o = hist[:, y, x] - mu, out[:, y, x] - mu
            # o is a non-negative multiple of d (same direction from the centre)
            t = np.dot(o, d) / np.dot(d, d)
            assert 0.0 <= t <= 1.0
            np.testing.assert_allclose(o, t * d, atol=1e-14)
            # and sits on the box's surface when h was outside it
            if np.any(np.abs(d) > half):
                assert np.max(np.abs(o) / half) == pytest.approx(1.0, rel=1e-12)
    np.testing.assert_allclose(O.clip(out, cur, 1.0), out, rtol=1e-13, atol=1e-15)


def test_clip_special_cases():
    H, W = 7, 6
    r = rng(42)
    cur = r.uniform(0, 1, (3, H, W))
    hist = r.uniform(-1, 2, (3, H, W))
    # gamma 0 and a huge box copy the history
    np.testing.assert_array_equal(O.clip(hist, cur, 0.0), hist)
    np.testing.assert_array_equal(O.clip(hist, cur, 1e12), hist)
    # a constant current frame (zero spread) sends any other history to it
    const = np.full((3, H, W), 0.375)
    np.testing.assert_array_equal(O.clip(hist, const, 1.0), const)
    # grey current and history: the box is a cube on the grey axis and the
    # segment runs along it, so clipping equals the per-channel clamp
    grey = np.broadcast_to(cur[:1], (3, H, W)).copy()
    hgrey = np.broadcast_to(hist[:1], (3, H, W)).copy()
    np.testing.assert_allclose(O.clip(hgrey, grey, 1.0), O.clamp(hgrey, grey, 1.0), rtol=1e-14)
    # a history off the centre in one channel only: clip == clamp
    mu = np.stack([corr(cur[c], np.ones((3, 3))) / corr(np.ones((H, W)), np.ones((3, 3)))
                   for c in range(3)])
    one = mu.copy()
    one[1] = hist[1]
    np.testing.assert_allclose(O.clip(one, cur, 1.0), O.clamp(one, cur, 1.0), rtol=1e-13)
    # empty centre pixels pass through; empty neighbours leave the box
    z = np.ones((H, W))
    z[3, 2] = 0.0
    z[0, 0] = -1.0
    out = O.clip(hist, cur, 1.0, z=z)
    np.testing.assert_array_equal(out[:, 3, 2], hist[:, 3, 2])
    win = [(yy, xx) for yy in range(2, 5) for xx in range(0, 3) if (yy, xx) != (3, 2)]
    m = np.array([np.mean([cur[c, yy, xx] for yy, xx in win]) for c in range(3)])
    hf = np.array([np.std([cur[c, yy, xx] for yy, xx in win]) for c in range(3)])
    d = hist[:, 3, 1] - m
    t = min([1.0] + [hf[c] / abs(d[c]) for c in range(3) if abs(d[c]) > hf[c]])
    np.testing.assert_allclose(out[:, 3, 1], m + t * d, rtol=1e-13)


def test_temporal_clip_flag_is_reproject_clip_blend():
    from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
    cfg = with_size(CONFIGS["hd_motion"], 40, 24, 3)
    frames = list(sequence(cfg))
    st = O.new_state(24, 40)
    p = O.OracleParams(clip=True, use_id=True)
    for fr in frames[:2]:
        t = O.temporal(fr, st, p)
        st = {"rgb": t["rgb"], "m1": t["m1"], "m2": t["m2"], "n": t["n"]}
    fr = frames[2]
    t = O.temporal(fr, st, p)
    rp = O.reproject(fr["z"], fr["n"], fr["mv"], fr["prev_z"], fr["prev_n"], st["rgb"],
                     st["m1"], st["m2"], st["n"], id=fr["id"], prev_id=fr["prev_id"],
                     use_id=True)
    h = O.clip(rp["rgb"], fr["rgb"], 1.0, z=fr["z"])
    b = O.blend(fr["rgb"], fr["z"], h, rp["m1"], rp["m2"], rp["n"], rp["valid"])
    np.testing.assert_array_equal(t["rgb"], b["rgb"])
    tc = O.temporal(fr, st, O.OracleParams(clamp=True, use_id=True))
    assert np.abs(tc["rgb"] - t["rgb"]).max() > 0  # the two rectifications differ here


# ---- temporal accumulation (Section 2) ----------------------------------------

def test_blend_closed_forms():
    H, W = 4, 5
    r = rng(6)
    cur = r.uniform(0, 1, (3, H, W))
    hist = r.uniform(0, 1, (3, H, W))
    m1, m2 = r.uniform(0, 1, (H, W)), r.uniform(0, 1, (H, W))
    z = np.ones((H, W))
    L = LUMA_W @ cur.reshape(3, -1)
    L = L.reshape(H, W)
    valid = np.ones((H, W), np.int32)
    for hn_val, a in [(10, 0.2), (1, 0.5), (2, 1.0 / 3.0), (254, 0.2)]:
        hn = np.full((H, W), hn_val, np.int32)
        out = O.blend(cur, z, hist, m1, m2, hn, valid, alpha=0.2, alpha_m=0.2)
        np.testing.assert_allclose(out["rgb"], (1 - a) * hist + a * cur, rtol=1e-14)
        np.testing.assert_allclose(out["m1"], (1 - a) * m1 + a * L, rtol=1e-14)
        np.testing.assert_allclose(out["m2"], (1 - a) * m2 + a * L * L, rtol=1e-14)
        assert np.all(out["n"] == min(hn_val + 1, 255))
    out = O.blend(cur, z, hist, m1, m2, np.full((H, W), 254, np.int32), valid, max_hist=255)
    assert np.all(out["n"] == 255)
    out = O.blend(cur, z, hist, m1, m2, np.full((H, W), 255, np.int32), valid, max_hist=255)
    assert np.all(out["n"] == 255)
    out = O.blend(cur, z, hist, m1, m2, np.full((H, W), 9, np.int32), np.zeros((H, W), np.int32))
    np.testing.assert_array_equal(out["rgb"], cur)
    np.testing.assert_allclose(out["m1"], L, rtol=1e-15)
    np.testing.assert_allclose(out["m2"], L * L, rtol=1e-15)
    assert np.all(out["n"] == 1)


def _static_frames(H, W, N, seed):
    r = rng(seed)
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    frames = []
    for _ in range(N):
        frames.append(dict(rgb=r.exponential(1.0, (3, H, W)), z=z, dzdx=dzdx, dzdy=dzdy,
                           n=n, mv=np.zeros((2, H, W)), prev_z=z, prev_n=n,
                           id=None, prev_id=None))
    return frames


def test_static_accumulation_with_alpha_zero_is_the_sample_mean():
    H, W, N = 12, 9, 8
    frames = _static_frames(H, W, N, 7)
    p = O.OracleParams(alpha=0.0, alpha_m=0.0, levels=0, feedback="temporal")
    st = O.new_state(H, W)
    for k, fr in enumerate(frames, start=1):
        _, st, ex = O.run_frame(fr, st, p)
        samples = np.stack([f["rgb"] for f in frames[:k]])
        Ls = np.einsum("c,kchw->khw", LUMA_W, samples)
        np.testing.assert_allclose(ex["temporal"]["rgb"], samples.mean(0), rtol=1e-12)
        np.testing.assert_allclose(ex["temporal"]["m1"], Ls.mean(0), rtol=1e-12)
        np.testing.assert_allclose(ex["temporal"]["m2"], (Ls ** 2).mean(0), rtol=1e-12)
        assert np.all(ex["temporal"]["n"] == k)
        if k >= 4:  # temporal variance = population variance of the samples
            np.testing.assert_allclose(ex["var"], Ls.var(0, ddof=0), rtol=1e-9, atol=1e-13)


def test_static_accumulation_alpha_schedule_mean_then_ema():
    H, W, N, a = 6, 7, 12, 0.2
    frames = _static_frames(H, W, N, 8)
    p = O.OracleParams(alpha=a, alpha_m=a, levels=0, feedback="temporal")
    st = O.new_state(H, W)
    xs = np.stack([f["rgb"] for f in frames])
    for k, fr in enumerate(frames, start=1):
        _, st, ex = O.run_frame(fr, st, p)
        if k <= 5:
            expect = xs[:k].mean(0)
        else:  # (1-a)^(k-5) * mean(x1..x5) + sum_j a (1-a)^(k-j) x_j
            expect = (1 - a) ** (k - 5) * xs[:5].mean(0)
            for j in range(6, k + 1):
                expect = expect + a * (1 - a) ** (k - j) * xs[j - 1]
        np.testing.assert_allclose(ex["temporal"]["rgb"], expect, rtol=1e-12)


def test_static_accumulation_ema_variance_ratio():
    # For i.i.d. samples an EMA with weight a has variance a / (2 - a) of
    # theirs (0.1111 for a = 0.2), once the start-up has decayed.
    H, W, N, a = 256, 256, 60, 0.2
    r = rng(9)
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    p = O.OracleParams(alpha=a, alpha_m=a, levels=0, feedback="temporal")
    st = O.new_state(H, W)
    for _ in range(N):
        fr = dict(rgb=np.broadcast_to(r.exponential(1.0, (1, H, W)), (3, H, W)), z=z,
                  dzdx=dzdx, dzdy=dzdy, n=n, mv=np.zeros((2, H, W)), prev_z=z,
                  prev_n=n, id=None, prev_id=None)
        _, st, ex = O.run_frame(fr, st, p)
    ratio = ex["temporal"]["rgb"][0].var() / 1.0  # Var[Exp(1)] = 1
    assert ratio == pytest.approx(a / (2 - a), rel=0.05)


# ---- variance estimate (Section 2) ----------------------------------------------

def test_variance_long_history_is_m2_minus_m1_squared():
    H, W = 5, 6
    r = rng(10)
    m1 = r.uniform(0, 1, (H, W))
    m2 = m1 ** 2 + r.uniform(-0.1, 0.3, (H, W))
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    hn = np.full((H, W), 4, np.int32)
    v = O.variance(m1, m2, hn, z, dzdx, dzdy, n)
    np.testing.assert_allclose(v, np.maximum(0.0, m2 - m1 ** 2), rtol=1e-15, atol=0)


def test_variance_short_history_unit_weights_is_window_variance():
    H, W = 9, 11
    r = rng(11)
    m1 = r.uniform(0, 1, (H, W))
    extra = 0.05
    m2 = m1 ** 2 + extra
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    hn = np.full((H, W), 2, np.int32)
    v = O.variance(m1, m2, hn, z, dzdx, dzdy, n)
    for y in range(H):
        for x in range(W):
            win = m1[max(0, y - 3):y + 4, max(0, x - 3):x + 4]
            assert v[y, x] == pytest.approx(win.var(ddof=0) + extra, rel=1e-12)


def test_variance_short_history_depth_and_normal_cuts():
    H, W = 8, 10
    r = rng(12)
    m1 = r.uniform(0, 1, (H, W))
    m2 = m1 ** 2
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    hn = np.ones((H, W), np.int32)
    zc = z.copy()
    zc[:, 5:] = 50.0  # depth step between columns 4 and 5
    v = O.variance(m1, m2, hn, zc, dzdx, dzdy, n)
    nc = n.copy()
    nc[:, :, 5:] = np.array([1.0, 0.0, 0.0])[:, None, None]  # perpendicular normals
    v2 = O.variance(m1, m2, hn, z, dzdx, dzdy, nc)
    for y in range(H):
        for x in range(W):
            lo, hi = (max(0, x - 3), min(x + 4, 5)) if x < 5 else (max(5, x - 3), x + 4)
            win = m1[max(0, y - 3):y + 4, lo:hi]
            assert v[y, x] == pytest.approx(win.var(), rel=1e-12, abs=1e-15)
            assert v2[y, x] == pytest.approx(win.var(), rel=1e-12, abs=1e-15)


def test_variance_short_history_weight_values():
    # Affine depth whose gradient matches the G-buffer: every neighbour's
    # depth weight is exp(-1/sigma_z).  Normals at a cosine of 0.5 on odd
    # columns: with sigma_n = 1 their normal weight is 0.5.
    H, W = 9, 9
    r = rng(13)
    m1 = r.uniform(0, 1, (H, W))
    m2 = m1 ** 2
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    gx, gy = 0.37, -0.21
    z = 20.0 + gx * xs + gy * ys
    n = np.zeros((3, H, W))
    n[1] = 1.0
    odd = (xs.astype(int) % 2) == 1
    n[:, odd] = np.array([math.sqrt(0.75), 0.5, 0.0])[:, None]
    hn = np.ones((H, W), np.int32)
    for sigma_z in (1.0, 2.0):
        v = O.variance(m1, m2, hn, z, np.full((H, W), gx), np.full((H, W), gy), n,
                       sigma_z=sigma_z, sigma_n=1.0, eps_z=0.0)
        e = math.exp(-1.0 / sigma_z)
        y, x = 4, 4  # even column: same normal as the even columns
        w = np.where(odd, 0.5, 1.0) * e
        w[y, x] = 1.0
        win_w = w[y - 3:y + 4, x - 3:x + 4]
        win = m1[y - 3:y + 4, x - 3:x + 4]
        mean = np.average(win, weights=win_w)
        assert v[y, x] == pytest.approx(np.average((win - mean) ** 2, weights=win_w), rel=1e-10)


# ---- a-trous level (Section 2, Fig. 1) -------------------------------------------

@pytest.mark.parametrize("shape", [(23, 37), (50, 70)])
@pytest.mark.parametrize("step", [1, 2, 4, 8, 16])
def test_atrous_unit_weights_is_dilated_b3_correlation(shape, step):
    H, W = shape
    r = rng(14 + step)
    c = r.uniform(0, 1, (3, H, W))
    var = r.uniform(0, 1, (H, W))
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    out, vo = O.atrous(c, var, z, dzdx, dzdy, n, step, unit_weights=True)
    K = kernel2d(step)
    norm = corr(np.ones((H, W)), K)
    for ch in range(3):
        np.testing.assert_allclose(out[ch], corr(c[ch], K) / norm, rtol=1e-13)
    np.testing.assert_allclose(vo, corr(var, K * K) / norm ** 2, rtol=1e-13)


def test_atrous_five_unit_levels_is_cascaded_b3_on_a_delta():
    # the support reaches 62 pixels and level 4 reads 32 beyond it: a 200
    # pixel image keeps every tap of every non-zero pixel inside
    H = W = 200
    c = np.zeros((3, H, W))
    c[:, 100, 100] = 1.0
    v = np.zeros((H, W))
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    for i in range(5):
        c, v = O.atrous(c, v, z, dzdx, dzdy, n, 1 << i, unit_weights=True)
    h = np.array([1.0])
    for i in range(5):
        h = np.convolve(h, dilated_b3(1 << i))
    R = len(h) // 2  # 62
    expect = np.outer(h, h)
    np.testing.assert_allclose(c[0, 100 - R:100 + R + 1, 100 - R:100 + R + 1], expect,
                               rtol=1e-12, atol=1e-18)


def test_atrous_constant_variance_unit_weights_closed_form():
    H, W = 40, 40
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    c = np.ones((3, H, W))
    V = 2.5
    _, vo = O.atrous(c, np.full((H, W), V), z, dzdx, dzdy, n, 1, unit_weights=True)
    assert vo[20, 20] == pytest.approx(V * (35.0 / 128.0) ** 2, rel=1e-14)
    assert (35.0 / 128.0) ** 2 == 0.07476806640625


def test_atrous_constant_image_is_a_fixed_point():
    H, W = 31, 29
    r = rng(15)
    c = np.ones((3, H, W)) * np.array([0.3, 0.6, 0.2])[:, None, None]
    var = r.uniform(0, 1, (H, W))
    z = r.uniform(5, 10, (H, W))
    dzdx, dzdy = r.normal(0, 0.1, (H, W)), r.normal(0, 0.1, (H, W))
    n = r.normal(0, 1, (3, H, W))
    n /= np.linalg.norm(n, axis=0)
    for step in (1, 4, 16):
        out, _ = O.atrous(c, var, z, dzdx, dzdy, n, step)
        np.testing.assert_allclose(out, c, rtol=1e-14)
        out, _, _ = O.atrous_sep(c, var, z, dzdx, dzdy, n, step)
        np.testing.assert_allclose(out, c, rtol=1e-14)


def test_atrous_depth_weight_on_affine_depth():
    # z = z0 + gx x + gy y with matching gradients: |z(p) - z(q)| equals
    # |grad . offset|, so every tap but the centre has weight exp(-1/sigma_z).
    H, W = 30, 34
    r = rng(16)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    gx, gy = 0.31, 0.113  # no tap offset is orthogonal to the gradient
    z = 40.0 + gx * xs + gy * ys
    c = equal_luma_rgb(r, H, W)
    n = flat_gbuf(H, W)[3]
    V = 0.7
    var = np.full((H, W), V)
    for step, sigma_z in [(1, 1.0), (2, 1.0), (4, 0.5), (1, 3.0)]:
        out, vo = O.atrous(c, var, z, np.full((H, W), gx), np.full((H, W), gy), n, step,
                           sigma_z=sigma_z, eps_z=0.0)
        e = math.exp(-1.0 / sigma_z)
        K = kernel2d(step)
        h00 = K[2 * step, 2 * step]
        den = e * corr(np.ones((H, W)), K) + (1 - e) * h00
        for ch in range(3):
            num = e * corr(c[ch], K) + (1 - e) * h00 * c[ch]
            np.testing.assert_allclose(out[ch], num / den, rtol=1e-12)
        vnum = e * e * corr(var, K * K) + (1 - e * e) * h00 ** 2 * var
        np.testing.assert_allclose(vo, vnum / den ** 2, rtol=1e-12)


def test_atrous_normal_weight_power_and_clamp():
    # Odd columns carry a normal at cosine d to the even columns' normal.
    H, W = 21, 24
    r = rng(17)
    c = equal_luma_rgb(r, H, W)
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    odd = (np.arange(W) % 2 == 1)[None, :] * np.ones((H, 1), bool)
    for d, sigma_n, w_other in [(0.5, 1.0, 0.5), (0.5, 3.0, 0.125), (-0.5, 1.0, 0.0)]:
        nn = n.copy()
        nn[:, odd] = np.array([math.sqrt(1 - d * d), d, 0.0])[:, None]
        out, _ = O.atrous(c, np.ones((H, W)), z, dzdx, dzdy, nn, 1, sigma_n=sigma_n)
        K = kernel2d(1)
        same = (~odd).astype(float)
        other = odd.astype(float)
        for ch in range(3):
            num = corr(c[ch] * same, K) + w_other * corr(c[ch] * other, K)
            den = corr(same, K) + w_other * corr(other, K)
            np.testing.assert_allclose(out[ch][~odd], (num / den)[~odd], rtol=1e-12)


@pytest.mark.parametrize("theta,eps_a,eps_b", [(0.05, 1e-3, -2e-3), (0.12, -1e-3, -1e-3),
                                             (0.02, 3e-3, 1e-3)])
def test_atrous_normal_weight_of_non_unit_normals_follows_the_angle(theta, eps_a, eps_b):
    """Reading R13: the cosine in (n_p . n_q)^sigma_n is taken as
    1 - |n_p - n_q|^2 / 2.  For normals of lengths 1 + ea, 1 + eb at angle
    theta that is, exactly,
        cos t + (ea + eb)(cos t - 1) + ea eb cos t - (ea^2 + eb^2) / 2,
    so the weight is cos(theta)^sigma_n up to a relative
    sigma_n (|ea| + |eb|)(1 - cos t) / cos t plus second order: a function
    of the angle alone where the weights matter, while the plain dot
    product (|n_p||n_q| cos t) is off by sigma_n (ea + eb) at every angle.
    Lengths off by 1e-3 make the two readings far apart in FP64."""
    H, W = 9, 10
    sigma_n = 128.0
    r = rng(23)
    c = equal_luma_rgb(r, H, W)
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    odd = (np.arange(W) % 2 == 1)[None, :] * np.ones((H, 1), bool)
    ua = np.array([0.3, 0.9, 0.1])
    ua /= np.linalg.norm(ua)
    perp = np.cross(ua, [0.0, 0.0, 1.0])
    perp /= np.linalg.norm(perp)
    ub = math.cos(theta) * ua + math.sin(theta) * perp
    a, b = (1 + eps_a) * ua, (1 + eps_b) * ub
    nn = n.copy()
    nn[:, ~odd] = a[:, None]
    nn[:, odd] = b[:, None]
    ct = math.cos(theta)
    chord = ct + (eps_a + eps_b) * (ct - 1) + eps_a * eps_b * ct - (eps_a ** 2 + eps_b ** 2) / 2
    w_other = chord ** sigma_n
    out, _ = O.atrous(c, np.ones((H, W)), z, dzdx, dzdy, nn, 1, sigma_n=sigma_n)
    K = kernel2d(1)
    same, other = (~odd).astype(float), odd.astype(float)
    for ch in range(3):
        num = corr(c[ch] * same, K) + w_other * corr(c[ch] * other, K)
        den = corr(same, K) + w_other * corr(other, K)
        np.testing.assert_allclose(out[ch][~odd], (num / den)[~odd], rtol=1e-11)
    # the weight follows the angle to first order in the length error ...
    first = sigma_n * (abs(eps_a) + abs(eps_b)) * (1 - ct) / ct
    second = sigma_n * 2 * max(abs(eps_a), abs(eps_b)) ** 2
    assert abs(w_other / ct ** sigma_n - 1) <= 1.05 * first + second
    # ... where the plain dot product does not
    dot = float(a @ b) ** sigma_n
    assert abs(dot / ct ** sigma_n - 1) > 10 * (first + second)


def test_atrous_luminance_weight_worked_example():
    with open(os.path.join(GOLDEN, "atrous_luma_example.json")) as f:
        gold = json.load(f)
    for case in gold["cases"]:
        grey = np.array(case["grey"], dtype=np.float64)[None, :]
        W = grey.shape[1]
        c = np.stack([grey, grey, grey])
        var = np.array(case["var"], dtype=np.float64)[None, :]
        z, dzdx, dzdy, n = flat_gbuf(1, W)
        out, _ = O.atrous(c, var, z, dzdx, dzdy, n, 1, sigma_l=case["sigma_l"], eps_l=0.0)
        assert out[0, 0, case["x"]] == pytest.approx(case["expect"], rel=1e-12)


def test_atrous_luminance_scale_invariance_and_kappa():
    # Colour x t and variance x t^2 leave the luminance weight unchanged.
    H, W = 25, 27
    r = rng(18)
    c = r.uniform(0.1, 1.0, (3, H, W))
    var = r.uniform(0.01, 0.2, (H, W))
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    out1, v1 = O.atrous(c, var, z, dzdx, dzdy, n, 2, eps_l=0.0)
    out2, v2 = O.atrous(3.0 * c, 9.0 * var, z, dzdx, dzdy, n, 2, eps_l=0.0)
    np.testing.assert_allclose(out2, 3.0 * out1, rtol=1e-12)
    np.testing.assert_allclose(v2, 9.0 * v1, rtol=1e-12)
    # kappa scales sigma_l per pixel
    outk, _ = O.atrous(c, var, z, dzdx, dzdy, n, 2, kappa=np.full((H, W), 2.0))
    out8, _ = O.atrous(c, var, z, dzdx, dzdy, n, 2, sigma_l=8.0)
    np.testing.assert_allclose(outk, out8, rtol=1e-14)
    # an infinite sigma_l turns the luminance weight off: unit result
    outi, _ = O.atrous(c, var, z, dzdx, dzdy, n, 2, sigma_l=1e300)
    K = kernel2d(2)
    for ch in range(3):
        np.testing.assert_allclose(outi[ch], corr(c[ch], K) / corr(np.ones((H, W)), K), rtol=1e-12)


def test_atrous_translation_equivariance_and_inverse_tonemap():
    H, W = 60, 64
    r = rng(19)
    c = r.uniform(0.1, 1.0, (3, H, W))
    var = r.uniform(0.01, 0.2, (H, W))
    z = r.uniform(5, 6, (H, W))
    dzdx, dzdy = r.normal(0, 0.05, (H, W)), r.normal(0, 0.05, (H, W))
    n = r.normal(0, 0.05, (3, H, W)) + np.array([0, 1.0, 0])[:, None, None]
    n /= np.linalg.norm(n, axis=0)
    out, vo = O.atrous(c, var, z, dzdx, dzdy, n, 2)
    sh = lambda a: np.roll(a, (3, -5), axis=(-2, -1))
    out_s, vo_s = O.atrous(sh(c), sh(var), sh(z), sh(dzdx), sh(dzdy), sh(n), 2)
    inner = (slice(12, H - 12), slice(12, W - 12))
    np.testing.assert_allclose(out_s[(slice(None),) + inner], sh(out)[(slice(None),) + inner], rtol=1e-13)
    np.testing.assert_allclose(vo_s[inner], sh(vo)[inner], rtol=1e-13)
    inv, _ = O.atrous(c, var, z, dzdx, dzdy, n, 2, inv_tonemap=True)
    np.testing.assert_allclose(inv, O.tonemap(out, inverse=True), rtol=1e-14)


def test_atrous_empty_pixels_pass_through_and_are_skipped():
    H, W = 15, 17
    r = rng(20)
    c = r.uniform(0, 1, (3, H, W))
    var = r.uniform(0, 1, (H, W))
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    z = z.copy()
    hole = r.random((H, W)) < 0.2
    z[hole] = 0.0
    out, vo = O.atrous(c, var, z, dzdx, dzdy, n, 1, unit_weights=True)
    np.testing.assert_array_equal(out[:, hole], c[:, hole])
    assert np.all(vo[hole] == 0.0)
    K = kernel2d(1)
    m = (~hole).astype(float)
    for ch in range(3):
        ref = corr(c[ch] * m, K) / corr(m, K)
        np.testing.assert_allclose(out[ch][~hole], ref[~hole], rtol=1e-13)


# ---- separable level (Section 3.3) --------------------------------------------

@pytest.mark.parametrize("step", [1, 2, 4, 8, 16])
def test_separable_unit_weights_equals_2d_colour_and_1d_variance(step):
    H, W = 40, 45
    r = rng(21 + step)
    c = r.uniform(0, 1, (3, H, W))
    var = r.uniform(0, 1, (H, W))
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    out, vo, _ = O.atrous_sep(c, var, z, dzdx, dzdy, n, step, unit_weights=True)
    out2, _ = O.atrous(c, var, z, dzdx, dzdy, n, step, unit_weights=True)
    np.testing.assert_allclose(out, out2, rtol=1e-13)
    k = dilated_b3(step)[:, None]  # vertical taps only
    norm = corr(np.ones((H, W)), k)
    np.testing.assert_allclose(vo, corr(var, k * k) / norm ** 2, rtol=1e-13)
    if H > 4 * step + 4:
        y = H // 2
        _, vc, _ = O.atrous_sep(c, np.full((H, W), 1.0), z, dzdx, dzdy, n, step, unit_weights=True)
        assert vc[y, W // 2] == pytest.approx(35.0 / 128.0, rel=1e-14)


def test_separable_variance_updated_only_in_vertical_pass():
    # Colour varies along x only: the horizontal pass has non-trivial
    # luminance weights, the vertical pass sees equal luminances (weight 1),
    # so the output variance is the plain vertical B3 propagation.
    H, W = 30, 36
    r = rng(27)
    row = r.uniform(0.1, 1.0, (3, 1, W))
    c = np.broadcast_to(row, (3, H, W)).copy()
    # variance varies along x only, so a horizontal mix of it would show
    var = np.broadcast_to(r.uniform(0.01, 0.05, (1, W)), (H, W)).copy()
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    for step in (1, 2):
        out, vo, sh = O.atrous_sep(c, var, z, dzdx, dzdy, n, step)
        k = dilated_b3(step)[:, None]
        norm = corr(np.ones((H, W)), k)
        np.testing.assert_allclose(vo, corr(var, k * k) / norm ** 2, rtol=1e-12)
        # the horizontal pass did filter the colour
        assert np.max(np.abs(sh - c)) > 1e-3
        # and the vertical pass kept it (equal values along y)
        np.testing.assert_allclose(out, sh, rtol=1e-13)


def test_separable_equals_2d_on_images_constant_along_one_axis():
    H, W = 28, 33
    r = rng(28)
    z, dzdx, dzdy, n = flat_gbuf(H, W)
    var = np.full((H, W), 0.03)
    row = r.uniform(0.1, 1.0, (3, 1, W))
    c = np.broadcast_to(row, (3, H, W)).copy()
    a, _, _ = O.atrous_sep(c, var, z, dzdx, dzdy, n, 2)
    b, _ = O.atrous(c, var, z, dzdx, dzdy, n, 2)
    np.testing.assert_allclose(a, b, rtol=1e-12)
    col = r.uniform(0.1, 1.0, (3, H, 1))
    c = np.broadcast_to(col, (3, H, W)).copy()
    a, _, _ = O.atrous_sep(c, var, z, dzdx, dzdy, n, 2)
    b, _ = O.atrous(c, var, z, dzdx, dzdy, n, 2)
    np.testing.assert_allclose(a, b, rtol=1e-12)


# ---- the whole chain -------------------------------------------------------------

def test_chain_constant_image_is_reproduced_under_motion():
    from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
    cfg = with_size(CONFIGS["hd_motion"], 96, 64, 5)
    p = O.OracleParams(clamp=True, tonemap=True, use_id=True)
    st = O.new_state(64, 96)
    c0 = np.array([0.8, 0.4, 1.7])
    for fr in sequence(cfg):
        fr = dict(fr)
        fr["rgb"] = np.broadcast_to(c0[:, None, None], (3, 64, 96)).copy()
        out, st, _ = O.run_frame(fr, st, p)
        np.testing.assert_allclose(out, fr["rgb"], rtol=1e-12)
    for sep in (True,):
        p2 = O.OracleParams(clamp=True, tonemap=True, separable=sep)
        out, _, _ = O.run_frame(fr, st, p2)
        np.testing.assert_allclose(out, fr["rgb"], rtol=1e-12)


# ---- blur adapted to scene features (Sections 3.2, 3.5) ---------------------------

def test_blur_control_follows_the_papers_thresholds():
    with open(os.path.join(GOLDEN, "blur_rule_paper.json")) as f:
        gold = json.load(f)
    f32 = np.float32
    up = lambda v: np.nextafter(f32(v), f32(np.inf))
    rs, an = gold["rough_shift"], gold["angle_shift"]
    t0, t1 = gold["table"][0]["rough_max"], gold["table"][1]["rough_max"]
    rough = np.array([-1.0, t0, up(t0), t1, up(t1), rs, up(rs), 1.0, np.nan], f32)[None, :]
    full = gold["full_cascade"]
    ctl = O.blur_control(rough, None, rough_shift=rs, rough_none=t0, rough_one=t1,
                         it_none=gold["table"][0]["iterations"],
                         it_one=gold["table"][1]["iterations"], it_rest=full)
    np.testing.assert_array_equal(ctl[0] & 15, [0, 0, 1, 1, full, full, full, full, full])
    np.testing.assert_array_equal(ctl[0] >> 4, [0, 0, 0, 0, 0, 0, 1, 1, 0])
    # the shadow angle alone
    ang = np.array([0.0, an, up(an), 90.0], f32)[None, :]
    ctl = O.blur_control(None, ang, angle_shift=an, table=False)
    np.testing.assert_array_equal(ctl[0], [15, 15, 16 + 15, 16 + 15])
    # either one shifts
    ctl = O.blur_control(np.array([[0.5, 0.1, 0.1]], f32), np.array([[0.0, 7.0, 1.0]], f32),
                         table=False)
    np.testing.assert_array_equal(ctl[0], [31, 31, 15])


def _adaptive_case(H=23, W=29, seed=50):
    r = rng(seed)
    c = r.uniform(0.1, 1.5, (3, H, W))
    var = r.uniform(0.0, 0.3, (H, W))
    z = 5.0 + 0.1 * r.standard_normal((H, W))
    dzdx = 0.01 * r.standard_normal((H, W))
    dzdy = 0.01 * r.standard_normal((H, W))
    n = r.standard_normal((3, H, W)) * 0.1
    n[2] += 1.0
    n /= np.linalg.norm(n, axis=0)
    return c, var, z, dzdx, dzdy, n


@pytest.mark.parametrize("sep", [False, True])
def test_adaptive_level_special_cases(sep):
    c, var, z, dzdx, dzdy, n = _adaptive_case()
    fn = O.atrous_sep if sep else O.atrous
    H, W = z.shape
    for level in (0, 1, 2):
        plain = fn(c, var, z, dzdx, dzdy, n, 1 << level)
        coarse = fn(c, var, z, dzdx, dzdy, n, 2 << level)
        every = np.full((H, W), 15, np.uint8)
        out = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, every, level, separable=sep)
        np.testing.assert_array_equal(out[0], plain[0])
        np.testing.assert_array_equal(out[1], plain[1])
        out = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, every | 16, level, separable=sep)
        np.testing.assert_array_equal(out[0], coarse[0])
        np.testing.assert_array_equal(out[1], coarse[1])
        # a spent budget keeps colour and variance
        spent = np.full((H, W), level, np.uint8) | 16
        out = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, spent, level, separable=sep)
        np.testing.assert_array_equal(out[0], c)
        np.testing.assert_array_equal(out[1], var)
        out = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, spent, level, separable=sep,
                                inv_tonemap=True, want_var=False)
        np.testing.assert_allclose(out[0], O.tonemap(c, inverse=True), rtol=1e-15)
    # Section 3.2: a shifted pixel's first iteration is the usual second one
    lvl1 = fn(c, var, z, dzdx, dzdy, n, 2)
    first = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, np.full((H, W), 31, np.uint8), 0,
                              separable=sep)
    np.testing.assert_array_equal(first[0], lvl1[0])


@pytest.mark.parametrize("sep", [False, True])
def test_adaptive_level_is_local_in_the_control_bytes(sep):
    # the output at p depends on ctl(p) alone (the level input is fixed)
    c, var, z, dzdx, dzdy, n = _adaptive_case(seed=51)
    H, W = z.shape
    r = rng(52)
    a = r.integers(0, 32, (H, W)).astype(np.uint8)
    b = r.integers(0, 32, (H, W)).astype(np.uint8)
    same = r.random((H, W)) < 0.5
    b[same] = a[same]
    oa = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, a, 1, separable=sep)
    ob = O.atrous_adaptive(c, var, z, dzdx, dzdy, n, b, 1, separable=sep)
    np.testing.assert_array_equal(oa[0][:, same], ob[0][:, same])
    np.testing.assert_array_equal(oa[1][same], ob[1][same])
    # and each class of pixel matches its own whole-image filter
    fn = O.atrous_sep if sep else O.atrous
    fine, coarse = fn(c, var, z, dzdx, dzdy, n, 2), fn(c, var, z, dzdx, dzdy, n, 4)
    kept = (a & 15) <= 1
    sh = ((a & 16) != 0) & ~kept
    fi = ~kept & ~sh
    np.testing.assert_array_equal(oa[0][:, kept], c[:, kept])
    np.testing.assert_array_equal(oa[0][:, sh], coarse[0][:, sh])
    np.testing.assert_array_equal(oa[0][:, fi], fine[0][:, fi])


def test_adaptive_cascade_with_the_papers_count_equals_every_level():
    # a count of 4 in a 4-level cascade is the same as no limit
    from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
    cfg = with_size(CONFIGS["hd_motion"], 48, 32, 2)
    fr = next(iter(sequence(cfg)))
    p = O.OracleParams(clamp=True, tonemap=True, use_id=True, levels=4)
    st = O.new_state(32, 48)
    plain, _, _ = O.run_frame(fr, st, p)
    four, _, _ = O.run_frame(fr, st, p, ctl=np.full((32, 48), 4, np.uint8))
    every, _, _ = O.run_frame(fr, st, p, ctl=np.full((32, 48), 15, np.uint8))
    np.testing.assert_array_equal(four, plain)
    np.testing.assert_array_equal(every, plain)
    one, _, ex = O.run_frame(fr, st, p, ctl=np.full((32, 48), 1, np.uint8))
    np.testing.assert_allclose(one, O.tonemap(ex["levels"][0], inverse=True), rtol=1e-15)


# ---- composition of the channels (Section 3, step 7) --------------------------------

def test_compose_closed_forms():
    r = rng(60)
    direct = r.uniform(0, 1, (3, 4, 5))
    vis = r.uniform(0, 1, (3, 4, 5))
    spec = r.uniform(0, 2, (3, 4, 5))
    np.testing.assert_array_equal(O.compose(direct), direct)
    np.testing.assert_array_equal(O.compose(direct, np.ones_like(vis)), direct)
    np.testing.assert_array_equal(O.compose(direct, np.zeros_like(vis), spec), spec)
    # a hand-worked pixel: 0.5 * 0.25 + 0.125
    d = np.full((3, 1, 1), 0.5)
    assert O.compose(d, np.full((3, 1, 1), 0.25), np.full((3, 1, 1), 0.125))[0, 0, 0] == 0.25
    np.testing.assert_allclose(O.compose(direct, vis, spec), direct * vis + spec, rtol=1e-15)


def test_two_channel_chain_reproduces_constant_channels():
    # constant visibility (no tone map) and constant specular light (tone
    # mapped) with valid history: each channel is reproduced, so the
    # composite is direct * v + s exactly where the chain invariant holds
    from dataclasses import replace
    from paper_2312_06827_amd.scene import CONFIGS, sequence, with_size
    cfg = replace(with_size(CONFIGS["hd_motion"], 64, 40, 4), channels=True)
    ps = O.OracleParams(clamp=True, use_id=True, levels=4)
    pr = O.OracleParams(clamp=True, tonemap=True, use_id=True, levels=4)
    ss, sp = O.new_state(40, 64), O.new_state(40, 64)
    v, c = 0.625, np.array([0.3, 0.2, 0.45])
    for fr in sequence(cfg):
        fs, fp = dict(fr), dict(fr)
        fs["rgb"] = np.full((3, 40, 64), v)
        fp["rgb"] = np.broadcast_to(c[:, None, None], (3, 40, 64)).copy()
        os_, ss, _ = O.run_frame(fs, ss, ps, ctl=O.blur_control(None, fr["shadow_angle"],
                                                                   table=False))
        op, sp, _ = O.run_frame(fp, sp, pr, ctl=O.blur_control(fr["roughness"]))
        out = O.compose(fr["direct"], os_, op)
        np.testing.assert_allclose(out, fr["direct"].astype(np.float64) * v + c[:, None, None],
                                   rtol=1e-12)
