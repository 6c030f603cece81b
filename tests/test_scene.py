"""Checks of the seeded input generator (CPU only).

The generator stands in for the paper's renderer (one sample per pixel,
Section 2), so every parity and quality figure rests on it: it must be
deterministic per seed, its noisy estimate must be unbiased, its backward
motion vectors must lead to the surface point the previous frame saw, and
the plane must fill every frame of every workload (no pixel without a
surface, which the filter treats specially).
"""

import math

import numpy as np
import pytest

from paper_2312_06827_amd import scene as S
from paper_2312_06827_amd.scene import CONFIGS, batched_configs, sequence, with_size


def _frames(cfg, start=0, count=None):
    return list(sequence(cfg, start, count))


def test_bytewise_deterministic_per_seed():
    cfg = with_size(CONFIGS["hd_motion"], 64, 40, 3)
    ch = S.SceneConfig(48, 32, 3, seed=7, channels=True)
    for c in (cfg, ch):
        a, b = _frames(c), _frames(c)
        for fa, fb in zip(a, b):
            assert fa.keys() == fb.keys()
            for k in fa:
                assert fa[k].dtype == fb[k].dtype and fa[k].tobytes() == fb[k].tobytes(), k
    # random access renders the same frame as the sequence
    fr = S.render_frame(cfg, 2)
    seq = _frames(cfg)
    for k in fr:
        assert fr[k].tobytes() == seq[2][k].tobytes(), k
    # another seed is another scene
    other = _frames(with_size(S.SceneConfig(64, 40, 3, seed=3), 64, 40, 3))
    assert other[0]["z"].tobytes() != seq[0]["z"].tobytes()
    assert other[0]["rgb"].tobytes() != seq[0]["rgb"].tobytes()


def test_noise_is_unbiased():
    """E[noisy] = clean: per pixel the estimate is clean * E * F / E[F] with
    E ~ Exp(1) per channel and F the firefly gain.  Over 65,536 lit pixels
    the mean ratio noisy / clean is within 3 standard errors of 1; the
    literal model (no division by E[F] = 1.245) would sit 24 standard
    errors away."""
    cfg = with_size(CONFIGS["small_static"], 256, 256, 1)
    fr = _frames(cfg)[0]
    clean = fr["clean"].astype(np.float64)
    noisy = fr["rgb"].astype(np.float64)
    lit = clean.min(0) > 1e-3
    ratio = (noisy[:, lit] / clean[:, lit]).mean(0)  # channels share F
    n = ratio.size
    assert n > 40000
    m, se = ratio.mean(), ratio.std(ddof=1) / math.sqrt(n)
    assert abs(m - 1.0) <= 3 * se, (m, se)
    assert abs(m * S._NOISE_NORM - 1.0) > 10 * se
    # fireflies: 0.5 % of the pixels, the three channels scaled together.
    # A firefly's channel-mean ratio is 50 / 1.245 times a Gamma(3, 1/3)
    # draw, above 8 with probability 0.977; without one it is beyond 8 with
    # probability below 1e-10.  Expected 0.00489, 3 sigma 0.0009.
    frac = float((ratio > 8).mean())
    assert 0.0038 < frac < 0.0060, frac


def _cast(scene, frame, px, py):
    """Independent ray cast through the (continuous) pixel position
    (px, py) of `frame`: returns (view depth, world normal, object id) of
    the nearest hit, or None."""
    C, fwd, right, up = scene.camera(frame)
    W, H, f = scene.cfg.width, scene.cfg.height, scene.f
    d = fwd + (px + 0.5 - W / 2.0) / f * right - (py + 0.5 - H / 2.0) / f * up
    best = (math.inf, None, None)
    if d[1] < 0:
        t = -C[1] / d[1]
        best = (t, np.array([0.0, 1.0, 0.0]), 0)
    for i, ctr in enumerate(scene.centers(frame)):
        oc = C - ctr
        a = d @ d
        b = 2 * (oc @ d)
        c = oc @ oc - scene.radius[i] ** 2
        disc = b * b - 4 * a * c
        if disc <= 0:
            continue
        t = (-b - math.sqrt(disc)) / (2 * a)
        if 1e-6 < t < best[0]:
            X = C + t * d
            best = (t, (X - ctr) / scene.radius[i], i + 1)
    return None if best[1] is None else best


def test_motion_vectors_lead_to_the_previous_frames_hit_point():
    """For every pixel p of frame f, the previous frame re-cast through the
    continuous position p + mv(p) sees the same surface point (moved back
    with its object): same object, depth equal to the point's depth in the
    previous camera and the same normal, to 1e-4.  Only disocclusions (the
    point hidden in the previous frame) may hit another object."""
    cfg = with_size(CONFIGS["hd_motion"], 96, 54, 4)
    scene = S._Scene(cfg)
    fr = _frames(cfg, 3, 1)[0]
    H, W = cfg.height, cfg.width
    gb = scene.gbuffer(3)
    mv = fr["mv"].astype(np.float64)
    Cp, fwdp, _, _ = scene.camera(2)
    checked = occluded = 0
    moving_obj = 0
    for y in range(0, H, 2):
        for x in range(0, W, 2):
            obj = int(gb["id"][y, x])
            X = gb["X"][:, y, x] - scene.vel[obj - 1] * (obj > 0)
            hit = _cast(scene, 2, x + mv[0, y, x], y + mv[1, y, x])
            assert hit is not None
            if hit[2] != obj:
                occluded += 1
                continue
            want_z = float((X - Cp) @ fwdp)
            assert abs(hit[0] - want_z) <= 1e-4 * want_z, (y, x, hit[0], want_z)
            n = gb["n"][:, y, x]
            assert np.abs(hit[1] / np.linalg.norm(hit[1]) - n).max() <= 1e-4, (y, x)
            checked += 1
            moving_obj += 1 <= obj <= cfg.n_moving
    assert checked > 0.95 * (checked + occluded)
    assert np.abs(mv).max() > 1.0 and moving_obj > 0


def _min_depth_and_finite(cfg, frame):
    gb = S._Scene(cfg).gbuffer(frame)
    z = gb["z"]
    return bool(np.all(np.isfinite(z)) and np.all(z > 0))


@pytest.mark.parametrize("name", ["small_static", "hd_motion", "uhd_half", "hd_learned"])
def test_no_empty_pixels_in_the_workloads(name):
    """The ground plane fills every frame (the camera looks 4.7 degrees or
    more below the horizon at the top row), so no pixel lacks a surface:
    first and last frame of each workload at its full size."""
    cfg = CONFIGS[name]
    for f in (0, cfg.frames - 1):
        assert _min_depth_and_finite(cfg, f), (name, f)


def test_no_empty_pixels_in_the_batched_streams():
    for cfg in batched_configs():
        assert _min_depth_and_finite(cfg, cfg.frames - 1), cfg
