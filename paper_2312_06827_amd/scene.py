"""Seeded synthetic inputs for the denoiser.

The paper's renderer traces one sample per pixel (Section 2) against scenes
that are not available here, so every input is generated: a procedural scene
(one ground plane and six spheres) seen through a pinhole camera, its
G-buffer (linear view depth, analytic depth gradients, unit normals, albedo,
object id), backward motion vectors, the previous frame's G-buffer, a clean
Lambert image and a noisy one-sample estimate of it.

This module draws and renders inputs only.  It holds none of the denoiser's
arithmetic (no tone map, no luminance, no reprojection rule, no filter): the
same arrays feed the HIP path and the CPU oracle.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import Dict, Iterator, List, Optional

import numpy as np

__all__ = [
    "SceneConfig",
    "Frame",
    "render_frame",
    "sequence",
    "CONFIGS",
    "batched_configs",
    "FIREFLY_P",
    "FIREFLY_GAIN",
    "with_size",
]

FIREFLY_P = 0.005  # probability that a pixel is a firefly
FIREFLY_GAIN = 50.0  # radiance multiplier of a firefly
# E[F] for F = 50 with probability 0.005 else 1; dividing by it keeps the
# noisy estimate unbiased (E[noisy] = clean).
_NOISE_NORM = (1.0 - FIREFLY_P) + FIREFLY_P * FIREFLY_GAIN

_CAM_POS0 = np.array([5.0, 9.0, -7.0])
_CAM_LOOK = np.array([5.0, 0.0, 6.0])
_WORLD_UP = np.array([0.0, 1.0, 0.0])
_LIGHT = np.array([1.0, 2.0, 0.5]) / math.sqrt(1.0 + 4.0 + 0.25)
_VFOV_DEG = 60.0


@dataclass(frozen=True)
class SceneConfig:
    width: int
    height: int
    frames: int
    seed: int
    stream: int = 0
    static: bool = False  # camera and spheres at rest: zero motion
    cam_px_per_frame: float = 2.0  # camera translation along its right axis
    yaw_deg_per_frame: float = 0.1  # camera rotation about the world up axis
    n_moving: int = 3  # spheres 0..n_moving-1 move in the image plane
    # the two channels the paper denoises separately (Section 3): a shadow
    # channel (one-sample visibility of a light of this angular diameter,
    # in degrees) and an indirect specular channel
    channels: bool = False
    shadow_angle_deg: float = 8.0
    sphere_px_per_frame: float = 5.0
    half: bool = False  # store every input plane as binary16


Frame = Dict[str, np.ndarray]


def _normalize(v):
    return v / np.linalg.norm(v)


def _focal(cfg: SceneConfig) -> float:
    return (cfg.height / 2.0) / math.tan(math.radians(_VFOV_DEG / 2.0))


class _Scene:
    """Objects and camera path of one seeded scene."""

    def __init__(self, cfg: SceneConfig):
        rng = np.random.Generator(
            np.random.Philox(np.random.SeedSequence([cfg.seed, cfg.stream, 1 << 20]))
        )
        self.cfg = cfg
        self.radius = rng.uniform(0.5, 2.0, size=6)
        self.center0 = rng.uniform(0.0, 10.0, size=(6, 3))
        # albedo of the plane (object id 0) then of spheres 1..6
        self.albedo = rng.uniform(0.2, 0.9, size=(7, 3))
        theta = rng.uniform(0.0, 2.0 * math.pi, size=6)
        self.f = _focal(cfg)
        fwd0, right0, up0 = self._basis(0.0)
        vel = np.zeros((6, 3))
        if not cfg.static:
            for i in range(min(cfg.n_moving, 6)):
                zc = float((self.center0[i] - _CAM_POS0) @ fwd0)
                speed = cfg.sphere_px_per_frame * zc / self.f
                vel[i] = speed * (math.cos(theta[i]) * right0 + math.sin(theta[i]) * up0)
        self.vel = vel
        # camera positions along the path, accumulated frame by frame
        z_ref = float(np.linalg.norm(_CAM_LOOK - _CAM_POS0))
        step = 0.0 if cfg.static else cfg.cam_px_per_frame * z_ref / self.f
        pos = [_CAM_POS0.copy()]
        for k in range(1, cfg.frames + 1):
            _, right_k, _ = self._basis(self._yaw(k))
            pos.append(pos[-1] + step * right_k)
        self.cam_pos = pos
        # surface roughness per object (plane, spheres), from its own stream
        # so that the draws above stay as they are: one value from each band
        # the adaptive blur tells apart (mirror, <= 0.05, <= 0.2, above)
        rr = np.random.Generator(
            np.random.Philox(np.random.SeedSequence([cfg.seed, cfg.stream, 1 << 20, 2])))
        bands = [0.0, 0.03, 0.1, 0.35, 0.6]
        self.roughness = np.concatenate(
            [[0.3], rr.permutation(bands + [float(rr.choice(bands))])]).astype(np.float32)

    def _yaw(self, frame: int) -> float:
        return 0.0 if self.cfg.static else math.radians(self.cfg.yaw_deg_per_frame * frame)

    @staticmethod
    def _basis(yaw: float):
        fwd = _normalize(_CAM_LOOK - _CAM_POS0)
        c, s = math.cos(yaw), math.sin(yaw)
        # rotation about world +y
        fwd = np.array([c * fwd[0] + s * fwd[2], fwd[1], -s * fwd[0] + c * fwd[2]])
        right = _normalize(np.cross(_WORLD_UP, fwd))
        up = np.cross(fwd, right)
        return fwd, right, up

    def camera(self, frame: int):
        fwd, right, up = self._basis(self._yaw(frame))
        return self.cam_pos[frame], fwd, right, up

    def centers(self, frame: int):
        return self.center0 + frame * self.vel

    def gbuffer(self, frame: int):
        """Ray-cast the scene at `frame`: depth, gradients, normals, ids."""
        cfg = self.cfg
        W, H, f = cfg.width, cfg.height, self.f
        C, fwd, right, up = self.camera(frame)
        u = (np.arange(W, dtype=np.float64) + 0.5 - W / 2.0) / f
        v = -(np.arange(H, dtype=np.float64) + 0.5 - H / 2.0) / f
        # ray direction with unit forward component: hit distance t is view depth
        d = (fwd[:, None, None] + u[None, None, :] * right[:, None, None]
             + v[None, :, None] * up[:, None, None])  # (3, H, W)
        t_best = np.full((H, W), np.inf)
        obj = np.zeros((H, W), dtype=np.uint8)
        # ground plane y = 0 (object 0)
        with np.errstate(divide="ignore", invalid="ignore"):
            tp = np.where(d[1] < 0.0, -C[1] / d[1], np.inf)
        t_best = np.minimum(t_best, tp)
        a = np.einsum("ihw,ihw->hw", d, d)
        for i, S in enumerate(self.centers(frame)):
            oc = C - S
            b = 2.0 * np.einsum("i,ihw->hw", oc, d)
            c = float(oc @ oc) - self.radius[i] ** 2
            disc = b * b - 4.0 * a * c
            hit = disc > 0.0
            sq = np.sqrt(np.where(hit, disc, 0.0))
            t0 = (-b - sq) / (2.0 * a)
            t0 = np.where(hit & (t0 > 1e-6), t0, np.inf)
            closer = t0 < t_best
            t_best = np.where(closer, t0, t_best)
            obj = np.where(closer, np.uint8(i + 1), obj)
        z = t_best
        X = C[:, None, None] + z[None] * d  # world hit points
        n = np.empty((3, H, W))
        n[0] = 0.0
        n[1] = 1.0
        n[2] = 0.0
        for i, S in enumerate(self.centers(frame)):
            m = obj == i + 1
            if np.any(m):
                n[:, m] = (X[:, m] - S[:, None]) / self.radius[i]
        n /= np.sqrt(np.einsum("ihw,ihw->hw", n, n))[None]
        ndotd = np.einsum("ihw,ihw->hw", n, d)
        dzdx = -z * np.einsum("i,ihw->hw", right, n) / (f * ndotd)
        dzdy = z * np.einsum("i,ihw->hw", up, n) / (f * ndotd)
        return dict(z=z, dzdx=dzdx, dzdy=dzdy, n=n, id=obj, X=X)

    def motion(self, frame: int, gb) -> np.ndarray:
        """Backward motion in pixels: where each pixel's surface point was
        seen in the previous frame, minus the pixel position."""
        cfg = self.cfg
        W, H, f = cfg.width, cfg.height, self.f
        if frame == 0 or cfg.static:
            return np.zeros((2, H, W))
        X = gb["X"].copy()
        for i in range(6):
            if np.any(self.vel[i] != 0.0):
                m = gb["id"] == i + 1
                X[:, m] -= self.vel[i][:, None]
        Cp, fwd, right, up = self.camera(frame - 1)
        rel = X - Cp[:, None, None]
        zc = np.einsum("i,ihw->hw", fwd, rel)
        xp = np.einsum("i,ihw->hw", right, rel) / zc * f + W / 2.0 - 0.5
        yp = -np.einsum("i,ihw->hw", up, rel) / zc * f + H / 2.0 - 0.5
        xs = np.arange(W, dtype=np.float64)[None, :]
        ys = np.arange(H, dtype=np.float64)[:, None]
        return np.stack([xp - xs, yp - ys])


def _noise(cfg: SceneConfig, frame: int, clean: np.ndarray) -> np.ndarray:
    rng = np.random.Generator(
        np.random.Philox(np.random.SeedSequence([cfg.seed, cfg.stream, frame]))
    )
    H, W = clean.shape[1:]
    e = rng.standard_exponential(size=(3, H, W))
    fire = rng.random(size=(H, W)) < FIREFLY_P
    gain = np.where(fire, FIREFLY_GAIN, 1.0) / _NOISE_NORM
    return clean * e * gain[None]


def _disc_overlap(d, r1, r2):
    """Area of the intersection of two discs of radii r1, r2 whose centres
    are d apart (all arrays, planar)."""
    d = np.maximum(d, 1e-12)
    a1 = np.clip((d * d + r1 * r1 - r2 * r2) / (2.0 * d * r1), -1.0, 1.0)
    a2 = np.clip((d * d + r2 * r2 - r1 * r1) / (2.0 * d * r2), -1.0, 1.0)
    k = (-d + r1 + r2) * (d + r1 - r2) * (d - r1 + r2) * (d + r1 + r2)
    lens = r1 * r1 * np.arccos(a1) + r2 * r2 * np.arccos(a2) - 0.5 * np.sqrt(np.maximum(k, 0.0))
    inner = np.pi * np.minimum(r1, r2) ** 2
    return np.where(d >= r1 + r2, 0.0, np.where(d <= np.abs(r1 - r2), inner, lens))


def _visibility(cfg, scene, frame, gb) -> np.ndarray:
    """Fraction of the light's disc (angular diameter shadow_angle_deg
    around the light direction) seen from each surface point: every sphere
    other than the point's own covers a disc of angular radius
    asin(R / distance); the covered fractions combine as independent
    occluders.  Small-angle (planar) disc geometry."""
    return _visibility_at(cfg, scene, frame, gb["X"], gb["id"])


def _visibility_at(cfg, scene, frame, X, obj) -> np.ndarray:
    theta = math.radians(cfg.shadow_angle_deg) / 2.0
    vis = np.ones(obj.shape)
    for i, S in enumerate(scene.centers(frame)):
        D = S[:, None, None] - X
        dist = np.sqrt(np.einsum("ihw,ihw->hw", D, D))
        beta = np.arcsin(np.clip(scene.radius[i] / np.maximum(dist, 1e-9), 0.0, 1.0))
        cosd = np.einsum("i,ihw->hw", _LIGHT, D) / np.maximum(dist, 1e-9)
        delta = np.arccos(np.clip(cosd, -1.0, 1.0))
        covered = _disc_overlap(delta, np.full_like(delta, theta), beta) / (np.pi * theta * theta)
        covered = np.where((obj == i + 1) | (dist <= scene.radius[i]), 0.0, covered)
        vis *= 1.0 - np.clip(covered, 0.0, 1.0)
    return vis


def _specular(cfg, scene, frame, gb) -> np.ndarray:
    """Indirect specular radiance: a sky gradient seen along the mirror
    direction, scaled by 0.25 (1 - roughness)."""
    C, _, _, _ = scene.camera(frame)
    V = gb["X"] - C[:, None, None]
    V /= np.sqrt(np.einsum("ihw,ihw->hw", V, V))[None]
    n = gb["n"]
    R = V - 2.0 * np.einsum("ihw,ihw->hw", V, n)[None] * n
    up = np.clip(R[1], 0.0, 1.0)[None]
    horizon = np.array([0.85, 0.8, 0.75])[:, None, None]
    zenith = np.array([0.25, 0.45, 0.95])[:, None, None]
    sky = horizon * (1.0 - up) + zenith * up
    ks = 0.25 * (1.0 - scene.roughness[gb["id"]].astype(np.float64))
    return 2.0 * sky * ks[None]


def _forward(cfg, scene, frame, gb_prev):
    """Where each pixel of frame - 1 lands in frame `frame`: its surface
    point moved with its object, projected with the current camera.
    Returns the moved points, the forward motion in pixels (2, H, W) and
    the moved points' view depth."""
    W, H, f = cfg.width, cfg.height, scene.f
    X = gb_prev["X"].copy()
    for i in range(6):
        if np.any(scene.vel[i] != 0.0):
            m = gb_prev["id"] == i + 1
            X[:, m] += scene.vel[i][:, None]
    C, fwd, right, up = scene.camera(frame)
    rel = X - C[:, None, None]
    zc = np.einsum("i,ihw->hw", fwd, rel)
    xp = np.einsum("i,ihw->hw", right, rel) / zc * f + W / 2.0 - 0.5
    yp = -np.einsum("i,ihw->hw", up, rel) / zc * f + H / 2.0 - 0.5
    xs = np.arange(W, dtype=np.float64)[None, :]
    ys = np.arange(H, dtype=np.float64)[:, None]
    return X, np.stack([xp - xs, yp - ys]), zc


def _channel_noise(cfg, frame: int, key: int, shape):
    """Uniforms of one channel's frame, from their own stream."""
    return np.random.Generator(
        np.random.Philox(np.random.SeedSequence([cfg.seed, cfg.stream, frame, 1 << 21, key])))


def _assemble(cfg, scene, frame, gb, gb_prev) -> Frame:
    n_dot_l = np.maximum(0.0, np.einsum("i,ihw->hw", _LIGHT, gb["n"]))
    alb = scene.albedo[gb["id"]].transpose(2, 0, 1)  # (3, H, W)
    clean = alb * n_dot_l[None]
    noisy = _noise(cfg, frame, clean)
    mv = scene.motion(frame, gb)
    ft = np.float16 if cfg.half else np.float32

    def q(a):
        return np.ascontiguousarray(a.astype(np.float32).astype(ft))

    out = {
        "rgb": q(noisy),
        "clean": np.ascontiguousarray(clean.astype(np.float32)),
        "albedo": q(alb),
        "z": q(gb["z"]),
        "dzdx": q(gb["dzdx"]),
        "dzdy": q(gb["dzdy"]),
        "n": q(gb["n"]),
        "id": np.ascontiguousarray(gb["id"]),
        "mv": q(mv),
        "prev_z": q(gb_prev["z"]),
        "prev_n": q(gb_prev["n"]),
        "prev_id": np.ascontiguousarray(gb_prev["id"]),
        "roughness": np.ascontiguousarray(scene.roughness[gb["id"]]),
    }
    if cfg.channels:
        H, W = gb["z"].shape
        vis = _visibility(cfg, scene, frame, gb)
        # one shadow ray per pixel: a Bernoulli sample of the visibility
        hit = _channel_noise(cfg, frame, 1, (H, W)).random(size=(H, W)) < vis
        shadow = np.broadcast_to(hit.astype(np.float64)[None], (3, H, W))
        spec_clean = _specular(cfg, scene, frame, gb)
        rs = _channel_noise(cfg, frame, 2, (H, W))
        e = rs.standard_exponential(size=(3, H, W))
        fire = rs.random(size=(H, W)) < FIREFLY_P
        spec = spec_clean * e * (np.where(fire, FIREFLY_GAIN, 1.0) / _NOISE_NORM)[None]
        out.update({
            "direct": q(clean),
            "shadow": q(shadow),
            "shadow_clean": np.ascontiguousarray(vis.astype(np.float32)),
            "spec": q(spec),
            "spec_clean": np.ascontiguousarray(spec_clean.astype(np.float32)),
            "shadow_angle": np.full((H, W), cfg.shadow_angle_deg, np.float32),
            "composite_clean": np.ascontiguousarray(
                (clean * vis[None] + spec_clean).astype(np.float32)),
        })
        # the temporal gradient's inputs (A-SVGF): every pixel of the
        # previous frame carried forward, its shadow ray traced again in
        # this frame with the previous frame's random number, and one
        # sample per 3x3 stratum of the previous frame chosen for it
        if frame > 0 and not cfg.static:
            Xf, fmv, fz = _forward(cfg, scene, frame, gb_prev)
            u_prev = _channel_noise(cfg, frame - 1, 1, (H, W)).random(size=(H, W))
            vis_f = _visibility_at(cfg, scene, frame, Xf, gb_prev["id"])
            reshade = (u_prev < vis_f).astype(np.float32)
        else:
            fmv = np.zeros((2, H, W))
            fz = gb_prev["z"]
            reshade = hit.astype(np.float32)
        pick = _channel_noise(cfg, frame, 3, (H, W)).integers(
            0, 9, size=((H + 2) // 3, (W + 2) // 3)).astype(np.uint8)
        out.update({
            "fmv": q(fmv),
            "fz": q(fz),
            "shadow_reshade": np.ascontiguousarray(reshade),
            "grad_pick": np.ascontiguousarray(pick),
        })
    return out


def render_frame(cfg: SceneConfig, frame: int) -> Frame:
    """Render one frame (random access)."""
    scene = _Scene(cfg)
    gb = scene.gbuffer(frame)
    gb_prev = scene.gbuffer(frame - 1) if (frame > 0 and not cfg.static) else gb
    return _assemble(cfg, scene, frame, gb, gb_prev)


def sequence(cfg: SceneConfig, start: int = 0, count: Optional[int] = None) -> Iterator[Frame]:
    """Render frames start .. start+count-1 in order, reusing each G-buffer
    as the next frame's previous G-buffer."""
    scene = _Scene(cfg)
    count = cfg.frames - start if count is None else count
    gb_prev = None
    for frame in range(start, start + count):
        gb = scene.gbuffer(frame)
        if cfg.static or frame == 0:
            gbp = gb
        elif gb_prev is None:
            gbp = scene.gbuffer(frame - 1)
        else:
            gbp = gb_prev
        yield _assemble(cfg, scene, frame, gb, gbp)
        gb_prev = gb


# The five workloads.  Sizes, frame counts and seeds are fixed here; filter
# settings live with the callers.
CONFIGS = {
    # 256x256, 8 frames, static camera
    "small_static": SceneConfig(256, 256, 8, seed=1, static=True),
    # 1920x1080, 60 frames, moving camera and spheres
    "hd_motion": SceneConfig(1920, 1080, 60, seed=2),
    # 3840x2160, 30 frames, binary16 storage
    "uhd_half": SceneConfig(3840, 2160, 30, seed=3, half=True),
    # 1920x1080, 60 frames (learned-filter evaluation sequences use seeds 5900+)
    "hd_learned": SceneConfig(1920, 1080, 60, seed=5900),
}


def batched_configs(n_streams: int = 16, frames: int = 30, seed: int = 4,
                    half: bool = True) -> List[SceneConfig]:
    """Sixteen independent streams of uneven size: W in [640, 2560] and
    H in [360, 1440] drawn independently, each with its own scene seed and
    camera speed."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, 0xB47C])))
    out = []
    for i in range(n_streams):
        w = int(rng.integers(640, 2561))
        h = int(rng.integers(360, 1441))
        out.append(SceneConfig(
            w, h, frames, seed=4000 + i, stream=i,
            cam_px_per_frame=float(rng.uniform(0.0, 4.0)),
            yaw_deg_per_frame=float(rng.uniform(0.0, 0.2)),
            half=half))
    return out


def with_size(cfg: SceneConfig, width: int, height: int, frames: Optional[int] = None) -> SceneConfig:
    """Same scene and motion at another resolution (for reduced test sizes)."""
    return replace(cfg, width=width, height=height,
                   frames=cfg.frames if frames is None else frames)
