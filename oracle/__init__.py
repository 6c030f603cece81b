"""FP64 CPU oracle of the denoiser (ctypes front end of ``svo.c``).

TEST INFRASTRUCTURE ONLY.  This package is the plain reference the HIP
library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never
does, and nothing here imports the product package.

Arrays are numpy, images ``(H, W)`` or channel-first ``(3, H, W)``; every
call converts its inputs to contiguous float64 and returns float64 (int32
for history lengths).  The steps and their order follow the paper:

* tone map before denoising and its inverse after (Section 3.4),
* temporal filter: backward reprojection, variance colour clamp of the
  history, accumulation of colour and luminance moments (Sections 2, 3.1),
* variance estimate (Section 2),
* edge-avoiding a-trous levels, 5x5 or separable (Section 2, Fig. 1;
  Section 3.3).

Yes/no decisions computed from floating point (the reprojection's depth and
normal tests) are taken in binary32, the precision of the device path.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass, replace
from typing import Dict, Optional

import numpy as np

__all__ = [
    "OracleParams", "tonemap", "reproject", "clamp", "clip", "blend", "temporal",
    "variance", "atrous", "atrous_sep", "quantize_half", "new_state",
    "run_frame", "luma", "blur_control", "atrous_adaptive", "compose",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsvoracle.so")
_lock = threading.Lock()
_lib = None

UNIT_WEIGHTS = 1
INV_TONEMAP = 2
HALF_OUT = 4
TM_MODES = {"luma": 0, "channel": 1, "paper": 2}
T_CLAMP = 1
T_USE_ID = 2
T_TONEMAP_IN = 4
T_CLIP = 8

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_up = ctypes.POINTER(ctypes.c_uint8)
_I, _L, _D = ctypes.c_int, ctypes.c_int64, ctypes.c_double


def _build():
    src = os.path.join(_HERE, "svo.c")
    if os.path.exists(_SO) and os.path.getmtime(_SO) >= os.path.getmtime(src):
        return
    subprocess.run(["make", "-s", "-C", _HERE, "libsvoracle.so"], check=True)


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        _build()
        lib = ctypes.CDLL(_SO)
        lib.svo_tonemap.argtypes = [_L, _dp, _dp, _dp, _dp, _dp, _dp, _I, _I, _D, _D]
        lib.svo_reproject.argtypes = (
            [_I, _I] + [_dp] * 4 + [_up] + [_dp] * 6 + [_up] + [_dp] * 5 + [_ip]
            + [_D, _D, _I] + [_dp] * 5 + [_ip, _ip])
        lib.svo_clamp.argtypes = [_I, _I] + [_dp] * 7 + [_D] + [_dp] * 3
        lib.svo_clip.argtypes = [_I, _I] + [_dp] * 7 + [_D] + [_dp] * 3
        lib.svo_blend.argtypes = (
            [_L] + [_dp] * 9 + [_ip, _ip, _D, _D, _dp, _I, _I] + [_dp] * 5 + [_ip])
        lib.svo_temporal.argtypes = (
            [_I, _I] + [_dp] * 7 + [_up] + [_dp] * 6 + [_up] + [_dp] * 5 + [_ip]
            + [_D] * 6 + [_I, _I, _I, _dp] + [_dp] * 5 + [_ip])
        lib.svo_temporal.restype = _I
        lib.svo_variance.argtypes = (
            [_I, _I, _dp, _dp, _ip] + [_dp] * 6 + [_D, _D, _D, _I, _I, _dp])
        lib.svo_atrous.argtypes = (
            [_I, _I] + [_dp] * 11 + [_I] + [_D] * 6 + [_I] + [_dp] * 4)
        lib.svo_atrous_sep.argtypes = (
            [_I, _I] + [_dp] * 11 + [_I] + [_D] * 6 + [_I] + [_dp] * 7)
        lib.svo_quantize_half.argtypes = [_L, _dp]
        lib.svo_version.restype = _I
        lib.svo_set_threads.argtypes = [_I]
        lib.svo_threads.restype = _I
        _lib = lib
        return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, kind=_dp):
    if a is None:
        return None
    return a.ctypes.data_as(kind)


def luma(rgb):
    """Rec. 709 luminance of a (3, ...) array (the listing's luma())."""
    rgb = np.asarray(rgb, dtype=np.float64)
    return 0.2126 * rgb[0] + 0.7152 * rgb[1] + 0.0722 * rgb[2]


@dataclass(frozen=True)
class OracleParams:
    """Filter constants.  Defaults: alpha 0.2, 5 levels, sigma_z 1,
    sigma_n 128, sigma_l 4, clamp gamma 1 (off unless `clamp`), depth and
    normal reprojection tolerances 0.1 and 0.9."""
    alpha: float = 0.2
    alpha_m: float = 0.2
    levels: int = 5
    sigma_z: float = 1.0
    sigma_n: float = 128.0
    sigma_l: float = 4.0
    eps_z: float = 1e-10
    eps_l: float = 1e-10
    tau_z: float = 0.1
    tau_n: float = 0.9
    gamma: float = 1.0
    clamp: bool = False
    clip: bool = False  # clip the history toward the box centre instead of clamping
    use_id: bool = False
    tonemap: bool = False
    tm_k: float = 1.0
    separable: bool = False
    max_hist: int = 255
    min_hist: int = 4
    var_radius: int = 3
    feedback: str = "atrous0"  # colour history: level-0 output, or "temporal"
    half: bool = False  # round stored colours to binary16


# ---- single steps --------------------------------------------------------

def tonemap(rgb, inverse=False, mode="luma", k=1.0, weight=1.0):
    rgb = _f64(rgb)
    out = np.empty_like(rgb)
    n = rgb[0].size
    _load().svo_tonemap(n, _ptr(rgb[0]), _ptr(rgb[1]), _ptr(rgb[2]),
                        _ptr(out[0]), _ptr(out[1]), _ptr(out[2]),
                        int(bool(inverse)), TM_MODES[mode], float(k), float(weight))
    return out


def reproject(z, n, mv, prev_z, prev_n, hist_rgb, hist_m1, hist_m2, hist_n,
              tau_z=0.1, tau_n=0.9, id=None, prev_id=None, use_id=False):
    z, n, mv, prev_z, prev_n = map(_f64, (z, n, mv, prev_z, prev_n))
    hist_rgb, hist_m1, hist_m2 = map(_f64, (hist_rgb, hist_m1, hist_m2))
    hist_n = np.ascontiguousarray(hist_n, dtype=np.int32)
    ids = [None if a is None else np.ascontiguousarray(a, dtype=np.uint8) for a in (id, prev_id)]
    H, W = z.shape
    o = np.empty((5, H, W))
    on = np.empty((H, W), np.int32)
    ov = np.empty((H, W), np.int32)
    _load().svo_reproject(
        W, H, _ptr(z), _ptr(n[0]), _ptr(n[1]), _ptr(n[2]), _ptr(ids[0], _up),
        _ptr(mv[0]), _ptr(mv[1]), _ptr(prev_z), _ptr(prev_n[0]), _ptr(prev_n[1]),
        _ptr(prev_n[2]), _ptr(ids[1], _up), _ptr(hist_rgb[0]), _ptr(hist_rgb[1]),
        _ptr(hist_rgb[2]), _ptr(hist_m1), _ptr(hist_m2), _ptr(hist_n, _ip),
        float(tau_z), float(tau_n), int(bool(use_id)),
        _ptr(o[0]), _ptr(o[1]), _ptr(o[2]), _ptr(o[3]), _ptr(o[4]), _ptr(on, _ip), _ptr(ov, _ip))
    return {"rgb": o[:3], "m1": o[3], "m2": o[4], "n": on, "valid": ov}


def clamp(hist_rgb, cur_rgb, gamma, z=None):
    hist_rgb, cur_rgb = _f64(hist_rgb), _f64(cur_rgb)
    z = None if z is None else _f64(z)
    H, W = hist_rgb.shape[1:]
    out = np.empty_like(hist_rgb)
    _load().svo_clamp(W, H, _ptr(hist_rgb[0]), _ptr(hist_rgb[1]), _ptr(hist_rgb[2]),
                      _ptr(cur_rgb[0]), _ptr(cur_rgb[1]), _ptr(cur_rgb[2]), _ptr(z),
                      float(gamma), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]))
    return out


def clip(hist_rgb, cur_rgb, gamma, z=None):
    hist_rgb, cur_rgb = _f64(hist_rgb), _f64(cur_rgb)
    z = None if z is None else _f64(z)
    H, W = hist_rgb.shape[1:]
    out = np.empty_like(hist_rgb)
    _load().svo_clip(W, H, _ptr(hist_rgb[0]), _ptr(hist_rgb[1]), _ptr(hist_rgb[2]),
                     _ptr(cur_rgb[0]), _ptr(cur_rgb[1]), _ptr(cur_rgb[2]), _ptr(z),
                     float(gamma), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]))
    return out


def blend(cur_rgb, z, hist_rgb, hist_m1, hist_m2, hist_n, valid, alpha=0.2,
          alpha_m=0.2, alpha_map=None, max_hist=255, half_out=False):
    cur_rgb, z, hist_rgb, hist_m1, hist_m2 = map(_f64, (cur_rgb, z, hist_rgb, hist_m1, hist_m2))
    hist_n = np.ascontiguousarray(hist_n, dtype=np.int32)
    valid = np.ascontiguousarray(valid, dtype=np.int32)
    am = None if alpha_map is None else _f64(alpha_map)
    H, W = z.shape
    o = np.empty((5, H, W))
    on = np.empty((H, W), np.int32)
    _load().svo_blend(
        W * H, _ptr(cur_rgb[0]), _ptr(cur_rgb[1]), _ptr(cur_rgb[2]), _ptr(z),
        _ptr(hist_rgb[0]), _ptr(hist_rgb[1]), _ptr(hist_rgb[2]), _ptr(hist_m1),
        _ptr(hist_m2), _ptr(hist_n, _ip), _ptr(valid, _ip), float(alpha), float(alpha_m),
        _ptr(am), int(max_hist), HALF_OUT if half_out else 0,
        _ptr(o[0]), _ptr(o[1]), _ptr(o[2]), _ptr(o[3]), _ptr(o[4]), _ptr(on, _ip))
    return {"rgb": o[:3], "m1": o[3], "m2": o[4], "n": on}


def temporal(frame: Dict[str, np.ndarray], state: Dict[str, np.ndarray],
             p: OracleParams, alpha_map=None):
    """Temporal filter of one frame.  `frame` holds the generator's planes
    (rgb, z, n, id, mv, prev_z, prev_n, prev_id); `state` the history
    (rgb, m1, m2, n)."""
    cur = _f64(frame["rgb"])
    z, n, mv = _f64(frame["z"]), _f64(frame["n"]), _f64(frame["mv"])
    pz, pn = _f64(frame["prev_z"]), _f64(frame["prev_n"])
    hr, h1, h2 = _f64(state["rgb"]), _f64(state["m1"]), _f64(state["m2"])
    hn = np.ascontiguousarray(state["n"], dtype=np.int32)
    ids = [np.ascontiguousarray(frame[k], dtype=np.uint8) if frame.get(k) is not None else None
           for k in ("id", "prev_id")]
    am = None if alpha_map is None else _f64(alpha_map)
    H, W = z.shape
    flags = (T_CLAMP if p.clamp else 0) | (T_CLIP if p.clip else 0) | \
        (T_USE_ID if p.use_id else 0) | (T_TONEMAP_IN if p.tonemap else 0)
    o = np.empty((5, H, W))
    on = np.empty((H, W), np.int32)
    rc = _load().svo_temporal(
        W, H, _ptr(cur[0]), _ptr(cur[1]), _ptr(cur[2]), _ptr(z), _ptr(n[0]),
        _ptr(n[1]), _ptr(n[2]), _ptr(ids[0], _up), _ptr(mv[0]), _ptr(mv[1]),
        _ptr(pz), _ptr(pn[0]), _ptr(pn[1]), _ptr(pn[2]), _ptr(ids[1], _up),
        _ptr(hr[0]), _ptr(hr[1]), _ptr(hr[2]), _ptr(h1), _ptr(h2), _ptr(hn, _ip),
        p.alpha, p.alpha_m, p.gamma, p.tau_z, p.tau_n, p.tm_k, p.max_hist, flags,
        HALF_OUT if p.half else 0, _ptr(am),
        _ptr(o[0]), _ptr(o[1]), _ptr(o[2]), _ptr(o[3]), _ptr(o[4]), _ptr(on, _ip))
    if rc != 0:
        raise MemoryError("oracle temporal: allocation failed")
    # m2c: the second central moment E[L^2] - E[L]^2 of the accumulated
    # luminance (the form in which the device path stores it)
    return {"rgb": o[:3], "m1": o[3], "m2": o[4], "m2c": o[4] - o[3] * o[3], "n": on}


def variance(m1, m2, hist_n, z, dzdx, dzdy, n, sigma_z=1.0, sigma_n=128.0,
             eps_z=1e-10, min_hist=4, radius=3):
    m1, m2, z, dzdx, dzdy, n = map(_f64, (m1, m2, z, dzdx, dzdy, n))
    hist_n = np.ascontiguousarray(hist_n, dtype=np.int32)
    H, W = z.shape
    out = np.empty((H, W))
    _load().svo_variance(W, H, _ptr(m1), _ptr(m2), _ptr(hist_n, _ip), _ptr(z),
                         _ptr(dzdx), _ptr(dzdy), _ptr(n[0]), _ptr(n[1]), _ptr(n[2]),
                         float(sigma_z), float(sigma_n), float(eps_z), int(min_hist),
                         int(radius), _ptr(out))
    return out


def _atrous_flags(unit_weights, inv_tonemap, half_out):
    return ((UNIT_WEIGHTS if unit_weights else 0) | (INV_TONEMAP if inv_tonemap else 0)
            | (HALF_OUT if half_out else 0))


def atrous(rgb, var, z, dzdx, dzdy, n, step, kappa=None, sigma_z=1.0,
           sigma_n=128.0, sigma_l=4.0, eps_z=1e-10, eps_l=1e-10, tm_k=1.0,
           unit_weights=False, inv_tonemap=False, half_out=False, want_var=True):
    """One 5x5 level; returns (rgb, var) (var None if not wanted)."""
    rgb, var, z, dzdx, dzdy, n = map(_f64, (rgb, var, z, dzdx, dzdy, n))
    kp = None if kappa is None else _f64(kappa)
    H, W = z.shape
    out = np.empty((3, H, W))
    vo = np.empty((H, W)) if want_var else None
    _load().svo_atrous(W, H, _ptr(rgb[0]), _ptr(rgb[1]), _ptr(rgb[2]), _ptr(var), _ptr(z),
                       _ptr(dzdx), _ptr(dzdy), _ptr(n[0]), _ptr(n[1]), _ptr(n[2]), _ptr(kp),
                       int(step), float(sigma_z), float(sigma_n), float(sigma_l),
                       float(eps_z), float(eps_l), float(tm_k),
                       _atrous_flags(unit_weights, inv_tonemap, half_out),
                       _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(vo))
    return out, vo


def atrous_sep(rgb, var, z, dzdx, dzdy, n, step, kappa=None, sigma_z=1.0,
               sigma_n=128.0, sigma_l=4.0, eps_z=1e-10, eps_l=1e-10, tm_k=1.0,
               unit_weights=False, inv_tonemap=False, half_out=False, want_var=True):
    """One separable level; returns (rgb, var, horizontal_rgb)."""
    rgb, var, z, dzdx, dzdy, n = map(_f64, (rgb, var, z, dzdx, dzdy, n))
    kp = None if kappa is None else _f64(kappa)
    H, W = z.shape
    out = np.empty((3, H, W))
    sh = np.empty((3, H, W))
    vo = np.empty((H, W)) if want_var else None
    _load().svo_atrous_sep(W, H, _ptr(rgb[0]), _ptr(rgb[1]), _ptr(rgb[2]), _ptr(var), _ptr(z),
                           _ptr(dzdx), _ptr(dzdy), _ptr(n[0]), _ptr(n[1]), _ptr(n[2]),
                           _ptr(kp), int(step), float(sigma_z), float(sigma_n),
                           float(sigma_l), float(eps_z), float(eps_l), float(tm_k),
                           _atrous_flags(unit_weights, inv_tonemap, half_out),
                           _ptr(sh[0]), _ptr(sh[1]), _ptr(sh[2]),
                           _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(vo))
    return out, vo, sh


# ---- blur adapted to scene features (Sections 3.2, 3.5) -----------------------

CTL_LEVELS_MASK, CTL_SHIFT = 15, 16


def blur_control(roughness=None, shadow_angle=None, rough_shift=0.2, angle_shift=6.0,
                 rough_none=0.0, rough_one=0.05, it_none=0, it_one=1, it_rest=15,
                 shift=True, table=True):
    """Per-pixel control bytes of the adaptive levels.

    Section 3.2: a pixel whose surface roughness exceeds 0.2, or whose
    shadow angle exceeds 6.0, starts the a-trous cascade one level coarser
    (its first level is the usual second one) with the same number of
    levels.  Section 3.5: the number of levels follows the roughness,
    none at roughness <= 0, one at <= 0.05, otherwise all of them (the
    paper's 4 is its full count; 15 here means every level).  Bits 0-3 hold
    the level count, bit 4 the shift.  The thresholds decide integers, so
    the comparisons are made in binary32, the precision of the device path."""
    ref = roughness if roughness is not None else shadow_angle
    f32 = np.float32
    shape = np.shape(ref)
    sh = np.zeros(shape, bool)
    if shift:
        if roughness is not None:
            sh |= np.asarray(roughness, f32) > f32(rough_shift)
        if shadow_angle is not None:
            sh |= np.asarray(shadow_angle, f32) > f32(angle_shift)
    lv = np.full(shape, 15, np.int32)
    if table:
        r = np.asarray(roughness, f32)
        lv = np.where(r <= f32(rough_none), it_none,
                      np.where(r <= f32(rough_one), it_one, it_rest)).astype(np.int32)
    return (sh.astype(np.uint8) * CTL_SHIFT) | lv.astype(np.uint8)


def atrous_adaptive(rgb, var, z, dzdx, dzdy, n, ctl, level, separable=False, kappa=None,
                    sigma_z=1.0, sigma_n=128.0, sigma_l=4.0, eps_z=1e-10, eps_l=1e-10,
                    tm_k=1.0, unit_weights=False, inv_tonemap=False, half_out=False,
                    want_var=True):
    """Level `level` of the adaptive cascade (Sections 3.2, 3.5): pixel p is
    the output at p of the whole level filtered at step 2^(level + shift(p))
    while level < levels(p), else its input (colour and variance) unchanged,
    inverse tone mapped on the last level like every other output.
    Returns (rgb, var)."""
    rgb, var = _f64(rgb), _f64(var)
    ctl = np.asarray(ctl, np.uint8)
    fn = atrous_sep if separable else atrous
    kw = dict(kappa=kappa, sigma_z=sigma_z, sigma_n=sigma_n, sigma_l=sigma_l, eps_z=eps_z,
              eps_l=eps_l, tm_k=tm_k, unit_weights=unit_weights, inv_tonemap=inv_tonemap,
              half_out=half_out, want_var=want_var)
    fine = fn(rgb, var, z, dzdx, dzdy, n, 1 << level, **kw)
    coarse = fn(rgb, var, z, dzdx, dzdy, n, 2 << level, **kw)
    keep = level >= (ctl & CTL_LEVELS_MASK).astype(np.int32)
    shifted = (ctl & CTL_SHIFT) != 0
    same = tonemap(rgb, inverse=True, k=tm_k) if inv_tonemap else rgb.copy()
    if half_out:
        same = quantize_half(same)
    out = np.where(keep, same, np.where(shifted, coarse[0], fine[0]))
    vo = np.where(keep, var, np.where(shifted, coarse[1], fine[1])) if want_var else None
    return out, vo


# ---- composition of the channels (Section 3, step 7) ---------------------------

def compose(direct, shadow=None, spec=None, half_out=False):
    """The denoised shadow and indirect specular channels blended with the
    noise-free direct lighting.  The paper names the step without a formula;
    the reading is the usual deferred one: direct light attenuated by the
    shadow visibility, plus the indirect specular light, per colour
    channel."""
    out = _f64(direct).copy()
    if shadow is not None:
        out = out * _f64(shadow)
    if spec is not None:
        out = out + _f64(spec)
    return quantize_half(out) if half_out else out


def quantize_half(x):
    """binary16 round-to-nearest-even of every element (as float64)."""
    x = np.array(x, dtype=np.float64, copy=True, order="C")
    _load().svo_quantize_half(x.size, _ptr(x))
    return x


# ---- one frame of the whole filter ---------------------------------------

def new_state(height: int, width: int):
    """Empty history: zero colour and moments, history length 0."""
    return {"rgb": np.zeros((3, height, width)), "m1": np.zeros((height, width)),
            "m2": np.zeros((height, width)), "n": np.zeros((height, width), np.int32)}


def run_frame(frame, state, p: OracleParams, alpha_map=None, kappa=None, ctl=None):
    """Temporal filter, variance, `p.levels` a-trous levels with steps
    1, 2, 4, ..., inverse tone map.  Returns (output rgb, new state,
    intermediates).  The colour history for the next frame is the level-0
    output (or the temporal output if p.feedback == "temporal"); the moment
    history is the temporal output.  With control bytes `ctl` the levels are
    the adaptive ones (Sections 3.2, 3.5)."""
    t = temporal(frame, state, p, alpha_map=alpha_map)
    z, dzdx, dzdy, n = frame["z"], frame["dzdx"], frame["dzdy"], frame["n"]
    var = variance(t["m1"], t["m2"], t["n"], z, dzdx, dzdy, n, p.sigma_z,
                   p.sigma_n, p.eps_z, p.min_hist, p.var_radius)
    c, v = t["rgb"], var
    hist_rgb = c
    step_fn = atrous_sep if p.separable else atrous
    levels = []
    for i in range(p.levels):
        last = i == p.levels - 1
        fuse_inv = p.tonemap and last and not (i == 0 and p.feedback == "atrous0")
        kw = dict(kappa=kappa, sigma_z=p.sigma_z, sigma_n=p.sigma_n, sigma_l=p.sigma_l,
                  eps_z=p.eps_z, eps_l=p.eps_l, tm_k=p.tm_k, inv_tonemap=fuse_inv,
                  half_out=p.half, want_var=not last)
        if ctl is not None:
            res = atrous_adaptive(c, v, z, dzdx, dzdy, n, ctl, i, separable=p.separable, **kw)
        else:
            res = step_fn(c, v, z, dzdx, dzdy, n, 1 << i, **kw)
        c, v = res[0], res[1]
        levels.append(c)
        if i == 0 and p.feedback == "atrous0":
            hist_rgb = c
        if last and p.tonemap and not fuse_inv:
            c = tonemap(c, inverse=True, k=p.tm_k)
            if p.half:
                c = quantize_half(c)
    if p.levels == 0 and p.tonemap:
        c = tonemap(c, inverse=True, k=p.tm_k)
        if p.half:
            c = quantize_half(c)
    if p.feedback == "temporal":
        hist_rgb = t["rgb"]
    new = {"rgb": hist_rgb, "m1": t["m1"], "m2": t["m2"], "n": t["n"]}
    return c, new, {"temporal": t, "var": var, "levels": levels}


def set_threads(n: int) -> None:
    """Host threads of the oracle's parallel loops (results do not depend
    on it)."""
    _load().svo_set_threads(int(n))


def threads() -> int:
    return int(_load().svo_threads())
