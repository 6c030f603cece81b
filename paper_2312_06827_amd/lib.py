"""ctypes binding of ``libsv.so`` (C ABI in ``include/sv.h``).

Argument marshalling only: every step runs in the library's HIP kernels.
Planes are torch tensors on the GPU: a 2-D ``(H, W)`` view (row pitch =
``stride(0)``, unit column stride) or, for colour and normals, a ``(3, H, W)``
tensor whose three planes share that layout.  ``float32`` planes select
``SV_F32`` storage, ``float16`` planes ``SV_F16``.  Calls are enqueued on
torch's current stream unless ``stream`` (a ``torch.cuda.Stream``) is given.

There is no CPU fallback: loading fails loudly when the library is missing,
and CPU tensors are rejected.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Union

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsv.so")

SV_OK, SV_EINVAL, SV_EALIAS, SV_EDTYPE, SV_EHIP, SV_EUNSUPPORTED, SV_ETOOBIG = range(7)
SV_F32, SV_F16 = 0, 1
SV_TM_LUMA, SV_TM_CHANNEL, SV_TM_PAPER = 0, 1, 2
SV_T_CLAMP, SV_T_USE_ID, SV_T_TONEMAP_IN, SV_T_CLIP = 1, 2, 4, 8
SV_A_UNIT_WEIGHTS, SV_A_INV_TONEMAP = 1, 2
SV_V_LISTED = 1
SV_CTL_LEVELS_MASK, SV_CTL_SHIFT = 15, 16
SV_BR_SHIFT, SV_BR_TABLE = 1, 2

_vp = ctypes.c_void_p


class sv_dims(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("h", ctypes.c_int32), ("pitch", ctypes.c_int32)]


class sv_rgb(ctypes.Structure):
    _fields_ = [("r", _vp), ("g", _vp), ("b", _vp)]


class sv_gbuf(ctypes.Structure):
    _fields_ = [("z", _vp), ("dzdx", _vp), ("dzdy", _vp), ("nx", _vp), ("ny", _vp),
                ("nz", _vp), ("id", _vp)]


class sv_tm_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_float), ("weight", ctypes.c_float), ("mode", ctypes.c_int32)]


class sv_temporal_io(ctypes.Structure):
    _fields_ = [("cur", sv_rgb), ("g", sv_gbuf), ("mvx", _vp), ("mvy", _vp),
                ("prev", sv_gbuf), ("hist", sv_rgb), ("hist_m1", _vp), ("hist_m2c", _vp),
                ("hist_n", _vp), ("out", sv_rgb), ("out_m1", _vp), ("out_m2c", _vp),
                ("out_n", _vp), ("alpha_map", _vp), ("mlp", _vp), ("albedo", sv_rgb),
                ("kappa_out", _vp), ("alpha_out", _vp), ("var", _vp), ("var_work", _vp),
                ("var_min_hist", ctypes.c_int32)]


class sv_temporal_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("alpha_m", ctypes.c_float),
                ("gamma", ctypes.c_float), ("tau_z", ctypes.c_float),
                ("tau_n", ctypes.c_float), ("tm_k", ctypes.c_float),
                ("max_hist", ctypes.c_int32), ("flags", ctypes.c_int32)]


class sv_variance_params(ctypes.Structure):
    _fields_ = [("sigma_z", ctypes.c_float), ("sigma_n", ctypes.c_float),
                ("eps_z", ctypes.c_float), ("min_hist", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("flags", ctypes.c_int32)]


class sv_atrous_params(ctypes.Structure):
    _fields_ = [("sigma_z", ctypes.c_float), ("sigma_n", ctypes.c_float),
                ("sigma_l", ctypes.c_float), ("eps_z", ctypes.c_float),
                ("eps_l", ctypes.c_float), ("tm_k", ctypes.c_float),
                ("flags", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("tile_rows", ctypes.c_int32)]


class sv_denoiser(ctypes.Structure):
    _fields_ = [("hist", sv_rgb * 2), ("m1", _vp * 2), ("m2c", _vp * 2), ("n", _vp * 2),
                ("temporal", sv_rgb), ("var", _vp), ("var_work", _vp), ("level", sv_rgb * 2),
                ("level_var", _vp * 2), ("scratch", sv_rgb), ("out", sv_rgb),
                ("cur", ctypes.c_int32), ("kappa", _vp)]


class sv_frame_in(ctypes.Structure):
    _fields_ = [("cur", sv_rgb), ("g", sv_gbuf), ("mvx", _vp), ("mvy", _vp),
                ("prev", sv_gbuf), ("alpha_map", _vp), ("kappa", _vp), ("mlp", _vp),
                ("albedo", sv_rgb), ("blur_ctl", _vp)]


class sv_grad_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_float), ("tau_z", ctypes.c_float),
                ("sigma_z", ctypes.c_float), ("levels", ctypes.c_int32)]


class sv_blur_rule(ctypes.Structure):
    _fields_ = [("rough_shift", ctypes.c_float), ("angle_shift", ctypes.c_float),
                ("rough_none", ctypes.c_float), ("rough_one", ctypes.c_float),
                ("it_none", ctypes.c_int32), ("it_one", ctypes.c_int32),
                ("it_rest", ctypes.c_int32), ("flags", ctypes.c_int32)]


class sv_frame_params(ctypes.Structure):
    _fields_ = [("temporal", sv_temporal_params), ("variance", sv_variance_params),
                ("atrous", sv_atrous_params), ("levels", ctypes.c_int32),
                ("separable", ctypes.c_int32), ("feedback", ctypes.c_int32),
                ("level_persistent", ctypes.c_int32 * 10),
                ("level_blocks_per_cu", ctypes.c_int32 * 10),
                ("level_tile_rows", ctypes.c_int32 * 10)]


_P = ctypes.POINTER
class sv_mlp(ctypes.Structure):
    _fields_ = [("params", _vp), ("wq", _vp), ("mu", _vp), ("inv_s", _vp)]


class sv_adam_params(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


SV_MLP_IN, SV_MLP_HIDDEN, SV_MLP_PARAMS = 14, 32, 1602

EXPORTS = {
    "sv_tonemap": ([_P(sv_rgb), _P(sv_rgb), sv_dims, ctypes.c_int, ctypes.c_int,
                    _P(sv_tm_params), _vp], ctypes.c_int),
    "sv_clamp": ([_P(sv_rgb), _P(sv_rgb), _P(sv_rgb), _vp, sv_dims, ctypes.c_int,
                  ctypes.c_float, _vp], ctypes.c_int),
    "sv_clip": ([_P(sv_rgb), _P(sv_rgb), _P(sv_rgb), _vp, sv_dims, ctypes.c_int,
                  ctypes.c_float, _vp], ctypes.c_int),
    "sv_temporal": ([_P(sv_temporal_io), sv_dims, ctypes.c_int, _P(sv_temporal_params), _vp],
                    ctypes.c_int),
    "sv_variance": ([_vp, _vp, _vp, _P(sv_gbuf), _vp, _vp, sv_dims, ctypes.c_int,
                     _P(sv_variance_params), _vp], ctypes.c_int),
    "sv_variance_work_bytes": ([sv_dims], ctypes.c_size_t),
    "sv_variance_noalloc": ([_vp, _vp, _vp, _P(sv_gbuf), _vp, sv_dims, ctypes.c_int,
                             _P(sv_variance_params), _vp], ctypes.c_int),
    "sv_atrous": ([_P(sv_rgb), _vp, _P(sv_gbuf), _vp, _P(sv_rgb), _vp, ctypes.c_int32,
                   sv_dims, ctypes.c_int, _P(sv_atrous_params), _vp], ctypes.c_int),
    "sv_atrous_sep": ([_P(sv_rgb), _vp, _P(sv_gbuf), _vp, _P(sv_rgb), _P(sv_rgb), _vp,
                       ctypes.c_int32, sv_dims, ctypes.c_int, _P(sv_atrous_params), _vp],
                      ctypes.c_int),
    "sv_atrous_adaptive": ([_P(sv_rgb), _vp, _P(sv_gbuf), _vp, _vp, _P(sv_rgb), _P(sv_rgb), _vp,
                            ctypes.c_int32, ctypes.c_int32, sv_dims, ctypes.c_int,
                            _P(sv_atrous_params), _vp], ctypes.c_int),
    "sv_grad_work_bytes": ([sv_dims], ctypes.c_size_t),
    "sv_temporal_gradient": ([_P(sv_rgb), _P(sv_rgb), _vp, _vp, _vp, _vp, _P(sv_gbuf), _vp, _vp,
                              _vp, sv_dims, ctypes.c_int, _P(sv_grad_params), _vp], ctypes.c_int),
    "sv_compose": ([_P(sv_rgb), _P(sv_rgb), _P(sv_rgb), _P(sv_rgb), sv_dims, ctypes.c_int, _vp],
                   ctypes.c_int),
    "sv_blur_control": ([_vp, _vp, _vp, sv_dims, _P(sv_blur_rule), _vp], ctypes.c_int),
    "sv_denoise_frame": ([_P(sv_frame_in), _P(sv_denoiser), sv_dims, ctypes.c_int,
                          _P(sv_frame_params), _vp], ctypes.c_int),
    "sv_mlp_features": ([_P(sv_temporal_io), _P(sv_rgb), _P(sv_mlp), _vp, _P(sv_rgb), sv_dims,
                         ctypes.c_int, _P(sv_temporal_params), _vp], ctypes.c_int),
    "sv_mlp_forward": ([_P(sv_mlp), _vp, _vp, _vp, sv_dims, _vp], ctypes.c_int),
    "sv_mlp_backward": ([_P(sv_mlp), _vp, _vp, _vp, ctypes.c_float, _vp, _vp, sv_dims, _vp],
                        ctypes.c_int),
    "sv_mlp_backward_work_bytes": ([sv_dims], ctypes.c_size_t),
    "sv_adam": ([_vp, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _P(sv_adam_params),
                 _vp], ctypes.c_int),
    "sv_mlp_alpha_grad": ([_P(sv_rgb), _P(sv_rgb), _P(sv_rgb), _P(sv_rgb), _vp, _vp, _vp,
                           ctypes.c_float, _vp, sv_dims, ctypes.c_int, _vp], ctypes.c_int),
    "sv_atrous_kappa_grad": ([_P(sv_rgb), _vp, _P(sv_gbuf), _vp, _P(sv_rgb), _P(sv_rgb), _vp,
                              ctypes.c_int32, sv_dims, ctypes.c_int, _P(sv_atrous_params), _vp],
                             ctypes.c_int),
    "sv_batch_create": ([_P(sv_dims), _P(_P(sv_denoiser)), ctypes.c_int32, ctypes.c_int,
                         _P(sv_frame_params), _P(_vp)], ctypes.c_int),
    "sv_batch_create_each": ([_P(sv_dims), _P(_P(sv_denoiser)), ctypes.c_int32, ctypes.c_int,
                              _P(sv_frame_params), _P(_vp)], ctypes.c_int),
    "sv_batch_frame": ([_vp, _P(sv_frame_in), _vp], ctypes.c_int),
    "sv_batch_passes": ([_vp], ctypes.c_int),
    "sv_batch_set_direct": ([_vp, ctypes.c_int32], ctypes.c_int),
    "sv_batch_destroy": ([_vp], None),
    "sv_struct_sizes": ([_P(ctypes.c_size_t), ctypes.c_int32], ctypes.c_int),
    "sv_status_str": ([ctypes.c_int], ctypes.c_char_p),
    "sv_version": ([], ctypes.c_int),
    "sv_last_hip_error": ([], ctypes.c_int),
    "sv_probe_copy": ([_vp, _vp, ctypes.c_size_t, _vp], ctypes.c_int),
    "sv_probe_issue": ([ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int32, _vp], ctypes.c_int),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_2312_06827_amd._build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (args, res) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class SVError(RuntimeError):
    def __init__(self, fn: str, status: int):
        lib = load()
        msg = lib.sv_status_str(status).decode()
        if status == SV_EHIP:
            msg += f" (hipError {lib.sv_last_hip_error()})"
        super().__init__(f"{fn}: {msg}")
        self.status = status


def _check(fn: str, status: int):
    if status != SV_OK:
        raise SVError(fn, status)


# ---- marshalling helpers ----------------------------------------------------

Planes = Union[torch.Tensor, Sequence[torch.Tensor]]


def _plane_ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected (the library takes device pointers)")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("a plane must be a 2-D (H, W) view with unit column stride")
    return t.data_ptr()


def _planes3(x: Planes):
    if isinstance(x, torch.Tensor):
        if x.dim() != 3 or x.shape[0] != 3:
            raise ValueError("colour must be a (3, H, W) tensor or three planes")
        return x[0], x[1], x[2]
    r, g, b = x
    return r, g, b


def _rgb(x: Planes) -> sv_rgb:
    r, g, b = _planes3(x)
    return sv_rgb(_plane_ptr(r), _plane_ptr(g), _plane_ptr(b))


def dims_of(t: torch.Tensor) -> sv_dims:
    p = t if t.dim() == 2 else t[0]
    return sv_dims(p.shape[1], p.shape[0], p.stride(0))


def dtype_of(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return SV_F32
    if t.dtype == torch.float16:
        return SV_F16
    raise ValueError(f"unsupported storage type {t.dtype}")


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


@dataclass
class GBuf:
    """G-buffer planes: depth, its screen gradients, normals (3, H, W), ids."""
    z: torch.Tensor
    dzdx: Optional[torch.Tensor]
    dzdy: Optional[torch.Tensor]
    n: torch.Tensor
    id: Optional[torch.Tensor] = None

    def c(self) -> sv_gbuf:
        nx, ny, nz = _planes3(self.n)
        return sv_gbuf(_plane_ptr(self.z), _plane_ptr(self.dzdx), _plane_ptr(self.dzdy),
                       _plane_ptr(nx), _plane_ptr(ny), _plane_ptr(nz), _plane_ptr(self.id))


@dataclass
class TemporalParams:
    alpha: float = 0.2
    alpha_m: float = 0.2
    gamma: float = 1.0
    tau_z: float = 0.1
    tau_n: float = 0.9
    tm_k: float = 1.0
    max_hist: int = 255
    clamp: bool = False
    use_id: bool = False
    tonemap: bool = False
    clip: bool = False  # clip the history toward the box centre instead of clamping

    def c(self) -> sv_temporal_params:
        flags = ((SV_T_CLAMP if self.clamp else 0) | (SV_T_USE_ID if self.use_id else 0)
                 | (SV_T_TONEMAP_IN if self.tonemap else 0) | (SV_T_CLIP if self.clip else 0))
        return sv_temporal_params(self.alpha, self.alpha_m, self.gamma, self.tau_z, self.tau_n,
                                  self.tm_k, self.max_hist, flags)


@dataclass
class VarianceParams:
    sigma_z: float = 1.0
    sigma_n: float = 128.0
    eps_z: float = 1e-10
    min_hist: int = 4
    radius: int = 3
    listed: bool = False  # the temporal step already wrote the pointwise part and the list

    def c(self) -> sv_variance_params:
        return sv_variance_params(self.sigma_z, self.sigma_n, self.eps_z, self.min_hist,
                                  self.radius, SV_V_LISTED if self.listed else 0)


@dataclass
class AtrousParams:
    sigma_z: float = 1.0
    sigma_n: float = 128.0
    sigma_l: float = 4.0
    eps_z: float = 1e-10
    eps_l: float = 1e-10
    tm_k: float = 1.0
    unit_weights: bool = False
    inv_tonemap: bool = False
    persistent: int = -1      # launch shape: -1 default, 0 / 1
    blocks_per_cu: int = 0    # persistent workgroups per CU, 0 default
    tile_rows: int = 0        # LDS tile height (5x5: 1 / 2; separable: 6 / 16), 0 default

    def c(self) -> sv_atrous_params:
        flags = ((SV_A_UNIT_WEIGHTS if self.unit_weights else 0)
                 | (SV_A_INV_TONEMAP if self.inv_tonemap else 0))
        return sv_atrous_params(self.sigma_z, self.sigma_n, self.sigma_l, self.eps_z,
                                self.eps_l, self.tm_k, flags, self.persistent,
                                self.blocks_per_cu, self.tile_rows)


# ---- the calls ------------------------------------------------------------------

def sv_tonemap(inp: Planes, out: Planes, inverse: bool = False, k: float = 1.0,
               weight: float = 1.0, mode: int = SV_TM_LUMA, stream=None):
    r = _planes3(inp)[0]
    p = sv_tm_params(k, weight, mode)
    _check("sv_tonemap", load().sv_tonemap(
        ctypes.byref(_rgb(inp)), ctypes.byref(_rgb(out)), dims_of(r), dtype_of(r),
        int(bool(inverse)), ctypes.byref(p), _stream(stream)))


def sv_clamp(hist: Planes, cur: Planes, out: Planes, gamma: float,
             z: Optional[torch.Tensor] = None, stream=None):
    r = _planes3(cur)[0]
    _check("sv_clamp", load().sv_clamp(
        ctypes.byref(_rgb(hist)), ctypes.byref(_rgb(cur)), ctypes.byref(_rgb(out)),
        _plane_ptr(z), dims_of(r), dtype_of(r), float(gamma), _stream(stream)))


def sv_clip(hist: Planes, cur: Planes, out: Planes, gamma: float,
            z: Optional[torch.Tensor] = None, stream=None):
    r = _planes3(cur)[0]
    _check("sv_clip", load().sv_clip(
        ctypes.byref(_rgb(hist)), ctypes.byref(_rgb(cur)), ctypes.byref(_rgb(out)),
        _plane_ptr(z), dims_of(r), dtype_of(r), float(gamma), _stream(stream)))


def sv_temporal(cur: Planes, g: GBuf, mv: Planes, prev: GBuf, hist: Planes,
                hist_m1: torch.Tensor, hist_m2c: torch.Tensor, hist_n: torch.Tensor,
                out: Planes, out_m1: torch.Tensor, out_m2c: torch.Tensor, out_n: torch.Tensor,
                params: TemporalParams, alpha_map: Optional[torch.Tensor] = None, stream=None,
                mlp: Optional["MLP"] = None, albedo: Optional[Planes] = None,
                kappa_out: Optional[torch.Tensor] = None,
                alpha_out: Optional[torch.Tensor] = None,
                var: Optional[torch.Tensor] = None, var_work: Optional[torch.Tensor] = None,
                var_min_hist: int = 4):
    """m2c planes hold the central moment E[L^2] - E[L]^2.  With `mlp` the
    network runs inside the step (needs albedo; alpha_map is ignored).
    With `var` (and its sv_variance workspace) the variance estimate's
    pointwise part is written here (finish with VarianceParams(listed=True))."""
    mvx, mvy = mv[0], mv[1]
    mc = None if mlp is None else mlp.c()
    io = sv_temporal_io(_rgb(cur), g.c(), _plane_ptr(mvx), _plane_ptr(mvy), prev.c(),
                        _rgb(hist), _plane_ptr(hist_m1), _plane_ptr(hist_m2c),
                        _plane_ptr(hist_n), _rgb(out), _plane_ptr(out_m1), _plane_ptr(out_m2c),
                        _plane_ptr(out_n), _plane_ptr(alpha_map),
                        None if mc is None else ctypes.addressof(mc),
                        _rgb(albedo) if albedo is not None else sv_rgb(),
                        _plane_ptr(kappa_out), _plane_ptr(alpha_out), _plane_ptr(var),
                        None if var_work is None else var_work.data_ptr(), int(var_min_hist))
    r = _planes3(cur)[0]
    pc = params.c()
    _check("sv_temporal", load().sv_temporal(ctypes.byref(io), dims_of(r), dtype_of(r),
                                             ctypes.byref(pc), _stream(stream)))


def variance_workspace(like: torch.Tensor) -> torch.Tensor:
    """A zeroed device workspace for sv_variance on planes shaped like `like`."""
    nbytes = load().sv_variance_work_bytes(dims_of(like))
    if nbytes == 0:
        raise ValueError("invalid dimensions")
    return torch.zeros((nbytes + 3) // 4, dtype=torch.int32, device=like.device)


def sv_variance(m1: torch.Tensor, m2c: torch.Tensor, n: torch.Tensor, g: GBuf,
                var: torch.Tensor, params: VarianceParams, work: torch.Tensor, stream=None):
    """`work`: a workspace from variance_workspace() (zeroed; stays zeroed)."""
    gc = g.c()
    pc = params.c()
    if work.numel() * work.element_size() < load().sv_variance_work_bytes(dims_of(m1)):
        raise ValueError("variance workspace too small")
    _check("sv_variance", load().sv_variance(
        _plane_ptr(m1), _plane_ptr(m2c), _plane_ptr(n), ctypes.byref(gc), _plane_ptr(var),
        work.data_ptr(), dims_of(m1), dtype_of(g.z), ctypes.byref(pc), _stream(stream)))


def sv_variance_noalloc(m1: torch.Tensor, m2c: torch.Tensor, n: torch.Tensor, g: GBuf,
                        var: torch.Tensor, params: VarianceParams, stream=None):
    """sv_variance with the library's fixed workspace (no allocation)."""
    gc = g.c()
    pc = params.c()
    _check("sv_variance_noalloc", load().sv_variance_noalloc(
        _plane_ptr(m1), _plane_ptr(m2c), _plane_ptr(n), ctypes.byref(gc), _plane_ptr(var),
        dims_of(m1), dtype_of(g.z), ctypes.byref(pc), _stream(stream)))


def sv_atrous(c_in: Planes, var_in: torch.Tensor, g: GBuf, c_out: Planes,
              var_out: Optional[torch.Tensor], step: int, params: AtrousParams,
              kappa: Optional[torch.Tensor] = None, stream=None):
    r = _planes3(c_in)[0]
    gc = g.c()
    pc = params.c()
    _check("sv_atrous", load().sv_atrous(
        ctypes.byref(_rgb(c_in)), _plane_ptr(var_in), ctypes.byref(gc), _plane_ptr(kappa),
        ctypes.byref(_rgb(c_out)), _plane_ptr(var_out), int(step), dims_of(r), dtype_of(r),
        ctypes.byref(pc), _stream(stream)))


def sv_atrous_sep(c_in: Planes, var_in: torch.Tensor, g: GBuf, scratch: Optional[Planes],
                  c_out: Planes, var_out: Optional[torch.Tensor], step: int, params: AtrousParams,
                  kappa: Optional[torch.Tensor] = None, stream=None):
    """scratch None: both passes in one kernel (steps 1..16)."""
    r = _planes3(c_in)[0]
    gc = g.c()
    pc = params.c()
    sc = None if scratch is None else ctypes.byref(_rgb(scratch))
    _check("sv_atrous_sep", load().sv_atrous_sep(
        ctypes.byref(_rgb(c_in)), _plane_ptr(var_in), ctypes.byref(gc), _plane_ptr(kappa),
        sc, ctypes.byref(_rgb(c_out)), _plane_ptr(var_out), int(step),
        dims_of(r), dtype_of(r), ctypes.byref(pc), _stream(stream)))


def sv_atrous_adaptive(c_in: Planes, var_in: torch.Tensor, g: GBuf, ctl: torch.Tensor,
                       scratch: Optional[Planes], c_out: Planes,
                       var_out: Optional[torch.Tensor], level: int, separable: bool,
                       params: AtrousParams, kappa: Optional[torch.Tensor] = None, stream=None):
    """Level `level` with per-pixel control bytes `ctl` (uint8 plane)."""
    r = _planes3(c_in)[0]
    gc = g.c()
    pc = params.c()
    sc = None if scratch is None else ctypes.byref(_rgb(scratch))
    _check("sv_atrous_adaptive", load().sv_atrous_adaptive(
        ctypes.byref(_rgb(c_in)), _plane_ptr(var_in), ctypes.byref(gc), _plane_ptr(kappa),
        _plane_ptr(ctl), sc, ctypes.byref(_rgb(c_out)), _plane_ptr(var_out), int(level),
        int(bool(separable)), dims_of(r), dtype_of(r), ctypes.byref(pc), _stream(stream)))


@dataclass
class BlurRule:
    """Thresholds of the adaptive blur: the coarser start above a roughness
    or shadow angle, and the roughness -> level count table."""
    rough_shift: float = 0.2
    angle_shift: float = 6.0
    rough_none: float = 0.0
    rough_one: float = 0.05
    it_none: int = 0
    it_one: int = 1
    it_rest: int = 15
    shift: bool = True
    table: bool = True

    def c(self) -> sv_blur_rule:
        flags = (SV_BR_SHIFT if self.shift else 0) | (SV_BR_TABLE if self.table else 0)
        return sv_blur_rule(self.rough_shift, self.angle_shift, self.rough_none, self.rough_one,
                            self.it_none, self.it_one, self.it_rest, flags)


def sv_blur_control(roughness: Optional[torch.Tensor], shadow_angle: Optional[torch.Tensor],
                    ctl: torch.Tensor, rule: BlurRule, stream=None):
    rc = rule.c()
    _check("sv_blur_control", load().sv_blur_control(
        _plane_ptr(roughness), _plane_ptr(shadow_angle), _plane_ptr(ctl), dims_of(ctl),
        ctypes.byref(rc), _stream(stream)))


def gradient_workspace(like: torch.Tensor) -> torch.Tensor:
    """Device workspace of sv_temporal_gradient for planes shaped like `like`."""
    n = load().sv_grad_work_bytes(dims_of(like))
    return torch.empty(max(n, 1), dtype=torch.uint8, device=like.device)


def sv_temporal_gradient(prev: Planes, reshade: Planes, fmv: torch.Tensor, fz: torch.Tensor,
                         pick: torch.Tensor, g: GBuf, alpha_map: torch.Tensor,
                         work: torch.Tensor, alpha: float = 0.2, tau_z: float = 0.1,
                         sigma_z: float = 1.0, levels: int = 3,
                         lam: Optional[torch.Tensor] = None, stream=None):
    """alpha_map <- the blend factor raised where the previous frame's
    samples, traced again, changed.  pick and lam are (ceil(H/3), ceil(W/3))
    contiguous."""
    r = _planes3(prev)[0]
    gc = g.c()
    p = sv_grad_params(alpha, tau_z, sigma_z, levels)
    _check("sv_temporal_gradient", load().sv_temporal_gradient(
        ctypes.byref(_rgb(prev)), ctypes.byref(_rgb(reshade)), _plane_ptr(fmv[0]),
        _plane_ptr(fmv[1]), _plane_ptr(fz), _plane_ptr(pick), ctypes.byref(gc),
        _plane_ptr(alpha_map), _plane_ptr(lam), work.data_ptr(), dims_of(r), dtype_of(r),
        ctypes.byref(p), _stream(stream)))


def sv_compose(direct: Planes, shadow: Optional[Planes], spec: Optional[Planes], out: Planes,
               stream=None):
    """out = direct * shadow + spec per colour channel."""
    r = _planes3(direct)[0]
    opt = lambda p: None if p is None else ctypes.byref(_rgb(p))
    _check("sv_compose", load().sv_compose(
        ctypes.byref(_rgb(direct)), opt(shadow), opt(spec), ctypes.byref(_rgb(out)),
        dims_of(r), dtype_of(r), _stream(stream)))


# ---- learned blend factor and edge scale -------------------------------------

class MLP:
    """Device parameters of the per-pixel network: binary32 flat vector
    (SV_MLP_PARAMS, order W1 b1 W2 b2 W3 b3, matrices [out][in]), its
    bfloat16 mirror, the feature standardisation, and Adam's moments."""

    def __init__(self, params, mu, inv_s, device="cuda"):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous()
        self.params = f(params)
        if self.params.numel() != SV_MLP_PARAMS:
            raise ValueError(f"expected {SV_MLP_PARAMS} parameters")
        self.mu, self.inv_s = f(mu), f(inv_s)
        if self.mu.numel() != SV_MLP_IN or self.inv_s.numel() != SV_MLP_IN:
            raise ValueError("standardisation needs 14 means and 14 inverse scales")
        self.wq = torch.empty(SV_MLP_PARAMS, dtype=torch.int16, device=device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.sync_mirror()

    def sync_mirror(self):
        """Refresh the bfloat16 mirror from the binary32 parameters (round to
        nearest even, torch's conversion)."""
        self.wq.copy_(self.params.to(torch.bfloat16).view(torch.int16))

    def c(self) -> sv_mlp:
        return sv_mlp(self.params.data_ptr(), self.wq.data_ptr(), self.mu.data_ptr(),
                      self.inv_s.data_ptr())


def feature_rows(H: int, W: int, device="cuda") -> torch.Tensor:
    """Buffer for sv_mlp_features: H*W rows of 16 bfloat16 (as int16)."""
    return torch.empty((H * W, 16), dtype=torch.int16, device=device)


def sv_mlp_features(cur: Planes, g: GBuf, mv: Planes, prev: GBuf, hist: Planes,
                    hist_m1: torch.Tensor, hist_m2c: torch.Tensor, hist_n: torch.Tensor,
                    albedo: Planes, mlp: MLP, feat: torch.Tensor, params: TemporalParams,
                    hist_out: Optional[Planes] = None, stream=None):
    r = _planes3(cur)[0]
    d = dims_of(r)
    if feat.numel() * feat.element_size() < d.w * d.h * 32 or not feat.is_contiguous():
        raise ValueError("feature buffer too small or not contiguous")
    mvx, mvy = mv[0], mv[1]
    io = sv_temporal_io(_rgb(cur), g.c(), _plane_ptr(mvx), _plane_ptr(mvy), prev.c(),
                        _rgb(hist), _plane_ptr(hist_m1), _plane_ptr(hist_m2c),
                        _plane_ptr(hist_n), sv_rgb(), None, None, None, None)
    pc, mc = params.c(), mlp.c()
    ho = None if hist_out is None else ctypes.byref(_rgb(hist_out))
    _check("sv_mlp_features", load().sv_mlp_features(
        ctypes.byref(io), ctypes.byref(_rgb(albedo)), ctypes.byref(mc), feat.data_ptr(), ho,
        d, dtype_of(r), ctypes.byref(pc), _stream(stream)))


def sv_mlp_forward(mlp: MLP, feat: torch.Tensor, alpha: Optional[torch.Tensor],
                   kappa: Optional[torch.Tensor], like: torch.Tensor, stream=None):
    """alpha / kappa: binary32 planes shaped like `like` (either may be None)."""
    mc = mlp.c()
    _check("sv_mlp_forward", load().sv_mlp_forward(
        ctypes.byref(mc), feat.data_ptr(), _plane_ptr(alpha), _plane_ptr(kappa), dims_of(like),
        _stream(stream)))


def mlp_workspace(like: torch.Tensor) -> torch.Tensor:
    nbytes = load().sv_mlp_backward_work_bytes(dims_of(like))
    return torch.empty(max(1, nbytes // 4), dtype=torch.float32, device=like.device)


def sv_mlp_backward(mlp: MLP, feat: torch.Tensor, d_alpha: Optional[torch.Tensor],
                    d_kappa: Optional[torch.Tensor], grad: torch.Tensor, work: torch.Tensor,
                    like: torch.Tensor, scale: float = 1.0, stream=None):
    d = dims_of(like)
    if work.numel() * work.element_size() < load().sv_mlp_backward_work_bytes(d):
        raise ValueError("backward workspace too small")
    mc = mlp.c()
    _check("sv_mlp_backward", load().sv_mlp_backward(
        ctypes.byref(mc), feat.data_ptr(), _plane_ptr(d_alpha), _plane_ptr(d_kappa),
        float(scale), grad.data_ptr(), work.data_ptr(), d, _stream(stream)))


def sv_adam(mlp: MLP, grad: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
            stream=None):
    mlp.t += 1
    p = sv_adam_params(lr, beta1, beta2, eps)
    _check("sv_adam", load().sv_adam(
        mlp.params.data_ptr(), mlp.wq.data_ptr(), mlp.m.data_ptr(), mlp.v.data_ptr(),
        grad.data_ptr(), SV_MLP_PARAMS, mlp.t, ctypes.byref(p), _stream(stream)))


def sv_mlp_alpha_grad(c_t: Planes, cur: Planes, hist: Planes, y: Planes, alpha: torch.Tensor,
                      n: torch.Tensor, z: torch.Tensor, d_alpha: torch.Tensor, tm_k: float = 1.0,
                      stream=None):
    r = _planes3(c_t)[0]
    _check("sv_mlp_alpha_grad", load().sv_mlp_alpha_grad(
        ctypes.byref(_rgb(c_t)), ctypes.byref(_rgb(cur)), ctypes.byref(_rgb(hist)),
        ctypes.byref(_rgb(y)), _plane_ptr(alpha), _plane_ptr(n), _plane_ptr(z), float(tm_k),
        _plane_ptr(d_alpha), dims_of(r), dtype_of(r), _stream(stream)))


def sv_atrous_kappa_grad(c_in: Planes, var_in: torch.Tensor, g: GBuf, kappa: torch.Tensor,
                         y: Planes, d_kappa: torch.Tensor, step: int, params: AtrousParams,
                         ref: Optional[Planes] = None, stream=None):
    r = _planes3(c_in)[0]
    gc, pc = g.c(), params.c()
    rf = None if ref is None else ctypes.byref(_rgb(ref))
    _check("sv_atrous_kappa_grad", load().sv_atrous_kappa_grad(
        ctypes.byref(_rgb(c_in)), _plane_ptr(var_in), ctypes.byref(gc), _plane_ptr(kappa),
        ctypes.byref(_rgb(y)), rf, _plane_ptr(d_kappa), int(step), dims_of(r), dtype_of(r),
        ctypes.byref(pc), _stream(stream)))


def sv_probe_copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    _check("sv_probe_copy", load().sv_probe_copy(dst.data_ptr(), src.data_ptr(), nbytes,
                                                 _stream(stream)))


def sv_probe_issue(out: torch.Tensor, kind: int, iters: int, stream=None):
    """`out`: float32 device tensor of blocks * 256 elements."""
    if out.dtype != torch.float32 or out.numel() % 256 or not out.is_cuda:
        raise ValueError("out must be a float32 device tensor of blocks * 256 elements")
    _check("sv_probe_issue", load().sv_probe_issue(int(kind), int(iters), out.data_ptr(),
                                                   out.numel() // 256, _stream(stream)))


def sv_denoise_frame(fin: sv_frame_in, st: sv_denoiser, dims: sv_dims, dtype: int,
                     params: sv_frame_params, stream=None):
    """One frame through the native driver (structures prepared by the
    caller; see pipeline.Denoiser)."""
    _check("sv_denoise_frame", load().sv_denoise_frame(
        ctypes.byref(fin), ctypes.byref(st), dims, dtype, ctypes.byref(params),
        _stream(stream)))


def sv_version() -> int:
    return load().sv_version()
