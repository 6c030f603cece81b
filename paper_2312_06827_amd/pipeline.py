"""One denoiser instance: its history buffers and the per-frame sequence of
library calls (Section 3, steps 4 and 5, with the tone map of Section 3.4).

Per frame, all on one stream:
  sv_temporal  (tone map in, reproject, clamp, blend colour and moments)
  sv_variance
  sv_atrous / sv_atrous_sep at steps 1, 2, 4, ... (inverse tone map fused
  into the last level)
The colour history of the next frame is the level-0 output; the moment
history is the temporal output.  Buffers are double-buffered so that a
frame never writes what it reads.
"""

from __future__ import annotations

import contextlib
from dataclasses import dataclass
from typing import Callable, Dict, Optional

import numpy as np
import torch

from . import lib
from .lib import AtrousParams, GBuf, TemporalParams, VarianceParams


@dataclass(frozen=True)
class FilterConfig:
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
    use_id: bool = False
    tonemap: bool = False
    tm_k: float = 1.0
    separable: bool = False
    max_hist: int = 255
    min_hist: int = 4
    var_radius: int = 3
    feedback: str = "atrous0"  # colour history: level-0 output or "temporal"

    def temporal(self) -> TemporalParams:
        return TemporalParams(self.alpha, self.alpha_m, self.gamma, self.tau_z, self.tau_n,
                              self.tm_k, self.max_hist, self.clamp, self.use_id, self.tonemap)

    def variance(self) -> VarianceParams:
        return VarianceParams(self.sigma_z, self.sigma_n, self.eps_z, self.min_hist,
                              self.var_radius)

    def atrous(self, inv_tonemap: bool = False) -> AtrousParams:
        return AtrousParams(self.sigma_z, self.sigma_n, self.sigma_l, self.eps_z, self.eps_l,
                            self.tm_k, False, inv_tonemap)


# The filter settings of the workloads: plain (static camera) and the
# paper's final configuration (clamp + tone map, with 2D or separable blur).
PLAIN = FilterConfig()
MOTION = FilterConfig(clamp=True, tonemap=True, use_id=True)
MOTION_SEP = FilterConfig(clamp=True, tonemap=True, use_id=True, separable=True)


@dataclass
class FrameInputs:
    """Device planes of one frame."""
    rgb: torch.Tensor          # (3, H, W) noisy radiance
    g: GBuf                    # current G-buffer
    mv: torch.Tensor           # (2, H, W) backward motion
    prev: GBuf                 # previous frame's z, n, id

    @staticmethod
    def from_numpy(fr: Dict[str, np.ndarray], device="cuda") -> "FrameInputs":
        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return FrameInputs(
            rgb=t(fr["rgb"]),
            g=GBuf(t(fr["z"]), t(fr["dzdx"]), t(fr["dzdy"]), t(fr["n"]), t(fr["id"])),
            mv=t(fr["mv"]),
            prev=GBuf(t(fr["prev_z"]), None, None, t(fr["prev_n"]), t(fr["prev_id"])),
        )


class Denoiser:
    def __init__(self, height: int, width: int, cfg: FilterConfig = PLAIN,
                 dtype: torch.dtype = torch.float32, device: str = "cuda"):
        lib.load()
        self.H, self.W, self.cfg, self.dtype = height, width, cfg, dtype
        dev = torch.device(device)
        rgb = lambda: torch.zeros((3, height, width), dtype=dtype, device=dev)
        f32 = lambda: torch.zeros((height, width), dtype=torch.float32, device=dev)
        u8 = lambda: torch.zeros((height, width), dtype=torch.uint8, device=dev)
        self.c_hist = [rgb(), rgb()]
        self.m1 = [f32(), f32()]
        self.m2 = [f32(), f32()]
        self.n = [u8(), u8()]
        self.t_rgb = [rgb(), rgb()]  # temporal output (double-buffered for "temporal" feedback)
        self.var = f32()
        self.lvl = [rgb(), rgb()]
        self.lvl_var = [f32(), f32()]
        self.scratch = rgb() if cfg.separable else None
        self.out = rgb()
        self.k = 0  # index of the current history buffers
        self.frames = 0

    def reset(self):
        for t in self.c_hist + self.m1 + self.m2 + self.n + self.t_rgb:
            t.zero_()
        self.k = 0
        self.frames = 0

    def state(self) -> Dict[str, torch.Tensor]:
        """The history the next frame will read."""
        k = self.k
        c = self.t_rgb[k] if self.cfg.feedback == "temporal" else self.c_hist[k]
        return {"rgb": c, "m1": self.m1[k], "m2": self.m2[k], "n": self.n[k]}

    def frame(self, inp: FrameInputs, alpha_map: Optional[torch.Tensor] = None,
              kappa: Optional[torch.Tensor] = None, stream=None,
              timer: Optional[Callable[[str], contextlib.AbstractContextManager]] = None
              ) -> torch.Tensor:
        """Enqueue one frame; returns the output tensor (valid once the
        stream reaches it; overwritten by the next frame).  `timer(name)`,
        if given, wraps each library call (for per-kernel events)."""
        cfg, k, k1 = self.cfg, self.k, 1 - self.k
        tm = timer if timer is not None else (lambda name: contextlib.nullcontext())
        hist = self.t_rgb[k] if cfg.feedback == "temporal" else self.c_hist[k]
        t_out = self.t_rgb[k1]
        with tm("temporal"):
            lib.sv_temporal(inp.rgb, inp.g, inp.mv, inp.prev, hist, self.m1[k], self.m2[k],
                            self.n[k], t_out, self.m1[k1], self.m2[k1], self.n[k1],
                            cfg.temporal(), alpha_map=alpha_map, stream=stream)
        with tm("variance"):
            lib.sv_variance(self.m1[k1], self.m2[k1], self.n[k1], inp.g, self.var,
                            cfg.variance(), stream=stream)
        c, v = t_out, self.var
        L = cfg.levels
        for i in range(L):
            last = i == L - 1
            fuse_inv = cfg.tonemap and last and not (i == 0 and cfg.feedback == "atrous0")
            if i == 0 and cfg.feedback == "atrous0":
                dst = self.c_hist[k1]
            elif last:
                dst = self.out
            else:
                dst = self.lvl[i % 2]
            dst_var = None if last else self.lvl_var[i % 2]
            p = cfg.atrous(inv_tonemap=fuse_inv)
            if cfg.separable:
                with tm(f"atrous_sep{i}"):
                    lib.sv_atrous_sep(c, v, inp.g, self.scratch, dst, dst_var, 1 << i, p,
                                      kappa=kappa, stream=stream)
            else:
                with tm(f"atrous{i}"):
                    lib.sv_atrous(c, v, inp.g, dst, dst_var, 1 << i, p, kappa=kappa,
                                  stream=stream)
            c, v = dst, dst_var
        if cfg.tonemap and (L == 0 or (L == 1 and cfg.feedback == "atrous0")):
            lib.sv_tonemap(c, self.out, inverse=True, k=cfg.tm_k, stream=stream)
            c = self.out
        elif c is not self.out:
            self.out.copy_(c)
        self.k = k1
        self.frames += 1
        return self.out

    def intermediates(self) -> Dict[str, torch.Tensor]:
        """Views of the last frame's temporal output, moments and variance."""
        k = self.k
        return {"t_rgb": self.t_rgb[k], "m1": self.m1[k], "m2": self.m2[k], "n": self.n[k],
                "var": self.var, "level0": self.c_hist[k]}
