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
import ctypes
import dataclasses
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
    clip: bool = False  # clip the history toward the box centre instead of clamping

    def temporal(self) -> TemporalParams:
        return TemporalParams(self.alpha, self.alpha_m, self.gamma, self.tau_z, self.tau_n,
                              self.tm_k, self.max_hist, self.clamp, self.use_id, self.tonemap,
                              self.clip)

    def variance(self) -> VarianceParams:
        return VarianceParams(self.sigma_z, self.sigma_n, self.eps_z, self.min_hist,
                              self.var_radius)

    def atrous(self, inv_tonemap: bool = False) -> AtrousParams:
        return AtrousParams(self.sigma_z, self.sigma_n, self.sigma_l, self.eps_z, self.eps_l,
                            self.tm_k, False, inv_tonemap)

    def frame_params(self, tiles=None) -> lib.sv_frame_params:
        """`tiles`: optional per-level launch shapes (persistent,
        blocks_per_cu[, tile_rows]), as the autotuner chooses them."""
        if self.feedback not in ("atrous0", "temporal"):
            raise ValueError(f"unknown feedback {self.feedback!r}")
        lp = (ctypes.c_int32 * 10)(*([-1] * 10))
        lb = (ctypes.c_int32 * 10)(*([0] * 10))
        lr = (ctypes.c_int32 * 10)(*([0] * 10))
        for i, shape in enumerate((tiles or [])[:10]):
            lp[i], lb[i] = shape[0], shape[1]
            if len(shape) > 2:
                lr[i] = shape[2]
        return lib.sv_frame_params(self.temporal().c(), self.variance().c(), self.atrous().c(),
                                   self.levels, int(self.separable),
                                   1 if self.feedback == "temporal" else 0, lp, lb, lr)


# The filter settings of the workloads: plain (static camera) and the
# paper's final configuration (clamp + tone map, with 2D or separable blur).
PLAIN = FilterConfig()
MOTION = FilterConfig(clamp=True, tonemap=True, use_id=True)
MOTION_SEP = FilterConfig(clamp=True, tonemap=True, use_id=True, separable=True)
# The two channels of Section 3: shadows without the tone map (Section 3.4
# applies it to the indirect specular channel only), four levels each (the
# paper's cascade).
SHADOW = FilterConfig(clamp=True, use_id=True, levels=4)
SPECULAR = FilterConfig(clamp=True, tonemap=True, use_id=True, levels=4)


@dataclass
class FrameInputs:
    """Device planes of one frame."""
    rgb: torch.Tensor          # (3, H, W) noisy radiance
    g: GBuf                    # current G-buffer
    mv: torch.Tensor           # (2, H, W) backward motion
    prev: GBuf                 # previous frame's z, n, id
    albedo: Optional[torch.Tensor] = None  # (3, H, W), for the learned mode
    blur_ctl: Optional[torch.Tensor] = None  # (H, W) uint8 control bytes: adaptive levels
    alpha_map: Optional[torch.Tensor] = None  # (H, W) binary32 blend factor (e.g. the gradient's)

    def c(self, alpha_map: Optional[torch.Tensor] = None,
          kappa: Optional[torch.Tensor] = None, mlp=None) -> lib.sv_frame_in:
        """mlp: a lib.sv_mlp structure (kept alive by the caller) for the
        learned mode."""
        if alpha_map is None:
            alpha_map = self.alpha_map
        key = (None if alpha_map is None else alpha_map.data_ptr(),
               None if kappa is None else kappa.data_ptr(),
               None if mlp is None else ctypes.addressof(mlp),
               None if self.blur_ctl is None else self.blur_ctl.data_ptr())
        cached = self.__dict__.get("_c")
        if cached is None or cached[0] != key:
            if mlp is not None and self.albedo is None:
                raise ValueError("the learned mode needs the albedo planes")
            fin = lib.sv_frame_in(lib._rgb(self.rgb), self.g.c(), lib._plane_ptr(self.mv[0]),
                                  lib._plane_ptr(self.mv[1]), self.prev.c(),
                                  lib._plane_ptr(alpha_map), lib._plane_ptr(kappa),
                                  None if mlp is None else ctypes.addressof(mlp),
                                  lib._rgb(self.albedo) if mlp is not None else lib.sv_rgb(),
                                  lib._plane_ptr(self.blur_ctl))
            self.__dict__["_c"] = cached = (key, fin)
        return cached[1]

    @staticmethod
    def from_numpy(fr: Dict[str, np.ndarray], device="cuda") -> "FrameInputs":
        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device)
        return FrameInputs(
            rgb=t(fr["rgb"]),
            g=GBuf(t(fr["z"]), t(fr["dzdx"]), t(fr["dzdy"]), t(fr["n"]), t(fr["id"])),
            mv=t(fr["mv"]),
            prev=GBuf(t(fr["prev_z"]), None, None, t(fr["prev_n"]), t(fr["prev_id"])),
            albedo=t(fr["albedo"]) if "albedo" in fr else None,
        )


class Denoiser:
    def __init__(self, height: int, width: int, cfg: FilterConfig = PLAIN,
                 dtype: torch.dtype = torch.float32, device: str = "cuda", tiles=None,
                 mlp: Optional[lib.MLP] = None):
        """mlp: run the learned network inside the temporal step (its alpha
        and kappa replace the constants)."""
        lib.load()
        self.H, self.W, self.cfg, self.dtype = height, width, cfg, dtype
        dev = torch.device(device)
        rgb = lambda: torch.zeros((3, height, width), dtype=dtype, device=dev)
        f32 = lambda: torch.zeros((height, width), dtype=torch.float32, device=dev)
        u8 = lambda: torch.zeros((height, width), dtype=torch.uint8, device=dev)
        self.c_hist = [rgb(), rgb()]
        self.m1 = [f32(), f32()]
        self.m2c = [f32(), f32()]  # central second moment
        self.n = [u8(), u8()]
        self.t_rgb = [rgb()]  # temporal output (the history itself under "temporal" feedback)
        self.var = f32()
        self.var_work = lib.variance_workspace(self.var)
        self.lvl = [rgb(), rgb()]
        self.lvl_var = [f32(), f32()]
        self.scratch = rgb() if cfg.separable else None
        self.out = rgb()
        self.frames = 0
        # the same buffers, as the native driver's structure
        R = lib._rgb
        scratch = R(self.scratch) if self.scratch is not None else lib.sv_rgb()
        self._st = lib.sv_denoiser(
            (lib.sv_rgb * 2)(R(self.c_hist[0]), R(self.c_hist[1])),
            (lib._vp * 2)(*[t.data_ptr() for t in self.m1]),
            (lib._vp * 2)(*[t.data_ptr() for t in self.m2c]),
            (lib._vp * 2)(*[t.data_ptr() for t in self.n]),
            R(self.t_rgb[0]), self.var.data_ptr(), self.var_work.data_ptr(),
            (lib.sv_rgb * 2)(R(self.lvl[0]), R(self.lvl[1])),
            (lib._vp * 2)(*[t.data_ptr() for t in self.lvl_var]),
            scratch, R(self.out), 0, None)
        self.mlp = mlp
        self._mlp_c = mlp.c() if mlp is not None else None
        self.kappa = f32() if mlp is not None else None
        if self.kappa is not None:
            self._st.kappa = self.kappa.data_ptr()
        self._dims = lib.dims_of(self.out)
        self._dtype = lib.dtype_of(self.out)
        self.tiles = tiles
        self._params = cfg.frame_params(tiles)

    @property
    def k(self) -> int:
        """Index of the buffers that hold the current history."""
        return self._st.cur

    @k.setter
    def k(self, v: int):
        self._st.cur = v

    def reset(self):
        for t in self.c_hist + self.m1 + self.m2c + self.n:
            t.zero_()
        self.k = 0
        self.frames = 0

    # ---- checkpoint / resume ------------------------------------------
    # Between frames the stream's state is its history buffers (both
    # halves of each ping-pong pair, and the temporal output that the
    # "temporal" feedback reads back), the index of the current half and
    # the frame count; everything else a frame writes before reading.

    def _state_tensors(self) -> Dict[str, torch.Tensor]:
        out = {}
        for name in ("c_hist", "m1", "m2c", "n"):
            for i, t in enumerate(getattr(self, name)):
                out[f"{name}{i}"] = t
        out["t_rgb"] = self.t_rgb[0]
        return out

    def save_state(self, path: str):
        """Write the stream's state to `path` (.npz; waits for the device)."""
        torch.cuda.synchronize()
        arrays = {k: t.cpu().numpy() for k, t in self._state_tensors().items()}
        np.savez(path, k=np.int32(self.k), frames=np.int64(self.frames),
                 dims=np.array([self.H, self.W], np.int64), **arrays)

    def load_state(self, path: str):
        """Resume from a state written by save_state for the same size and
        storage type: the next frame continues bitwise as the saved stream
        would have."""
        with np.load(path, allow_pickle=False) as f:
            if tuple(int(v) for v in f["dims"]) != (self.H, self.W):
                raise ValueError(f"state of a {tuple(f['dims'])} stream, this one is "
                                 f"{(self.H, self.W)}")
            for name, t in self._state_tensors().items():
                a = f[name]
                want = torch.empty(0, dtype=t.dtype).numpy().dtype
                if a.shape != tuple(t.shape) or a.dtype != want:
                    raise ValueError(f"{name}: {a.dtype}{a.shape} does not fit "
                                     f"{t.dtype}{tuple(t.shape)}")
                t.copy_(torch.from_numpy(a))
            self.k = int(f["k"])
            self.frames = int(f["frames"])
        torch.cuda.synchronize()

    def state(self) -> Dict[str, torch.Tensor]:
        """The history the next frame will read."""
        k = self.k
        return {"rgb": self.c_hist[k], "m1": self.m1[k], "m2c": self.m2c[k], "n": self.n[k]}

    def frame(self, inp: FrameInputs, alpha_map: Optional[torch.Tensor] = None,
              kappa: Optional[torch.Tensor] = None, stream=None,
              timer: Optional[Callable[[str], contextlib.AbstractContextManager]] = None
              ) -> torch.Tensor:
        """Enqueue one frame; returns the output tensor (valid once the
        stream reaches it; overwritten by the next frame).  `timer(name)`,
        if given, wraps each library call (for per-kernel events)."""
        if alpha_map is None:
            alpha_map = inp.alpha_map
        if timer is None:
            lib.sv_denoise_frame(inp.c(alpha_map, kappa, self._mlp_c), self._st, self._dims,
                                 self._dtype, self._params, stream=stream)
            self.frames += 1
            return self.out
        if self.mlp is not None:
            alpha_map, kappa = None, self.kappa
        # the same sequence call by call, for per-kernel timing
        cfg, k, k1 = self.cfg, self.k, 1 - self.k
        tm = timer
        fb_t = cfg.feedback == "temporal" or cfg.levels == 0
        hist = self.c_hist[k]
        t_out = self.c_hist[k1] if fb_t else self.t_rgb[0]
        with tm("temporal"):
            lib.sv_temporal(inp.rgb, inp.g, inp.mv, inp.prev, hist, self.m1[k], self.m2c[k],
                            self.n[k], t_out, self.m1[k1], self.m2c[k1], self.n[k1],
                            cfg.temporal(), alpha_map=alpha_map, stream=stream,
                            mlp=self.mlp, albedo=inp.albedo,
                            kappa_out=self.kappa if self.mlp is not None else None,
                            var=self.var, var_work=self.var_work, var_min_hist=cfg.min_hist)
        with tm("variance"):
            vp = cfg.variance()
            vp.listed = True
            lib.sv_variance(self.m1[k1], self.m2c[k1], self.n[k1], inp.g, self.var, vp,
                            self.var_work, stream=stream)
        c, v = t_out, self.var
        L = cfg.levels
        for i in range(L):
            last = i == L - 1
            fuse_inv = cfg.tonemap and last and not (i == 0 and not fb_t)
            if i == 0 and not fb_t:
                dst = self.c_hist[k1]
            elif last:
                dst = self.out
            else:
                dst = self.lvl[i % 2]
            dst_var = None if last else self.lvl_var[i % 2]
            p = cfg.atrous(inv_tonemap=fuse_inv)
            if self.tiles and i < len(self.tiles):
                shape = self.tiles[i]  # (persistent, blocks per CU[, tile rows])
                p.persistent, p.blocks_per_cu = shape[0], shape[1]
                if len(shape) > 2:
                    p.tile_rows = shape[2]
            if inp.blur_ctl is not None:
                with tm(f"atrous_adaptive{i}"):
                    fused = (2 << i) <= 32
                    lib.sv_atrous_adaptive(c, v, inp.g, inp.blur_ctl,
                                           self.scratch if cfg.separable and not fused else None,
                                           dst, dst_var, i, cfg.separable, p, kappa=kappa,
                                           stream=stream)
            elif cfg.separable:
                with tm(f"atrous_sep{i}"):
                    # the fused single-kernel form where the step has one
                    lib.sv_atrous_sep(c, v, inp.g, None if (1 << i) <= 32 else self.scratch, dst,
                                      dst_var, 1 << i, p, kappa=kappa, stream=stream)
            else:
                with tm(f"atrous{i}"):
                    lib.sv_atrous(c, v, inp.g, dst, dst_var, 1 << i, p, kappa=kappa,
                                  stream=stream)
            c, v = dst, dst_var
        if L == 0 or (L == 1 and not fb_t):
            if cfg.tonemap:
                lib.sv_tonemap(c, self.out, inverse=True, k=cfg.tm_k, stream=stream)
            else:
                self.out.copy_(c)
        self.k = k1
        self.frames += 1
        return self.out

    def intermediates(self) -> Dict[str, torch.Tensor]:
        """Views of the last frame's temporal output, moments and variance."""
        k = self.k
        fb_t = self.cfg.feedback == "temporal" or self.cfg.levels == 0
        t_rgb = self.c_hist[k] if fb_t else self.t_rgb[0]
        return {"t_rgb": t_rgb, "m1": self.m1[k], "m2c": self.m2c[k], "n": self.n[k],
                "var": self.var, "level0": self.c_hist[k]}


class BatchDenoiser:
    """Many independent streams of uneven sizes filtered together: one
    launch per pass over all of them, the frame's passes replayed as a HIP
    graph (sv_batch_*).  Each stream owns a Denoiser's buffers and its
    results are bitwise those of that Denoiser run alone."""

    def __init__(self, sizes, cfg=MOTION, dtype: torch.dtype = torch.float32,
                 tiles=None, device: str = "cuda", mlp: Optional[lib.MLP] = None,
                 graph: bool = True):
        """cfg: one FilterConfig for every stream, or a list with one per
        stream (the streams must then run the same kernels pass by pass).
        graph: replay the frame's passes as a HIP graph (else launch them
        one by one; the same results)."""
        cfgs = list(cfg) if isinstance(cfg, (list, tuple)) else [cfg] * len(sizes)
        if len(cfgs) != len(sizes):
            raise ValueError("one FilterConfig per stream")
        self.streams = [Denoiser(h, w, c, dtype, device, tiles, mlp)
                        for (h, w), c in zip(sizes, cfgs)]
        n = len(self.streams)
        self._dims = (lib.sv_dims * n)(*[d._dims for d in self.streams])
        self._states = (ctypes.POINTER(lib.sv_denoiser) * n)(
            *[ctypes.pointer(d._st) for d in self.streams])
        self._params = (lib.sv_frame_params * n)(*[d._params for d in self.streams])
        self._plan = ctypes.c_void_p()
        so = lib.load()
        lib._check("sv_batch_create_each", so.sv_batch_create_each(
            self._dims, self._states, n, self.streams[0]._dtype, self._params,
            ctypes.byref(self._plan)))
        lib._check("sv_batch_set_direct", so.sv_batch_set_direct(self._plan, 0 if graph else 1))

    def frame(self, inputs, stream=None):
        """One frame of every stream; inputs[i] are stream i's FrameInputs.
        Returns the streams' output tensors."""
        if len(inputs) != len(self.streams):
            raise ValueError("one FrameInputs per stream")
        fins = (lib.sv_frame_in * len(inputs))(
            *[inp.c(mlp=d._mlp_c) for inp, d in zip(inputs, self.streams)])
        lib._check("sv_batch_frame", lib.load().sv_batch_frame(
            self._plan, fins, lib._stream(stream)))
        for d in self.streams:
            d.frames += 1
        return [d.out for d in self.streams]

    def passes(self) -> int:
        return lib.load().sv_batch_passes(self._plan)

    def close(self):
        if self._plan:
            torch.cuda.synchronize()
            lib.load().sv_batch_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ChannelDenoiser:
    """The paper's pipeline shape (Section 3): a shadow channel and an
    indirect specular channel denoised separately, each with its own
    settings and its own adaptive-blur rule (shadow angle for shadows,
    roughness for reflections), in one batch plan (one launch per pass over
    both channels), then blended with the noise-free direct light by
    sv_compose."""

    def __init__(self, height: int, width: int, shadow: FilterConfig = SHADOW,
                 specular: FilterConfig = SPECULAR, dtype: torch.dtype = torch.float32,
                 adaptive: bool = True, device: str = "cuda", graph: bool = True):
        """graph: the batch plan replays its passes as a HIP graph (else it
        launches them one by one; the same results)."""
        self.H, self.W, self.adaptive = height, width, adaptive
        self.batch = BatchDenoiser([(height, width)] * 2, [shadow, specular], dtype,
                                   device=device, graph=graph)
        dev = torch.device(device)
        self.out = torch.zeros((3, height, width), dtype=dtype, device=dev)
        self.ctl = [torch.zeros((height, width), dtype=torch.uint8, device=dev) for _ in range(2)]
        self.shadow_rule = lib.BlurRule(table=False)  # shift above the shadow angle
        self.spec_rule = lib.BlurRule()               # shift and level table by roughness
        # the temporal gradient's blend factor for the shadow channel
        self.grad_alpha = torch.full((height, width), shadow.alpha, dtype=torch.float32,
                                     device=dev)
        self.grad_work = lib.gradient_workspace(self.grad_alpha)
        self.shadow_cfg = shadow

    def frame(self, geo: FrameInputs, shadow_rgb: torch.Tensor, spec_rgb: torch.Tensor,
              direct: torch.Tensor, roughness: Optional[torch.Tensor] = None,
              shadow_angle: Optional[torch.Tensor] = None, gradient: Optional[dict] = None,
              stream=None) -> torch.Tensor:
        """geo: the frame's G-buffer and motion (its rgb is not used);
        shadow_rgb: the one-sample visibility (3, H, W); spec_rgb: the
        one-sample indirect specular light; direct: the direct light.
        gradient (optional): the temporal gradient's inputs for the shadow
        channel - prev (the previous frame's visibility samples), reshade
        (them traced again), fmv, fz, pick - whose blend factor then replaces
        the shadow channel's constant one."""
        am = None
        if gradient is not None:
            lib.sv_temporal_gradient(gradient["prev"], gradient["reshade"], gradient["fmv"],
                                     gradient["fz"], gradient["pick"], geo.g, self.grad_alpha,
                                     self.grad_work, alpha=self.shadow_cfg.alpha, stream=stream)
            am = self.grad_alpha
        ins = [dataclasses.replace(geo, rgb=shadow_rgb, blur_ctl=None, alpha_map=am),
               dataclasses.replace(geo, rgb=spec_rgb, blur_ctl=None, alpha_map=None)]
        if self.adaptive:
            lib.sv_blur_control(None, shadow_angle, self.ctl[0], self.shadow_rule, stream=stream)
            lib.sv_blur_control(roughness, None, self.ctl[1], self.spec_rule, stream=stream)
            ins[0].blur_ctl, ins[1].blur_ctl = self.ctl
        shadow_out, spec_out = self.batch.frame(ins, stream=stream)
        lib.sv_compose(direct, shadow_out, spec_out, self.out, stream=stream)
        return self.out

    def close(self):
        self.batch.close()
