"""The learned variant: the filter with a per-pixel network that predicts
the temporal blend factor and the luminance edge-scale, trained on the GPU
by the library's own kernels against the generator's clean images.

Frame chain (one stream):

    sv_mlp_features -> sv_mlp_forward -> (alpha, kappa)
    sv_temporal (alpha_map = alpha) -> sv_variance
    -> a-trous levels (kappa) -> inverse tone map

Training (truncated gradients, one Adam step per frame):
  * dL/dalpha: the blend's local derivative (history held fixed) weighted
    by the residual of the chain's final output (sv_mlp_alpha_grad with
    the final output in place of the temporal output);
  * dL/dkappa: every level's local derivative (its input held fixed)
    weighted by the same final residual, summed over levels
    (sv_atrous_kappa_grad with ref = the final output);
  * L = mean over pixels of the per-pixel RelMSE term
    (1/3) sum_c (x - y)^2 / (y^2 + 0.01) in tone-mapped space, y = the tone-
    mapped clean image; sv_mlp_backward then sv_adam.

Torch provides memory, streams and a few reductions for statistics; every
step of the filter and of training runs in the library's kernels.
"""

from __future__ import annotations

import math
import os
from dataclasses import dataclass, replace
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import lib
from .pipeline import MOTION, FilterConfig, FrameInputs
from .scene import CONFIGS, render_frame, with_size

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "mlp_hd.npz")


@dataclass
class TrainConfig:
    width: int = 320
    height: int = 180
    frames: int = 8          # frames per training sequence
    sequences: int = 200     # training sequences (seeds seed0, seed0 + 1, ...)
    seed0: int = 5000
    warm: int = 1            # frames of each sequence run before gradients start
    lr: float = 1e-3
    init_seed: int = 0
    stat_frames: int = 16    # frames used for the feature standardisation


def relmse(x: torch.Tensor, y: torch.Tensor) -> float:
    """mean over pixels and channels of (x - y)^2 / (y^2 + 0.01)."""
    x, y = x.double(), y.double()
    return float((((x - y) ** 2) / (y * y + 0.01)).mean().item())


def train_sequence_config(cfg: TrainConfig, i: int):
    return replace(with_size(CONFIGS["hd_motion"], cfg.width, cfg.height, cfg.frames),
                   seed=cfg.seed0 + i)


def _dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class LearnedDenoiser:
    """One stream of the learned chain, call by call through the C ABI."""

    def __init__(self, H: int, W: int, mlp: lib.MLP, cfg: FilterConfig = MOTION,
                 dtype: torch.dtype = torch.float32):
        self.H, self.W, self.mlp, self.cfg, self.dtype = H, W, mlp, cfg, dtype
        z = lambda *s, dt=dtype: torch.zeros(s, dtype=dt, device="cuda")
        self.c_hist = [z(3, H, W), z(3, H, W)]
        self.m1 = [z(H, W, dt=torch.float32), z(H, W, dt=torch.float32)]
        self.m2c = [z(H, W, dt=torch.float32), z(H, W, dt=torch.float32)]
        self.n = [z(H, W, dt=torch.uint8), z(H, W, dt=torch.uint8)]
        self.t_rgb = z(3, H, W)
        self.var = z(H, W, dt=torch.float32)
        self.var_work = lib.variance_workspace(self.var)
        self.lvl = [z(3, H, W), z(3, H, W)]
        self.lvl_var = [z(H, W, dt=torch.float32), z(H, W, dt=torch.float32)]
        self.scratch = z(3, H, W)
        self.out = z(3, H, W)
        self.feat = lib.feature_rows(H, W)
        self.alpha = z(H, W, dt=torch.float32)
        self.kappa = z(H, W, dt=torch.float32)
        # training buffers
        self.hist_out = z(3, H, W, dt=torch.float32)
        self.y = z(3, H, W, dt=torch.float32)
        self.d_alpha = z(H, W, dt=torch.float32)
        self.d_kappa = z(H, W, dt=torch.float32)
        self.grad = z(lib.SV_MLP_PARAMS, dt=torch.float32)
        self.work = lib.mlp_workspace(self.var)
        self.k = 0

    def _training_levels(self):
        if getattr(self, "tr_c", None) is None:
            L, H, W = self.cfg.levels, self.H, self.W
            self.tr_c = [None] + [torch.zeros((3, H, W), dtype=self.dtype, device="cuda")
                                  for _ in range(1, L)]
            self.tr_v = [torch.zeros((H, W), dtype=torch.float32, device="cuda")
                         for _ in range(max(0, L - 1))]

    def reset(self):
        for t in self.c_hist + self.m1 + self.m2c + self.n:
            t.zero_()
        self.k = 0

    def frame(self, inp: FrameInputs, albedo: torch.Tensor, clean: Optional[torch.Tensor] = None,
              train: bool = False) -> torch.Tensor:
        """One frame; with `train`, also one Adam step on the network
        (needs `clean`, the linear clean image)."""
        c, k = self.cfg, self.k
        tp, ap = c.temporal(), c.atrous()
        lib.sv_mlp_features(inp.rgb, inp.g, inp.mv, inp.prev, self.c_hist[k], self.m1[k],
                            self.m2c[k], self.n[k], albedo, self.mlp, self.feat, tp,
                            hist_out=self.hist_out if train else None)
        lib.sv_mlp_forward(self.mlp, self.feat, self.alpha, self.kappa, self.var)
        lib.sv_temporal(inp.rgb, inp.g, inp.mv, inp.prev, self.c_hist[k], self.m1[k],
                        self.m2c[k], self.n[k], self.t_rgb, self.m1[1 - k], self.m2c[1 - k],
                        self.n[1 - k], tp, alpha_map=self.alpha)
        lib.sv_variance(self.m1[1 - k], self.m2c[1 - k], self.n[1 - k], inp.g, self.var,
                        c.variance(), self.var_work)
        if train:
            # tone-mapped clean target and the blend's gradient
            lib.sv_tonemap(clean, self.y, k=c.tm_k if c.tonemap else 1.0)
            self.d_kappa.zero_()
            self._training_levels()
        src, vsrc = self.t_rgb, self.var
        level_inputs = []
        for i in range(c.levels):
            last = i == c.levels - 1
            if train:  # every level's input is kept for the gradients
                dst = self.c_hist[1 - k] if i == 0 else self.tr_c[i]
                vdst = None if last else self.tr_v[i]
            else:
                dst = self.c_hist[1 - k] if i == 0 else self.lvl[i % 2]
                vdst = None if last else self.lvl_var[i % 2]
            level_inputs.append((src, vsrc))
            if c.separable:
                lib.sv_atrous_sep(src, vsrc, inp.g, None, dst, vdst, 1 << i, ap,
                                  kappa=self.kappa)
            else:
                lib.sv_atrous(src, vsrc, inp.g, dst, vdst, 1 << i, ap, kappa=self.kappa)
            src, vsrc = dst, vdst
        if train:
            # the blend's and each level's local derivatives, weighted by the
            # residual of the chain's final (tone-mapped) output: the colour
            # history is the level-0 output fed back every frame, so a
            # one-step loss on the temporal output alone rewards blur that
            # accumulates over frames
            lib.sv_mlp_alpha_grad(src, inp.rgb, self.hist_out, self.y, self.alpha,
                                  self.n[1 - k], inp.g.z, self.d_alpha,
                                  tm_k=c.tm_k if c.tonemap else 0.0)
            for i, (ci, vi) in enumerate(level_inputs):
                lib.sv_atrous_kappa_grad(ci, vi, inp.g, self.kappa, self.y, self.d_kappa, 1 << i,
                                         ap, ref=src)
        if c.tonemap:
            lib.sv_tonemap(src, self.out, inverse=True, k=c.tm_k)
        else:
            self.out.copy_(src)
        if train:
            npx = self.H * self.W
            lib.sv_mlp_backward(self.mlp, self.feat, self.d_alpha, self.d_kappa, self.grad,
                                self.work, self.var, scale=1.0 / npx)
        self.k = 1 - k
        return self.out


def _sequence_frames(cfg: TrainConfig, s: int, frames=None):
    """Frames of training sequence s: pre-generated, or rendered now."""
    if frames is not None:
        return frames[s]
    scfg = train_sequence_config(cfg, s)
    return (render_frame(scfg, f) for f in range(cfg.frames))


def render_sequence(args):
    cfg, s = args
    scfg = train_sequence_config(cfg, s)
    return [render_frame(scfg, f) for f in range(cfg.frames)]


def feature_statistics(cfg: TrainConfig, filt: FilterConfig = MOTION, frames=None):
    """Per-feature mean and 1/std over a few training frames, from the
    device's own raw features (standardisation off)."""
    mlp = lib.MLP(np.zeros(lib.SV_MLP_PARAMS), np.zeros(14), np.ones(14))
    den = LearnedDenoiser(cfg.height, cfg.width, mlp, filt)
    rows = []
    nseq = max(1, math.ceil(cfg.stat_frames / max(1, cfg.frames)))
    for s in range(nseq):
        den.reset()
        for fr in _sequence_frames(cfg, s, frames):
            den.frame(FrameInputs.from_numpy(fr), _dev(fr["albedo"]))
            x = den.feat.view(torch.bfloat16)[:, :14].float()
            rows.append(x[::max(1, x.shape[0] // 20000)])
    x = torch.cat(rows).double()
    mu = x.mean(0)
    sd = x.std(0)
    inv_s = torch.where(sd > 1e-6, 1.0 / sd, torch.ones_like(sd))
    return mu.cpu().numpy(), inv_s.cpu().numpy()


def init_params(seed: int, alpha0: float = 0.2) -> np.ndarray:
    """He-normal hidden layers and a zero output layer whose biases give the
    plain filter's settings everywhere (alpha = alpha0, kappa = 1): training
    starts from the method without the network."""
    r = np.random.default_rng(seed)
    w1 = r.normal(0, math.sqrt(2 / 14), (32, 14))
    w2 = r.normal(0, math.sqrt(2 / 32), (32, 32))
    s = (alpha0 - 0.05) / 0.95
    b3 = np.array([math.log(s / (1.0 - s)), 0.0])
    return np.concatenate([w1.ravel(), np.zeros(32), w2.ravel(), np.zeros(32),
                           np.zeros(64), b3]).astype(np.float32)


def train(cfg: TrainConfig, filt: FilterConfig = MOTION, log=None, frames=None) -> lib.MLP:
    """Train from scratch; returns the device network.  `frames[s]`, if
    given, are training sequence s's pre-generated frames."""
    mu, inv_s = feature_statistics(cfg, filt, frames)
    mlp = lib.MLP(init_params(cfg.init_seed), mu, inv_s)
    den = LearnedDenoiser(cfg.height, cfg.width, mlp, filt)
    for s in range(cfg.sequences):
        den.reset()
        for f, fr in enumerate(_sequence_frames(cfg, s, frames)):
            inp = FrameInputs.from_numpy(fr)
            alb, clean = _dev(fr["albedo"]), _dev(fr["clean"])
            tr = f >= cfg.warm
            den.frame(inp, alb, clean, train=tr)
            if tr:
                lib.sv_adam(mlp, den.grad, lr=cfg.lr)
        if log is not None and (s % 20 == 0 or s == cfg.sequences - 1):
            log(f"sequence {s}: alpha mean {den.alpha.mean().item():.3f} "
                f"kappa mean {den.kappa.mean().item():.3f}")
    torch.cuda.synchronize()
    return mlp


def save(mlp: lib.MLP, path: str = DEFAULT_WEIGHTS, meta: Optional[Dict] = None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=mlp.params.cpu().numpy(), mu=mlp.mu.cpu().numpy(),
             inv_s=mlp.inv_s.cpu().numpy(),
             meta=np.array(repr(meta or {})))


def load_weights(path: str = DEFAULT_WEIGHTS) -> lib.MLP:
    with np.load(path, allow_pickle=False) as z:
        return lib.MLP(z["params"], z["mu"], z["inv_s"])


def evaluate(seeds: Sequence[int], width: int, height: int, frames: int,
             mlp: Optional[lib.MLP], filt: FilterConfig = MOTION, first: int = 10) -> float:
    """Mean RelMSE of the final output against the clean image over frames
    first..frames-1 of each sequence; mlp None = the plain filter."""
    from .pipeline import Denoiser
    errs: List[float] = []
    for sd in seeds:
        scfg = replace(with_size(CONFIGS["hd_motion"], width, height, frames), seed=sd)
        if mlp is None:
            den = Denoiser(height, width, filt)
        else:
            den = LearnedDenoiser(height, width, mlp, filt)
        for f in range(frames):
            fr = render_frame(scfg, f)
            inp = FrameInputs.from_numpy(fr)
            out = den.frame(inp) if mlp is None else den.frame(inp, _dev(fr["albedo"]))
            if f >= first:
                errs.append(relmse(out, _dev(fr["clean"])))
    return float(np.mean(errs))


if __name__ == "__main__":
    import argparse
    import multiprocessing as mp
    import sys
    import time

    ap = argparse.ArgumentParser(description="train the blend/edge network and save it")
    ap.add_argument("--sequences", type=int, default=200)
    ap.add_argument("--frames", type=int, default=12)
    ap.add_argument("--width", type=int, default=320)
    ap.add_argument("--height", type=int, default=180)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args()
    cfg = TrainConfig(width=args.width, height=args.height, frames=args.frames,
                      sequences=args.sequences, warm=2, lr=args.lr, stat_frames=24)
    log = lambda m: print(m, flush=True)
    # every training frame is generated before the GPU is first touched
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(max(1, args.workers)) as pool:
        frames = pool.map(render_sequence, [(cfg, s) for s in range(cfg.sequences)])
    log(f"generated {cfg.sequences} sequences of {cfg.frames} frames at "
        f"{cfg.width}x{cfg.height} in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    net = train(cfg, log=log, frames=frames)
    log(f"trained in {time.perf_counter() - t0:.1f} s")
    del frames
    save(net, args.out, meta=cfg.__dict__)
    plain = evaluate([5900, 5901], 480, 270, 24, None)
    learned = evaluate([5900, 5901], 480, 270, 24, net)
    log(f"held-out RelMSE (480x270, frames 10..23) plain {plain:.5f} learned {learned:.5f}")
    sys.exit(0)
