"""Throughput of the denoiser on one MI355X.

Workload: the 1920x1080 moving-camera sequence (camera translating 2 px
and yawing 0.1 deg per frame, three spheres moving 5 px per frame), binary32
storage, with the paper's final filter: Reinhard tone map in, temporal
accumulation with variance colour clamping (gamma 1), variance estimate,
five edge-avoiding a-trous levels, inverse tone map.  One step = one frame
of the whole chain; inputs for all frames are resident in HBM before the
timed region.  The separable-blur chain is timed the same way and reported
as a variant.

Prints one JSON line.  See --help.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import multiprocessing as mp
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2312_06827_amd.scene import CONFIGS, render_frame, with_size  # noqa: E402

HBM_PEAK_GBS = 8000.0
# VALU issue rate: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78.6 T
# lane-operations per second, the published 157.3 TFLOP/s FP32 vector peak
# with an FMA counted as one operation.  Non-packed FP32 instructions reach
# it on this chip (the issue-rate probe's FMA links issue a wave64
# instruction in about two cycles), so it is the a-trous level's ALU peak.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
WORKLOAD = CONFIGS["hd_motion"]
PROFILES = os.path.join(ROOT, "profiles")

# Algorithmic bytes per pixel (each input plane read once, each output
# written once), binary32 storage, ids on.
BYTES_PER_PX = {
    # cur rgb, z, normal, mv, prev z, prev normal, ids x2, history rgb,
    # m1, m2, n -> rgb, m1, m2, n
    "temporal": 12 + 4 + 12 + 8 + 4 + 12 + 2 + 12 + 8 + 1 + 12 + 8 + 1,
    # m2c, n, z -> var (history long enough; the short-history pixels'
    # window reads are extra)
    "variance": 4 + 1 + 4 + 4,
    # rgb, var, z, dzdx, dzdy, normal -> rgb, var
    "atrous": 12 + 4 + 4 + 4 + 4 + 12 + 12 + 4,
    "atrous_last": 12 + 4 + 4 + 4 + 4 + 12 + 12,
    # separable level in one kernel: the same inputs and outputs (the
    # horizontal result never reaches memory)
    "atrous_sep": 12 + 4 + 4 + 4 + 4 + 12 + 12 + 4,
    "atrous_sep_last": 12 + 4 + 4 + 4 + 4 + 12 + 12,
}


# Algorithmic VALU slots per output pixel of the 5x5 a-trous level: the
# FP32 operations of the level's definition, one full-rate issue slot each
# but for the transcendentals, which are priced at their issue cost measured
# on the GPU the benchmark runs on (issue_costs).  Per non-centre tap: depth term 2,
# luminance term 2, normal term 8 + log2 (chord 6, u, scale), exp2, and the
# accumulation 6 (sum of weights, three colour FMAs, w^2 var).  Per pixel:
# 71 plain operations (3x3 variance prefilter 19, luminance scale 3, the 12
# distinct depth scales 36, own luminance 3, centre tap 5, normalisation 5)
# plus 15 reciprocals (prefilter, luminance scale, 12 depth scales,
# normalisation) and one square root.
def atrous_ops_per_px(cost):
    return 24 * (18 + cost["log2"] + cost["exp2"]) + 71 + 15 * cost["rcp"] + cost["sqrt"]


def issue_costs(torch, blocks=8192, iters=2048, reps=3):
    """Issue cost of exp2, log2, rcp and sqrt in full-rate VALU slots (the
    issue time of the probe's FMA link, which runs at the full rate), from
    the library's issue-rate probe: each chain link is the operation beside
    one or two full-rate ones, timed against FMA links."""
    from paper_2312_06827_amd import lib

    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t = {}
    for kind in range(5):
        lib.sv_probe_issue(out, kind, iters)  # warm
        best = float("inf")
        for _ in range(reps):
            a.record()
            lib.sv_probe_issue(out, kind, iters)
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b))
        t[kind] = best
    unit = t[0]  # one FMA per link
    return {"exp2": round(t[1] / unit - 1, 2), "log2": round(t[2] / unit - 2, 2),
            "rcp": round(t[3] / unit - 2, 2), "sqrt": round(t[4] / unit - 2, 2)}


# Source files that make up the 2D a-trous kernel; PMC traffic measured on
# them is reported only while they are unchanged.
ATROUS_SOURCES = ("paper_2312_06827_amd/csrc/atrous_impl.h",
                  "paper_2312_06827_amd/csrc/atrous_f32_2d.hip",
                  "paper_2312_06827_amd/csrc/atrous.hip",
                  "paper_2312_06827_amd/csrc/sv_internal.h")
TRAFFIC_FILE = os.path.join(PROFILES, "atrous2d_f32_1920x1080_pmc_traffic.txt")


def source_digest(paths) -> str:
    import hashlib

    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per a-trous launch (mean over the five levels) from the
    committed PMC summary, or None if it is missing or the kernel sources
    changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(l.split(":", 1) for l in f.read().splitlines() if ":" in l and not
                      l.startswith(("#", " ")))
    except OSError:
        return None
    if kv.get("kernel_source_sha256", "").strip() != source_digest(ATROUS_SOURCES):
        return None
    try:
        return float(kv["hbm_bytes_per_launch_mean"])
    except (KeyError, ValueError):
        return None


# Binary16 storage, 2D levels: temporal 56 (+ 2 for the id planes),
# variance 13, level 32, last level 28.
FP16_FRAME_BYTES = 56 + 2 + 13 + 4 * 32 + 28


def frame_bytes_per_px(levels: int, sep: bool) -> int:
    a, al = ("atrous_sep", "atrous_sep_last") if sep else ("atrous", "atrous_last")
    return (BYTES_PER_PX["temporal"] + BYTES_PER_PX["variance"]
            + (levels - 1) * BYTES_PER_PX[a] + BYTES_PER_PX[al])


def _render(args):
    cfg, f = args
    return render_frame(cfg, f)


def generate(cfg, n_frames, workers):
    cfg = type(cfg)(**{**cfg.__dict__, "frames": n_frames})
    if workers <= 1:
        return [render_frame(cfg, f) for f in range(n_frames)]
    ctx = mp.get_context("fork")
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        return list(ex.map(_render, [(cfg, f) for f in range(n_frames)]))


class KernelTimer:
    """HIP events around each library call, recorded on torch's current
    stream (the stream the calls launch on).  Events are created up front so
    that no event creation happens inside the timed loop."""

    def __init__(self, torch, n):
        self.pool = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                     for _ in range(n)]
        self.used = []

    def __call__(self, name):
        a, b = self.pool[len(self.used)]
        self.used.append((name, a, b))

        class _Ctx:
            def __enter__(self_):
                a.record()

            def __exit__(self_, *exc):
                b.record()
        return _Ctx()

    def summary(self):
        out = {}
        for name, a, b in self.used:
            out.setdefault(name, []).append(a.elapsed_time(b))
        return {k: (float(np.mean(v)), len(v)) for k, v in out.items()}


def run_chain(torch, frames_dev, cfg, H, W, warmup, steps, per_kernel, tiles=None):
    """Warm up, then time `steps` frames.  Headline mode enqueues each frame
    with one native call and nothing else; per-kernel mode brackets every
    library call with events (which adds a few microseconds per call)."""
    from paper_2312_06827_amd.pipeline import Denoiser

    den = Denoiser(H, W, cfg, tiles=tiles)
    timer = KernelTimer(torch, 16 * (warmup + steps)) if per_kernel else None
    for f in range(warmup):
        den.frame(frames_dev[f], timer=timer)
    torch.cuda.synchronize()
    if timer is not None:
        timer.used.clear()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for f in range(warmup, warmup + steps):
        den.frame(frames_dev[f], timer=timer)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = start.elapsed_time(stop)
    return gpu_ms, wall, (timer.summary() if timer else None)


def frame_times(torch, frames_dev, cfg, H, W, warmup, steps, tiles=None):
    """Per-frame GPU times (us) of the chain: an event between consecutive
    native frame calls on the launch stream, nothing else added."""
    from paper_2312_06827_amd.pipeline import Denoiser

    den = Denoiser(H, W, cfg, tiles=tiles)
    for f in range(warmup):
        den.frame(frames_dev[f])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record()
    for i, f in enumerate(range(warmup, warmup + steps)):
        den.frame(frames_dev[f])
        ev[i + 1].record()
    torch.cuda.synchronize()
    t = np.array([ev[i].elapsed_time(ev[i + 1]) * 1e3 for i in range(steps)])
    return {"median": round(float(np.median(t)), 2), "p90": round(float(np.percentile(t, 90)), 2),
            "min": round(float(t.min()), 2), "max": round(float(t.max()), 2)}


def graph_replay(torch, frames_dev, cfg, H, W, warmup, tiles=None):
    """The headline chain as a one-stream batch plan: the frame's passes
    captured once as a HIP graph and replayed with refreshed arguments."""
    from paper_2312_06827_amd.pipeline import BatchDenoiser

    plan = BatchDenoiser([(H, W)], cfg, torch.float32, tiles=tiles)
    try:
        ms = _timed_frames(torch, plan.frame, [[fd] for fd in frames_dev], warmup)
        passes = plan.passes()
    finally:
        plan.close()
    return {"value": round(H * W / (ms * 1e-3) / 1e6, 1), "unit": "Mpix/s",
            "ms_per_step": round(ms, 4), "launches_per_frame": passes}


def copy_probe(torch, nbytes=1 << 30, reps=10):
    from paper_2312_06827_amd import lib

    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    lib.sv_probe_copy(dst, src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        lib.sv_probe_copy(dst, src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return 2 * nbytes / (ms * 1e-3) / 1e9  # read + write


def _timed_frames(torch, fn, frames, warmup):
    """Run fn(frame) over frames; time the ones after `warmup` with events."""
    for f in frames[:warmup]:
        fn(f)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for f in frames[warmup:]:
        fn(f)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / max(1, len(frames) - warmup)


UHD_WARMUP, UHD_STEPS = 4, 10
BATCH_WARMUP, BATCH_STEPS = 3, 5
SMALL_STREAMS, SMALL_SIZE = 64, (180, 320)  # (H, W)
CH_WARMUP, CH_STEPS = 5, 15
# the learned component's quality judge: the held-out sequences (never
# trained on), 1920x1080, RelMSE-to-clean over frames 10..13 of each
LEARN_SEEDS = tuple(range(5900, 5908))
LEARN_FRAMES, LEARN_FIRST = 14, 10
# the plain filter at its best constant blend factor and luminance-edge
# width, the grid the learned per-pixel values are judged against (wider
# than the network's own ranges: alpha in [0.05, 1], kappa in [1/4, 4])
PLAIN_GRID_ALPHA = (0.05, 0.1, 0.2, 0.4, 0.6, 0.8, 1.0)
PLAIN_GRID_KAPPA = (0.5, 1.0, 2.0, 4.0, 8.0, 16.0, 64.0, 256.0)
_LEARN_KEYS = ("rgb", "clean", "albedo", "z", "dzdx", "dzdy", "n", "id", "mv", "prev_z",
               "prev_n", "prev_id")


def _render_learn(args):
    fr = render_frame(*args)
    return {k: fr[k] for k in _LEARN_KEYS}


def generate_variant_frames(workers, want):
    """Host frames of the 4K, sixteen-stream and two-channel variants
    (generated before the GPU is touched, like the headline frames)."""
    from paper_2312_06827_amd.scene import batched_configs
    uhd = CONFIGS["uhd_half"]
    uhd = type(uhd)(**{**uhd.__dict__, "frames": UHD_WARMUP + UHD_STEPS})
    n = BATCH_WARMUP + BATCH_STEPS
    scfg = batched_configs(16, n, half=True)
    # many small streams, where one stream alone cannot fill the GPU
    small = [with_size(c, SMALL_SIZE[1], SMALL_SIZE[0])
             for c in batched_configs(SMALL_STREAMS, n, seed=5, half=True)]
    ch = type(WORKLOAD)(**{**WORKLOAD.__dict__, "frames": CH_WARMUP + CH_STEPS, "channels": True})
    jobs = []
    if "uhd_half" in want:
        jobs += [(uhd, f) for f in range(uhd.frames)]
    if "batched" in want:
        jobs += [(c, f) for f in range(n) for c in scfg]
        jobs += [(c, f) for f in range(n) for c in small]
    if want & {"channels", "gradient"}:
        jobs += [(ch, f) for f in range(ch.frames)]
    held = [type(WORKLOAD)(**{**WORKLOAD.__dict__, "frames": LEARN_FRAMES, "seed": sd})
            for sd in LEARN_SEEDS]
    ljobs = [(c, f) for c in held for f in range(LEARN_FRAMES)] if "learned" in want else []
    if workers <= 1:
        out = [_render(j) for j in jobs]
        lout = [_render_learn(j) for j in ljobs]
    else:
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
            out = list(ex.map(_render, jobs))
            lout = list(ex.map(_render_learn, ljobs))
    res, k = {}, 0
    if "uhd_half" in want:
        res["uhd"], k = out[:uhd.frames], uhd.frames
    if "batched" in want:
        res["batch_cfg"] = scfg
        res["batch"] = [out[k + f * 16:k + (f + 1) * 16] for f in range(n)]
        k += 16 * n
        m = SMALL_STREAMS
        res["small_cfg"] = small
        res["small"] = [out[k + f * m:k + (f + 1) * m] for f in range(n)]
        k += m * n
    if want & {"channels", "gradient"}:
        res["channels"] = out[k:k + ch.frames]
    if "learned" in want:
        res["held_out"] = [lout[i * LEARN_FRAMES:(i + 1) * LEARN_FRAMES]
                           for i in range(len(LEARN_SEEDS))]
    return res


def variant_uhd_half(torch, frames_np, warmup=UHD_WARMUP, steps=UHD_STEPS, tune=True):
    """Binary16 storage at 3840x2160 (2D levels), launch shapes from the
    autotuner at that size and storage type."""
    from paper_2312_06827_amd.autotune import tiles_for
    from paper_2312_06827_amd.pipeline import MOTION, Denoiser, FrameInputs
    cfg = CONFIGS["uhd_half"]
    frames = [FrameInputs.from_numpy(fr) for fr in frames_np]
    tiles = tiles_for(cfg.height, cfg.width, torch.float16, cache=None) if tune else None
    den = Denoiser(cfg.height, cfg.width, MOTION, dtype=torch.float16, tiles=tiles)
    ms = _timed_frames(torch, den.frame, frames, warmup)
    px = cfg.width * cfg.height
    return {"value": round(px / (ms * 1e-3) / 1e6, 1), "unit": "Mpix/s", "ms_per_step": round(ms, 4),
            "dtype": "f16 storage / f32 math", "frame_bytes_per_px": FP16_FRAME_BYTES,
            "launch_shapes": tiles and [list(t) for t in tiles],
            "frame_hbm_frac": round(px * FP16_FRAME_BYTES / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "config": f"{cfg.width}x{cfg.height}, {steps} frames timed after {warmup}"}


def _batch_vs_singles(torch, scfg, frames_np, warmup, tune):
    from paper_2312_06827_amd.autotune import tiles_for
    from paper_2312_06827_amd.pipeline import MOTION, BatchDenoiser, Denoiser, FrameInputs
    frames = [[FrameInputs.from_numpy(fr) for fr in per] for per in frames_np]
    sizes = [(c.height, c.width) for c in scfg]
    px = sum(h * w for h, w in sizes)
    mh, mw = sorted(sizes, key=lambda s: s[0] * s[1])[len(sizes) // 2]
    tiles = tiles_for(mh, mw, torch.float16, cache=None) if tune else None
    batch = BatchDenoiser(sizes, MOTION, torch.float16, tiles=tiles)
    ms_b = _timed_frames(torch, batch.frame, frames, warmup)
    passes = batch.passes()
    batch.close()
    # the same plan with its passes launched one by one instead of a graph
    direct = BatchDenoiser(sizes, MOTION, torch.float16, tiles=tiles, graph=False)
    ms_d = _timed_frames(torch, direct.frame, frames, warmup)
    direct.close()
    singles = [Denoiser(h, w, MOTION, torch.float16, tiles=tiles) for h, w in sizes]
    ms_s = _timed_frames(torch, lambda fr: [d.frame(x) for d, x in zip(singles, fr)], frames, warmup)
    return {"value": round(px / (ms_b * 1e-3) / 1e6, 1), "unit": "Mpix/s",
            "ms_per_step": round(ms_b, 4), "launches_per_frame": passes,
            "launch_shapes": tiles and [list(t) for t in tiles],
            "tuned_at": f"{mw}x{mh}",
            "direct_launches": {"value": round(px / (ms_d * 1e-3) / 1e6, 1),
                                "ms_per_step": round(ms_d, 4)},
            "one_by_one": {"value": round(px / (ms_s * 1e-3) / 1e6, 1), "ms_per_step": round(ms_s, 4),
                           "launches_per_frame": len(sizes) * passes},
            "config": f"{len(sizes)} streams {min(sizes)}..{max(sizes)} (HxW), {px / 1e6:.1f} Mpix "
                      f"per frame, {len(frames_np) - warmup} frames timed after {warmup}"}


def variant_batched(torch, scfg, frames_np, small_cfg, small_np, warmup=BATCH_WARMUP, tune=True):
    """Sixteen streams of uneven size, binary16: one launch per pass under a
    HIP graph, against the same streams run one by one.  One set of launch
    shapes for every stream (a pass is one launch over all of them), from
    the autotuner at the median stream size.  Beside it, the same for 64
    streams of 320x180, each too small to fill the GPU alone."""
    out = _batch_vs_singles(torch, scfg, frames_np, warmup, tune)
    out["small_streams"] = _batch_vs_singles(torch, small_cfg, small_np, warmup, tune)
    return out


def variant_learned(torch, frames_np, held_np, warmup, steps):
    """The learned blend/edge network inside the temporal step, against
    plain SVGF.  Throughput: the headline frames, for {plain, learned} x
    {2D, separable} x {5, 4, 3} levels.  Quality: RelMSE-to-clean over
    frames 10..13 of the eight held-out 1080p sequences (seeds 5900-5907).
    Two plain references: the paper's constants (alpha 0.2, sigma_l 4) and
    the best constant (alpha, sigma_l scale) of a 7 x 8 grid chosen on those
    same held-out frames (the strongest constant the network could be
    replaced by).  The claim holds against a reference if some learned point
    has RelMSE no higher and throughput no lower than plain 5-level 2D."""
    from dataclasses import replace as dc_replace

    from paper_2312_06827_amd import learn
    from paper_2312_06827_amd.pipeline import MOTION, MOTION_SEP, Denoiser, FrameInputs
    if not os.path.exists(learn.DEFAULT_WEIGHTS):
        return None
    net = learn.load_weights(learn.DEFAULT_WEIGHTS)
    H, W = WORKLOAD.height, WORKLOAD.width
    n = warmup + steps
    frames = [FrameInputs.from_numpy(fr) for fr in frames_np[:n]]
    held = [[(FrameInputs.from_numpy(fr), torch.from_numpy(fr["clean"]).cuda()) for fr in seq]
            for seq in held_np]

    def quality(cfg, mlp):
        errs = []
        for seq in held:
            den = Denoiser(H, W, cfg, mlp=mlp)
            for f, (fr, clean) in enumerate(seq):
                out = den.frame(fr)
                if f >= LEARN_FIRST:
                    errs.append(learn.relmse(out, clean))
        return float(np.mean(errs))

    out = {"weights": os.path.relpath(learn.DEFAULT_WEIGHTS, ROOT),
           "judge": f"RelMSE over frames {LEARN_FIRST}..{LEARN_FRAMES - 1} of held-out 1080p "
                    f"sequences, seeds {LEARN_SEEDS[0]}-{LEARN_SEEDS[-1]}",
           "points": {}}
    for mode in ("plain", "learned"):
        mlp = net if mode == "learned" else None
        for form, base in (("2d", MOTION), ("sep", MOTION_SEP)):
            for levels in (5, 4, 3):
                cfg = dc_replace(base, levels=levels)
                ms = _timed_frames(torch, Denoiser(H, W, cfg, mlp=mlp).frame, frames, warmup)
                out["points"][f"{mode}_{form}_{levels}"] = {
                    "value": round(H * W / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
                    "relmse": round(quality(cfg, mlp), 6)}
    grid = {}
    for a in PLAIN_GRID_ALPHA:
        for k in PLAIN_GRID_KAPPA:
            grid[(a, k)] = quality(dc_replace(MOTION, alpha=a,
                                              sigma_l=MOTION.sigma_l * k), None)
    (ba, bk), best = min(grid.items(), key=lambda kv: kv[1])
    out["plain_best_constant"] = {
        "alpha": ba, "sigma_l_scale": bk, "relmse": round(best, 6),
        "grid": {f"a{a}_k{k}": round(v, 6) for (a, k), v in grid.items()}}
    ref = out["points"]["plain_2d_5"]

    def winners(rel):
        return [k for k, v in out["points"].items() if k.startswith("learned")
                and v["relmse"] <= rel and v["value"] >= ref["value"]]

    out["winning_points"] = winners(ref["relmse"])
    out["claim_holds"] = bool(out["winning_points"])
    out["winning_points_vs_best_constant"] = winners(best)
    out["claim_holds_vs_best_constant"] = bool(out["winning_points_vs_best_constant"])
    return out


def variant_scene_features(torch, frames_np, warmup, steps):
    """The paper's alternatives on the headline workload: variance colour
    clipping instead of the clamp (Section 3.1), and the blur adapted to
    scene features (Sections 3.2, 3.5) with the control bytes computed
    from the scene's roughness every frame (inside the timed region).
    Throughput and RelMSE-to-clean over the timed frames."""
    from dataclasses import replace as dc_replace

    from paper_2312_06827_amd import learn
    from paper_2312_06827_amd import lib as L
    from paper_2312_06827_amd.pipeline import MOTION, MOTION_SEP, Denoiser, FrameInputs
    H, W = WORKLOAD.height, WORKLOAD.width
    n = warmup + steps
    frames = [FrameInputs.from_numpy(fr) for fr in frames_np[:n]]
    clean = [torch.from_numpy(fr["clean"]).cuda() for fr in frames_np[:n]]
    rough = [torch.from_numpy(fr["roughness"]).cuda() for fr in frames_np[:n]]
    ctl = [torch.empty((H, W), dtype=torch.uint8, device="cuda") for _ in range(n)]
    rule = L.BlurRule()

    def run(cfg, adaptive):
        for i, fr in enumerate(frames):
            fr.blur_ctl = ctl[i] if adaptive else None
        den = Denoiser(H, W, cfg)

        def step(i):
            if adaptive:
                L.sv_blur_control(rough[i], None, ctl[i], rule)
            return den.frame(frames[i])
        ms = _timed_frames(torch, step, list(range(n)), warmup)
        den = Denoiser(H, W, cfg)
        q = float(np.mean([learn.relmse(step(i), clean[i]) for i in range(n)][warmup:]))
        return {"value": round(H * W / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
                "relmse": round(q, 6)}

    out = {"rule": "shift above roughness 0.2; levels 0 / 1 / all at roughness <= 0 / <= 0.05 / above"}
    out["clamp_2d"] = run(MOTION, False)
    out["clip_2d"] = run(dc_replace(MOTION, clamp=False, clip=True), False)
    out["adaptive_2d"] = run(MOTION, True)
    out["clamp_sep"] = run(MOTION_SEP, False)
    out["adaptive_sep"] = run(MOTION_SEP, True)
    for fr in frames:
        fr.blur_ctl = None
    return out


def variant_channels(torch, frames_np, warmup=CH_WARMUP, steps=CH_STEPS):
    """The paper's pipeline shape (Section 3): a shadow channel and an
    indirect specular channel, each filtered with its own settings and
    adaptive-blur rule in one batch plan, then composed with the direct
    light.  Throughput (pixels of the composed frame per second) and
    RelMSE of the composite against the clean one, with and without the
    adaptive blur; the plain single-channel filter of the composite's
    noisy estimate is reported beside it."""
    from paper_2312_06827_amd import learn
    from paper_2312_06827_amd.pipeline import ChannelDenoiser, Denoiser, FrameInputs, MOTION
    H, W = WORKLOAD.height, WORKLOAD.width
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    geo = [FrameInputs.from_numpy(fr) for fr in frames_np]
    planes = [{k: t(fr[k]) for k in ("shadow", "spec", "direct", "roughness", "shadow_angle")}
              for fr in frames_np]
    clean = [t(fr["composite_clean"]) for fr in frames_np]
    out = {"config": f"{W}x{H}, two channels, {steps} frames timed after {warmup}"}
    for adaptive in (True, False):
        timed = {}
        for graph in (True, False):  # the batch plan as a graph, or launched directly
            den = ChannelDenoiser(H, W, adaptive=adaptive, graph=graph)
            step = lambda i: den.frame(geo[i], planes[i]["shadow"], planes[i]["spec"],
                                       planes[i]["direct"], roughness=planes[i]["roughness"],
                                       shadow_angle=planes[i]["shadow_angle"])
            timed[graph] = _timed_frames(torch, step, list(range(len(geo))), warmup)
            den.close()
        ms = timed[True]
        den = ChannelDenoiser(H, W, adaptive=adaptive)
        step = lambda i: den.frame(geo[i], planes[i]["shadow"], planes[i]["spec"],
                                   planes[i]["direct"], roughness=planes[i]["roughness"],
                                   shadow_angle=planes[i]["shadow_angle"])
        q = float(np.mean([learn.relmse(step(i), clean[i]) for i in range(len(geo))][warmup:]))
        den.close()
        out["adaptive" if adaptive else "fixed"] = {
            "value": round(H * W / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "relmse": round(q, 6),
            "direct_launches": {"value": round(H * W / (timed[False] * 1e-3) / 1e6, 1),
                                "ms_per_step": round(timed[False], 4)}}
    # one filter over the noisy composite (direct * shadow sample + specular sample)
    comp = [FrameInputs.from_numpy({**fr, "rgb": fr["direct"] * fr["shadow"] + fr["spec"]})
            for fr in frames_np]
    den = Denoiser(H, W, MOTION)
    q = float(np.mean([learn.relmse(den.frame(c), clean[i]) for i, c in enumerate(comp)][warmup:]))
    out["one_filter_relmse"] = round(q, 6)
    return out


def variant_gradient(torch, frames_np, warmup=CH_WARMUP, steps=CH_STEPS):
    """The temporal gradient (A-SVGF) on the shadow channel, whose moving
    shadows lag behind under a constant blend factor: throughput of the
    shadow channel's frame with the gradient passes included, and RelMSE of
    its output against the clean visibility, with and without the gradient."""
    from paper_2312_06827_amd import learn
    from paper_2312_06827_amd import lib as L
    from paper_2312_06827_amd.pipeline import SHADOW, Denoiser, FrameInputs
    H, W = WORKLOAD.height, WORKLOAD.width
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ins, grads = [], []
    for f, fr in enumerate(frames_np):
        ins.append(FrameInputs.from_numpy({**fr, "rgb": fr["shadow"]}))
        if f == 0:
            grads.append(None)
            continue
        re = np.broadcast_to(fr["shadow_reshade"][None], (3, H, W))
        grads.append({"prev": t(frames_np[f - 1]["shadow"]), "reshade": t(re),
                      "fmv": t(fr["fmv"]), "fz": t(fr["fz"]), "pick": t(fr["grad_pick"])})
    clean = [t(np.broadcast_to(fr["shadow_clean"][None], (3, H, W))) for fr in frames_np]
    am = torch.full((H, W), SHADOW.alpha, dtype=torch.float32, device="cuda")
    work = L.gradient_workspace(am)
    out = {"config": f"{W}x{H} shadow channel, {steps} frames timed after {warmup}"}
    for use in (False, True):
        def run():
            den = Denoiser(H, W, SHADOW)

            def step(i):
                g = grads[i]
                if use and g is not None:
                    L.sv_temporal_gradient(g["prev"], g["reshade"], g["fmv"], g["fz"], g["pick"],
                                           ins[i].g, am, work, alpha=SHADOW.alpha)
                    return den.frame(ins[i], alpha_map=am)
                return den.frame(ins[i])
            return step
        ms = _timed_frames(torch, run(), list(range(len(ins))), warmup)
        step = run()
        q = float(np.mean([learn.relmse(step(i), clean[i]) for i in range(len(ins))][warmup:]))
        out["gradient" if use else "constant_alpha"] = {
            "value": round(H * W / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "relmse": round(q, 6)}
    return out


def host_cpu():
    """CPU model and the logical CPUs this process may run on."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(frames_np, warm, timed, timed_one=1, timed_eight=2, uhd_np=None):
    """The oracle as it stands, on the host cores, on a bounded sample: the
    chain over `timed` frames with every usable core, then `timed_one`
    further frames on one thread and `timed_eight` on eight (the same frames
    the GPU filters); beside it the small static workload in full and, when
    its frames are at hand, the first two 3840x2160 binary16 frames (every
    pixel short of history there, so the spatial variance runs everywhere)."""
    import oracle as O
    from paper_2312_06827_amd.scene import sequence

    p = O.OracleParams(clamp=True, tonemap=True, use_id=True)
    H, W = frames_np[0]["z"].shape
    st = O.new_state(H, W)
    cpu = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", cpu["usable_cpus"]))
    O.set_threads(threads)
    for f in range(warm):
        _, st, _ = O.run_frame(frames_np[f], st, p)

    def run(first, count, n_threads):
        nonlocal st
        O.set_threads(n_threads)
        t0 = time.perf_counter()
        for f in range(first, first + count):
            _, st, _ = O.run_frame(frames_np[f], st, p)
        return time.perf_counter() - t0

    dt = run(warm, timed, threads)
    f1 = warm + timed
    dt1 = run(f1, timed_one, 1)
    f8 = f1 + timed_one
    dt8 = run(f8, timed_eight, 8) if timed_eight and f8 + timed_eight <= len(frames_np) else None
    O.set_threads(threads)
    frames = lambda a, n: f"frame{'s' if n > 1 else ''} {a}{'..' + str(a + n - 1) if n > 1 else ''}"
    out = {"value": W * H * timed / dt / 1e6, "unit": "Mpix/s", "cores": O.threads(),
           "kind": "oracle",
           "sample": f"{W}x{H} {frames(warm, timed)} of the same sequence after {warm} untimed "
                     f"frames, FP64 C oracle with OpenMP ({dt:.1f} s)",
           "single_thread": {"value": W * H * timed_one / dt1 / 1e6, "unit": "Mpix/s", "cores": 1,
                             "sample": f"{frames(f1, timed_one)} on one thread ({dt1:.1f} s)"},
           "cpu": cpu}
    if dt8 is not None:
        out["eight_threads"] = {"value": W * H * timed_eight / dt8 / 1e6, "unit": "Mpix/s",
                                "cores": 8, "sample": f"{frames(f8, timed_eight)} ({dt8:.1f} s)"}
    # the small static workload, all eight frames
    small = list(sequence(CONFIGS["small_static"]))
    sh, sw = small[0]["z"].shape
    s_st = O.new_state(sh, sw)
    t0 = time.perf_counter()
    for fr in small:
        _, s_st, _ = O.run_frame(fr, s_st, O.OracleParams())
    dts = time.perf_counter() - t0
    out["small_static"] = {"value": sw * sh * len(small) / dts / 1e6, "unit": "Mpix/s",
                           "cores": O.threads(),
                           "sample": f"{sw}x{sh}, all {len(small)} frames ({dts:.2f} s)"}
    if uhd_np:
        hp = O.OracleParams(clamp=True, tonemap=True, use_id=True, half=True)
        uh, uw = uhd_np[0]["z"].shape
        u_st = O.new_state(uh, uw)
        n = min(2, len(uhd_np))
        t0 = time.perf_counter()
        for fr in uhd_np[:n]:
            _, u_st, _ = O.run_frame(fr, u_st, hp)
        dtu = time.perf_counter() - t0
        out["uhd_half"] = {"value": uw * uh * n / dtu / 1e6, "unit": "Mpix/s", "cores": O.threads(),
                           "sample": f"{uw}x{uh} binary16, frames 0..{n - 1} ({dtu:.1f} s)"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--variants",
                    default="separable,uhd_half,batched,scene_features,channels,gradient,learned",
                    help="comma-separated variants to run after the headline chain")
    ap.add_argument("--no-tune", action="store_true",
                    help="the library's default a-trous launch shapes instead of the"
                         " autotuner's (which are timed on this GPU before the run)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    H, W = WORKLOAD.height, WORKLOAD.width
    n_frames = args.warmup + args.steps
    t0 = time.perf_counter()
    frames_np = generate(WORKLOAD, n_frames, args.workers)  # before any GPU call (fork)
    want = set() if args.no_variants else set(v for v in args.variants.split(",") if v)
    vframes = (generate_variant_frames(args.workers, want)
               if want & {"uhd_half", "batched", "channels", "gradient", "learned"} else None)
    gen_s = time.perf_counter() - t0
    print(f"# generated {n_frames} frames in {gen_s:.1f} s", file=sys.stderr, flush=True)

    import torch

    from paper_2312_06827_amd.pipeline import MOTION, MOTION_SEP, FrameInputs

    frames_dev = [FrameInputs.from_numpy(fr) for fr in frames_np]
    torch.cuda.synchronize()

    # launch shapes of the a-trous levels, measured on this device and size
    from paper_2312_06827_amd.autotune import tiles_for
    if args.no_tune:
        tiles_2d = tiles_sep = None
    else:
        tiles_2d = tiles_for(H, W, separable=False, cache=None)
        tiles_sep = tiles_for(H, W, separable=True, cache=None)
    print(f"# tuned launch shapes 2d {tiles_2d} sep {tiles_sep}", file=sys.stderr, flush=True)
    # a throwaway pass warms clocks, code objects and allocator
    tw = min(2, args.warmup)
    run_chain(torch, frames_dev, MOTION, H, W, tw, min(8, n_frames - tw), per_kernel=False,
              tiles=tiles_2d)
    gpu_ms, wall, _ = run_chain(torch, frames_dev, MOTION, H, W, args.warmup, args.steps,
                                per_kernel=False, tiles=tiles_2d)
    ms_per_step = gpu_ms / args.steps
    mpix = W * H * args.steps / (gpu_ms * 1e-3) / 1e6
    print(f"# 2d chain: {ms_per_step * 1e3:.1f} us/frame (host wall {wall / args.steps * 1e6:.1f}"
          f" us/frame)", file=sys.stderr, flush=True)
    # per-kernel durations: the same frames again, every call between events
    _, _, ktimes = run_chain(torch, frames_dev, MOTION, H, W, args.warmup, args.steps,
                             per_kernel=True, tiles=tiles_2d)

    # roofline of the dominant kernel: the 5x5 a-trous level (VALU-bound;
    # its HBM figures are reported beside)
    npx = W * H
    lv = [k for k in ktimes if k.startswith("atrous")]
    launches = sum(ktimes[k][1] for k in lv)
    tot_ms = sum(ktimes[k][0] * ktimes[k][1] for k in lv)
    mean_us = tot_ms / launches * 1e3
    tot_bytes = sum(ktimes[k][1] * npx * BYTES_PER_PX["atrous_last" if k.endswith("4") else "atrous"]
                    for k in lv)
    costs = issue_costs(torch)
    ops_px = atrous_ops_per_px(costs)
    achieved = npx * ops_px / (mean_us * 1e-6) / 1e12
    hbm_gbs = tot_bytes / (tot_ms * 1e-3) / 1e9
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": measured_traffic(),
                "kernel": "atrous 5x5 level (mean over the five levels)",
                "ops_per_px": round(ops_px, 1), "transcendental_slots": costs,
                "px_per_launch": npx,
                "launch_us": round(mean_us, 2),
                "algorithmic_bytes_per_launch": round(tot_bytes / launches),
                "hbm_achieved_gbs": round(hbm_gbs, 1),
                "hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 4)}
    per_kernel = {k: {"us": round(v[0] * 1e3, 2), "launches": v[1]} for k, v in sorted(ktimes.items())}
    # the spread of single frames, and the same chain replayed as a HIP graph
    frame_us = frame_times(torch, frames_dev, MOTION, H, W, args.warmup, args.steps, tiles=tiles_2d)
    graph = graph_replay(torch, frames_dev, MOTION, H, W, args.warmup, tiles=tiles_2d)
    print(f"# per frame: {frame_us}; as a graph: {graph['ms_per_step'] * 1e3:.1f} us/frame",
          file=sys.stderr, flush=True)

    variants = {}
    if "separable" in want:
        g2, w2, _ = run_chain(torch, frames_dev, MOTION_SEP, H, W, args.warmup, args.steps,
                              per_kernel=False, tiles=tiles_sep)
        _, _, kt2 = run_chain(torch, frames_dev, MOTION_SEP, H, W, args.warmup, args.steps,
                              per_kernel=True, tiles=tiles_sep)
        variants["separable"] = {
            "value": round(W * H * args.steps / (g2 * 1e-3) / 1e6, 1), "unit": "Mpix/s",
            "ms_per_step": round(g2 / args.steps, 4),
            "frame_bytes_per_px": frame_bytes_per_px(5, True),
            "frame_hbm_frac": round(W * H * args.steps * frame_bytes_per_px(5, True)
                                    / (g2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "per_kernel_us": {k: round(v[0] * 1e3, 2) for k, v in sorted(kt2.items())}}
        print(f"# separable chain: {variants['separable']['ms_per_step'] * 1e3:.1f} us/frame",
              file=sys.stderr, flush=True)
    if "uhd_half" in want:
        variants["uhd_half"] = variant_uhd_half(torch, vframes["uhd"], tune=not args.no_tune)
        print(f"# 4K binary16: {variants['uhd_half']['ms_per_step'] * 1e3:.1f} us/frame",
              file=sys.stderr, flush=True)
    if "batched" in want:
        variants["batched"] = variant_batched(torch, vframes["batch_cfg"], vframes["batch"],
                                              vframes["small_cfg"], vframes["small"],
                                              tune=not args.no_tune)
        bv = variants["batched"]
        sm = bv['small_streams']
        print(f"# 16 streams batched: {bv['ms_per_step'] * 1e3:.1f} us/frame (direct "
              f"{bv['direct_launches']['ms_per_step'] * 1e3:.1f}, one by one"
              f" {bv['one_by_one']['ms_per_step'] * 1e3:.1f}); 64 small streams: "
              f"{sm['ms_per_step'] * 1e3:.1f} us/frame (direct "
              f"{sm['direct_launches']['ms_per_step'] * 1e3:.1f}, one by one "
              f"{sm['one_by_one']['ms_per_step'] * 1e3:.1f})", file=sys.stderr, flush=True)
    if "channels" in want:
        variants["channels"] = variant_channels(torch, vframes["channels"])
        print(f"# channels: {variants['channels']}", file=sys.stderr, flush=True)
    if "gradient" in want:
        variants["gradient"] = variant_gradient(torch, vframes["channels"])
        print(f"# gradient: {variants['gradient']}", file=sys.stderr, flush=True)
    if "scene_features" in want:
        variants["scene_features"] = variant_scene_features(torch, frames_np, args.warmup,
                                                            args.steps)
        print(f"# clip / adaptive: {variants['scene_features']}", file=sys.stderr, flush=True)
    if "learned" in want:
        learned = variant_learned(torch, frames_np, vframes["held_out"], args.warmup, args.steps)
        if learned is not None:
            variants["learned"] = learned
    copy_gbs = copy_probe(torch)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(frames_np, warm=4, timed=4,
                           uhd_np=vframes.get("uhd") if vframes else None)

    fb = frame_bytes_per_px(5, False)
    line = {
        "metric": "1080p denoise Mpix/s + HBM roofline frac; learned vs plain at equal RelMSE",
        "value": round(mpix, 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded procedural scene, 1 spp Exp(1) noise with 0.5% x50 fireflies)",
        "config": {"workload": "svgf denoise, 1920x1080, moving camera + 3 moving spheres, "
                               "clamp gamma 1, Reinhard tone map, 5 a-trous levels (2D)",
                   "width": W, "height": H, "frames_timed": args.steps, "levels": 5,
                   "alpha": 0.2, "sigma_z": 1, "sigma_n": 128, "sigma_l": 4},
        "roofline": roofline,
        # a-trous launch shapes per level (persistent, workgroups per CU,
        # tile rows), from the autotuner on this GPU; null: library defaults
        "launch_shapes": {"2d": tiles_2d and [list(t) for t in tiles_2d],
                          "separable": tiles_sep and [list(t) for t in tiles_sep]},
        "frame_hbm_frac": round(mpix * 1e6 * fb / 1e9 / HBM_PEAK_GBS, 4),
        # the whole frame against the HBM roofline at its algorithmic bytes:
        # the target is 0.60 of 8 TB/s
        "hbm_target": {"frame_hbm_frac": round(mpix * 1e6 * fb / 1e9 / HBM_PEAK_GBS, 4),
                       "frame_copy_frac": round(mpix * 1e6 * fb / 1e9 / copy_gbs, 4),
                       "target": 0.60,
                       "met": bool(mpix * 1e6 * fb / 1e9 / HBM_PEAK_GBS >= 0.60)},
        "frame_us": frame_us,
        "graph_replay": graph,
        "frame_bytes_per_px": fb,
        "copy_probe_gbs": round(copy_gbs, 1),
        "per_kernel_us": per_kernel,
        "variants": variants,
        "cpu_baseline": cpu,
        "host": {**host_cpu(), "gen_s": round(gen_s, 1)},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
