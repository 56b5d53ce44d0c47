#!/usr/bin/env python3
"""Fit-step benchmark of the MI355X Gaussian-splatting fit path.

Default workload (foveal refinement, the configuration the metric's
ms/regeneration is defined on): a 256^3 uint16 CT-like phantom (20 random
ellipsoids, HU-like values, noise sigma 20, seed 3); one Gaussian per voxel
above 1200 capped at 500,000 (seed 4), isotropic one-voxel scale, opacity 0.1,
linear transfer-function colour (SH degree 0); 16 views of 1920x1920, 60 degree
FOV, poses on the radius-3 sphere (seed 2); L1 loss masked to a circular fovea
of radius 0.2 W around a random gaze point per view (seed 6), against FP32
emission-absorption ray marches of the same volume; Adam lr 1e-3.  One
regeneration = device seeding from the resident volume + plan + capture + 300
captured steps.  All inputs are seeded and synthetic (the paper's CT datasets
are not available).

Other workloads (--workload): small (1,000 random Gaussians, one 128^2 view,
target rendered by the oracle), phantom (50,000 Gaussians from a 128^3
phantom, one 1024^2 view), batched (200,000 SH3 Gaussians, 8 views of uneven
resolution), stereo (1,000,000 SH3 Gaussians, two eyes of 2064x2208,
recomputed / checkpointed / stored transmittance compared), p0 (the paper's
initial-fit shape: 20,000 Gaussians from the 128^3 phantom, 12 views of 512^2,
one view per step, a 700-step fit), reproject, firsthit.

A "step" is one forward + loss + backward + Adam pass over all views.  The
timed path is the fused step captured in a HIP graph (one launch per stage
for all views, key count on the device), replayed K times after W warm-up
replays, bracketed by device synchronisation and timed with HIP events.
Alongside: the plain path (one host-synchronised plan per view, eager, the
same loss normalisation and fovea culling), the eager fused path, per-stage
kernel times (HIP events recorded by the library on the stream the kernels run
on, over the same step indices as the timed replays), the roofline of the
dominant kernel and the FP64 CPU oracle on a bounded sample.  Each phase
announces itself on stderr before it starts.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload NAME]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gaussian fit-steps/s (fwd+bwd+Adam), Mpix/s, ms/regeneration vs plain"

# Per-pair FP32 operation counts of the compositing definition (FMA = 2):
# alpha evaluation of a (pixel, splat) pair; extra work when the pair is
# included in the forward image; extra adjoint work per included pair.
FLOPS_ALPHA = 18
FLOPS_FWD_INCLUDED = 10
FLOPS_BWD_INCLUDED = 48
# MI355X FP32 vector peak: 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz x 2
# (packed dual-issue FP32) = 157.3 TFLOP/s.  Without packed FP32 instructions
# (the library is compiled without them) the attainable peak is half that, 78.6 TFLOP/s,
# which is quoted beside the published figure.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
GSF_FLAG_CAPACITY = 1


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def phase(msg):
    """Announce a phase before it starts (flushed), so a long phase is named."""
    log(f"[bench] >> {msg}")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


@dataclasses.dataclass
class Workload:
    name: str
    description: str
    data: str
    P: object                       # planar float32 [C][n]
    cams: list
    targets: object = None          # float32, per view [3][H][W], views concatenated (flat)
    gaze: object = None             # float32 [V][2] or None
    target_params: object = None    # Gaussian set whose render is the target
    volume: object = None
    device_targets: bool = False    # targets: FP32 ray march of `volume` on the device
    views_per_step: int = 0         # 0: every view each step; 1: one view per step, cycled
    fit_steps: int = 0              # steps of one fit (p0), reported as ms per fit


def _phantom(n_vol, cap):
    import synth
    phase(f"phantom {n_vol}^3 and voxel seeding (cap {cap}) on the host")
    vol = synth.phantom(n_vol, seed=synth.SEED_VOLUME)
    P = synth.seed_from_volume(vol, cap=cap, seed=synth.SEED_CAP_SUBSET)
    return P, vol


def _marched_targets(vol, cams):
    import numpy as np

    import synth
    phase(f"FP64 ray march of {len(cams)} target view(s) on the host")
    return np.concatenate([synth.raymarch_volume(vol, c)[:3].reshape(-1) for c in cams])


def build_workload(name="foveal"):
    import numpy as np

    import synth
    if name == "small":
        P = synth.random_gaussians(1000, seed=synth.SEED_GAUSSIANS)
        cam = synth.axis_camera(128, 128)
        tgt = np.load(os.path.join(ROOT, "tests", "golden", "cfg1_target_128.npy"))[:3]
        return Workload(name, "plain single view: 1,000 random Gaussians (SH0), one 128x128 view, "
                              "L1 vs the seed-1 set rendered by the oracle, Adam lr 1e-3",
                        "synthetic: seeded random Gaussians; target from the FP64 oracle",
                        P, [cam], targets=np.ascontiguousarray(tgt.reshape(-1)))
    if name == "phantom":
        d = synth.sphere_directions(1, seed=synth.SEED_POSES)[0]
        cam = synth.look_at_camera(3.0 * d, width=1024, height=1024, fov_x_deg=60.0)
        P, vol = _phantom(128, 50_000)
        return Workload(name, "phantom-seeded fit: 128^3 phantom, 50,000 Gaussians (SH0), one "
                              "1024x1024 view, L1 vs ray-marched target, Adam lr 1e-3",
                        "synthetic: seeded CT-like phantom, voxel-seeded Gaussians, ray-marched target",
                        P, [cam], targets=_marched_targets(vol, [cam]), volume=vol)
    if name == "p0":
        cams = synth.sphere_cameras([(512, 512)] * 12, radius=3.0, seed=synth.SEED_POSES)
        P, vol = _phantom(128, 20_000)
        return Workload(name, "paper-shape initial fit: 128^3 phantom, 20,000 Gaussians (SH0), 12 "
                              "views of 512x512, one view per step (cycled), 700-step fit, L1 vs "
                              "ray-marched targets, Adam lr 1e-3",
                        "synthetic: seeded CT-like phantom, voxel-seeded Gaussians, ray-marched targets",
                        P, cams, targets=_marched_targets(vol, cams), volume=vol,
                        views_per_step=1, fit_steps=700)
    if name == "batched":
        n = 200_000
        mu = synth.scaled_logscale_mean(n)
        P = synth.random_gaussians(n, seed=synth.SEED_GAUSSIANS, sh_degree=3, logscale_mean=mu)
        Pt = synth.random_gaussians(n, seed=synth.SEED_TARGET_SET, sh_degree=3, logscale_mean=mu)
        cams = synth.sphere_cameras(synth.draw_resolutions(8, seed=synth.SEED_RESOLUTIONS),
                                    radius=3.0, seed=synth.SEED_POSES)
        return Workload(name, "batched uneven views: 200,000 random Gaussians (SH3), 8 views with "
                              "resolutions drawn from {512^2, 768x1024, 1024^2, 1536^2, 2048^2}, "
                              "L1 vs the seed-1 set, Adam lr 1e-3",
                        "synthetic: seeded random Gaussians; target = the seed-1 set rendered by "
                        "this library's forward", P, cams, target_params=Pt)
    if name == "foveal":
        dirs = synth.sphere_directions(16, seed=synth.SEED_POSES)
        cams = [synth.look_at_camera(3.0 * d, width=1920, height=1920, fov_x_deg=60.0) for d in dirs]
        gaze = synth.gaze_points(cams, seed=synth.SEED_GAZE)
        P, vol = _phantom(256, 500_000)
        return Workload(name, "foveal refinement: 256^3 phantom, 500,000 Gaussians (SH0), 16 views "
                              "of 1920x1920, L1 masked to a fovea of radius 0.2 W at a random gaze "
                              "point per view, FP32 ray-marched targets, 300-step regeneration, "
                              "Adam lr 1e-3",
                        "synthetic: seeded CT-like phantom, voxel-seeded Gaussians, FP32 ray-marched "
                        "targets", P, cams, gaze=gaze, volume=vol, device_targets=True)
    if name == "stereo":
        n = 1_000_000
        mu = synth.scaled_logscale_mean(n)
        P = synth.random_gaussians(n, seed=synth.SEED_GAUSSIANS, sh_degree=3, logscale_mean=mu)
        Pt = synth.random_gaussians(n, seed=synth.SEED_TARGET_SET, sh_degree=3, logscale_mean=mu)
        cams = synth.stereo_cameras(2064, 2208, radius=3.0, baseline=0.064, seed=synth.SEED_POSES)
        return Workload(name, "stereo HMD: 1,000,000 random Gaussians (SH3), two eyes of 2064x2208 "
                              "with a 64 mm baseline, L1 vs the seed-1 set, Adam lr 1e-3",
                        "synthetic: seeded random Gaussians; target = the seed-1 set rendered by "
                        "this library's forward", P, cams, target_params=Pt)
    raise SystemExit(f"unknown workload {name!r}")


def render_targets(ctx, wl, dev):
    """RGB of the target Gaussian set through the library's forward (a plain
    host-sized plan with recomputed transmittance)."""
    import numpy as np
    import torch

    import paper_2601_22026_amd as gs
    Pt = torch.from_numpy(np.ascontiguousarray(wl.target_params)).to(dev)
    deg = int(round(((Pt.shape[0] - 11) // 3) ** 0.5)) - 1
    sizes = [(c.width, c.height) for c in wl.cams]
    plan = gs.Plan(ctx, Pt.shape[1], sizes, deg, 16, 128, host_sized=True)
    rgba = torch.zeros(4 * sum(w * h for w, h in sizes), dtype=torch.float32, device=dev)
    plan.forward(Pt, Pt.shape[1], gs.cameras_to_device(wl.cams, dev), rgba)
    out, off = [], 0
    for w, h in sizes:
        out.append(rgba[4 * off:4 * off + 3 * w * h])
        off += w * h
    plan.close()
    return torch.cat(out).contiguous()


def device_marched_targets(ctx, vol_dev, cams):
    """RGB planes of the FP32 ray march of every view on the device."""
    import torch

    import paper_2601_22026_amd as gs
    rgba = gs.raymarch(ctx, vol_dev, cams)
    out, off = [], 0
    for c in cams:
        w, h = c.width, c.height
        out.append(rgba[4 * off:4 * off + 3 * w * h])
        off += w * h
    return torch.cat(out).contiguous()


def time_steps(fn, steps, stream):
    """(mean ms over `steps` back-to-back calls, median ms of one call): an
    event between consecutive calls, device synchronised before and after."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        fn()
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    per = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
    return ev[0].elapsed_time(ev[steps]) / steps, per[len(per) // 2]


def radix_passes(bits):
    """Passes of the library's radix sorts: digits of at most 8 bits."""
    return 0 if bits <= 0 else (bits + 7) // 8


def composited_pixels(cams, gaze, radius_frac, tile):
    """Pixels of the tiles a fovea-culled step composites, back-propagates and
    takes the loss over: per view, the tiles that meet the box of pixel centres
    within the radius of the gaze point plus one pixel, clipped to the view,
    and of those the ones whose rectangle of pixel centres comes within the
    radius plus one pixel of the gaze point (the box's corners are skipped);
    the FP32 arithmetic of the kernels' tests."""
    import numpy as np
    f32 = np.float32
    n = 0
    for c, (gx, gy) in zip(cams, gaze):
        gx, gy = f32(gx), f32(gy)
        r = f32(radius_frac) * f32(c.width)
        x0 = max(np.floor(gx - r - f32(0.5)) - 1, 0)
        x1 = min(np.ceil(gx + r - f32(0.5)) + 1, c.width - 1)
        y0 = max(np.floor(gy - r - f32(0.5)) - 1, 0)
        y1 = min(np.ceil(gy + r - f32(0.5)) + 1, c.height - 1)
        if x0 > x1 or y0 > y1:
            continue
        tx0, tx1, ty0, ty1 = int(x0) // tile, int(x1) // tile, int(y0) // tile, int(y1) // tile
        rl = r + f32(1)
        for ty in range(ty0, ty1 + 1):
            py0, py1 = f32(ty * tile) + f32(0.5), f32(min((ty + 1) * tile, c.height)) - f32(0.5)
            dy = max(py0 - gy, gy - py1, f32(0))
            for tx in range(tx0, tx1 + 1):
                px0, px1 = f32(tx * tile) + f32(0.5), f32(min((tx + 1) * tile, c.width)) - f32(0.5)
                dx = max(px0 - gx, gx - px1, f32(0))
                if dx * dx + dy * dy <= rl * rl:
                    n += (min((tx + 1) * tile, c.width) - tx * tile) * (min((ty + 1) * tile, c.height) - ty * tile)
    return n


def depth_sort_passes(keys):
    """Passes of the library's depth sort over these depth keys (the records
    that list a tile): three when every key lies below 2^24 above the smallest
    key with its low 8 bits cleared, else four."""
    if keys.size == 0:
        return 3
    base = int(keys.min()) & ~0xFF
    return 3 if int(keys.max()) - base < (1 << 24) else 4


def hbm_bytes_per_launch(stage, N, R, M, npix, planes, tiles, A, depth_passes=4):
    """Algorithmic HBM bytes one launch of a stage must move: N Gaussians,
    R = N * views records, A of them listing a tile, M keys, npix pixels
    composited (the fovea tiles' pixels when the step is fovea-culled),
    `planes` floats per Gaussian, `depth_passes` passes of the depth sort."""
    tile_passes = radix_passes(max(1, (tiles - 1).bit_length()))
    return {
        "project": planes * 4 * N + 88 * R,                   # params in; splat, key, box, count, ellipse, spans
        # counts in; slots, depth keys in, (depth, entry) pairs and 32-byte entries out; ranges cleared
        "duplicate": 4 * R + 48 * A + 8 * tiles,
        # depth sort of the A entries (per pass: key histogram, pair in, pair out; the
        # last pass writes no keys), the emission's count totals and the emission
        # (sorted entries, 32-byte entries in; (tile, record) keys out)
        "depth_sort": (depth_passes - 1) * 20 * A + 16 * A + 8 * A + 36 * A + 8 * M,
        "tile_sort": tile_passes * 20 * M,                    # per pass: key histogram, pair in, pair out
        "ranges": 4 * M + 28 * tiles,                         # sorted tile ids in; ranges out; order
        "render": 40 * M + 24 * npix,                         # splat gather per key; RGBA, T, count out
        "loss": 40 * npix,                                    # RGBA, target in; dL/dRGBA out
        "render_bwd": 76 * M + 24 * npix,                     # splat gather; pixel state in; per-key gradient out
        # params in, grads out; SH 0-1: the per-key gradients (with count and offset) summed
        # inside, SH 2-3: g2d, which grad_sum wrote
        "project_bwd": planes * 8 * N + (36 * M + 8 * R if planes <= 23 else 36 * R),
        "adam": 28 * planes * N,
        "grad_sum": 36 * M + 44 * R,                          # per-key gradient, count, offset in; g2d out
    }.get(stage)


def profiled_traffic(workload, kernel, tile, batch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summaries (FETCH_SIZE and WRITE_SIZE, scaled by a copy-kernel calibration),
    or None when no summary matches this workload, kernel, tile and LDS batch,
    or the compositing source has changed since the counters were taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2601_22026_amd", "csrc", "raster.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic:"):
                continue
            kv = dict(f.split("=", 1) for f in line.split()[1:])
            if (kv.get("workload") == workload and kv.get("kernel") == kernel
                    and int(kv.get("tile", 0)) == tile and int(kv.get("lds_batch", 0)) == batch
                    and kv.get("raster_sha256") == h):
                return int(kv["bytes_per_launch"])
    return None


def cpu_baseline(wl, targets_np, budget_s=15.0):
    """FP64 oracle fit step (render, masked L1, adjoint, Adam) timed on a
    bounded sample of the pixels that carry loss (every pixel, or the fovea's
    when the loss is masked), spread evenly over each view.  Two sample sizes
    per view give the oracle's fixed per-view cost (projection and depth sort,
    once for the render and once for the adjoint) and its cost per pixel; the
    step is extrapolated to every loss-carrying pixel of every view, plus one
    dense Adam update."""
    import numpy as np

    import oracle
    Pd = wl.P.astype(np.float64)
    offs = np.cumsum([0] + [c.width * c.height for c in wl.cams])
    views = wl.cams if wl.views_per_step == 0 else wl.cams[:1]

    def loss_pixels(k, cam):
        W, H = cam.width, cam.height
        if wl.gaze is None:
            return np.arange(W * H)
        gx, gy = float(wl.gaze[k][0]), float(wl.gaze[k][1])
        r = 0.2 * W
        ii, jj = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
        return np.flatnonzero(((ii - gx) ** 2 + (jj - gy) ** 2 <= r * r).reshape(-1))

    full = [loss_pixels(k, c) for k, c in enumerate(views)]

    def run_view(k, cam, count):
        pix_all = full[k]
        pix = pix_all[np.linspace(0, pix_all.size - 1, min(count, pix_all.size)).astype(np.int64)]
        t0 = time.perf_counter()
        r = oracle.render(Pd, cam, pixels=pix)
        tgt = targets_np[3 * offs[k]:3 * offs[k + 1]].reshape(3, -1)[:, pix]
        s, cnt, dl = oracle.loss_l1_view(r.rgba, tgt, type("c", (), {"width": pix.size, "height": 1})())
        oracle.backward(Pd, cam, dl / max(cnt, 1), pixels=pix)
        return time.perf_counter() - t0, pix.size

    t_start = time.perf_counter()
    most = max(f.size for f in full)
    k, prev, cur = 4, None, None
    while True:
        t0 = time.perf_counter()
        cur = (k, [run_view(v, c, k) for v, c in enumerate(views)])
        took = time.perf_counter() - t0
        log(f"[bench] oracle sample: {k} px per view in {took:.1f} s")
        if prev is not None and (took >= budget_s / 3 or k >= most):
            break
        prev, k = cur, min(4 * k, most)
    est, used = 0.0, 0
    for v in range(len(views)):
        (t1, n1), (t2, n2) = prev[1][v], cur[1][v]
        slope = max((t2 - t1) / max(n2 - n1, 1), 0.0)
        fixed = max(t1 - n1 * slope, 0.0)
        est += fixed + slope * full[v].size
        used += n2
    k1 = prev[0]
    G = np.zeros_like(Pd)
    t0 = time.perf_counter()
    oracle.adam(Pd.copy(), G, np.zeros_like(Pd), np.zeros_like(Pd), 1)
    est += time.perf_counter() - t0
    spent = time.perf_counter() - t_start
    carried = int(sum(f.size for f in full))
    return {"value": 1.0 / est, "unit": "fit-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{used} of the step's {carried} loss-carrying pixels over {len(views)} "
                      f"view(s) (plus {k1} per view to split the per-view cost from the per-pixel "
                      f"cost), {spent:.1f} s, extrapolated to the whole step; all "
                      f"{wl.P.shape[1]} Gaussians per pixel, no tiles",
            "s_per_step_extrapolated": round(est, 2)}


def bench_reproject(args):
    """Viewer-side workload: the depth-guided reprojection warp of one eye's
    foveal image (2064 x 2208, the stereo rig's eye resolution; the paper's
    512 x 512 foveal size is timed too) to the head pose a frame later."""
    import numpy as np
    import torch

    import paper_2601_22026_amd as gs
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)
    sizes = [(2064, 2208), (512, 512)]
    out = {}
    with torch.cuda.stream(stream):
        ctx = gs.Context(0)
        for (w, h) in sizes:
            old = synth.look_at_camera([0.2, -0.1, -2.5], [0.0, 0.0, 0.0], w, h, 60.0)
            new = synth.look_at_camera([0.23, -0.09, -2.52], [0.03, 0.02, 0.0], w, h, 60.0)
            depth = synth.sphere_depth(old, radius=1.0)
            rgba = np.random.default_rng(synth.SEED_GAUSSIANS).uniform(size=(4, h, w)).astype(np.float32)
            P0, V0 = synth.clip_matrices(old)
            P1, V1 = synth.clip_matrices(new)
            d_dev = torch.from_numpy(depth).to(dev)
            c_dev = torch.from_numpy(rgba).to(dev)
            zbuf = torch.empty(w * h, dtype=torch.int64, device=dev)
            res = {}

            def warp():
                res["o"] = gs.reproject_warp(ctx, c_dev, d_dev, P0, V0, old.campos, P1, V1, w, h,
                                             zbuf=zbuf)
            warp()
            torch.cuda.synchronize()
            # the three launches captured once and replayed, so host call overhead
            # stays out of the timed region
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                warp()
            for _ in range(args.warmup):
                graph.replay()
            ms, _ = time_steps(graph.replay, args.steps, stream)
            landed = int((res["o"][1] >= 0).sum().item())
            # algorithmic bytes: depth and colour in, z-buffer cleared, one 64-bit
            # atomic per landing point, resolve reads the z-buffer and the winner's
            # colour and writes colour and source index
            bytes_ = 4 * w * h + 8 * w * h + 16 * landed + 8 * w * h + 16 * landed + 20 * w * h
            out[(w, h)] = {"ms": ms, "mpix_per_s": w * h / (ms * 1e-3) / 1e6, "bytes": bytes_,
                           "landed": landed}
            log(f"[bench] reproject {w}x{h}: {ms * 1e3:.1f} us per warp, landed {landed}, "
                f"{bytes_ / (ms * 1e-3) / 1e9:.0f} GB/s")
    main_w, main_h = sizes[0]
    r = out[sizes[0]]
    gbs = r["bytes"] / (r["ms"] * 1e-3) / 1e9
    res = {
        "metric": METRIC, "value": round(r["mpix_per_s"], 1), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: unit-sphere first-hit depth, seeded colours, 3 cm / 1 degree head motion",
        "config": {"workload": f"depth-guided reprojection warp of a {main_w}x{main_h} foveal image "
                               "to the next head pose (Eqs. (2)-(4), nearest-wins forward warp)",
                   "name": "reproject", "width": main_w, "height": main_h},
        "paper_foveal_512": {"us_per_warp": round(out[(512, 512)]["ms"] * 1e3, 2),
                             "mpix_per_s": round(out[(512, 512)]["mpix_per_s"], 1)},
        "roofline": {"kernel": "reproject_warp (clear, splat, resolve)", "bound": "hbm",
                     "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None},
    }
    if not args.no_cpu_baseline:
        import oracle
        w, h = 512, 512
        old = synth.look_at_camera([0.2, -0.1, -2.5], [0.0, 0.0, 0.0], w, h, 60.0)
        new = synth.look_at_camera([0.23, -0.09, -2.52], [0.03, 0.02, 0.0], w, h, 60.0)
        depth = synth.sphere_depth(old, radius=1.0)
        rgba = np.random.default_rng(synth.SEED_GAUSSIANS).uniform(size=(4, h, w))
        P0, V0 = synth.clip_matrices(old)
        P1, V1 = synth.clip_matrices(new)
        t0 = time.perf_counter()
        oracle.reproject_warp(rgba, depth, P0, V0, old.campos, P1, V1, w, h)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(w * h / dt / 1e6, 4), "unit": "Mpix/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one 512x512 warp in {dt:.2f} s (numpy, one thread)"}
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


def bench_first_hits(args):
    """Initial point cloud: the first significant hits of the pixel rays of 8
    views (256 x 256 each, poses on the radius-3 sphere) of the 128^3 phantom,
    capped at the paper's 20,000 points; one call per timed step (it
    synchronises, so the time is the whole seeding as a caller sees it)."""
    import numpy as np
    import torch

    import paper_2601_22026_amd as gs
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    vol = synth.phantom(128, seed=synth.SEED_VOLUME)
    cams = synth.sphere_cameras([(256, 256)] * 8)
    kw = dict(step=0.01, extinction=synth.EXTINCTION, threshold=synth.TF_THRESHOLD,
              range_=synth.TF_RANGE, lo=synth.TF_LO, hi=synth.TF_HI)
    cap = 20_000
    ctx = gs.Context(0)
    v_dev = torch.from_numpy(vol.view(np.int16)).to(dev)
    for _ in range(max(1, args.warmup)):
        P, ids = gs.seed_first_hits(ctx, v_dev, cams, cap, synth.SEED_CAP_SUBSET, **kw)
    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, ids = gs.seed_first_hits(ctx, v_dev, cams, cap, synth.SEED_CAP_SUBSET, **kw)
        times.append(time.perf_counter() - t0)
    ms = 1e3 * float(np.median(times))
    nrays = sum(c.width * c.height for c in cams)
    log(f"[bench] first hits: {ids.numel()} points from {nrays} rays in {ms:.2f} ms (median)")
    res = {
        "metric": METRIC, "value": round(1e3 / ms, 2), "unit": "point clouds/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: seeded CT-like phantom, sphere poses",
        "config": {"workload": "first-hit point cloud: 128^3 phantom, 8 views of 256x256 rays, "
                               "hit at accumulated opacity 0.5, 20,000 points",
                   "name": "firsthit", "rays": nrays, "points": int(ids.numel())},
        "paper_context": "about 50 ms for 20,000 points with 64 path-traced samples each on an "
                         "RTX 4090 (a different colouring, context only)",
        "roofline": None, "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        oracle.seed_first_hits(vol, cams, cap, synth.SEED_CAP_SUBSET, **kw)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(1.0 / dt, 4), "unit": "point clouds/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"the whole seeding once, {dt:.2f} s"}
    print(json.dumps(res), flush=True)


def check_flags(flags, what):
    if flags & GSF_FLAG_CAPACITY:
        raise SystemExit(f"[bench] {what}: key capacity overflowed during timed steps "
                         f"(flags {flags}); those steps did no fitting, so the timing is void")
    if flags:
        raise SystemExit(f"[bench] {what}: device flags {flags} (non-finite loss)")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="foveal",
                    choices=["foveal", "small", "phantom", "batched", "stereo", "p0", "reproject",
                             "firsthit"])
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--lds-batch", type=int, default=128)
    ap.add_argument("--t-mode", type=int, default=1, choices=[0, 1, 2],
                    help="transmittance of the timed step: 0 recomputed, 1 checkpointed, 2 stored")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --tile/--lds-batch/--t-mode instead of sweeping tile x LDS batch x "
                         "transmittance mode (recomputed, checkpointed)")
    ap.add_argument("--compare-t-modes", action="store_true",
                    help="also time the captured step and record peak device memory with each "
                         "transmittance mode (always on for --workload stereo)")
    ap.add_argument("--no-fovea-cull", action="store_true",
                    help="composite full frames even when the loss is masked to a fovea")
    ap.add_argument("--full-frame", action="store_true",
                    help="with a fovea-masked loss, also time the captured step without fovea "
                         "culling (the culling gain)")
    ap.add_argument("--regen-steps", type=int, default=300,
                    help="steps of one regeneration (foveal workload)")
    ap.add_argument("--regen-runs", type=int, default=3)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 256 MiB device buffer 5 times (reference for HBM byte "
                         "counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": x.numel() * 4,
                          "copy_bytes_written_per_launch": x.numel() * 4, "launches": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the multi-GPU "
              "sharding of this path (views split across GPUs, gradients all-reduced) is not "
              "built.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "reproject":
        bench_reproject(args)
        return
    if args.workload == "firsthit":
        bench_first_hits(args)
        return

    import numpy as np
    import torch

    import paper_2601_22026_amd as gs

    t0 = time.perf_counter()
    phase(f"building workload {args.workload}")
    wl = build_workload(args.workload)
    P, cams = wl.P, wl.cams
    N, planes, V = P.shape[1], P.shape[0], len(cams)
    step_cams = cams if wl.views_per_step == 0 else cams[:1]
    npix = sum(c.width * c.height for c in step_cams)
    log(f"[bench] workload {wl.name}: {N} Gaussians, {V} view(s), {npix} px per step, built in "
        f"{time.perf_counter() - t0:.1f} s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)
    # a masked loss lets the fused step composite only the tiles that meet each fovea
    cull = wl.gaze is not None and not args.no_fovea_cull
    cfg = gs.FitConfig(lr=1e-3, tile=args.tile, lds_batch=args.lds_batch, t_mode=args.t_mode,
                       fovea_cull=cull)
    with torch.cuda.stream(stream):
        ctx = gs.Context(0)
        vol_dev = None
        if wl.volume is not None:
            vol_dev = torch.from_numpy(np.ascontiguousarray(wl.volume).view(np.int16)).to(dev)
        if wl.device_targets:
            phase(f"FP32 ray march of {V} target views on the device")
            tgt_dev = device_marched_targets(ctx, vol_dev, cams)
        elif wl.targets is None:
            phase("rendering the target Gaussian set")
            tgt_dev = render_targets(ctx, wl, dev)
        else:
            tgt_dev = torch.from_numpy(np.ascontiguousarray(wl.targets)).to(dev)
        gaze_dev = None if wl.gaze is None else torch.from_numpy(np.ascontiguousarray(wl.gaze)).to(dev)
        P_dev = torch.from_numpy(np.ascontiguousarray(P)).to(dev)
        cams_all = gs.cameras_to_device(cams, dev)
        view_off = np.cumsum([0] + [c.width * c.height for c in cams])

        def fit(c, fused=True, params=None):
            if wl.views_per_step == 0:
                return gs.FitStep(ctx, (P_dev if params is None else params).clone(), cams,
                                  tgt_dev, gaze_dev, cfg=c, fused=fused)
            # one view per step: the step's camera and target are copied into its
            # buffers before each step, so size the keys for the heaviest view
            if c.key_capacity == 0:
                c = dataclasses.replace(c, key_capacity=max_view_keys(c) * 3 // 2 + (1 << 16))
            return gs.FitStep(ctx, P_dev.clone(), cams[:1],
                              tgt_dev[:3 * cams[0].width * cams[0].height].clone(), None, cfg=c,
                              fused=fused)

        def max_view_keys(c):
            m = 0
            for k, cam in enumerate(cams):
                pl = gs.Plan(ctx, N, [(cam.width, cam.height)], 0, c.tile, c.lds_batch,
                             host_sized=True)
                out = torch.empty(4 * cam.width * cam.height, dtype=torch.float32, device=dev)
                pl.forward(P_dev, N, cams_all[128 * k:128 * (k + 1)], out)
                m = max(m, pl.poll()[1])
                pl.close()
            return m

        counter = [0]

        def runner(fs, captured):
            """The callable of one step: for one view per step, select the next
            view's camera and target first."""
            def one():
                if wl.views_per_step:
                    k = counter[0] % V
                    counter[0] += 1
                    fs.cams_dev.copy_(cams_all[128 * k:128 * (k + 1)], non_blocking=True)
                    fs.targets.copy_(tgt_dev[3 * view_off[k]:3 * view_off[k + 1]], non_blocking=True)
                (fs.replay if captured else fs.step)()
            return one

        tune = None
        if not args.no_autotune:
            phase("autotune: captured step per tile x LDS batch x transmittance mode")
            tp, tc, tt = (P_dev, cams, tgt_dev) if wl.views_per_step == 0 else \
                (P_dev, cams[:1], tgt_dev[:3 * cams[0].width * cams[0].height])
            best, sweep = gs.autotune(ctx, tp, tc, tt, gaze_dev, cfg=cfg, t_modes=(0, 1),
                                      stream=stream)
            tune = {"best": list(best), "us_per_step": {f"{t}x{b}/t{m}": round(ms * 1e3, 1)
                                                        for (t, b, m), ms in sorted(sweep.items())}}
            cfg = dataclasses.replace(cfg, tile=best[0], lds_batch=best[1], t_mode=best[2])
            log(f"[bench] autotune: best tile {best[0]} batch {best[1]} t_mode {best[2]}; "
                f"{tune['us_per_step']}")

        # fused, captured: the timed path
        phase(f"fused captured step: {args.warmup} warm-up + {args.steps} timed replays")
        fused = fit(cfg)
        fused.capture()
        one = runner(fused, True)
        for _ in range(args.warmup):
            one()
        ms_fused, med_fused = time_steps(one, args.steps, stream)
        flags, M = fused.poll()
        check_flags(flags, "fused captured step")
        # records that list a tile (the depth sort's input) in the last step
        act = fused.plan.debug(gs._abi.GSF_DBG_COUNT, np.uint32, N * len(step_cams)) > 0
        act_depth = fused.plan.debug(gs._abi.GSF_DBG_DEPTH, np.uint32, N * len(step_cams))[act]
        A = int(act_depth.size)
        depth_passes = depth_sort_passes(act_depth)
        loss_fused = float(fused.loss.item())
        log(f"[bench] fused+captured: {ms_fused * 1e3:.1f} us/step (median {med_fused * 1e3:.1f}), "
            f"keys {M}, flags {flags}, loss {loss_fused:.5f}")
        ws_fused = fused.plan.workspace_bytes
        total_tiles = fused.plan.total_tiles
        fused.plan.close()
        del fused

        fit_run = None
        if wl.fit_steps:
            phase(f"one {wl.fit_steps}-step fit, captured, one view per step")
            fr = fit(cfg)
            fr.capture()
            one = runner(fr, True)
            counter[0] = 0
            torch.cuda.synchronize()
            t_fit = time.perf_counter()
            for _ in range(wl.fit_steps):
                one()
            torch.cuda.synchronize()
            ms_fit = (time.perf_counter() - t_fit) * 1e3
            flags, _ = fr.poll()
            check_flags(flags, "fit")
            fit_run = {"steps": wl.fit_steps, "ms_per_fit": round(ms_fit, 2),
                       "ms_per_step": round(ms_fit / wl.fit_steps, 4),
                       "loss_after_fit": round(float(fr.loss.item()), 6),
                       "paper_context": "about 0.85 s for 700 iterations at 512^2 on an RTX 4090 "
                                        "(about 1.2 ms per iteration; context only)"}
            fr.plan.close()
            del fr
            log(f"[bench] {wl.fit_steps}-step fit: {ms_fit:.1f} ms")

        culled_gain = None
        if cull and args.full_frame:
            phase("fused captured step over full frames (no fovea culling), for the culling gain")
            fu = fit(dataclasses.replace(cfg, fovea_cull=False))
            fu.capture()
            for _ in range(args.warmup):
                fu.replay()
            ms_full, _ = time_steps(fu.replay, args.steps, stream)
            check_flags(fu.poll()[0], "full-frame step")
            fu.plan.close()
            del fu
            culled_gain = {"full_frame_ms_per_step": round(ms_full, 4),
                           "culling_speedup": round(ms_full / ms_fused, 3)}
            log(f"[bench] fused full-frame: {ms_full * 1e3:.1f} us/step")

        regen = None
        if wl.name == "foveal" and args.regen_runs > 0:
            # one regeneration: seed the Gaussians on the device from the resident
            # volume, plan, capture, run the steps - wall clock, synchronised
            import synth
            runs, seeds, plans, caps, replans = [], [], [], [], 0
            same = None
            for k in range(args.regen_runs):
                phase(f"regeneration {k + 1}/{args.regen_runs} ({args.regen_steps} steps)")
                torch.cuda.synchronize()
                t_start = time.perf_counter()
                Ps = gs.seed_volume(ctx, vol_dev, cap=N, seed=synth.SEED_CAP_SUBSET)
                t_seeded = time.perf_counter()
                rf = gs.FitStep(ctx, Ps, cams, tgt_dev, gaze_dev, cfg=cfg, fused=True)
                torch.cuda.synchronize()
                t_planned = time.perf_counter()
                rf.capture()
                torch.cuda.synchronize()
                t_captured = time.perf_counter()
                replans += rf.run(args.regen_steps)
                torch.cuda.synchronize()
                runs.append((time.perf_counter() - t_start) * 1e3)
                seeds.append((t_seeded - t_start) * 1e3)
                plans.append((t_planned - t_seeded) * 1e3)
                caps.append((t_captured - t_planned) * 1e3)
                if same is None:   # the device seeding reproduces the workload's Gaussians
                    again = gs.seed_volume(ctx, vol_dev, cap=N, seed=synth.SEED_CAP_SUBSET)
                    same = bool(torch.equal(again.cpu(), torch.from_numpy(P)))
                rf.plan.close()
                del rf
            # the targets' ray march on the device, reported apart (S24)
            march = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                gs.raymarch(ctx, vol_dev, cams)
                e1.record(stream)
                e1.synchronize()
                march.append(e0.elapsed_time(e1))
            regen = {"ms_per_regeneration": round(sorted(runs)[len(runs) // 2], 2),
                     "steps": args.regen_steps, "runs_ms": [round(r, 2) for r in runs],
                     "seeding_ms": round(sorted(seeds)[len(seeds) // 2], 2),
                     "plan_ms": round(sorted(plans)[len(plans) // 2], 2),
                     "capture_ms": round(sorted(caps)[len(caps) // 2], 2),
                     "key_replans": replans,
                     "seeded_on_device_equals_workload": same,
                     "target_raymarch_ms": round(sorted(march)[1], 2),
                     "includes": "seeding from the device-resident volume, plan creation, graph "
                                 "capture and the captured fit steps, with a flag poll every 100 "
                                 "steps (the targets' ray march is timed apart)",
                     "paper_context": "full peripheral-model regeneration in about 1.0 s on an RTX "
                                      "4090, including path tracing the views (context only)"}
            log(f"[bench] regeneration ({args.regen_steps} steps): {regen['ms_per_regeneration']} ms "
                f"(seeding {regen['seeding_ms']} ms, plan {regen['plan_ms']} ms, capture "
                f"{regen['capture_ms']} ms, same Gaussians as the workload: {same}, "
                f"key re-plans {replans}); target ray march {regen['target_raymarch_ms']} ms")

        # fused, eager (same plan shape, no graph)
        phase("fused eager step")
        eager = fit(cfg)
        one = runner(eager, False)
        for _ in range(args.warmup):
            one()
        ms_eager, _ = time_steps(one, args.steps, stream)
        check_flags(eager.poll()[0], "eager step")
        eager.plan.close()
        del eager
        log(f"[bench] fused eager: {ms_eager * 1e3:.1f} us/step")

        # per-stage kernel times: a fresh eager fused step taken through the same
        # step indices as the timed replays (W warm-up, then K), with HIP events
        # recorded by the library around each stage on the stream it launches on
        phase("per-stage kernel times (eager, library HIP events)")
        staged = fit(cfg)
        one = runner(staged, False)
        counter[0] = 0
        for _ in range(args.warmup):
            one()
        staged.plan.set_timing(True)
        for _ in range(args.steps):
            one()
        st = staged.plan.stage_times()
        staged.plan.set_timing(False)
        staged.plan.close()
        del staged
        stages = {k: (ms / max(c, 1)) for k, (ms, c) in st.items() if c}
        log("[bench] stage us/launch: " + ", ".join(f"{k} {v * 1e3:.1f}" for k, v in stages.items()))
        # pair counts of the same K steps (a separate run: counting synchronises)
        phase("pair counts of the same steps")
        counted = fit(cfg)
        one = runner(counted, False)
        counter[0] = 0
        for _ in range(args.warmup):
            one()
        pairs = {}
        for _ in range(args.steps):
            one()
            for k, v in counted.plan.count_pairs().items():
                pairs[k] = pairs.get(k, 0) + v / args.steps
        counted.plan.close()
        del counted
        pairs = {k: int(round(v)) for k, v in pairs.items()}
        log(f"[bench] pairs per step (mean of the K steps): {pairs}")

        # plain path: one host-synchronised plan per view, eager
        ms_plain = None
        if not args.no_plain:
            phase("plain step (one host-synchronised plan per view, eager)")
            plain = fit(cfg, fused=False)
            one = runner(plain, False)
            counter[0] = 0
            for _ in range(args.warmup):
                one()
            ms_plain, _ = time_steps(one, args.steps, stream)
            plain.close()
            del plain
            log(f"[bench] plain: {ms_plain * 1e3:.1f} us/step")

        # transmittance modes: step time and peak device memory
        modes = None
        if args.compare_t_modes or wl.name == "stereo":
            modes = {}
            for m, label in enumerate(["recompute", "checkpointed", "stored"]):
                phase(f"transmittance mode {label}")
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
                torch.cuda.reset_peak_memory_stats(dev)
                base = torch.cuda.memory_allocated(dev)
                fm = fit(dataclasses.replace(cfg, t_mode=m))
                fm.capture()
                for _ in range(args.warmup):
                    fm.replay()
                ms_m, _ = time_steps(fm.replay, args.steps, stream)
                check_flags(fm.poll()[0], f"t_mode {m}")
                peak = torch.cuda.max_memory_allocated(dev)
                modes[label] = {"ms_per_step": round(ms_m, 4),
                                "workspace_bytes": fm.plan.workspace_bytes,
                                "peak_device_bytes_above_inputs": int(peak - base)}
                fm.plan.close()
                del fm
                log(f"[bench] t_mode {m} ({label}): {ms_m * 1e3:.1f} us/step, workspace "
                    f"{modes[label]['workspace_bytes'] / 2**30:.2f} GiB")
        tgt_np = tgt_dev.detach().cpu().numpy() if not args.no_cpu_baseline else None
    torch.cuda.synchronize()

    # roofline of the dominant kernel
    R = N * len(step_cams)
    apix = (composited_pixels(step_cams, wl.gaze, cfg.radius_frac, cfg.tile) if cull else npix)
    dom = max(stages, key=stages.get)
    traffic = profiled_traffic(wl.name, dom, cfg.tile, cfg.lds_batch)
    if dom in ("render", "render_bwd"):
        if dom == "render":
            flops = FLOPS_ALPHA * pairs["visited_fwd"] + FLOPS_FWD_INCLUDED * pairs["included"]
        else:
            flops = FLOPS_ALPHA * pairs["visited_bwd"] + FLOPS_BWD_INCLUDED * pairs["included"]
        ach = flops / (stages[dom] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                "frac_of_nonpacked": round(ach / PEAK_FP32_NONPACKED_TFLOPS, 4),
                "us_per_launch": round(stages[dom] * 1e3, 2),
                "work": {"flops_per_launch": int(flops), **pairs}}
    else:
        byt = hbm_bytes_per_launch(dom, N, R, M, apix, planes, total_tiles, A, depth_passes)
        ach = byt / (stages[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic,
                "us_per_launch": round(stages[dom] * 1e3, 2)}
    stage_roof = {}
    for k, ms in stages.items():
        byt = hbm_bytes_per_launch(k, N, R, M, apix, planes, total_tiles, A, depth_passes)
        stage_roof[k] = {"us": round(ms * 1e3, 2), "gbs": round(byt / (ms * 1e-3) / 1e9, 1)}
        if k in ("render", "render_bwd"):
            fl = (FLOPS_ALPHA * pairs["visited_fwd"] + FLOPS_FWD_INCLUDED * pairs["included"]
                  if k == "render" else
                  FLOPS_ALPHA * pairs["visited_bwd"] + FLOPS_BWD_INCLUDED * pairs["included"])
            stage_roof[k]["tflops"] = round(fl / (ms * 1e-3) / 1e12, 3)
    step_bytes = sum(hbm_bytes_per_launch(k, N, R, M, apix, planes, total_tiles, A, depth_passes)
                     for k in stages)

    steps_per_s = 1000.0 / ms_fused
    res = {
        "metric": METRIC,
        "value": round(steps_per_s, 2),
        "unit": "fit-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_fused, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": wl.data,
        "config": {"workload": wl.description, "name": wl.name, "gaussians": N, "views": V,
                   "views_per_step": len(step_cams),
                   "sizes": [[c.width, c.height] for c in cams], "pixels_per_step": npix,
                   "sh_degree": int(round(((planes - 11) // 3) ** 0.5)) - 1,
                   "tile": cfg.tile, "lds_batch": cfg.lds_batch, "t_mode": cfg.t_mode,
                   "fovea_cull": bool(cfg.fovea_cull),
                   "keys_per_step": M, "records_with_keys": A,
                   "depth_sort_passes": depth_passes, "form": "fused, hipGraph-captured"},
        "median_step_ms": round(med_fused, 4),
        "flags_after_timed_steps": flags,
        "mpix_per_s": round(npix * steps_per_s / 1e6, 1),
        "composited_pixels_per_step": apix,
        "composited_mpix_per_s": round(apix * steps_per_s / 1e6, 1),
        "eager_fused_steps_per_s": round(1000.0 / ms_eager, 2),
        "plain_steps_per_s": round(1000.0 / ms_plain, 2) if ms_plain else None,
        "vs_plain": round(ms_plain / ms_fused, 3) if ms_plain else None,
        "loss_after_timed_steps": round(loss_fused, 6),
        "workspace_bytes": ws_fused,
        "step_hbm": {"algorithmic_bytes": int(step_bytes),
                     "gbs": round(step_bytes / (ms_fused * 1e-3) / 1e9, 1),
                     "frac_of_peak": round(step_bytes / (ms_fused * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
        "autotune": tune,
        "stages": stage_roof,
        "roofline": roof,
    }
    if regen:
        res["ms_per_regeneration"] = regen["ms_per_regeneration"]
        res["regeneration"] = regen
    if fit_run:
        res["fit"] = fit_run
    if culled_gain:
        res["fovea_culling"] = culled_gain
    if modes:
        res["transmittance_modes"] = modes
    if not args.no_cpu_baseline:
        phase("FP64 CPU oracle baseline on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(wl, tgt_np)
        log(f"[bench] CPU oracle: {res['cpu_baseline']['value']:.3g} fit-steps/s on "
            f"{res['cpu_baseline']['cores']} threads")
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
