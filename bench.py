#!/usr/bin/env python3
"""Fit-step benchmark of the MI355X Gaussian-splatting fit path.

Default workload (phantom-seeded fit): a 128^3 uint16 CT-like phantom (20
random ellipsoids, HU-like values, noise sigma 20, seed 3); one Gaussian per
voxel above 1200 capped at 50,000 (seed 4), isotropic one-voxel scale,
opacity 0.1, linear transfer-function colour (SH degree 0); one 1024x1024
view, 60 degree FOV, on the radius-3 sphere (pose seed 2); L1 loss against an
emission-absorption ray march of the same volume; Adam lr 1e-3.  All inputs
are seeded and synthetic (the paper's CT datasets are not available).

Other workloads (--workload): small (1,000 random Gaussians, one 128^2 view,
target rendered by the oracle), batched (200,000 SH3 Gaussians, 8 views of
uneven resolution), foveal (500,000 Gaussians seeded from a 256^3 phantom, 16
views of 1920^2, loss masked to a fovea of radius 0.2 W at a random gaze point,
ms per 300-step regeneration), stereo (1,000,000 SH3 Gaussians, two eyes of
2064x2208, recomputed / checkpointed / stored transmittance compared).

A "step" is one forward + loss + backward + Adam pass over all views.  The
timed path is the fused step captured in a HIP graph (one launch per stage
for all views, key count on the device), replayed K times after W warm-up
replays, bracketed by stream synchronisation and timed with HIP events.
Alongside: the plain path (one host-synchronised plan per view, eager), the
eager fused path, per-stage kernel times (HIP events recorded by the library
on the stream the kernels run on, over the same step indices as the timed
replays), the roofline of the dominant kernel and the FP64 CPU oracle on a
bounded sample of rows.

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
# Non-packed FP32 vector peak: 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.
PEAK_FP32_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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


def _phantom_fit(n_vol, cap, cams, gaze=None):
    import numpy as np

    import synth
    vol = synth.phantom(n_vol, seed=synth.SEED_VOLUME)
    P = synth.seed_from_volume(vol, cap=cap, seed=synth.SEED_CAP_SUBSET)
    tg = []
    for k, c in enumerate(cams):
        if gaze is None:
            tg.append(synth.raymarch_volume(vol, c)[:3])
            continue
        # only rows that meet the fovea carry loss; the others stay zero
        r = 0.2 * c.width
        y0 = max(0, int(np.floor(gaze[k][1] - r - 1)))
        y1 = min(c.height, int(np.ceil(gaze[k][1] + r + 1)))
        img = np.zeros((3, c.height, c.width), np.float32)
        img[:, y0:y1] = synth.raymarch_volume(vol, c, rows=np.arange(y0, y1))[:3]
        tg.append(img)
    targets = np.concatenate([t.reshape(-1) for t in tg])
    return P, targets, vol


def build_workload(name="phantom"):
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
        P, targets, vol = _phantom_fit(128, 50_000, [cam])
        return Workload(name, "phantom-seeded fit: 128^3 phantom, 50,000 Gaussians (SH0), one "
                              "1024x1024 view, L1 vs ray-marched target, Adam lr 1e-3",
                        "synthetic: seeded CT-like phantom, voxel-seeded Gaussians, ray-marched target",
                        P, [cam], targets=targets, volume=vol)
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
        P, targets, vol = _phantom_fit(256, 500_000, cams, gaze)
        return Workload(name, "foveal refinement: 256^3 phantom, 500,000 Gaussians (SH0), 16 views "
                              "of 1920x1920, L1 masked to a fovea of radius 0.2 W at a random gaze "
                              "point per view, ray-marched targets, Adam lr 1e-3",
                        "synthetic: seeded CT-like phantom, voxel-seeded Gaussians, ray-marched target",
                        P, cams, targets=targets, gaze=gaze, volume=vol)
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


def time_steps(fn, steps, stream):
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def hbm_bytes_per_launch(stage, N, R, M, npix, planes, tiles):
    """Algorithmic HBM bytes one launch of a stage must move: N Gaussians,
    R = N * views records, M keys, npix pixels, `planes` floats per Gaussian."""
    passes = (max(1, (tiles - 1).bit_length()) + 7) // 8
    return {
        "project": planes * 4 * N + 88 * R,                   # params in; splat, key, box, count, ellipse, spans
        "duplicate": 20 * R + 8 * M + 8 * tiles,              # counts (twice), boxes in; first-key offset, pairs out; ranges cleared
        "tile_sort": passes * 20 * M,                         # per pass: key histogram, pair in, pair out
        "ranges": 4 * M + 28 * tiles,                         # sorted tile ids in; ranges out; order
        "depth_sort": 12 * M,                                 # record ids in, depth gather, record ids out
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
    """FP64 oracle fit step (render, L1 sign, adjoint, Adam) on a bounded sample
    of image rows of every view, extrapolated linearly in rows per view."""
    import numpy as np

    import oracle
    Pd = wl.P.astype(np.float64)
    m, v = np.zeros_like(Pd), np.zeros_like(Pd)
    offs = np.cumsum([0] + [c.width * c.height for c in wl.cams])

    def run(rows_per_view):
        est, used = 0.0, 0
        G = np.zeros_like(Pd)
        t_start = time.perf_counter()
        for k, cam in enumerate(wl.cams):
            H, W = cam.height, cam.width
            nrows = min(H, rows_per_view)
            rows = np.linspace(0, H - 1, nrows).astype(np.int64)
            pix = (rows[:, None] * W + np.arange(W)[None, :]).reshape(-1)
            t0 = time.perf_counter()
            r = oracle.render(Pd, cam, pixels=pix)
            tgt = targets_np[3 * offs[k]:3 * offs[k + 1]].reshape(3, -1)[:, pix]
            s, cnt, dl = oracle.loss_l1_view(r.rgba, tgt, type("c", (), {"width": W, "height": nrows})())
            G += oracle.backward(Pd, cam, dl / max(cnt, 1), pixels=pix)
            est += (time.perf_counter() - t0) * H / nrows
            used += nrows
        t0 = time.perf_counter()
        oracle.adam(Pd.copy(), G, m.copy(), v.copy(), 1)
        est += time.perf_counter() - t0
        return est, used, time.perf_counter() - t_start

    _, _, t_probe = run(2)
    rows = max(2, int(2 * budget_s / max(t_probe, 1e-3)))
    full, used, spent = run(rows)
    tot_rows = sum(c.height for c in wl.cams)
    return {"value": 1.0 / full, "unit": "fit-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{used} of {tot_rows} rows over {len(wl.cams)} view(s) of one step, "
                      f"{spent:.1f} s, extrapolated per view in rows (all {wl.P.shape[1]} Gaussians "
                      f"per pixel)"}


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
            ms = time_steps(graph.replay, args.steps, stream)
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


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="phantom",
                    choices=["small", "phantom", "batched", "foveal", "stereo", "reproject",
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
    ap.add_argument("--regen-steps", type=int, default=300,
                    help="steps of one regeneration (foveal workload)")
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
    wl = build_workload(args.workload)
    P, cams = wl.P, wl.cams
    N, planes, V = P.shape[1], P.shape[0], len(cams)
    npix = sum(c.width * c.height for c in cams)
    log(f"[bench] workload {wl.name}: {N} Gaussians, {V} view(s), {npix} px, built in "
        f"{time.perf_counter() - t0:.1f} s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)
    # a masked loss lets the fused step composite only the tiles that meet each fovea
    cfg = gs.FitConfig(lr=1e-3, tile=args.tile, lds_batch=args.lds_batch, t_mode=args.t_mode,
                       fovea_cull=wl.gaze is not None and not args.no_fovea_cull)
    with torch.cuda.stream(stream):
        ctx = gs.Context(0)
        if wl.targets is None:
            tgt_dev = render_targets(ctx, wl, dev)
        else:
            tgt_dev = torch.from_numpy(np.ascontiguousarray(wl.targets)).to(dev)
        gaze_dev = None if wl.gaze is None else torch.from_numpy(np.ascontiguousarray(wl.gaze)).to(dev)
        P_dev = torch.from_numpy(np.ascontiguousarray(P)).to(dev)

        def fit(c, fused=True):
            return gs.FitStep(ctx, P_dev.clone(), cams, tgt_dev, gaze_dev, cfg=c, fused=fused)

        tune = None
        if not args.no_autotune:
            best, sweep = gs.autotune(ctx, P_dev, cams, tgt_dev, gaze_dev, cfg=cfg, t_modes=(0, 1),
                                      stream=stream)
            tune = {"best": list(best), "us_per_step": {f"{t}x{b}/t{m}": round(ms * 1e3, 1)
                                                        for (t, b, m), ms in sorted(sweep.items())}}
            cfg = dataclasses.replace(cfg, tile=best[0], lds_batch=best[1], t_mode=best[2])
            log(f"[bench] autotune: best tile {best[0]} batch {best[1]} t_mode {best[2]}; "
                f"{tune['us_per_step']}")

        # fused, captured: the timed path
        fused = fit(cfg)
        fused.capture()
        for _ in range(args.warmup):
            fused.replay()
        ms_fused = time_steps(fused.replay, args.steps, stream)
        flags, M = fused.poll()
        loss_fused = float(fused.loss.item())
        log(f"[bench] fused+captured: {ms_fused * 1e3:.1f} us/step, keys {M}, flags {flags}, "
            f"loss {loss_fused:.5f}")
        ws_fused = fused.plan.workspace_bytes
        total_tiles = fused.plan.total_tiles
        fused.plan.close()
        del fused

        regen = None
        if wl.name == "foveal":
            # one regeneration: seed the Gaussians on the device from the resident
            # volume, plan, capture, run the steps - wall clock, synchronised
            import synth
            vol_dev = torch.from_numpy(np.ascontiguousarray(wl.volume).view(np.int16)).to(dev)
            runs, seeds = [], []
            for _ in range(3):
                torch.cuda.synchronize()
                t_start = time.perf_counter()
                Ps = gs.seed_volume(ctx, vol_dev, cap=N, seed=synth.SEED_CAP_SUBSET)
                t_seeded = time.perf_counter()
                if not runs:   # the device seeding reproduces the workload's Gaussians
                    same = bool(torch.equal(Ps.cpu(), torch.from_numpy(P)))
                rf = gs.FitStep(ctx, Ps, cams, tgt_dev, gaze_dev, cfg=cfg, fused=True)
                rf.capture()
                for _ in range(args.regen_steps):
                    rf.replay()
                torch.cuda.synchronize()
                runs.append((time.perf_counter() - t_start) * 1e3)
                seeds.append((t_seeded - t_start) * 1e3)
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
            regen = {"ms_per_regeneration": round(sorted(runs)[1], 2), "steps": args.regen_steps,
                     "runs_ms": [round(r, 2) for r in runs],
                     "seeding_ms": round(sorted(seeds)[1], 2),
                     "seeded_on_device_equals_workload": same,
                     "target_raymarch_ms": round(sorted(march)[1], 2),
                     "includes": "seeding from the device-resident volume, plan creation, graph "
                                 "capture and the captured fit steps (the targets' ray march is "
                                 "timed apart)"}
            log(f"[bench] regeneration ({args.regen_steps} steps): {regen['ms_per_regeneration']} ms "
                f"(seeding {regen['seeding_ms']} ms, same Gaussians as the workload: {same}); "
                f"target ray march {regen['target_raymarch_ms']} ms")

        # fused, eager (same plan shape, no graph)
        eager = fit(cfg)
        for _ in range(args.warmup):
            eager.step()
        ms_eager = time_steps(eager.step, args.steps, stream)
        eager.plan.close()
        del eager
        log(f"[bench] fused eager: {ms_eager * 1e3:.1f} us/step")

        # per-stage kernel times: a fresh eager fused step taken through the same
        # step indices as the timed replays (W warm-up, then K), with HIP events
        # recorded by the library around each stage on the stream it launches on
        staged = fit(cfg)
        for _ in range(args.warmup):
            staged.step()
        staged.plan.set_timing(True)
        for _ in range(args.steps):
            staged.step()
        st = staged.plan.stage_times()
        staged.plan.set_timing(False)
        staged.plan.close()
        del staged
        stages = {k: (ms / max(c, 1)) for k, (ms, c) in st.items() if c}
        log("[bench] stage us/launch: " + ", ".join(f"{k} {v * 1e3:.1f}" for k, v in stages.items()))
        # pair counts of the same K steps (a separate run: counting synchronises)
        counted = fit(cfg)
        for _ in range(args.warmup):
            counted.step()
        pairs = {}
        for _ in range(args.steps):
            counted.step()
            for k, v in counted.plan.count_pairs().items():
                pairs[k] = pairs.get(k, 0) + v / args.steps
        counted.plan.close()
        del counted
        pairs = {k: int(round(v)) for k, v in pairs.items()}
        log(f"[bench] pairs per step (mean of the K steps): {pairs}")

        # plain path: one host-synchronised plan per view, eager, full frames
        ms_plain = None
        if not args.no_plain:
            plain = fit(cfg, fused=False)
            for _ in range(args.warmup):
                plain.step()
            ms_plain = time_steps(plain.step, args.steps, stream)
            for p, _, _ in plain.view_plans:
                p.close()
            del plain
            log(f"[bench] plain: {ms_plain * 1e3:.1f} us/step")

        # transmittance modes: step time and peak device memory
        modes = None
        if args.compare_t_modes or wl.name == "stereo":
            modes = {}
            for m, label in enumerate(["recompute", "checkpointed", "stored"]):
                torch.cuda.synchronize()
                torch.cuda.empty_cache()
                torch.cuda.reset_peak_memory_stats(dev)
                base = torch.cuda.memory_allocated(dev)
                fm = fit(dataclasses.replace(cfg, t_mode=m))
                fm.capture()
                for _ in range(args.warmup):
                    fm.replay()
                ms_m = time_steps(fm.replay, args.steps, stream)
                peak = torch.cuda.max_memory_allocated(dev)
                modes[label] = {"ms_per_step": round(ms_m, 4),
                                "workspace_bytes": fm.plan.workspace_bytes,
                                "peak_device_bytes_above_inputs": int(peak - base)}
                fm.plan.close()
                del fm
                log(f"[bench] t_mode {m} ({label}): {ms_m * 1e3:.1f} us/step, workspace "
                    f"{modes[label]['workspace_bytes'] / 2**30:.2f} GiB")
    torch.cuda.synchronize()

    # roofline of the dominant kernel
    R = N * V
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
                "work": {"flops_per_launch": int(flops), **pairs}}
    else:
        byt = hbm_bytes_per_launch(dom, N, R, M, npix, planes, total_tiles)
        ach = byt / (stages[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic}
    stage_roof = {}
    for k, ms in stages.items():
        byt = hbm_bytes_per_launch(k, N, R, M, npix, planes, total_tiles)
        stage_roof[k] = {"us": round(ms * 1e3, 2), "gbs": round(byt / (ms * 1e-3) / 1e9, 1)}
        if k in ("render", "render_bwd"):
            fl = (FLOPS_ALPHA * pairs["visited_fwd"] + FLOPS_FWD_INCLUDED * pairs["included"]
                  if k == "render" else
                  FLOPS_ALPHA * pairs["visited_bwd"] + FLOPS_BWD_INCLUDED * pairs["included"])
            stage_roof[k]["tflops"] = round(fl / (ms * 1e-3) / 1e12, 3)
    step_bytes = sum(hbm_bytes_per_launch(k, N, R, M, npix, planes, total_tiles) for k in stages)

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
                   "sizes": [[c.width, c.height] for c in cams], "pixels": npix,
                   "sh_degree": int(round(((planes - 11) // 3) ** 0.5)) - 1,
                   "tile": cfg.tile, "lds_batch": cfg.lds_batch, "t_mode": cfg.t_mode,
                   "fovea_cull": bool(cfg.fovea_cull),
                   "keys_per_step": M, "form": "fused, hipGraph-captured"},
        "mpix_per_s": round(npix * steps_per_s / 1e6, 1),
        "ms_per_100_step_fit": round(100 * ms_fused, 2),
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
        res["regeneration"] = regen
    if modes:
        res["transmittance_modes"] = modes
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        res["cpu_baseline"] = cpu_baseline(wl, tgt_dev.detach().cpu().numpy())
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
