#!/usr/bin/env python3
"""Fit-step benchmark of the MI355X Gaussian-splatting fit path.

Workload (phantom-seeded fit): a 128^3 uint16 CT-like phantom (20 random
ellipsoids, HU-like values, noise sigma 20, seed 3); one Gaussian per voxel
above 1200 capped at 50,000 (seed 4), isotropic one-voxel scale, opacity 0.1,
linear transfer-function colour (SH degree 0); one 1024x1024 view, 60 degree
FOV, on the radius-3 sphere (pose seed 2); L1 loss against an emission-
absorption ray march of the same volume; Adam lr 1e-3.  All inputs are seeded
and synthetic (the paper's CT datasets are not available).

A "step" is one forward + loss + backward + Adam pass over the view.  The
timed path is the fused step captured in a HIP graph (one launch per stage,
key count on the device), replayed K times after W warm-up replays, bracketed
by stream synchronisation and timed with HIP events.  Alongside: the plain
path (host-synchronised, eager launches), the eager fused path, per-stage
kernel times (HIP events in the library, on the stream the kernels run on),
the roofline of the dominant kernel and the FP64 CPU oracle on a bounded
sample of rows.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
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


def build_workload(n_vol=128, cap=50_000, size=1024):
    import synth
    vol = synth.phantom(n_vol, seed=synth.SEED_VOLUME)
    P = synth.seed_from_volume(vol, cap=cap, seed=synth.SEED_CAP_SUBSET)
    d = synth.sphere_directions(1, seed=synth.SEED_POSES)[0]
    cam = synth.look_at_camera(3.0 * d, width=size, height=size, fov_x_deg=60.0)
    target = synth.raymarch_volume(vol, cam)[:3]
    return P, cam, target


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


def hbm_bytes_per_launch(stage, N, M, npix, planes, tiles):
    """Algorithmic HBM bytes one launch of a stage must move."""
    rec = N  # one view
    passes = (max(1, (tiles - 1).bit_length()) + 7) // 8
    return {
        "project": planes * 4 * N + 92 * rec,                # params in; splat, key, box, count, g2d clear
        "duplicate": 16 * rec + 8 * M + 8 * tiles,           # counts (twice), boxes in; pairs out; ranges cleared
        "tile_sort": passes * 20 * M,                        # per pass: key histogram, pair in, pair out
        "ranges": 4 * M + 8 * tiles,                         # sorted tile ids in; ranges out
        "depth_sort": 12 * M,                                # record ids in, depth gather, record ids out
        "loss": 40 * npix,
        "project_bwd": planes * 4 * N + 36 * rec + planes * 4 * N,
        "adam": 28 * planes * N,
        "zero": 36 * rec,
    }.get(stage)


def profiled_traffic(kernel, tile, batch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summaries (FETCH_SIZE and WRITE_SIZE, scaled by a copy-kernel calibration),
    or None when no summary matches this kernel, tile and LDS batch, or the
    compositing source has changed since the counters were taken."""
    import glob
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "paper_2601_22026_amd", "csrc", "raster.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(here, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic:"):
                continue
            kv = dict(f.split("=", 1) for f in line.split()[1:])
            if (kv.get("kernel") == kernel and int(kv.get("tile", 0)) == tile
                    and int(kv.get("lds_batch", 0)) == batch and kv.get("raster_sha256") == h):
                return int(kv["bytes_per_launch"])
    return None


def cpu_baseline(P, cam, target, budget_s=15.0):
    """FP64 oracle fit step on a bounded sample of image rows, extrapolated
    linearly in rows to the full image."""
    import numpy as np

    import oracle
    H, W = cam.height, cam.width
    Pd = P.astype(np.float64)
    m, v = np.zeros_like(Pd), np.zeros_like(Pd)

    def run(nrows):
        rows = np.linspace(0, H - 1, nrows).astype(np.int64)
        pix = (rows[:, None] * W + np.arange(W)[None, :]).reshape(-1)
        t0 = time.perf_counter()
        r = oracle.render(Pd, cam, pixels=pix)
        tgt = target.reshape(3, -1)[:, pix]
        s, cnt, dl = oracle.loss_l1_view(r.rgba, tgt, type("c", (), {"width": W, "height": nrows})())
        G = oracle.backward(Pd, cam, dl / max(cnt, 1), pixels=pix)
        oracle.adam(Pd.copy(), G, m.copy(), v.copy(), 1)
        return time.perf_counter() - t0

    t_small = run(4)
    nrows = int(min(H, max(8, 4 * budget_s / max(t_small, 1e-3))))
    t = run(nrows)
    full = t * H / nrows
    return {"value": 1.0 / full, "unit": "fit-steps/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{nrows} of {H} rows ({nrows * W} px) of one step, {t:.1f} s, "
                      f"extrapolated x{H / nrows:.1f} in rows (all {P.shape[1]} Gaussians per pixel)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--lds-batch", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --tile/--lds-batch instead of sweeping tile x LDS batch")
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
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is described in DESIGN.md but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2601_22026_amd as gs

    t0 = time.perf_counter()
    P, cam, target = build_workload()
    N = P.shape[1]
    planes = P.shape[0]
    npix = cam.npix
    log(f"[bench] workload: {N} Gaussians, {cam.width}x{cam.height}, built in "
        f"{time.perf_counter() - t0:.1f} s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)
    tgt_dev = torch.from_numpy(np.ascontiguousarray(target.reshape(-1))).to(dev)
    cfg = gs.FitConfig(lr=1e-3, tile=args.tile, lds_batch=args.lds_batch)
    out = {}
    with torch.cuda.stream(stream):
        ctx = gs.Context(0)

        tune = None
        if not args.no_autotune:
            best, sweep = gs.autotune(ctx, torch.from_numpy(P).to(dev), [cam], tgt_dev, cfg=cfg,
                                      stream=stream)
            tune = {"best": list(best), "us_per_step": {f"{t}x{b}": round(ms * 1e3, 1)
                                                        for (t, b), ms in sorted(sweep.items())}}
            cfg = gs.FitConfig(lr=1e-3, tile=best[0], lds_batch=best[1])
            log(f"[bench] autotune: best tile {best[0]} batch {best[1]}; {tune['us_per_step']}")

        # fused, captured
        fused = gs.FitStep(ctx, torch.from_numpy(P).to(dev), [cam], tgt_dev, cfg=cfg, fused=True)
        fused.capture()
        for _ in range(args.warmup):
            fused.replay()
        ms_fused = time_steps(fused.replay, args.steps, stream)
        flags, M = fused.poll()
        loss_fused = float(fused.loss.item())
        log(f"[bench] fused+captured: {ms_fused * 1e3:.1f} us/step, keys {M}, flags {flags}, "
            f"loss {loss_fused:.5f}")

        # fused, eager (same plan shape, no graph)
        eager = gs.FitStep(ctx, torch.from_numpy(P).to(dev), [cam], tgt_dev, cfg=cfg, fused=True)
        for _ in range(args.warmup):
            eager.step()
        ms_eager = time_steps(eager.step, args.steps, stream)
        log(f"[bench] fused eager: {ms_eager * 1e3:.1f} us/step")

        # per-stage kernel times on the eager fused step (HIP events in the library)
        eager.plan.set_timing(True)
        n_prof = max(10, min(args.steps, 50))
        for _ in range(n_prof):
            eager.step()
        st = eager.plan.stage_times()
        eager.plan.set_timing(False)
        stages = {k: (ms / max(c, 1)) for k, (ms, c) in st.items() if c}
        eager.plan.forward(eager.params, N, eager.cams_dev, eager.rgba)
        pairs = eager.plan.count_pairs()
        log("[bench] stage us/launch: " + ", ".join(f"{k} {v * 1e3:.1f}" for k, v in stages.items()))
        log(f"[bench] pairs: {pairs}")

        # plain path: host-synchronised, eager
        ms_plain = None
        if not args.no_plain:
            plain = gs.FitStep(ctx, torch.from_numpy(P).to(dev), [cam], tgt_dev, cfg=cfg, fused=False)
            for _ in range(args.warmup):
                plain.step()
            ms_plain = time_steps(plain.step, args.steps, stream)
            log(f"[bench] plain: {ms_plain * 1e3:.1f} us/step")
    torch.cuda.synchronize()

    # roofline of the dominant kernel
    dom = max(stages, key=stages.get)
    tiles = fused.plan.total_tiles
    if dom in ("render", "render_bwd"):
        if dom == "render":
            flops = FLOPS_ALPHA * pairs["visited_fwd"] + FLOPS_FWD_INCLUDED * pairs["included"]
        else:
            flops = FLOPS_ALPHA * pairs["visited_bwd"] + FLOPS_BWD_INCLUDED * pairs["included"]
        ach = flops / (stages[dom] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                "traffic": profiled_traffic(dom, cfg.tile, cfg.lds_batch),
                "work": {"flops_per_launch": int(flops), **pairs}}
    else:
        byt = hbm_bytes_per_launch(dom, N, M, npix, planes, tiles)
        ach = byt / (stages[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
                "traffic": profiled_traffic(dom, cfg.tile, cfg.lds_batch)}
    stage_roof = {}
    for k, ms in stages.items():
        if k in ("render", "render_bwd"):
            fl = (FLOPS_ALPHA * pairs["visited_fwd"] + FLOPS_FWD_INCLUDED * pairs["included"]
                  if k == "render" else
                  FLOPS_ALPHA * pairs["visited_bwd"] + FLOPS_BWD_INCLUDED * pairs["included"])
            stage_roof[k] = {"us": round(ms * 1e3, 2), "tflops": round(fl / (ms * 1e-3) / 1e12, 3)}
        else:
            byt = hbm_bytes_per_launch(k, N, M, npix, planes, tiles)
            stage_roof[k] = {"us": round(ms * 1e3, 2)}
            if byt:
                stage_roof[k]["gbs"] = round(byt / (ms * 1e-3) / 1e9, 1)

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
        "data": "synthetic: seeded CT-like phantom, voxel-seeded Gaussians, ray-marched target",
        "config": {"workload": "phantom-seeded fit: 128^3 phantom, 50,000 Gaussians (SH0), "
                               "one 1024x1024 view, L1 vs ray-marched target, Adam lr 1e-3",
                   "gaussians": N, "views": 1, "width": cam.width, "height": cam.height,
                   "tile": cfg.tile, "lds_batch": cfg.lds_batch, "keys_per_step": M,
                   "form": "fused, hipGraph-captured"},
        "mpix_per_s": round(npix * steps_per_s / 1e6, 1),
        "ms_per_100_step_fit": round(100 * ms_fused, 2),
        "eager_fused_steps_per_s": round(1000.0 / ms_eager, 2),
        "plain_steps_per_s": round(1000.0 / ms_plain, 2) if ms_plain else None,
        "vs_plain": round(ms_plain / ms_fused, 3) if ms_plain else None,
        "loss_after_timed_steps": round(loss_fused, 6),
        "autotune": tune,
        "stages": stage_roof,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        res["cpu_baseline"] = cpu_baseline(P, cam, target)
    else:
        res["cpu_baseline"] = None
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
