"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the oracle (inputs come from ``synth``; expected values from
``oracle``)."""
from __future__ import annotations

import numpy as np
import torch

import oracle
import paper_2601_22026_amd as gs
from paper_2601_22026_amd import _abi

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)


class GpuScene:
    """Device copies of a parameter set and cameras plus one plan."""

    def __init__(self, ctx, P, cams, tile=16, batch=128, host_sized=True, key_capacity=0,
                 t_mode=0):
        self.P = P
        self.cams = list(cams)
        self.deg = oracle.sh_degree_of(P)
        self.n = P.shape[1]
        self.params = torch.from_numpy(np.ascontiguousarray(P, np.float32)).to(DEV)
        self.cams_dev = gs.cameras_to_device(self.cams, DEV)
        self.plan = gs.Plan(ctx, self.n, [(c.width, c.height) for c in self.cams], self.deg,
                            tile, batch, host_sized=host_sized, key_capacity=key_capacity,
                            t_mode=t_mode)
        self.npix = [c.width * c.height for c in self.cams]
        self.rgba = torch.zeros(4 * sum(self.npix), dtype=torch.float32, device=DEV)

    def forward(self):
        self.plan.forward(self.params, self.n, self.cams_dev, self.rgba)
        torch.cuda.synchronize()
        return self.images()

    def images(self):
        out, off = [], 0
        flat = self.rgba.cpu().numpy()
        for k in self.npix:
            out.append(flat[4 * off:4 * (off + k)].reshape(4, k))
            off += k
        return out

    def backward(self, dls):
        dl = torch.from_numpy(np.concatenate([np.asarray(d, np.float32).reshape(-1) for d in dls])).to(DEV)
        g = torch.zeros_like(self.params)
        self.plan.backward(self.params, self.n, self.cams_dev, dl, g)
        torch.cuda.synchronize()
        return g.cpu().numpy()

    def debug(self, which, dtype, count):
        return self.plan.debug(which, dtype, count)

    def proj(self):
        R = self.n * len(self.cams)
        return self.debug(_abi.GSF_DBG_PROJ, np.float32, 11 * R).reshape(R, 11)


def image_close(gpu, ref, flags, rtol=1e-4, atol=1e-6):
    ok = flags == 0
    diff = np.abs(gpu[:, ok] - ref[:, ok])
    bad = diff > rtol * np.abs(ref[:, ok]) + atol
    return int(bad.sum()), float(diff.max()) if diff.size else 0.0, int((~ok).sum())


def grads_close(gpu, ref, rtol=1e-3, floor_frac=1e-2, atol_frac=1e-5):
    """Per parameter group: relative 1e-3 where |ref| >= 1e-2 max|ref|, else
    absolute 1e-5 max|ref|.  Returns list of (group, n_bad, worst)."""
    groups = {"mean": slice(0, 3), "logscale": slice(3, 6), "quat": slice(6, 10),
              "opacity": slice(10, 11), "sh": slice(11, gpu.shape[0])}
    report = []
    overall = np.abs(ref).max()
    for name, sl in groups.items():
        g, r = gpu[sl], ref[sl]
        mx = np.abs(r).max()
        if mx < 1e-4 * overall:
            # a group that is zero in exact arithmetic (e.g. rotations of isotropic
            # Gaussians): float32 cancellation noise against the largest gradient
            err = np.abs(g - r)
            report.append((name, int((err > atol_frac * overall).sum()), float(err.max() / overall)))
            continue
        big = np.abs(r) >= floor_frac * mx
        err = np.abs(g - r)
        bad = np.where(big, err > rtol * np.abs(r), err > atol_frac * mx)
        worst = float(np.max(np.where(big, err / np.maximum(np.abs(r), 1e-30), err / mx)))
        report.append((name, int(bad.sum()), worst))
    return report
