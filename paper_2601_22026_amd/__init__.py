"""MI355X (gfx950) differentiable Gaussian-splatting fit path - Python binding.

The compute path is the HIP library ``libgsfit.so`` behind the C ABI in
``include/gsfit.h``; this module only marshals arguments (PyTorch supplies
device memory and streams).  The C functions are re-exported under their own
names by ``paper_2601_22026_amd._abi``; the classes here wrap them:

* ``Context``   - device + stream (``gsf_ctx_*``)
* ``Plan``      - view sizes, SH degree, tile/batch, key capacity and the
                  caller-owned workspace (``gsf_plan_*``)
* ``rasterize`` - ``torch.autograd.Function`` around ``gsf_forward`` /
                  ``gsf_backward``
* ``adam``      - ``gsf_adam`` on a flat parameter buffer
* ``FitStep``   - one forward + L1 loss + backward + Adam step, either fused
                  over all views and captured in a HIP graph, or plain (one
                  host-synchronised plan per view, eager launches)
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import GsfError, gsf_camera, gsf_plan_desc, gsf_step_args, lib

__all__ = ["GsfError", "Context", "Plan", "rasterize", "adam", "adam_masked", "adam_reset",
           "FitStep", "FitConfig", "autotune", "select_views", "plane_learning_rates", "Refiner",
           "seed_volume", "seed_first_hits", "raymarch", "reproject", "reproject_warp",
           "reproject_warp_noalloc",
           "pack_cameras", "cameras_to_device", "n_planes", "lib"]


def n_planes(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise GsfError(_abi.GSF_E_INVALID, "tensor must live on the GPU")
    return ct.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def pack_cameras(cams) -> bytes:
    """gsf_camera records of camera objects with attributes R (3x3), t (3),
    campos (3), fx, fy, cx, cy, tanx, tany, znear, bg (3), width, height."""
    arr = (gsf_camera * len(cams))()
    for k, c in enumerate(cams):
        R = np.asarray(c.R, np.float32).reshape(3, 3)
        t = np.asarray(c.t, np.float32).reshape(3)
        vm = np.concatenate([R, t[:, None]], axis=1).reshape(-1)
        arr[k].viewmat[:] = [float(x) for x in vm]
        arr[k].campos[:] = [float(x) for x in np.asarray(c.campos, np.float32)]
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = c.fx, c.fy, c.cx, c.cy
        arr[k].tan_half_fov_x, arr[k].tan_half_fov_y = c.tanx, c.tany
        arr[k].znear = c.znear
        arr[k].bg[:] = [float(x) for x in np.asarray(c.bg, np.float32)]
        arr[k].width, arr[k].height = int(c.width), int(c.height)
    return bytes(arr)


def cameras_to_device(cams, device="cuda") -> torch.Tensor:
    raw = np.frombuffer(pack_cameras(cams), dtype=np.uint8).copy()
    return torch.from_numpy(raw).to(device)


class Context:
    """A device and the stream calls are enqueued on (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        self.device = device
        h = ct.c_void_p()
        st = lib().gsf_ctx_create(device, _stream_ptr(stream), ct.byref(h))
        if st != 0:
            raise GsfError(st, f"gsf_ctx_create(device={device}) failed")
        self.handle = h

    def check(self, status: int, what: str = ""):
        if status != 0:
            msg = lib().gsf_last_error(self.handle).decode()
            raise GsfError(status, f"{what}: {msg}" if what else msg)

    def use_stream(self, stream=None):
        self.check(lib().gsf_ctx_set_stream(self.handle, _stream_ptr(stream)), "gsf_ctx_set_stream")

    def close(self):
        if self.handle:
            lib().gsf_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Plan over fixed view sizes with its own device workspace."""

    def __init__(self, ctx: Context, n_max: int, sizes: Sequence[tuple], sh_degree: int = 0,
                 tile: int = 16, lds_batch: int = 128, host_sized: bool = False,
                 key_capacity: int = 0, t_mode: int = 0):
        self.ctx = ctx
        self.sizes = [(int(w), int(h)) for w, h in sizes]
        self.n_max, self.sh_degree, self.tile, self.lds_batch = n_max, sh_degree, tile, lds_batch
        self.host_sized = bool(host_sized)
        V = len(self.sizes)
        self._w = (ct.c_int32 * V)(*[w for w, _ in self.sizes])
        self._h = (ct.c_int32 * V)(*[h for _, h in self.sizes])
        d = gsf_plan_desc(n_max=n_max, sh_degree=sh_degree, n_views=V,
                          widths=ct.cast(self._w, ct.POINTER(ct.c_int32)),
                          heights=ct.cast(self._h, ct.POINTER(ct.c_int32)), tile=tile,
                          lds_batch=lds_batch, t_mode=t_mode, host_sized=int(host_sized),
                          key_capacity=int(key_capacity))
        h = ct.c_void_p()
        ctx.check(lib().gsf_plan_create(ctx.handle, ct.byref(d), ct.byref(h)), "gsf_plan_create")
        self.handle = h
        nb = ct.c_size_t()
        ctx.check(lib().gsf_plan_workspace_bytes(h, ct.byref(nb)), "gsf_plan_workspace_bytes")
        self.workspace = torch.empty(max(int(nb.value), 256), dtype=torch.uint8,
                                     device=f"cuda:{ctx.device}")
        ctx.use_stream()
        ctx.check(lib().gsf_plan_bind_workspace(h, _ptr(self.workspace), nb.value),
                  "gsf_plan_bind_workspace")
        tt, tp = ct.c_int64(), ct.c_int64()
        lib().gsf_plan_info(h, ct.byref(tt), ct.byref(tp))
        self.total_tiles, self.total_pixels = tt.value, tp.value

    # -- raw calls (tensors in, status checked) ------------------------------------
    def forward(self, params, n, cams_dev, out_rgba, cull_gaze=None, cull_radius_frac=0.0):
        """gsf_forward; with cull_gaze ([V][2] device) only the pixels of each
        view's fovea disk are composited (the rest of their tiles as background)."""
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_forward(self.handle, _ptr(params), int(n), _ptr(cams_dev),
                                         _ptr(cull_gaze), float(cull_radius_frac), _ptr(out_rgba)),
                       "gsf_forward")

    def loss_l1(self, rgba, target, loss, dl, gaze=None, radius_frac=0.0, norm_count=0,
                accumulate=False):
        """gsf_loss_l1; norm_count > 0 divides by that entry count (a loss split
        over several plans), accumulate adds this plan's share to loss[0]."""
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_loss_l1(self.handle, _ptr(rgba), _ptr(target), _ptr(gaze),
                                         float(radius_frac), int(norm_count), int(bool(accumulate)),
                                         _ptr(loss), _ptr(dl)), "gsf_loss_l1")

    def loss_count(self, gaze=None, radius_frac=0.0) -> int:
        """gsf_loss_count: the entries gsf_loss_l1 averages over (synchronises)."""
        c = ct.c_int64()
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_loss_count(self.handle, _ptr(gaze), float(radius_frac),
                                            ct.byref(c)), "gsf_loss_count")
        return int(c.value)

    def loss_l1_rgba(self, rgba, target_rgba, loss, dl, bg=None, alpha=True, gaze=None,
                     radius_frac=0.0):
        """Alpha-training L1 against RGBA targets composited over bg ([V][3] device
        tensor or None for black)."""
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_loss_l1_rgba(self.handle, _ptr(rgba), _ptr(target_rgba), _ptr(bg),
                                              int(bool(alpha)), _ptr(gaze), float(radius_frac),
                                              _ptr(loss), _ptr(dl)), "gsf_loss_l1_rgba")

    def backward(self, params, n, cams_dev, dl, grads, accumulate=False):
        """gsf_backward; accumulate adds to grads instead of overwriting them."""
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_backward(self.handle, _ptr(params), int(n), _ptr(cams_dev),
                                          _ptr(dl), int(bool(accumulate)), _ptr(grads)),
                       "gsf_backward")

    def poll(self):
        f, m = ct.c_uint32(), ct.c_int64()
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_poll(self.handle, ct.byref(f), ct.byref(m)), "gsf_poll")
        return int(f.value), int(m.value)

    def debug(self, which: int, dtype, count: int) -> np.ndarray:
        out = np.zeros(max(count, 1), dtype=dtype)
        written = ct.c_size_t()
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_debug_copy(self.handle, which, out.ctypes.data_as(ct.c_void_p),
                                            out.nbytes, ct.byref(written)), "gsf_debug_copy")
        return out[: written.value // out.itemsize]

    def count_pairs(self) -> dict:
        """Pairs visited / included by the last forward, and visited by its adjoint."""
        out = (ct.c_int64 * 3)()
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_count_pairs(self.handle, out), "gsf_count_pairs")
        return {"visited_fwd": out[0], "included": out[1], "visited_bwd": out[2]}

    def set_timing(self, enable: bool = True):
        self.ctx.check(lib().gsf_plan_set_timing(self.handle, int(enable)), "gsf_plan_set_timing")

    def stage_times(self) -> dict:
        """{stage: (total ms, calls)} of the eager calls since timing was enabled."""
        n = len(_abi.STAGES)
        ms, calls = (ct.c_double * n)(), (ct.c_int64 * n)()
        self.ctx.check(lib().gsf_plan_stage_times(self.handle, ms, calls), "gsf_plan_stage_times")
        return {name: (ms[k], calls[k]) for k, name in enumerate(_abi.STAGES)}

    def close(self):
        if getattr(self, "handle", None):
            lib().gsf_plan_destroy(self.handle)
            self.handle = None
        self.workspace = None

    @property
    def workspace_bytes(self) -> int:
        return 0 if self.workspace is None else int(self.workspace.numel())

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Rasterize(torch.autograd.Function):
    @staticmethod
    def forward(fctx, params, plan, cams_dev):
        params = params.contiguous()
        n = params.shape[1]
        out = torch.empty(4 * plan.total_pixels, dtype=torch.float32, device=params.device)
        plan.forward(params, n, cams_dev, out)
        fctx.plan, fctx.cams = plan, cams_dev
        fctx.save_for_backward(params)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        (params,) = fctx.saved_tensors
        grads = torch.empty_like(params)
        fctx.plan.backward(params, params.shape[1], fctx.cams, grad_out.contiguous(), grads)
        return grads, None, None


def rasterize(params: torch.Tensor, plan: Plan, cams_dev: torch.Tensor) -> torch.Tensor:
    """Concatenated per-view [4][H][W] images of planar float32 params [C][n].
    Differentiable w.r.t. params (gsf_backward).  The state the backward needs
    lives in the plan, so use one plan per forward in flight."""
    return _Rasterize.apply(params, plan, cams_dev)


def adam(ctx: Context, p, g, m, v, step_dev, seg_off, seg_lr, betas=(0.9, 0.999), eps=1e-15):
    """gsf_adam over flat float32 buffers with per-segment learning rates."""
    so = (ct.c_int64 * len(seg_off))(*[int(x) for x in seg_off])
    sl = (ct.c_float * len(seg_lr))(*[float(x) for x in seg_lr])
    ctx.use_stream()
    ctx.check(lib().gsf_adam(ctx.handle, _ptr(p), _ptr(g), _ptr(m), _ptr(v), int(p.numel()), so, sl,
                             len(seg_lr), float(betas[0]), float(betas[1]), float(eps),
                             _ptr(step_dev)), "gsf_adam")


def adam_masked(ctx: Context, p, g, m, v, step_dev, plane_lr, visible, betas=(0.9, 0.999),
                eps=1e-15):
    """gsf_adam_masked over planar float32 state [C][n]: only the Gaussians with
    visible[i] != 0 (device uint8 [n]) are updated; plane c at plane_lr[c]."""
    C, n = p.shape
    assert visible.dtype == torch.uint8 and visible.numel() == n
    lr = (ct.c_float * C)(*[float(x) for x in plane_lr])
    ctx.use_stream()
    ctx.check(lib().gsf_adam_masked(ctx.handle, _ptr(p), _ptr(g), _ptr(m), _ptr(v), int(n), int(C),
                                    lr, _ptr(visible), float(betas[0]), float(betas[1]),
                                    float(eps), _ptr(step_dev)), "gsf_adam_masked")


def adam_reset(ctx: Context, m, v, step_dev):
    """gsf_adam_reset: m = v = 0 and the step counter = 0 (optimiser restart)."""
    ctx.use_stream()
    ctx.check(lib().gsf_adam_reset(ctx.handle, _ptr(m), _ptr(v), int(m.numel()), _ptr(step_dev)),
              "gsf_adam_reset")


def select_views(kept, candidates, delta_pos: float = 0.05, theta_view_deg: float = 5.0):
    """gsf_view_select (Eq. (1), host only): which candidate cameras join the
    kept set when offered in order.  Returns one bool per candidate."""
    kept, candidates = list(kept), list(candidates)
    if not candidates:
        return []
    ks = (gsf_camera * max(len(kept), 1)).from_buffer_copy(
        pack_cameras(kept) if kept else bytes(ct.sizeof(gsf_camera)))
    cs = (gsf_camera * len(candidates)).from_buffer_copy(pack_cameras(candidates))
    keep = (ct.c_int32 * len(candidates))()
    nk = ct.c_int32()
    st = lib().gsf_view_select(ks, len(kept), cs, len(candidates), float(delta_pos),
                               float(theta_view_deg), keep, ct.byref(nk))
    if st != _abi.GSF_OK:
        raise GsfError(st, "gsf_view_select: invalid argument")
    return [bool(x) for x in keep]


# Planes whose learning rate the initial fit raises: log-scale (3..5), opacity
# (10) and colour (11 onwards); the paper raises them by about 50 % (Method,
# "Periphery Model Training").
REFINE_LR_BOOST = 1.5


def plane_learning_rates(sh_degree: int, lr=1e-3, boost: float = 1.0):
    """Learning rate per parameter plane: ``lr`` (scalar or per plane), times
    ``boost`` on the scale, opacity and colour planes."""
    C = n_planes(sh_degree)
    base = [float(x) for x in lr] if isinstance(lr, (list, tuple, np.ndarray)) else [float(lr)] * C
    if len(base) != C:
        raise ValueError(f"need {C} learning rates, got {len(base)}")
    return [b * boost if (3 <= c <= 5 or c >= 10) else b for c, b in enumerate(base)]


@dataclass
class FitConfig:
    lr: float | Sequence[float] = 1e-3
    betas: tuple = (0.9, 0.999)
    eps: float = 1e-15
    tile: int = 16
    lds_batch: int = 128
    radius_frac: float = 0.2
    key_capacity: int = 0
    t_mode: int = 1          # adjoint transmittance of the fused step: 0 recomputed, 1 checkpointed, 2 stored
    fovea_cull: bool = False  # fused step with a gaze: composite only the fovea disks' pixels
    alpha_loss: bool = False  # targets are RGBA ([4][H][W] per view) and the L1 covers alpha
    random_bg: bool = False   # fused step: a new background per view each step (needs alpha_loss)
    bg_seed: int = 0
    masked_adam: bool = False  # fused step: Adam only for Gaussians that touched a tile this step
    lr_boost: float = 1.0     # factor on the scale, opacity and colour planes' learning rates


class FitStep:
    """One fit step (forward, L1 loss, backward, Adam) over all views.

    fused=True: one plan over all views (one launch per stage), key count kept
    on the device, checkpointed transmittance (cfg.t_mode), and ``capture()``
    records the whole step in a HIP graph that ``replay()`` launches.
    fused=False: the plain path - one host-synchronised plan per view (same
    tile, LDS batch, transmittance mode and fovea culling), eager launches,
    views one after another; the library normalises each view's L1 by the
    entry count over all views and adds the views' losses and gradients, so
    the step optimises the same objective as the fused one.
    """

    def __init__(self, ctx: Context, params: torch.Tensor, cams, targets: torch.Tensor,
                 gaze: Optional[torch.Tensor] = None, cfg: FitConfig = FitConfig(),
                 fused: bool = True):
        self.ctx, self.cfg, self.fused = ctx, cfg, fused
        self.params = params
        self.C, self.n = params.shape
        self.sh_degree = int(round(((self.C - 11) // 3) ** 0.5)) - 1
        dev = params.device
        self.cams = list(cams)
        self.sizes = [(c.width, c.height) for c in self.cams]
        self.cams_dev = cameras_to_device(self.cams, dev)
        self.targets = targets.contiguous()
        self.gaze = gaze
        total = sum(w * h for w, h in self.sizes)
        self.rgba = torch.zeros(4 * total, dtype=torch.float32, device=dev)
        self.dl = torch.zeros_like(self.rgba)
        self.grads = torch.zeros_like(params)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        lr = plane_learning_rates(self.sh_degree, cfg.lr, cfg.lr_boost)
        self._seg_lr = (ct.c_float * self.C)(*[float(x) for x in lr])
        if cfg.random_bg and not cfg.alpha_loss:
            raise ValueError("random_bg needs alpha_loss (RGBA targets)")
        if not fused and (cfg.alpha_loss or cfg.random_bg or cfg.masked_adam):
            raise ValueError("alpha training, random backgrounds and the masked Adam are "
                             "fused-step options")
        if fused:
            self.key_capacity = cfg.key_capacity or self._measure_capacity()
            self._make_plan()
        else:
            self.view_plans = []
            off = 0
            for k, (w, h) in enumerate(self.sizes):
                p = Plan(ctx, self.n, [(w, h)], self.sh_degree, cfg.tile, cfg.lds_batch,
                         host_sized=True, key_capacity=cfg.key_capacity, t_mode=cfg.t_mode)
                sl = slice(off, off + w * h)
                self.view_plans.append((p, self.cams_dev[128 * k:128 * (k + 1)], sl))
                off += w * h
            # the fused step's normaliser: masked entries over all views
            self.norm_count = sum(
                p.loss_count(self._view_gaze(k), cfg.radius_frac)
                for k, (p, _, _) in enumerate(self.view_plans))
        self.captured = False

    def _view_gaze(self, k):
        return self.gaze[k] if self.gaze is not None else None

    @property
    def culls(self) -> bool:
        return bool(self.cfg.fovea_cull and self.gaze is not None)

    def _make_plan(self):
        self.plan = Plan(self.ctx, self.n, self.sizes, self.sh_degree, self.cfg.tile,
                         self.cfg.lds_batch, host_sized=False, key_capacity=self.key_capacity,
                         t_mode=self.cfg.t_mode)
        self.args = self._args(self.plan, self.cams_dev, self.targets, self.rgba, self.dl,
                               self.gaze)

    def ensure_capacity(self) -> bool:
        """Poll the fused step's flags (synchronises).  After a key-capacity
        overflow (the overflowing steps left parameters, moments and the step
        counter as they were) re-plan with room for 1.5 times the keys needed
        (at least twice the old capacity), recapture if captured, and return
        True: the caller repeats the step.  Raises on a non-finite loss."""
        if not self.fused:
            raise GsfError(_abi.GSF_E_STATE, "the plain path reports overflow on each forward")
        flags, m = self.plan.poll()
        if flags & _abi.GSF_FLAG_NONFINITE:
            raise GsfError(_abi.GSF_E_NONFINITE, "non-finite loss")
        if not flags & _abi.GSF_FLAG_CAPACITY:
            return False
        self.plan.close()
        self.key_capacity = max(2 * self.key_capacity, int(m * 1.5) + (1 << 16))
        self._make_plan()
        if self.captured:
            self.capture()
        return True

    def _measure_capacity(self) -> int:
        return measure_keys(self.ctx, self.params, self.cams_dev, self.sizes, self.sh_degree,
                            self.cfg.tile, self.gaze if self.culls else None,
                            self.cfg.radius_frac) * 3 // 2 + (1 << 16)

    def _args(self, plan, cams_dev, targets, rgba, dl, gaze):
        return gsf_step_args(
            params=self.params.data_ptr(), n=self.n, cams=cams_dev.data_ptr(),
            target_rgb=targets.data_ptr(), gaze_px=gaze.data_ptr() if gaze is not None else None,
            mask_radius_frac=self.cfg.radius_frac, loss=self.loss.data_ptr(),
            rgba=rgba.data_ptr(), dl_drgba=dl.data_ptr(), grads=self.grads.data_ptr(),
            adam_m=self.m.data_ptr(), adam_v=self.v.data_ptr(), step_dev=self.step_dev.data_ptr(),
            seg_lr=ct.cast(self._seg_lr, ct.POINTER(ct.c_float)), beta1=self.cfg.betas[0],
            beta2=self.cfg.betas[1], eps=self.cfg.eps,
            fovea_cull=int(bool(self.cfg.fovea_cull and gaze is not None)),
            alpha_loss=int(bool(self.cfg.alpha_loss)), random_bg=int(bool(self.cfg.random_bg)),
            bg_seed=int(self.cfg.bg_seed) & ((1 << 64) - 1),
            masked_adam=int(bool(self.cfg.masked_adam)))

    def step(self):
        """One eager step."""
        self.ctx.use_stream()
        if self.fused:
            self.ctx.check(lib().gsf_step(self.plan.handle, ct.byref(self.args)), "gsf_step")
            return
        # plain: per view forward + loss share + backward, the library adding the
        # views' losses and gradients, then Adam
        for k, (p, cam, sl) in enumerate(self.view_plans):
            rgba = self.rgba[4 * sl.start:4 * sl.stop]
            dl = self.dl[4 * sl.start:4 * sl.stop]
            tgt = self.targets[3 * sl.start:3 * sl.stop]
            gz = self._view_gaze(k)
            p.forward(self.params, self.n, cam, rgba, gz if self.culls else None,
                      self.cfg.radius_frac)
            p.loss_l1(rgba, tgt, self.loss, dl, gz, self.cfg.radius_frac,
                      norm_count=self.norm_count, accumulate=k > 0)
            p.backward(self.params, self.n, cam, dl, self.grads, accumulate=k > 0)
        seg_off = [c * self.n for c in range(self.C + 1)]
        lr = list(self._seg_lr)
        so, sl_ = [0], [lr[0]]
        for c in range(1, self.C):
            if lr[c] != sl_[-1]:
                so.append(seg_off[c])
                sl_.append(lr[c])
        so.append(seg_off[self.C])
        adam(self.ctx, self.params, self.grads, self.m, self.v, self.step_dev, so, sl_,
             self.cfg.betas, self.cfg.eps)

    def capture(self):
        if not self.fused:
            raise GsfError(_abi.GSF_E_STATE, "only the fused step can be captured")
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_step_capture(self.plan.handle, ct.byref(self.args)),
                       "gsf_step_capture")
        self.captured = True

    def replay(self):
        self.ctx.use_stream()
        self.ctx.check(lib().gsf_step_replay(self.plan.handle), "gsf_step_replay")

    def steps_done(self) -> int:
        """The device step counter (synchronises): steps that updated the model
        since the last optimiser reset."""
        return int(self.step_dev.item())

    def run(self, steps: int, check_every: int = 100) -> int:
        """Replay the captured step until ``steps`` steps have updated the model.
        The device flags are polled every ``check_every`` replays (one
        synchronisation each).  A step that overflows the key capacity changes
        nothing (parameters, moments and step counter stay), so after an
        overflow the plan is re-made with room (``ensure_capacity``) and the
        missing steps are replayed.  Returns the number of re-plans."""
        if not self.captured:
            raise GsfError(_abi.GSF_E_STATE, "capture() first")
        target = self.steps_done() + int(steps)
        replans = 0
        while True:
            left = target - self.steps_done()
            if left <= 0:
                return replans
            for _ in range(min(left, max(1, int(check_every)))):
                self.replay()
            if self.ensure_capacity():
                replans += 1

    def close(self):
        """Release the plans (and their workspaces)."""
        if self.fused:
            self.plan.close()
        else:
            for p, _, _ in self.view_plans:
                p.close()

    def backgrounds(self):
        """The per-view backgrounds [V][3] drawn by the last random_bg step."""
        if not (self.fused and self.cfg.random_bg):
            raise GsfError(_abi.GSF_E_STATE, "no random backgrounds in this step")
        return self.plan.debug(_abi.GSF_DBG_BG, np.float32, 3 * len(self.cams)).reshape(-1, 3)

    def reset_optimizer(self):
        """Continual refinement restarts Adam: zero m, v and the step counter
        (gsf_adam_reset)."""
        adam_reset(self.ctx, self.m, self.v, self.step_dev)

    def restart(self, params: Optional[torch.Tensor] = None):
        """Restart optimisation: reload ``params`` (same shape) as the Gaussians,
        if given, and discard the optimiser state.  A captured graph stays valid
        (same buffers)."""
        if params is not None:
            if tuple(params.shape) != tuple(self.params.shape):
                raise ValueError("restart: the Gaussian count is fixed by the plan")
            self.ctx.use_stream()
            self.params.copy_(params)
        self.reset_optimizer()

    def visibility(self):
        """Per-Gaussian visibility (uint8 [n]) of the last masked_adam step."""
        if not (self.fused and self.cfg.masked_adam):
            raise GsfError(_abi.GSF_E_STATE, "no masked Adam in this step")
        return self.plan.debug(_abi.GSF_DBG_VIS, np.uint8, self.n)

    def poll(self):
        if self.fused:
            return self.plan.poll()
        flags, m = 0, 0
        for p, _, _ in self.view_plans:
            f, mm = p.poll()
            flags |= f
            m += mm
        return flags, m


class Refiner:
    """Continual refinement by restart (Method, "Periphery Model Training").

    Holds the training views (cameras, per-view targets, optional gaze points).
    ``offer`` admits a new view only when Eq. (1) finds it novel against every
    kept view (gsf_view_select).  ``restart`` builds the fused, captured step
    over all kept views (at most 64), starting from the current Gaussians with
    the optimiser state discarded; ``run`` replays it.  Either every view has a
    gaze point (fovea-masked loss) or none has.
    """

    def __init__(self, ctx: Context, params: torch.Tensor, cams, targets, gazes=None,
                 cfg: FitConfig = FitConfig(), delta_pos: float = 0.05,
                 theta_view_deg: float = 5.0):
        self.ctx, self.cfg = ctx, cfg
        self.params = params
        self.delta_pos, self.theta_view_deg = float(delta_pos), float(theta_view_deg)
        self.cams = list(cams)
        self.targets = [t.reshape(-1) for t in targets]
        if len(self.targets) != len(self.cams):
            raise ValueError("one target per camera")
        self.gazes = None if gazes is None else [np.asarray(g, np.float32).reshape(2) for g in gazes]
        self.fit: Optional[FitStep] = None
        self.pending = 0          # views admitted since the last restart

    def offer(self, cam, target: torch.Tensor, gaze=None) -> bool:
        """Eq. (1): keep the view if it is novel against every kept view."""
        if (gaze is None) != (self.gazes is None):
            raise ValueError("either every view has a gaze point or none has")
        if not select_views(self.cams, [cam], self.delta_pos, self.theta_view_deg)[0]:
            return False
        self.cams.append(cam)
        self.targets.append(target.reshape(-1))
        if gaze is not None:
            self.gazes.append(np.asarray(gaze, np.float32).reshape(2))
        self.pending += 1
        return True

    def restart(self) -> FitStep:
        """Fused step over every kept view from the current Gaussians, Adam state
        discarded (new zero moments and step counter), captured in a graph."""
        if len(self.cams) > 64:
            raise GsfError(_abi.GSF_E_INVALID, "at most 64 views per fused step")
        if self.fit is not None:
            self.fit.plan.close()
        dev = self.params.device
        tgt = torch.cat(self.targets)
        gz = None
        if self.gazes is not None:
            gz = torch.from_numpy(np.stack(self.gazes)).to(dev)
        self.fit = FitStep(self.ctx, self.params, self.cams, tgt, gz, cfg=self.cfg, fused=True)
        self.fit.reset_optimizer()
        self.fit.capture()
        self.pending = 0
        return self.fit

    def run(self, steps: int):
        """``steps`` captured fit steps that update the model (a step lost to a
        key overflow is repeated after a re-plan, see FitStep.run)."""
        if self.fit is None:
            raise GsfError(_abi.GSF_E_STATE, "restart() first")
        return self.fit.run(steps)


def seed_first_hits(ctx: Context, vol: torch.Tensor, cams, cap: int, seed: int, step: float,
                    extinction: float = 40.0, threshold: float = 1200.0, range_: float = 1800.0,
                    lo=(0.8, 0.3, 0.2), hi=(1.0, 0.95, 0.9), hit_alpha: float = 0.5,
                    color_steps: int = 8, opacity: float = 0.1):
    """gsf_seed_first_hits: Gaussians at the first significant hits of every
    pixel ray of `cams` (planar float32 [14][m]) and the ray of each (int32 [m]).
    Synchronises."""
    n = int(vol.shape[0])
    cams = list(cams)
    dev = vol.device
    cams_dev = cameras_to_device(cams, dev)
    ws = (ct.c_int32 * len(cams))(*[c.width for c in cams])
    hs = (ct.c_int32 * len(cams))(*[c.height for c in cams])
    nrays = sum(c.width * c.height for c in cams)
    nb = ct.c_size_t()
    ctx.check(lib().gsf_first_hit_scratch_bytes(nrays, ct.byref(nb)), "gsf_first_hit_scratch_bytes")
    scratch = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=dev)
    base = scratch.data_ptr()
    aligned = (base + 255) & ~255
    out = torch.empty(14 * int(cap), dtype=torch.float32, device=dev)
    ids = torch.empty(int(cap), dtype=torch.int32, device=dev)
    m = ct.c_int64()
    lo_a = (ct.c_float * 3)(*[float(x) for x in lo])
    hi_a = (ct.c_float * 3)(*[float(x) for x in hi])
    ctx.use_stream()
    ctx.check(lib().gsf_seed_first_hits(ctx.handle, _ptr(vol), n, _ptr(cams_dev), len(cams), ws, hs,
                                        float(step), float(extinction), float(threshold),
                                        float(range_), lo_a, hi_a, float(hit_alpha),
                                        int(color_steps), float(opacity), int(cap),
                                        int(seed) & ((1 << 64) - 1), _ptr(out), _ptr(ids),
                                        ct.byref(m), ct.c_void_p(aligned), nb.value),
              "gsf_seed_first_hits")
    k = int(m.value)
    return out[:14 * k].view(14, k), ids[:k]


def _mat16(m):
    a = np.ascontiguousarray(np.asarray(m, np.float32).reshape(16))
    return (ct.c_float * 16)(*[float(x) for x in a])


def _vec3(v):
    return (ct.c_float * 3)(*[float(x) for x in np.asarray(v, np.float32).reshape(3)])


def reproject(ctx: Context, depth: torch.Tensor, P_old, V_old, pos_old, P_new, V_new) -> torch.Tensor:
    """gsf_reproject (Eqs. (2)-(4)): clip coordinates [4][H][W] of every pixel
    of a depth image [H][W] (NaN where the depth is missing).  Matrices: 4x4
    row-major, column-vector convention."""
    H, W = depth.shape
    clip = torch.empty((4, H, W), dtype=torch.float32, device=depth.device)
    ctx.use_stream()
    ctx.check(lib().gsf_reproject(ctx.handle, _ptr(depth), int(W), int(H), _mat16(P_old),
                                  _mat16(V_old), _vec3(pos_old), _mat16(P_new), _mat16(V_new),
                                  _ptr(clip)), "gsf_reproject")
    return clip


def reproject_warp(ctx: Context, rgba: torch.Tensor, depth: torch.Tensor, P_old, V_old, pos_old,
                   P_new, V_new, out_w: int, out_h: int, zbuf: Optional[torch.Tensor] = None):
    """gsf_reproject_warp: the image [4][H][W] moved to the new view by its
    depth, as (out_rgba [4][out_h][out_w], src int32 [out_h][out_w])."""
    H, W = depth.shape
    dev = depth.device
    if zbuf is None:
        zbuf = torch.empty(int(out_w) * int(out_h), dtype=torch.int64, device=dev)
    out = torch.empty((4, out_h, out_w), dtype=torch.float32, device=dev)
    src = torch.empty((out_h, out_w), dtype=torch.int32, device=dev)
    ctx.use_stream()
    ctx.check(lib().gsf_reproject_warp(ctx.handle, _ptr(rgba), _ptr(depth), int(W), int(H),
                                       _mat16(P_old), _mat16(V_old), _vec3(pos_old),
                                       _mat16(P_new), _mat16(V_new), int(out_w), int(out_h),
                                       _ptr(zbuf), _ptr(out), _ptr(src)), "gsf_reproject_warp")
    return out, src


def reproject_warp_noalloc(ctx: Context, rgba: torch.Tensor, depth: torch.Tensor, P_old, V_old,
                           pos_old, P_new, V_new, out_rgba: torch.Tensor, out_src: torch.Tensor):
    """gsf_reproject_warp_noalloc: reproject_warp into caller-given outputs
    (out_rgba float32 [4][out_h][out_w], out_src int32 [out_h][out_w]) with the
    library's device-resident z-buffer; the call allocates no device memory."""
    H, W = depth.shape
    out_h, out_w = out_src.shape
    ctx.use_stream()
    ctx.check(lib().gsf_reproject_warp_noalloc(ctx.handle, _ptr(rgba), _ptr(depth), int(W), int(H),
                                               _mat16(P_old), _mat16(V_old), _vec3(pos_old),
                                               _mat16(P_new), _mat16(V_new), int(out_w), int(out_h),
                                               _ptr(out_rgba), _ptr(out_src)),
              "gsf_reproject_warp_noalloc")
    return out_rgba, out_src


def seed_volume(ctx: Context, vol: torch.Tensor, cap: int, seed: int, threshold: float = 1200.0,
                range_: float = 1800.0, lo=(0.8, 0.3, 0.2), hi=(1.0, 0.95, 0.9),
                opacity: float = 0.1) -> torch.Tensor:
    """Gaussians seeded on the device from a uint16 volume [n][n][n] (one per
    voxel above the threshold, capped by a seeded priority subset): planar
    float32 [14][m] (see gsf_seed_volume).  Synchronises."""
    n = int(vol.shape[0])
    assert vol.dtype == torch.int16 or vol.dtype == torch.uint16 or vol.element_size() == 2
    nb = ct.c_size_t()
    ctx.check(lib().gsf_seed_scratch_bytes(n, ct.byref(nb)), "gsf_seed_scratch_bytes")
    scratch = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=vol.device)
    out = torch.empty(14 * int(cap), dtype=torch.float32, device=vol.device)
    m = ct.c_int64()
    lo_a, hi_a = (ct.c_double * 3)(*lo), (ct.c_double * 3)(*hi)
    ctx.use_stream()
    ctx.check(lib().gsf_seed_volume(ctx.handle, _ptr(vol), n, float(threshold), float(range_), lo_a,
                                    hi_a, float(opacity), int(cap), int(seed) & ((1 << 64) - 1),
                                    _ptr(out), ct.byref(m), _ptr(scratch), nb.value),
              "gsf_seed_volume")
    return out[:14 * m.value].view(14, m.value)


def raymarch(ctx: Context, vol: torch.Tensor, cams, step: Optional[float] = None,
             extinction: float = 40.0, t_stop: float = 1e-4, threshold: float = 1200.0,
             range_: float = 1800.0, lo=(0.8, 0.3, 0.2), hi=(1.0, 0.95, 0.9),
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Emission-absorption RGBA of the volume for each camera (float32 [4][H][W]
    per view, concatenated); step defaults to half a voxel (1/n)."""
    n = int(vol.shape[0])
    cams = list(cams)
    sizes = [(c.width, c.height) for c in cams]
    if out is None:
        out = torch.empty(4 * sum(w * h for w, h in sizes), dtype=torch.float32, device=vol.device)
    cams_dev = cameras_to_device(cams, vol.device)
    w = (ct.c_int32 * len(cams))(*[a for a, _ in sizes])
    h = (ct.c_int32 * len(cams))(*[b for _, b in sizes])
    ctx.use_stream()
    ctx.check(lib().gsf_raymarch(ctx.handle, _ptr(vol), n, _ptr(cams_dev), len(cams), w, h,
                                 float(step if step is not None else 1.0 / n), float(extinction),
                                 float(t_stop), float(threshold), float(range_),
                                 (ct.c_float * 3)(*lo), (ct.c_float * 3)(*hi), _ptr(out)),
              "gsf_raymarch")
    return out


def measure_keys(ctx: Context, params: torch.Tensor, cams_dev: torch.Tensor, sizes, sh_degree: int,
                 tile: int, cull_gaze: Optional[torch.Tensor] = None, radius_frac: float = 0.0) -> int:
    """Keys one forward of these Gaussians lists at this tile size (a host-sized
    plan; fovea-culled when cull_gaze is given).  Synchronises."""
    n = params.shape[1]
    cap = 4 * n * len(sizes) + (1 << 20)
    while True:
        # the key total a host-sized forward reports is exact even when it exceeds
        # the capacity, so the probe's workspace can stay modest
        probe = Plan(ctx, n, sizes, sh_degree, tile, 64, host_sized=True, key_capacity=cap)
        out = torch.empty(4 * probe.total_pixels, dtype=torch.float32, device=params.device)
        ctx.use_stream()
        st = lib().gsf_forward(probe.handle, _ptr(params), int(n), _ptr(cams_dev), _ptr(cull_gaze),
                               float(radius_frac), _ptr(out))
        if st not in (_abi.GSF_OK, _abi.GSF_E_CAPACITY):
            ctx.check(st, "gsf_forward")
        _, m = probe.poll()
        probe.close()
        if m > 0 or st == _abi.GSF_OK:
            return int(m)
        cap *= 4   # no total reported: try again with room


_TUNE_CACHE: dict = {}


def autotune(ctx: Context, params: torch.Tensor, cams, targets: torch.Tensor,
             gaze: Optional[torch.Tensor] = None, cfg: FitConfig = FitConfig(),
             tiles=(8, 16, 32), batches=(64, 128, 256), t_modes=None, warmup: int = 3,
             reps: int = 10, stream=None):
    """gsf_autotune: the tile size, LDS batch and adjoint transmittance mode that
    make the captured fused step fastest on this input.  Each tile size's key
    capacity is 1.5 times the keys one forward lists there.  The library times
    every candidate's captured forward + loss + backward with HIP events over
    ``reps`` replays (Adam left out, so params are not changed).  ``t_modes``
    defaults to ``(cfg.t_mode,)``.  Results are cached per input shape and step
    options.  Returns (best (tile, batch, t_mode), {(tile, batch, t_mode):
    ms/step}); overflowing candidates are left out of the dict."""
    t_modes = tuple(t_modes) if t_modes is not None else (cfg.t_mode,)
    key = (params.shape[1], params.shape[0], tuple((c.width, c.height) for c in cams),
           tuple(tiles), tuple(batches), t_modes, bool(cfg.fovea_cull), bool(cfg.alpha_loss),
           bool(cfg.random_bg), bool(cfg.masked_adam), gaze is not None, float(cfg.radius_frac))
    if key in _TUNE_CACHE:
        return _TUNE_CACHE[key]
    stream = stream or torch.cuda.current_stream()
    if stream.cuda_stream == 0:          # graphs cannot be captured on the null stream
        stream = torch.cuda.Stream()
    C, n = params.shape
    sh_degree = int(round(((C - 11) // 3) ** 0.5)) - 1
    sizes = [(c.width, c.height) for c in cams]
    cull = bool(cfg.fovea_cull and gaze is not None)
    with torch.cuda.stream(stream):
        ctx.use_stream()
        dev = params.device
        cams_dev = cameras_to_device(cams, dev)
        space = _abi.gsf_tune_space(n_tiles=len(tiles), n_batches=len(batches),
                                    n_t_modes=len(t_modes), warmup=int(warmup), reps=int(reps))
        for k, t in enumerate(tiles):
            space.tiles[k] = int(t)
            space.key_capacity[k] = measure_keys(ctx, params, cams_dev, sizes, sh_degree, t,
                                                 gaze if cull else None,
                                                 cfg.radius_frac) * 3 // 2 + (1 << 16)
        for j, b in enumerate(batches):
            space.batches[j] = int(b)
        for m, tm in enumerate(t_modes):
            space.t_modes[m] = int(tm)
        w = (ct.c_int32 * len(sizes))(*[a for a, _ in sizes])
        h = (ct.c_int32 * len(sizes))(*[b for _, b in sizes])
        desc = gsf_plan_desc(n_max=n, sh_degree=sh_degree, n_views=len(sizes),
                             widths=ct.cast(w, ct.POINTER(ct.c_int32)),
                             heights=ct.cast(h, ct.POINTER(ct.c_int32)), tile=int(tiles[0]),
                             lds_batch=int(batches[0]), t_mode=int(t_modes[0]), host_sized=0,
                             key_capacity=0)
        nb = ct.c_size_t()
        ctx.check(lib().gsf_autotune_workspace_bytes(ctx.handle, ct.byref(desc), ct.byref(space),
                                                     ct.byref(nb)), "gsf_autotune_workspace_bytes")
        raw = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=dev)
        ws = (raw.data_ptr() + 255) & ~255
        total = sum(a * b for a, b in sizes)
        rgba = torch.zeros(4 * total, dtype=torch.float32, device=dev)
        dl = torch.zeros_like(rgba)
        grads = torch.zeros_like(params)
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        step_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        lr = (ct.c_float * C)(*([0.0] * C))
        tgt = targets.contiguous()
        args = gsf_step_args(
            params=params.data_ptr(), n=n, cams=cams_dev.data_ptr(), target_rgb=tgt.data_ptr(),
            gaze_px=gaze.data_ptr() if gaze is not None else None,
            mask_radius_frac=cfg.radius_frac, loss=loss.data_ptr(), rgba=rgba.data_ptr(),
            dl_drgba=dl.data_ptr(), grads=grads.data_ptr(), adam_m=grads.data_ptr(),
            adam_v=grads.data_ptr(), step_dev=step_dev.data_ptr(),
            seg_lr=ct.cast(lr, ct.POINTER(ct.c_float)), beta1=cfg.betas[0], beta2=cfg.betas[1],
            eps=cfg.eps, fovea_cull=int(cull), alpha_loss=int(bool(cfg.alpha_loss)),
            random_bg=int(bool(cfg.random_bg)), bg_seed=int(cfg.bg_seed) & ((1 << 64) - 1),
            masked_adam=int(bool(cfg.masked_adam)))
        res = _abi.gsf_tune_result()
        ctx.check(lib().gsf_autotune(ctx.handle, ct.byref(desc), ct.byref(space), ct.byref(args),
                                     ct.c_void_p(ws), nb.value, ct.byref(res)), "gsf_autotune")
        del raw
    times = {}
    for k, t in enumerate(tiles):
        for j, b in enumerate(batches):
            for m, tm in enumerate(t_modes):
                ms = float(res.ms[9 * k + 3 * j + m])
                if ms >= 0 and ms != float("inf"):
                    times[(int(t), int(b), int(tm))] = ms
    best = (int(res.tile), int(res.lds_batch), int(res.t_mode))
    _TUNE_CACHE[key] = (best, times)
    return best, times
