"""FP64 CPU oracle for the Gaussian-splatting fit step (ctypes wrapper of gsorc.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the package smoke check
and the benchmark's CPU-baseline leg.  The product path never imports it.

Functions follow the plain definitions written out in ``gsorc.c`` (projection by
the local affine approximation of the pinhole map, brute-force front-to-back
compositing over all Gaussians in depth order, the exact adjoint, the
(tile, depth) discrete stage by nested loops and a comparison sort, L1 loss,
bias-corrected Adam) and, in Python, the refinement loop's Eq. (1) view
selection, Gaussian visibility and visibility-masked Adam.  Inputs are the float32 arrays produced by ``synth``,
widened to float64.
"""
from __future__ import annotations

import ctypes as ct
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsorc.c")
_LIB = os.path.join(_HERE, "libgsorc.so")

NREC = 22
F_NEAR_ALPHA, F_NEAR_STOP, F_NEAR_TIE, F_NEAR_CLAMP = 1, 2, 4, 8
F_NEAR_CULL, F_NEAR_BOX, F_NEAR_GRAD = 16, 32, 64
# pixel flags that make the fp32 image legitimately differ
IMAGE_FLAGS = F_NEAR_ALPHA | F_NEAR_STOP | F_NEAR_TIE
REC_FIELDS = ["valid", "tz", "tx", "ty", "mx", "my", "A", "B", "C", "o", "r", "g", "b",
              "sa", "sb", "sc", "ex0", "ex1", "ey0", "ey1", "d32", "colraw"]

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.{os.getpid()}.tmp"   # concurrent test workers each build their own
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ct.CDLL(_LIB)
        dp, i64p, i32p = ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32)
        L.orc_project.argtypes = [dp, ct.c_int64, ct.c_int, dp, dp, i32p]
        L.orc_render.argtypes = [dp, ct.c_int64, ct.c_int, dp, i64p, ct.c_int64, dp, dp, i64p,
                                 i64p, i32p]
        L.orc_backward.argtypes = [dp, ct.c_int64, ct.c_int, dp, i64p, ct.c_int64, dp, dp, dp]
        L.orc_discrete.argtypes = [dp, ct.c_int64, ct.c_int, dp, ct.c_int, ct.c_int, i64p, i64p,
                                   ct.c_int64, i64p, i64p, i32p]
        L.orc_loss_l1.argtypes = [dp, dp, ct.c_int64, ct.c_int64, dp, ct.c_double, dp, i64p]
        L.orc_loss_l1.restype = ct.c_double
        L.orc_loss_l1_rgba.argtypes = [dp, dp, dp, ct.c_int64, ct.c_int64, dp, ct.c_double, ct.c_int,
                                       dp, i64p]
        L.orc_loss_l1_rgba.restype = ct.c_double
        L.orc_adam.argtypes = [dp, dp, dp, dp, ct.c_int64, ct.c_double, ct.c_double, ct.c_double,
                               ct.c_double, ct.c_int64]
        L.orc_adam.restype = None
        L.orc_sh_basis.argtypes = [ct.c_int, dp, ct.c_int64, dp]
        L.orc_first_hits.argtypes = [ct.c_void_p, ct.c_int, dp, ct.c_int, ct.c_double, ct.c_double,
                                     ct.c_double, ct.c_double, dp, dp, ct.c_double, ct.c_int, i32p,
                                     dp, dp, dp]
        L.orc_num_threads.restype = ct.c_int
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=ct.c_double):
    return a.ctypes.data_as(ct.POINTER(t)) if a is not None else None


def cam_array(cam) -> np.ndarray:
    """27-double camera record of a ``synth.Camera``."""
    return _d(np.concatenate([cam.R.reshape(-1), cam.t, cam.campos,
                              [cam.fx, cam.fy, cam.cx, cam.cy, cam.tanx, cam.tany, cam.znear],
                              cam.bg, [cam.width, cam.height]]))


def sh_degree_of(params) -> int:
    C = params.shape[0]
    K = (C - 11) // 3
    deg = int(round(K ** 0.5)) - 1
    assert 11 + 3 * (deg + 1) ** 2 == C, "bad parameter plane count"
    return deg


def num_threads() -> int:
    return lib().orc_num_threads()


def project(params, cam):
    """FP64 per-Gaussian projection records as a dict of arrays, plus flags."""
    P = _d(params)
    n = P.shape[1]
    rec = np.zeros((n, NREC))
    fl = np.zeros(n, np.int32)
    rc = lib().orc_project(_p(P), n, sh_degree_of(P), _p(cam_array(cam)), _p(rec),
                           _p(fl, ct.c_int32))
    assert rc == 0
    out = {k: rec[:, j] for j, k in enumerate(REC_FIELDS)}
    out["flags"] = fl
    return out


@dataclass
class Render:
    rgba: np.ndarray      # [4][npix]
    tfinal: np.ndarray    # [npix]
    last: np.ndarray      # [npix] Gaussian index of the last included Gaussian, -1 if none
    ncontrib: np.ndarray  # [npix]
    flags: np.ndarray     # [npix]


def render(params, cam, pixels=None) -> Render:
    P = _d(params)
    n = P.shape[1]
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int64)
    npix = cam.npix if pix is None else pix.size
    rgba = np.zeros((4, npix))
    tf = np.zeros(npix)
    last = np.zeros(npix, np.int64)
    nc = np.zeros(npix, np.int64)
    fl = np.zeros(npix, np.int32)
    rc = lib().orc_render(_p(P), n, sh_degree_of(P), _p(cam_array(cam)), _p(pix, ct.c_int64),
                          npix, _p(rgba), _p(tf), _p(last, ct.c_int64), _p(nc, ct.c_int64),
                          _p(fl, ct.c_int32))
    assert rc == 0
    return Render(rgba, tf, last, nc, fl)


def backward(params, cam, dl_drgba, pixels=None, with_g2d=False):
    """Gradient of sum <dl, rgba> over the listed pixels w.r.t. the raw
    parameters ([C][n], float64); optionally also the per-Gaussian 2D gradient
    (dmx, dmy, dA, dB, dC, do, dr, dg, db) as [9][n]."""
    P = _d(params)
    n = P.shape[1]
    pix = None if pixels is None else np.ascontiguousarray(pixels, np.int64)
    npix = cam.npix if pix is None else pix.size
    dl = _d(dl_drgba).reshape(4, npix)
    G = np.zeros_like(P)
    g2 = np.zeros((9, n))
    rc = lib().orc_backward(_p(P), n, sh_degree_of(P), _p(cam_array(cam)), _p(pix, ct.c_int64),
                            npix, _p(dl), _p(G), _p(g2))
    assert rc == 0
    return (G, g2) if with_g2d else G


@dataclass
class Discrete:
    keys: np.ndarray      # global tile id per key
    vals: np.ndarray      # record r = v*n + i per key
    ranges: np.ndarray    # [tiles][2] start, end
    rflags: np.ndarray    # [V*n] per-record ambiguity flags
    m: int


def discrete(params, cams, tile: int) -> Discrete:
    P = _d(params)
    n = P.shape[1]
    C = _d(np.concatenate([cam_array(c) for c in cams]))
    tiles = sum(((c.width + tile - 1) // tile) * ((c.height + tile - 1) // tile) for c in cams)
    ranges = np.zeros((tiles, 2), np.int64)
    rflags = np.zeros(len(cams) * n, np.int32)
    m = np.zeros(1, np.int64)
    # first pass counts, second pass fills
    lib().orc_discrete(_p(P), n, sh_degree_of(P), _p(C), len(cams), tile, None, None, 0,
                       _p(m, ct.c_int64), _p(ranges, ct.c_int64), _p(rflags, ct.c_int32))
    M = int(m[0])
    keys = np.zeros(max(M, 1), np.int64)
    vals = np.zeros(max(M, 1), np.int64)
    lib().orc_discrete(_p(P), n, sh_degree_of(P), _p(C), len(cams), tile, _p(keys, ct.c_int64),
                       _p(vals, ct.c_int64), M, _p(m, ct.c_int64), _p(ranges, ct.c_int64),
                       _p(rflags, ct.c_int32))
    return Discrete(keys[:M], vals[:M], ranges, rflags, M)


def fovea_radius(radius_frac, width):
    """The fovea radius in pixels as the compositing path forms it: the
    fraction and the width in float32, their product rounded to float32 (the
    mask decides an integer, so both sides take it in the same precision)."""
    return float(np.float32(np.float32(radius_frac) * np.float32(width)))


def loss_l1_view(rgba, target, cam, gaze=None, radius=0.0):
    """(sum, count, sign[4][npix]) of one view's masked L1 term."""
    rgba = _d(rgba).reshape(4, -1)
    target = _d(target).reshape(-1, rgba.shape[1])[:3]
    target = np.ascontiguousarray(target)
    dl = np.zeros_like(rgba)
    cnt = np.zeros(1, np.int64)
    g = None if gaze is None else _d(gaze)
    s = lib().orc_loss_l1(_p(rgba), _p(target), cam.width, cam.height, _p(g), float(radius),
                          _p(dl), _p(cnt, ct.c_int64))
    return s, int(cnt[0]), dl


def loss_l1(rgbas, targets, cams, gazes=None, radius_frac=0.2):
    """Mean |RGB - target| over all masked (view, pixel, channel) entries and
    dL/dRGBA per view."""
    sums, cnts, dls = 0.0, 0, []
    for v, cam in enumerate(cams):
        g = None if gazes is None else gazes[v]
        s, c, dl = loss_l1_view(rgbas[v], targets[v], cam, g, fovea_radius(radius_frac, cam.width))
        sums += s
        cnts += c
        dls.append(dl)
    denom = max(cnts, 1)
    return sums / denom, [d / denom for d in dls]


def loss_l1_rgba(rgbas, targets, cams, bgs=None, alpha=True, gazes=None, radius_frac=0.2):
    """Alpha training over backgrounds: mean |prediction - target| over all
    masked (view, pixel, channel) entries, the RGBA target composited over the
    view's background bgs[v] (None: black), channels R, G, B and (alpha) A.
    Returns (loss, [dL/dRGBA per view])."""
    sums, cnts, dls = 0.0, 0, []
    for v, cam in enumerate(cams):
        rgba = _d(rgbas[v]).reshape(4, -1)
        tgt = np.ascontiguousarray(_d(targets[v]).reshape(4, -1))
        dl = np.zeros_like(rgba)
        cnt = np.zeros(1, np.int64)
        g = None if gazes is None else _d(gazes[v])
        bg = None if bgs is None else _d(bgs[v])
        sums += lib().orc_loss_l1_rgba(_p(rgba), _p(tgt), _p(bg), cam.width, cam.height, _p(g),
                                       fovea_radius(radius_frac, cam.width), int(bool(alpha)), _p(dl),
                                       _p(cnt, ct.c_int64))
        cnts += int(cnt[0])
        dls.append(dl)
    denom = max(cnts, 1)
    return sums / denom, [d / denom for d in dls]


_M64 = (1 << 64) - 1


def splitmix64(seed: int, k: int) -> int:
    """k-th output (k >= 1) of the SplitMix64 generator (Steele, Lea and Flood,
    "Fast splittable pseudorandom number generators", OOPSLA 2014) started from
    state ``seed``: the state advances by the golden-ratio increment and each
    output is the state passed through the published 64-bit finaliser."""
    z = (seed + k * 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def background_draw(seed: int, step: int, nviews: int, max_views: int = 64) -> np.ndarray:
    """Random background of every view for fit step ``step`` (0-based): channel
    c of view v is the top 24 bits of output 1 + (step * max_views + v) * 4 + c
    of SplitMix64(seed), scaled to [0, 1).  [nviews][3] float64 (exact float32
    values)."""
    out = np.zeros((nviews, 3))
    for v in range(nviews):
        for c in range(3):
            z = splitmix64(seed, 1 + (step * max_views + v) * 4 + c)
            out[v, c] = (z >> 40) * 2.0 ** -24
    return out


def adam(p, g, m, v, t, lr=1e-3, betas=(0.9, 0.999), eps=1e-15):
    """In-place bias-corrected Adam on float64 arrays; ``t`` is the step number
    after increment (1 for the first step).  ``lr`` may be a per-element array."""
    for a in (p, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lr_arr = np.broadcast_to(np.asarray(lr, np.float64), p.shape)
    if np.all(lr_arr == lr_arr.flat[0]):
        lib().orc_adam(_p(p), _p(g), _p(m), _p(v), p.size, float(lr_arr.flat[0]), betas[0],
                       betas[1], eps, int(t))
        return
    # per-segment learning rates: one call per distinct value on a masked copy
    for val in np.unique(lr_arr):
        sel = np.nonzero(lr_arr.reshape(-1) == val)[0]
        ps, gs, ms, vs = (np.ascontiguousarray(a.reshape(-1)[sel]) for a in (p, g, m, v))
        lib().orc_adam(_p(ps), _p(gs), _p(ms), _p(vs), ps.size, float(val), betas[0], betas[1],
                       eps, int(t))
        p.reshape(-1)[sel], m.reshape(-1)[sel], v.reshape(-1)[sel] = ps, ms, vs


def fit_step(params, m, v, t, cams, targets, gazes=None, radius_frac=0.2, lr=1e-3,
             betas=(0.9, 0.999), eps=1e-15, masked=False, tile=16):
    """One full oracle step (render, L1 loss, adjoint, Adam) on float64 state.
    Returns the loss; params, m, v are updated in place.  masked: the
    visibility-masked Adam of ``adam_masked`` with ``visibility(params, cams,
    tile)`` taken before the update."""
    rgbas = [render(params, c).rgba for c in cams]
    loss, dls = loss_l1(rgbas, targets, cams, gazes, radius_frac)
    G = np.zeros_like(params)
    for cam, dl in zip(cams, dls):
        G += backward(params, cam, dl)
    if masked:
        adam_masked(params, G, m, v, t, visibility(params, cams, tile), lr, betas, eps)
    else:
        adam(params, G, m, v, t, lr, betas, eps)
    return loss


# ------------------------------------------------------------ continual refinement
# Method, "Periphery Model Training": the refinement keeps a set of training
# views, admits a new foveal view only when Eq. (1) finds it novel against every
# view already kept, and restarts optimisation from the current Gaussians with
# the optimiser state discarded (m = v = 0, t = 0).  The visibility-masked
# update is the sparse Adam of Taming 3DGS, which the paper's optimiser builds on.

def view_pose(cam):
    """Camera centre and unit viewing direction in world coordinates (FP64).  The
    viewing direction is the camera's +z axis: the third row of the world-to-
    camera rotation, normalised."""
    c = [float(x) for x in np.asarray(cam.campos, np.float64)]
    d = [float(x) for x in np.asarray(cam.R, np.float64)[2]]
    norm = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
    return c, [x / norm for x in d]


def view_is_novel(pose, kept_poses, delta_pos=0.05, theta_view_deg=5.0) -> bool:
    """Eq. (1): for every kept view i, the centres lie more than delta_pos apart
    or the viewing directions' dot product is below cos(theta_view)."""
    (p, d), cos_t = pose, math.cos(math.radians(theta_view_deg))
    for q, e in kept_poses:
        dist = math.sqrt(sum((p[k] - q[k]) ** 2 for k in range(3)))
        dot = sum(d[k] * e[k] for k in range(3))
        if not (dist > delta_pos or dot < cos_t):
            return False
    return True


def select_views(kept, candidates, delta_pos=0.05, theta_view_deg=5.0):
    """Candidates offered one after another to the kept set (cameras): each one
    that Eq. (1) finds novel joins the set before the next is tested.  Returns
    one bool per candidate."""
    poses = [view_pose(c) for c in kept]
    out = []
    for cam in candidates:
        pose = view_pose(cam)
        novel = view_is_novel(pose, poses, delta_pos, theta_view_deg)
        if novel:
            poses.append(pose)
        out.append(novel)
    return out


def visibility(params, cams, tile: int = 16) -> np.ndarray:
    """Gaussians that emit at least one (tile, depth) key in some view: bool [n]."""
    n = params.shape[1]
    d = discrete(params, cams, tile)
    vis = np.zeros(n, bool)
    vis[d.vals % n] = True
    return vis


def adam_masked(p, g, m, v, t, visible, lr=1e-3, betas=(0.9, 0.999), eps=1e-15):
    """Visibility-masked Adam on planar float64 state [C][n]: the columns of the
    visible Gaussians take one bias-corrected Adam step at step number t; the
    others keep p, m and v.  ``lr``: scalar or per-plane [C]."""
    C, n = p.shape
    sel = np.nonzero(np.asarray(visible, bool))[0]
    if sel.size == 0:
        return
    lr_planes = np.broadcast_to(np.asarray(lr, np.float64).reshape(-1, 1), (C, 1))
    cols = [np.ascontiguousarray(a[:, sel]) for a in (p, g, m, v)]
    adam(*cols, t, lr=np.ascontiguousarray(np.broadcast_to(lr_planes, cols[0].shape)),
         betas=betas, eps=eps)
    p[:, sel], m[:, sel], v[:, sel] = cols[0], cols[2], cols[3]


def sh_basis(deg, dirs):
    d = _d(dirs).reshape(-1, 3)
    out = np.zeros((d.shape[0], 16))
    lib().orc_sh_basis(deg, _p(d), d.shape[0], _p(out))
    return out[:, :(deg + 1) ** 2]


# ------------------------------------------------------------ depth-guided reprojection
# Method, "Real-time Viewer", Eqs. (2)-(4): a pixel with texture coordinate uv
# and first-hit distance d is lifted to the world point at distance d from the
# old camera centre along the ray through the far-plane point that
# (P_old V_old)^-1 maps (2 uv - 1, 1, 1) to, and projected with P_new V_new.

def reproject(depth, P_old, V_old, pos_old, P_new, V_new):
    """Eqs. (2)-(4) per pixel in FP64: clip coordinates [H][W][4] of the world
    points; pixel (i, j) has uv = ((i + 0.5) / W, (j + 0.5) / H).  Pixels whose
    depth is not finite and positive get NaN."""
    d = np.asarray(depth, np.float64)
    H, W = d.shape
    inv_old = np.linalg.inv(np.asarray(P_old, np.float64) @ np.asarray(V_old, np.float64))
    u = (np.arange(W) + 0.5) / W
    v = (np.arange(H) + 0.5) / H
    ndc = np.stack(np.broadcast_arrays((2.0 * u - 1.0)[None, :], (2.0 * v - 1.0)[:, None],
                                       np.ones((H, W)), np.ones((H, W))), -1)
    far = ndc @ inv_old.T                                   # Eq. (2), before the divide
    p_far = far[..., :3] / far[..., 3:4]
    c = np.asarray(pos_old, np.float64)
    ray = p_far - c
    with np.errstate(invalid="ignore", over="ignore"):
        p_world = c + ray / np.linalg.norm(ray, axis=-1, keepdims=True) * d[..., None]   # Eq. (3)
    hom = np.concatenate([p_world, np.ones((H, W, 1))], -1)
    with np.errstate(invalid="ignore", over="ignore"):
        clip = hom @ (np.asarray(P_new, np.float64) @ np.asarray(V_new, np.float64)).T    # Eq. (4)
    clip[~(np.isfinite(d) & (d > 0))] = np.nan
    return clip


def reproject_warp(rgba, depth, P_old, V_old, pos_old, P_new, V_new, out_w, out_h, eps=1e-4):
    """The foveal image moved to the new view: every pixel with a depth lands on
    the output pixel containing its reprojected position (NDC x, y in [-1, 1)
    mapped to [0, W') x [0, H'), clip w > 0, NDC z in [-1, 1]); where several
    land, the smallest clip w (nearest to the new camera) wins, ties to the
    lower source index.  Returns (out_rgba [4][H'][W'], src [H'][W'] with -1
    where nothing lands, flags [H'][W']).  flags marks output pixels whose
    winner FP32 rounding could change: a candidate within eps of a pixel edge,
    or the two nearest candidates within 1e-5 relative in w."""
    rgba = np.asarray(rgba, np.float64).reshape(4, -1)
    clip = reproject(depth, P_old, V_old, pos_old, P_new, V_new).reshape(-1, 4)
    n = clip.shape[0]
    w = clip[:, 3]
    with np.errstate(invalid="ignore", divide="ignore"):
        ndc = clip[:, :3] / w[:, None]
        x = (ndc[:, 0] + 1.0) * 0.5 * out_w
        y = (ndc[:, 1] + 1.0) * 0.5 * out_h
        ok = np.isfinite(w) & (w > 0) & (np.abs(ndc[:, 2]) <= 1.0) & (x >= 0) & (x < out_w) & \
            (y >= 0) & (y < out_h)
    src = np.nonzero(ok)[0]
    tx, ty = np.floor(x[src]).astype(np.int64), np.floor(y[src]).astype(np.int64)
    tgt = ty * out_w + tx
    edge = (np.abs(x[src] - np.round(x[src])) < eps) | (np.abs(y[src] - np.round(y[src])) < eps)
    order = np.lexsort((src, w[src], tgt))                 # by target, then w, then index
    out = np.zeros((4, out_h * out_w))
    who = np.full(out_h * out_w, -1, np.int64)
    flags = np.zeros(out_h * out_w, bool)
    first = np.ones(order.size, bool)
    first[1:] = tgt[order][1:] != tgt[order][:-1]
    for k in np.nonzero(first)[0]:
        t = tgt[order[k]]
        win = order[k]
        who[t] = src[win]
        out[:, t] = rgba[:, src[win]]
        group = [order[k]]
        q = k + 1
        while q < order.size and tgt[order[q]] == t:
            group.append(order[q])
            q += 1
        if edge[group].any():
            flags[t] = True
        if len(group) > 1 and w[src[group[1]]] - w[src[group[0]]] <= 1e-5 * w[src[group[0]]]:
            flags[t] = True
    # a candidate near an edge may belong to a neighbouring output pixel instead
    for s_, t in zip(np.nonzero(edge)[0], tgt[edge]):
        ty_, tx_ = divmod(int(t), out_w)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                yy, xx = ty_ + dy, tx_ + dx
                if 0 <= yy < out_h and 0 <= xx < out_w:
                    flags[yy * out_w + xx] = True
    return out.reshape(4, out_h, out_w), who.reshape(out_h, out_w), flags.reshape(out_h, out_w)


# ------------------------------------------------------------ first-hit point cloud
def first_hits(vol, cams, step, extinction, threshold, range_, lo, hi, hit_alpha=0.5,
               color_steps=8):
    """Per pixel-centre ray of every camera (rays in view, row, column order):
    dict(hit bool [R], pos [R][3], col [R][3], margin [R]) as defined in
    orc_first_hits."""
    vol = np.ascontiguousarray(vol, np.uint16)
    n = vol.shape[0]
    C = _d(np.concatenate([cam_array(c) for c in cams]))
    R = sum(c.width * c.height for c in cams)
    hit = np.zeros(R, np.int32)
    pos = np.zeros((R, 3))
    col = np.zeros((R, 3))
    margin = np.zeros(R)
    lib().orc_first_hits(vol.ctypes.data_as(ct.c_void_p), n, _p(C), len(cams), float(step),
                         float(extinction), float(threshold), float(range_), _p(_d(lo)), _p(_d(hi)),
                         float(hit_alpha), int(color_steps), _p(hit, ct.c_int32), _p(pos), _p(col),
                         _p(margin))
    return {"hit": hit.astype(bool), "pos": pos, "col": col, "margin": margin}


def ray_priority(idx, seed: int, n_rays: int) -> np.ndarray:
    """Cap priority of ray idx: SplitMix64 output idx + 1 from state seed with
    its low b bits (b = bits of n_rays - 1) replaced by idx (distinct)."""
    b = max(1, int(n_rays - 1).bit_length())
    out = np.zeros(len(idx), np.uint64)
    for q, r in enumerate(np.asarray(idx, np.int64)):
        h = splitmix64(seed, int(r) + 1)
        out[q] = np.uint64(((h >> b) << b) | int(r))
    return out


def seed_first_hits(vol, cams, cap, seed, step, extinction, threshold, range_, lo, hi,
                    hit_alpha=0.5, color_steps=8, opacity=0.1, flag_margin=1e-4):
    """Gaussians at the first significant hits (Method, "Volumetric Path
    Tracing"): one per hit ray, capped to the `cap` rays of smallest
    ray_priority, in ray order; mean at the hit, isotropic scale of one voxel,
    identity rotation, the given opacity, the hit colour as degree-0 SH.
    Returns (params [14][m] float64, ray ids [m], flagged ray ids): a ray is
    flagged when its hit decision lies within flag_margin of the threshold."""
    n = np.asarray(vol).shape[0]
    h = first_hits(vol, cams, step, extinction, threshold, range_, lo, hi, hit_alpha, color_steps)
    R = h["hit"].size
    idx = np.nonzero(h["hit"])[0]
    if idx.size > cap:
        pri = ray_priority(idx, seed, R)
        idx = np.sort(idx[np.argsort(pri, kind="stable")[:cap]])
    P = np.zeros((14, idx.size))
    P[0:3] = h["pos"][idx].T
    P[3:6] = math.log(2.0 / n)
    P[6] = 1.0
    P[10] = math.log(opacity / (1.0 - opacity))
    P[11:14] = ((h["col"][idx] - 0.5) / (0.5 / math.sqrt(math.pi))).T
    return P, idx, np.nonzero(h["margin"] < flag_margin)[0]
