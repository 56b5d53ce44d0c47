"""Seeded synthetic inputs for the Gaussian-fit hot path.

This module only *produces inputs*: Gaussian parameter sets, pinhole cameras,
a CT-like phantom volume, voxel-seeded Gaussians and emission-absorption
ray-marched target images.  It contains none of the rasterizer's arithmetic
(projection, compositing, adjoint, optimizer) and is the only code shared by
the FP64 oracle and the HIP path.  Every value it returns is float32-exact, so
both sides read bit-identical inputs (the oracle widens them to float64).

The paper's CT datasets (its Datasets section) and its path tracer are not
available; these generators stand in for them:

* ``random_gaussians``  - independent Gaussians (means uniform in a cube,
  log-normal scales, random unit quaternions, logit-normal opacity,
  RGB-uniform degree-0 colour, optional higher SH bands).
* ``phantom`` / ``seed_from_volume`` - a sum of random ellipsoids with HU-like
  values and noise, and one Gaussian per voxel above a threshold (the paper
  seeds its fit from points placed on the volume's surfaces, Method section,
  "Volumetric Path Tracing").
* ``raymarch`` - an emission-absorption ray march of that volume, standing in
  for the path-traced training views.

Parameter layout (planar float32, ``[C][n]``)::

    0..2   mean (x, y, z)            world units
    3..5   log-scale (x, y, z)       scale = exp(log-scale)
    6..9   quaternion (w, x, y, z)   normalised by the rasterizer
    10     opacity logit             opacity = sigmoid(logit)
    11 + 3k + c   SH coefficient k (k = l*l + l + m) for colour channel c
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Seeds fixed by the workload recipes (each a separate stream).
SEED_GAUSSIANS = 0
SEED_TARGET_SET = 1
SEED_POSES = 2
SEED_VOLUME = 3
SEED_CAP_SUBSET = 4
SEED_RESOLUTIONS = 5
SEED_GAZE = 6
SEED_VIEW_STREAM = 7

RESOLUTION_CHOICES = [(512, 512), (768, 1024), (1024, 1024), (1536, 1536), (2048, 2048)]

_SH_DC = 0.5 / math.sqrt(math.pi)   # value of the constant (l = 0) basis function


def n_sh_coeffs(sh_degree: int) -> int:
    return (sh_degree + 1) ** 2


def n_planes(sh_degree: int) -> int:
    return 11 + 3 * n_sh_coeffs(sh_degree)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _f32(x):
    return np.asarray(x, dtype=np.float32)


# --------------------------------------------------------------------------------------
# Gaussian sets
# --------------------------------------------------------------------------------------

def random_gaussians(n: int, seed: int = SEED_GAUSSIANS, sh_degree: int = 0,
                     logscale_mean: float = -3.0, logscale_std: float = 0.5,
                     mean_range: float = 1.0, sh_rest_std: float = 0.05) -> np.ndarray:
    """Random Gaussian set, planar float32 ``[C][n]``.

    means ~ U[-r, r]^3, log-scales ~ N(mu, sd^2) per axis, quaternions =
    normalised N(0, I4) draws (uniform on the unit sphere), opacity logit ~
    N(0, 1), colour: RGB ~ U[0, 1]^3 stored as degree-0 SH (rgb - 0.5) / Y00,
    higher SH bands ~ N(0, sh_rest_std^2).
    """
    rng = _rng(seed)
    K = n_sh_coeffs(sh_degree)
    P = np.zeros((n_planes(sh_degree), n), dtype=np.float64)
    P[0:3] = rng.uniform(-mean_range, mean_range, size=(3, n))
    P[3:6] = rng.normal(logscale_mean, logscale_std, size=(3, n))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    P[6:10] = q
    P[10] = rng.normal(0.0, 1.0, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(3, n))
    P[11:14] = (rgb - 0.5) / _SH_DC
    if K > 1:
        P[14:11 + 3 * K] = rng.normal(0.0, sh_rest_std, size=(3 * (K - 1), n))
    return _f32(P)


def with_near_splats(P: np.ndarray, n_near: int, seed: int = SEED_GAUSSIANS,
                     depth=(1.0, 1.6), scale=(0.08, 0.25), spread: float = 0.4) -> np.ndarray:
    """``P`` followed by ``n_near`` large splats close to an axis camera at
    distance 3 (camera-space depth U[depth], so world z = depth - 3), centred
    within +-spread of the optical axis, log-scales of U[scale] per axis (so
    anisotropic), random rotation, opacity logit U[1, 4]; the rest of each
    column as ``random_gaussians`` draws it.  Their support boxes span tens of
    tile rows at 8-pixel tiles in a 512-pixel view."""
    rng = _rng(seed + 1000)
    Q = random_gaussians(n_near, seed=seed + 1000, sh_degree=int(round(math.sqrt((P.shape[0] - 11) // 3))) - 1)
    Q = Q.astype(np.float64)
    Q[0] = rng.uniform(-spread, spread, size=n_near)
    Q[1] = rng.uniform(-spread, spread, size=n_near)
    Q[2] = rng.uniform(depth[0], depth[1], size=n_near) - 3.0
    Q[3:6] = np.log(rng.uniform(scale[0], scale[1], size=(3, n_near)))
    Q[10] = rng.uniform(1.0, 4.0, size=n_near)
    return _f32(np.concatenate([np.asarray(P, np.float64), Q], axis=1))


def scaled_logscale_mean(n: int) -> float:
    """Log-scale mean that keeps world-space overlap equal to the 1k-Gaussian set."""
    return -3.0 - math.log(n / 1000.0) / 3.0


# --------------------------------------------------------------------------------------
# Cameras (OpenCV axes: x right, y down, z forward; pixel (i, j) centre at (i+.5, j+.5))
# --------------------------------------------------------------------------------------

@dataclass
class Camera:
    R: np.ndarray          # (3, 3) float32, world -> camera rotation
    t: np.ndarray          # (3,)   float32, world -> camera translation
    campos: np.ndarray     # (3,)   float32, camera centre in world
    fx: float
    fy: float
    cx: float
    cy: float
    tanx: float            # tan of the half field of view along x
    tany: float
    width: int
    height: int
    znear: float = 0.2
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))

    def __post_init__(self):
        self.R = _f32(self.R).reshape(3, 3)
        self.t = _f32(self.t).reshape(3)
        self.campos = _f32(self.campos).reshape(3)
        self.bg = _f32(self.bg).reshape(3)
        for k in ("fx", "fy", "cx", "cy", "tanx", "tany", "znear"):
            setattr(self, k, float(np.float32(getattr(self, k))))
        self.width = int(self.width)
        self.height = int(self.height)

    @property
    def npix(self) -> int:
        return self.width * self.height


def _intrinsics(width: int, height: int, fov_x_deg: float):
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    f32 = float(np.float32(f))
    return dict(fx=f32, fy=f32, cx=width / 2.0, cy=height / 2.0,
                tanx=(width / 2.0) / f32, tany=(height / 2.0) / f32)


def axis_camera(width: int = 128, height: int = 128, distance: float = 3.0,
                fov_x_deg: float = 60.0, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera with identity rotation at (0, 0, -distance), looking at the origin."""
    return Camera(R=np.eye(3), t=[0.0, 0.0, distance], campos=[0.0, 0.0, -distance],
                  width=width, height=height, bg=bg, **_intrinsics(width, height, fov_x_deg))


def look_at_camera(center, target=(0.0, 0.0, 0.0), width: int = 512, height: int = 512,
                   fov_x_deg: float = 60.0, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Pinhole camera at ``center`` looking at ``target``; world up is -y
    (fallback +z when the view direction is nearly vertical)."""
    c = np.asarray(center, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    up = np.array([0.0, -1.0, 0.0])
    if abs(float(f @ up)) > 0.99:
        up = np.array([0.0, 0.0, 1.0])
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f])
    R32 = _f32(R)
    t = -(R32.astype(np.float64) @ c)
    return Camera(R=R32, t=t, campos=c, width=width, height=height, bg=bg,
                  **_intrinsics(width, height, fov_x_deg))


def sphere_directions(count: int, seed: int = SEED_POSES) -> np.ndarray:
    d = _rng(seed).normal(size=(count, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def sphere_cameras(resolutions, radius: float = 3.0, seed: int = SEED_POSES,
                   fov_x_deg: float = 60.0):
    dirs = sphere_directions(len(resolutions), seed)
    return [look_at_camera(radius * d, width=w, height=h, fov_x_deg=fov_x_deg)
            for d, (w, h) in zip(dirs, resolutions)]


def draw_resolutions(count: int, seed: int = SEED_RESOLUTIONS):
    idx = _rng(seed).integers(0, len(RESOLUTION_CHOICES), size=count)
    return [RESOLUTION_CHOICES[i] for i in idx]


def stereo_cameras(width: int = 2064, height: int = 2208, radius: float = 3.0,
                   baseline: float = 0.064, seed: int = SEED_POSES, fov_x_deg: float = 60.0):
    """Two eyes at +-baseline/2 along the head camera's x axis, parallel axes."""
    head = look_at_camera(radius * sphere_directions(1, seed)[0], width=width,
                          height=height, fov_x_deg=fov_x_deg)
    cams = []
    for s in (-0.5, 0.5):
        c = head.campos.astype(np.float64) + s * baseline * head.R[0].astype(np.float64)
        t = -(head.R.astype(np.float64) @ c)
        cams.append(Camera(R=head.R, t=t, campos=c, width=width, height=height,
                           **_intrinsics(width, height, fov_x_deg)))
    return cams


def view_stream(count: int, radius: float = 3.0, seed: int = SEED_VIEW_STREAM,
                step: float = 0.04, jitter: float = 0.15, width: int = 128, height: int = 128,
                fov_x_deg: float = 20.0):
    """Foveal views along a wandering head path, as offered to the refinement's
    view selection: camera centres on a random walk (isotropic steps of about
    ``step`` scene units) starting on the sphere of the given radius, each
    looking at a point drawn around the origin (standard deviation ``jitter``
    per axis), so consecutive directions differ by a few degrees; narrow field of
    view."""
    rng = _rng(seed)
    c = radius * sphere_directions(1, seed)[0]
    cams = []
    for _ in range(count):
        c = c + rng.normal(scale=step / math.sqrt(3.0), size=3)
        target = rng.normal(scale=jitter, size=3)
        cams.append(look_at_camera(c, target, width, height, fov_x_deg))
    return cams


def clip_matrices(cam: Camera, near: float = 0.1, far: float = 100.0):
    """Projection P and view V (float32 4x4, row-major) of a pinhole camera for
    column vectors: V = [R | t; 0 0 0 1]; P maps camera space (x right, y
    down, z forward) to clip space with NDC x = 2 px / W - 1, y = 2 py / H - 1
    (px, py the pixel coordinates, pixel i covering [i, i + 1)), NDC z = -1 at
    the near and +1 at the far plane, and clip w = camera z."""
    W, H = float(cam.width), float(cam.height)
    P = np.zeros((4, 4))
    P[0, 0], P[0, 2] = 2.0 * cam.fx / W, 2.0 * cam.cx / W - 1.0
    P[1, 1], P[1, 2] = 2.0 * cam.fy / H, 2.0 * cam.cy / H - 1.0
    P[2, 2], P[2, 3] = (far + near) / (far - near), -2.0 * far * near / (far - near)
    P[3, 2] = 1.0
    V = np.eye(4)
    V[:3, :3] = cam.R
    V[:3, 3] = cam.t
    return _f32(P), _f32(V)


def sphere_depth(cam: Camera, radius: float = 1.0, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """First-hit distance along each pixel-centre ray to a sphere (float32
    [H][W]; 0 where the ray misses): the depth a path tracer's first hits give
    for a round object, standing in for the paper's foveal depth images."""
    j, i = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    xc = (i + 0.5 - cam.cx) / cam.fx
    yc = (j + 0.5 - cam.cy) / cam.fy
    d_cam = np.stack([xc, yc, np.ones_like(xc)], -1)
    d = d_cam @ cam.R.astype(np.float64)          # camera -> world direction (R^T d)
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    o = cam.campos.astype(np.float64) - np.asarray(center, np.float64)
    b = d @ o
    disc = b * b - (o @ o - radius * radius)
    t = -b - np.sqrt(np.maximum(disc, 0.0))
    return _f32(np.where((disc > 0) & (t > 0), t, 0.0))


def gaze_points(cams, seed: int = SEED_GAZE) -> np.ndarray:
    rng = _rng(seed)
    g = [(rng.uniform(0.2 * c.width, 0.8 * c.width), rng.uniform(0.2 * c.height, 0.8 * c.height))
         for c in cams]
    return _f32(g)


# --------------------------------------------------------------------------------------
# CT-like phantom, voxel seeding, linear transfer function
# --------------------------------------------------------------------------------------

TF_LO = np.array([0.8, 0.3, 0.2])
TF_HI = np.array([1.0, 0.95, 0.9])
TF_THRESHOLD = 1200.0
TF_RANGE = 1800.0
EXTINCTION = 40.0     # per world unit at full transfer-function density


def voxel_centres(n: int) -> np.ndarray:
    return (np.arange(n) + 0.5) * (2.0 / n) - 1.0


def _haar_rotation(rng: np.random.Generator) -> np.ndarray:
    a = rng.normal(size=(3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def phantom(n: int = 128, seed: int = SEED_VOLUME, n_ellipsoids: int = 20,
            noise_sigma: float = 20.0) -> np.ndarray:
    """uint16 volume ``vol[ix, iy, iz]`` spanning [-1, 1]^3 (voxel centres at
    (idx + 1/2) * 2/n - 1): a sum of random rotated ellipsoids adding
    U[400, 1600] inside each, plus N(0, sigma^2) noise, clipped to [0, 3000]."""
    rng = _rng(seed)
    c = voxel_centres(n)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    pts = np.stack([X, Y, Z], axis=-1).reshape(-1, 3)
    vol = np.zeros(pts.shape[0], np.float64)
    for _ in range(n_ellipsoids):
        ctr = rng.uniform(-0.6, 0.6, size=3)
        axes = rng.uniform(0.1, 0.5, size=3)
        rot = _haar_rotation(rng)
        val = rng.uniform(400.0, 1600.0)
        local = (pts - ctr) @ rot          # coordinates in the ellipsoid frame
        inside = np.sum((local / axes) ** 2, axis=1) <= 1.0
        vol[inside] += val
    vol += rng.normal(0.0, noise_sigma, size=vol.shape)
    vol = np.clip(vol, 0.0, 3000.0)
    return np.rint(vol).astype(np.uint16).reshape(n, n, n)


def tf_density(v):
    return np.clip((np.asarray(v, np.float64) - TF_THRESHOLD) / TF_RANGE, 0.0, 1.0)


def tf_colour(t):
    t = np.asarray(t, np.float64)[..., None]
    return TF_LO * (1.0 - t) + TF_HI * t


def _splitmix64(state: int, k: np.ndarray) -> np.ndarray:
    """Outputs k (uint64 array, k >= 1) of SplitMix64 (Steele, Lea and Flood,
    OOPSLA 2014) from state ``state``: state + k * golden-ratio increment
    through the published finaliser (uint64 arithmetic wraps)."""
    z = np.uint64(state) + k.astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def cap_priority(idx: np.ndarray, seed: int, nvox: int) -> np.ndarray:
    """Priority of voxel ``idx`` for the seeding cap: SplitMix64 output idx + 1
    from state ``seed`` with its low b bits replaced by idx (b = bits of
    nvox - 1), so priorities are distinct; the cap smallest are kept."""
    b = np.uint64(max(1, int(nvox - 1).bit_length()))
    idx = np.asarray(idx, np.uint64)
    with np.errstate(over="ignore"):
        h = _splitmix64(seed, idx + np.uint64(1))
    return ((h >> b) << b) | idx


def seed_from_volume(vol: np.ndarray, threshold: float = TF_THRESHOLD, cap: int = 50_000,
                     seed: int = SEED_CAP_SUBSET, opacity: float = 0.1) -> np.ndarray:
    """One Gaussian per voxel above ``threshold`` (raster order), capped by a
    seeded uniform subset without replacement (the candidates of smallest
    ``cap_priority``, kept in raster order).  Mean at
    the voxel centre, isotropic scale of one voxel, identity rotation, the
    given initial opacity and the transfer-function colour as degree-0 SH."""
    n = vol.shape[0]
    flat = vol.reshape(-1)
    idx = np.nonzero(flat > threshold)[0]
    if idx.size > cap:
        # the cap candidates of smallest priority (a seeded uniform subset)
        pri = cap_priority(idx, seed, flat.size)
        idx = np.sort(idx[np.argsort(pri, kind="stable")[:cap]])
    ix, iy, iz = np.unravel_index(idx, vol.shape)
    c = voxel_centres(n)
    m = idx.size
    P = np.zeros((n_planes(0), m), np.float64)
    P[0], P[1], P[2] = c[ix], c[iy], c[iz]
    P[3:6] = math.log(2.0 / n)
    P[6] = 1.0
    P[10] = math.log(opacity / (1.0 - opacity))
    col = tf_colour(tf_density(flat[idx]))
    P[11:14] = ((col - 0.5) / _SH_DC).T
    return _f32(P)


# --------------------------------------------------------------------------------------
# Emission-absorption ray march (target images)
# --------------------------------------------------------------------------------------

def trilinear_sampler(vol: np.ndarray):
    """Sampler returning (density t in [0,1], rgb) at world points, trilinear in
    the raw values with zero outside the grid (scipy's C interpolator)."""
    from scipy.ndimage import map_coordinates
    n = vol.shape[0]
    v = vol.astype(np.float64)

    def sample(p):
        u = (p + 1.0) * (n / 2.0) - 0.5
        acc = map_coordinates(v, u.T, order=1, mode="grid-constant", cval=0.0, prefilter=False)
        t = tf_density(acc)
        return t, tf_colour(t)

    return sample


def trilinear_sampler_reference(vol: np.ndarray):
    """Explicit eight-corner form of ``trilinear_sampler`` (for checking it)."""
    n = vol.shape[0]
    v = vol.astype(np.float64)

    def sample(p):
        u = (p + 1.0) * (n / 2.0) - 0.5
        i0 = np.floor(u).astype(np.int64)
        f = u - i0
        acc = np.zeros(p.shape[0])
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    ix, iy, iz = i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz
                    w = ((f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1])
                         * (f[:, 2] if dz else 1 - f[:, 2]))
                    ok = (ix >= 0) & (ix < n) & (iy >= 0) & (iy < n) & (iz >= 0) & (iz < n)
                    val = np.zeros(p.shape[0])
                    val[ok] = v[ix[ok], iy[ok], iz[ok]]
                    acc += w * val
        t = tf_density(acc)
        return t, tf_colour(t)

    return sample


def raymarch(sampler, cam: Camera, step: float, extinction: float = EXTINCTION,
             t_stop: float = 1e-4, rows=None, chunk: int = 1 << 17) -> np.ndarray:
    """Front-to-back emission-absorption march through the box [-1, 1]^3.

    Segments of length ``step`` from the box entry point, the last one
    shortened to end at the exit point; each segment takes the sample at its
    midpoint, alpha = 1 - exp(-extinction * t * length).  Stops once the
    transmittance falls below ``t_stop``.  Returns float32 RGBA ``[4][H][W]``
    (or ``[4][len(rows)][W]`` for a row subset) with RGB = C + T * bg and
    A = 1 - T.
    """
    W, H = cam.width, cam.height
    rows = np.arange(H) if rows is None else np.asarray(rows)
    jj, ii = np.meshgrid(rows, np.arange(W), indexing="ij")
    dc = np.stack([(ii + 0.5 - cam.cx) / cam.fx, (jj + 0.5 - cam.cy) / cam.fy,
                   np.ones_like(ii, dtype=np.float64)], axis=-1).reshape(-1, 3)
    R = cam.R.astype(np.float64)
    d = dc @ R                                  # R^T d_cam for each row vector
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = cam.campos.astype(np.float64)
    npx = d.shape[0]
    out_c = np.zeros((npx, 3))
    out_T = np.ones(npx)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        ta = (-1.0 - o) * inv
        tb = (1.0 - o) * inv
    t0 = np.max(np.minimum(ta, tb), axis=1)
    t1 = np.min(np.maximum(ta, tb), axis=1)
    t0 = np.maximum(t0, 0.0)
    hit = np.nonzero(t1 > t0)[0]
    for s in range(0, hit.size, chunk):
        ids = hit[s:s + chunk]
        a, b = t0[ids], t1[ids]
        dd = d[ids]
        C = np.zeros((ids.size, 3))
        T = np.ones(ids.size)
        act = np.arange(ids.size)
        k = 0
        while act.size:
            seg0 = a[act] + k * step
            seg1 = np.minimum(seg0 + step, b[act])
            live = seg1 > seg0
            act, seg0, seg1 = act[live], seg0[live], seg1[live]
            if not act.size:
                break
            mid = 0.5 * (seg0 + seg1)
            p = o + dd[act] * mid[:, None]
            dens, col = sampler(p)
            alpha = 1.0 - np.exp(-extinction * dens * (seg1 - seg0))
            C[act] += col * (alpha * T[act])[:, None]
            T[act] *= 1.0 - alpha
            act = act[T[act] >= t_stop]
            k += 1
        out_c[ids] = C
        out_T[ids] = T
    rgb = out_c + out_T[:, None] * cam.bg.astype(np.float64)[None, :]
    img = np.concatenate([rgb, (1.0 - out_T)[:, None]], axis=1).T
    return _f32(img.reshape(4, rows.size, W))


_RM_SRC = __import__("os").path.join(__import__("os").path.dirname(__file__), "raymarch.c")
_RM_LIB = _RM_SRC[:-2] + ".so"
_rm = None


def _raymarch_lib():
    """ctypes handle of raymarch.c (built with gcc on first use)."""
    global _rm
    import ctypes as ct
    import os
    import subprocess
    if _rm is None:
        if not os.path.exists(_RM_LIB) or os.path.getmtime(_RM_LIB) < os.path.getmtime(_RM_SRC):
            tmp = _RM_LIB + f".tmp{os.getpid()}"
            subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _RM_SRC, "-lm"],
                           check=True)
            os.replace(tmp, _RM_LIB)
        L = ct.CDLL(_RM_LIB)
        dp = ct.POINTER(ct.c_double)
        L.syn_raymarch.argtypes = [ct.c_void_p, ct.c_int, dp, ct.POINTER(ct.c_int64), ct.c_int64,
                                   ct.c_double, ct.c_double, ct.c_double, dp, dp, ct.c_double,
                                   ct.c_double, ct.c_void_p]
        L.syn_raymarch.restype = None
        _rm = L
    return _rm


def raymarch_volume(vol: np.ndarray, cam: Camera, rows=None, t_stop: float = 1e-4) -> np.ndarray:
    """Target image of the phantom with half-voxel steps (C implementation of
    ``raymarch`` with ``trilinear_sampler``)."""
    import ctypes as ct
    L = _raymarch_lib()
    n = vol.shape[0]
    v = np.ascontiguousarray(vol, np.uint16)
    rows = np.arange(cam.height) if rows is None else np.asarray(rows)
    rows = np.ascontiguousarray(rows, np.int64)
    c = np.ascontiguousarray(np.concatenate([cam.R.reshape(-1), cam.campos,
                                             [cam.fx, cam.fy, cam.cx, cam.cy], cam.bg,
                                             [cam.width, cam.height]]).astype(np.float64))
    out = np.zeros((4, rows.size, cam.width), np.float32)
    lo, hi = np.ascontiguousarray(TF_LO, np.float64), np.ascontiguousarray(TF_HI, np.float64)
    dp = ct.POINTER(ct.c_double)
    L.syn_raymarch(v.ctypes.data_as(ct.c_void_p), n, c.ctypes.data_as(dp),
                   rows.ctypes.data_as(ct.POINTER(ct.c_int64)), rows.size, 1.0 / n, EXTINCTION,
                   t_stop, lo.ctypes.data_as(dp), hi.ctypes.data_as(dp), TF_THRESHOLD, TF_RANGE,
                   out.ctypes.data_as(ct.c_void_p))
    return out
