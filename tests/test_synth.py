"""Checks of the seeded input generators (no rasterizer arithmetic involved)."""
import math

import numpy as np

import synth


def test_random_gaussians_shapes_and_determinism():
    a = synth.random_gaussians(500, seed=0, sh_degree=3)
    b = synth.random_gaussians(500, seed=0, sh_degree=3)
    assert a.dtype == np.float32 and a.shape == (59, 500)
    np.testing.assert_array_equal(a, b)
    q = a[6:10].astype(np.float64)
    np.testing.assert_allclose(np.linalg.norm(q, axis=0), 1.0, atol=1e-6)
    assert np.abs(a[0:3]).max() <= 1.0
    rgb = a[11:14] * (0.5 / math.sqrt(math.pi)) + 0.5
    assert rgb.min() >= -1e-6 and rgb.max() <= 1 + 1e-6


def test_look_at_camera_axes():
    cam = synth.look_at_camera([0.0, 0.0, -3.0], width=64, height=32)
    np.testing.assert_allclose(cam.R, np.eye(3), atol=1e-7)
    np.testing.assert_allclose(cam.t, [0, 0, 3], atol=1e-6)
    assert cam.fx == cam.fy and abs(cam.tanx - math.tan(math.radians(30))) < 1e-6
    c2 = synth.look_at_camera([1.0, 2.0, 2.0])
    R = c2.R.astype(np.float64)
    np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-6)
    # the target (origin) projects to the principal point
    t = R @ np.zeros(3) + c2.t
    assert abs(t[0] / t[2]) < 1e-6 and abs(t[1] / t[2]) < 1e-6 and t[2] > 0


def test_stereo_baseline():
    L, R = synth.stereo_cameras()
    np.testing.assert_allclose(np.linalg.norm(L.campos.astype(np.float64) - R.campos), 0.064, rtol=1e-5)
    np.testing.assert_array_equal(L.R, R.R)


def test_phantom_and_seeding():
    vol = synth.phantom(32, seed=3)
    assert vol.dtype == np.uint16 and vol.shape == (32, 32, 32) and vol.max() <= 3000
    P = synth.seed_from_volume(vol, cap=200, seed=4)
    assert P.shape == (14, min(200, int((vol > 1200).sum())))
    np.testing.assert_allclose(np.exp(P[3:6].astype(np.float64)), 2.0 / 32, rtol=1e-6)
    assert np.all(np.abs(P[0:3]) < 1)


def test_cap_subset_is_the_smallest_splitmix_priorities():
    """The seeding cap keeps the candidates of smallest priority: SplitMix64
    outputs (first output from state 0 as published: 0xE220A8397B1DCDAF) with
    the low bits replaced by the voxel index - distinct, so the kept set is
    exactly determined - in raster order."""
    pri = synth.cap_priority(np.array([0]), 0, 2)
    assert int(pri[0]) == 0xE220A8397B1DCDAF & ~1
    vol = synth.phantom(24, seed=3)
    flat = vol.reshape(-1)
    cand = np.nonzero(flat > synth.TF_THRESHOLD)[0]
    cap = cand.size // 3
    P = synth.seed_from_volume(vol, cap=cap, seed=9)
    pr = synth.cap_priority(cand, 9, flat.size)
    assert np.unique(pr).size == pr.size
    keep = np.sort(cand[np.argsort(pr)[:cap]])
    c = synth.voxel_centres(24)
    ix, iy, iz = np.unravel_index(keep, vol.shape)
    np.testing.assert_array_equal(P[0], c[ix].astype(np.float32))
    np.testing.assert_array_equal(P[1], c[iy].astype(np.float32))
    np.testing.assert_array_equal(P[2], c[iz].astype(np.float32))
    # a cap above the candidate count keeps them all
    assert synth.seed_from_volume(vol, cap=cand.size + 5, seed=9).shape[1] == cand.size


def test_raymarch_constant_slab_closed_form():
    """Constant density in the box: A = 1 - exp(-sigma * L) with L the chord length
    (the midpoint rule is exact for a piecewise-constant medium)."""
    cam = synth.look_at_camera([0.3, -0.2, -3.0], width=24, height=20)
    dens = 0.37

    def sampler(p):
        t = np.full(p.shape[0], dens)
        return t, np.tile([0.2, 0.5, 0.7], (p.shape[0], 1))

    img = synth.raymarch(sampler, cam, step=0.013, extinction=4.0, t_stop=0.0)
    # chord length through [-1, 1]^3 per pixel ray
    jj, ii = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    dc = np.stack([(ii + 0.5 - cam.cx) / cam.fx, (jj + 0.5 - cam.cy) / cam.fy, np.ones_like(ii, float)], -1)
    d = dc.reshape(-1, 3) @ cam.R.astype(np.float64)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = cam.campos.astype(np.float64)
    with np.errstate(divide="ignore"):
        ta, tb = (-1 - o) / d, (1 - o) / d
    L = np.clip(np.min(np.maximum(ta, tb), 1) - np.max(np.minimum(ta, tb), 1), 0, None)
    np.testing.assert_allclose(img[3].reshape(-1), 1 - np.exp(-4.0 * dens * L), atol=1e-12)
    assert L.max() > 1.5


def test_trilinear_sampler_matches_eight_corner_form():
    vol = synth.phantom(16, seed=3)
    p = np.random.default_rng(0).uniform(-1.1, 1.1, size=(2000, 3))
    a, ca = synth.trilinear_sampler(vol)(p)
    b, cb = synth.trilinear_sampler_reference(vol)(p)
    np.testing.assert_allclose(a, b, atol=1e-12)
    np.testing.assert_allclose(ca, cb, atol=1e-12)


def test_c_raymarch_matches_numpy_definition():
    vol = synth.phantom(24, seed=3)
    cam = synth.look_at_camera([0.4, -2.5, 1.6], width=40, height=30, bg=(0.1, 0.0, 0.2))
    ref = synth.raymarch(synth.trilinear_sampler_reference(vol), cam, step=1.0 / 24)
    got = synth.raymarch_volume(vol, cam)
    assert ref[3].max() > 0.3
    np.testing.assert_allclose(got, ref, atol=2e-6)
    rows = np.array([3, 17, 29])
    np.testing.assert_array_equal(synth.raymarch_volume(vol, cam, rows=rows), got[:, rows])
