"""Pins of the oracle's first-hit point cloud (Method, "Volumetric Path
Tracing"): the hit position at a sharp slab in closed form, the hit colour in a
uniform medium, misses, monotonicity in the hit threshold, and the cap rule."""
import math

import numpy as np

import oracle
import synth

THR, RANGE = 1200.0, 1800.0
LO, HI = synth.TF_LO, synth.TF_HI


def _slab(n=32, v0=65535):
    """Voxels with x index >= n/2 at v0, the rest empty."""
    vol = np.zeros((n, n, n), np.uint16)
    vol[n // 2:] = v0
    return vol


def test_slab_hit_position_closed_form():
    n, step = 32, 0.01
    vol = _slab(n, 20000)
    cam = synth.look_at_camera([-3.0, 0.0, 0.0], [0.0, 0.0, 0.0], 9, 9, 10.0)
    h = oracle.first_hits(vol, [cam], step, 40.0, THR, RANGE, LO, HI, hit_alpha=1e-12)
    centre = 4 * 9 + 4                      # pixel (4, 4): the ray along +x through the origin
    assert h["hit"][centre]
    # along the ray the value ramps from 0 at the last empty voxel centre (x = -1/n)
    # to 20000 at the first full one (x = +1/n); density > 0 once v > THR
    x_th = -1.0 / n + (THR / 20000.0) * (2.0 / n)
    k = math.ceil((x_th + 1.0) / step - 0.5)
    if -1.0 + (k + 0.5) * step <= x_th:
        k += 1
    np.testing.assert_allclose(h["pos"][centre], [-1.0 + (k + 0.5) * step, 0.0, 0.0], atol=1e-12)
    # every hit lies on the slab's ramp, just past the same plane
    assert (np.abs(h["pos"][h["hit"], 0] - x_th) < step).all()


def test_uniform_medium_colour_is_the_transfer_function_colour():
    n, step = 64, 0.004
    t0 = 0.5
    vol = np.full((n, n, n), int(THR + t0 * RANGE), np.uint16)
    cams = synth.sphere_cameras([(12, 10)] * 3)
    h = oracle.first_hits(vol, cams, step, 40.0, THR, RANGE, LO, HI, hit_alpha=0.5,
                          color_steps=8)
    assert h["hit"].sum() > 100
    # the hit lies more than a voxel inside, so its segments all sample t = 0.5
    expect = LO * (1.0 - t0) + HI * t0
    inside = np.abs(h["pos"]).max(axis=1) < 1.0 - 2.0 * (2.0 / n) - 8 * step
    assert inside.sum() > 50
    np.testing.assert_allclose(h["col"][h["hit"] & inside], np.broadcast_to(expect, (int((h["hit"] & inside).sum()), 3)),
                               rtol=1e-12)
    # and the optical depth ln 2 is reached within one segment of the uniform medium
    # past the first segment of the ramp
    assert (h["margin"][h["hit"]] < 1.0).all()


def test_misses_and_empty_volume():
    vol = _slab(16)
    away = synth.look_at_camera([-3.0, 0.0, 0.0], [-6.0, 0.0, 0.0], 6, 6, 20.0)
    h = oracle.first_hits(vol, [away], 0.01, 40.0, THR, RANGE, LO, HI)
    assert not h["hit"].any() and np.isinf(h["margin"]).all()      # no ray meets the box
    empty = np.zeros((16, 16, 16), np.uint16)
    cam = synth.look_at_camera([-3.0, 0.0, 0.0], [0.0, 0.0, 0.0], 6, 6, 20.0)
    h = oracle.first_hits(empty, [cam], 0.01, 40.0, THR, RANGE, LO, HI, hit_alpha=0.3)
    assert not h["hit"].any()
    np.testing.assert_allclose(h["margin"], 0.3)                    # T stays 1 on every ray


def test_a_higher_threshold_hits_farther_along_the_ray():
    vol = synth.phantom(48, seed=synth.SEED_VOLUME)
    cams = synth.sphere_cameras([(16, 16)] * 2)
    a = oracle.first_hits(vol, cams, 0.01, 40.0, THR, RANGE, LO, HI, hit_alpha=0.2)
    b = oracle.first_hits(vol, cams, 0.01, 40.0, THR, RANGE, LO, HI, hit_alpha=0.6)
    assert b["hit"].sum() <= a["hit"].sum() and (a["hit"] | ~b["hit"]).all()
    both = a["hit"] & b["hit"]
    c = np.concatenate([[np.asarray(cam.campos, np.float64)] * cam.width * cam.height for cam in cams])
    da = np.linalg.norm(a["pos"][both] - c[both], axis=1)
    db = np.linalg.norm(b["pos"][both] - c[both], axis=1)
    assert (db >= da - 1e-12).all() and (db > da).any()


def test_cap_keeps_the_smallest_priorities_in_ray_order():
    vol = synth.phantom(48, seed=synth.SEED_VOLUME)
    cams = synth.sphere_cameras([(20, 20)] * 3)
    args = (vol, cams)
    kw = dict(step=0.01, extinction=40.0, threshold=THR, range_=RANGE, lo=LO, hi=HI)
    P_all, ids_all, _ = oracle.seed_first_hits(*args, cap=10**9, seed=5, **kw)
    cap = ids_all.size // 3
    P, ids, _ = oracle.seed_first_hits(*args, cap=cap, seed=5, **kw)
    assert ids.size == cap and (np.diff(ids) > 0).all() and np.isin(ids, ids_all).all()
    R = sum(c.width * c.height for c in cams)
    kept = oracle.ray_priority(ids, 5, R)
    dropped = oracle.ray_priority(np.setdiff1d(ids_all, ids), 5, R)
    assert kept.max() < dropped.min()
    assert np.unique(oracle.ray_priority(ids_all, 5, R)).size == ids_all.size
    # the Gaussians sit at the kept rays' hits
    np.testing.assert_array_equal(P, P_all[:, np.searchsorted(ids_all, ids)])
