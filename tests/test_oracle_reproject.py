"""Pins of the oracle's depth-guided reprojection (Method, "Real-time Viewer",
Eqs. (2)-(4)): closed forms for an unmoved camera, for the disparity of a
fronto-parallel plane under a sideways camera move, and the nearest-wins rule
of the warp where a near layer slides over a far one."""
import numpy as np

import oracle
import synth


def _plane_depth(cam, z0):
    """First-hit distance of each pixel ray to the plane at camera depth z0."""
    j, i = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    xc = (i + 0.5 - cam.cx) / cam.fx
    yc = (j + 0.5 - cam.cy) / cam.fy
    return z0 * np.sqrt(1.0 + xc * xc + yc * yc)


def _moved(cam, b):
    """The same camera moved by b along its own x axis (rotation identity)."""
    c = cam.campos.astype(np.float64) + np.array([b, 0.0, 0.0])
    return synth.Camera(R=np.eye(3), t=-c, campos=c, fx=cam.fx, fy=cam.fy, cx=cam.cx, cy=cam.cy,
                        tanx=cam.tanx, tany=cam.tany, width=cam.width, height=cam.height)


def test_unmoved_camera_maps_every_pixel_to_itself():
    cam = synth.axis_camera(24, 20)
    P, V = synth.clip_matrices(cam)
    rng = np.random.default_rng(3)
    d = rng.uniform(1.0, 6.0, size=(20, 24))
    clip = oracle.reproject(d, P, V, cam.campos, P, V)
    ndc = clip[..., :2] / clip[..., 3:4]
    u = (np.arange(24) + 0.5) / 24
    v = (np.arange(20) + 0.5) / 20
    np.testing.assert_allclose(ndc[..., 0], np.broadcast_to(2 * u - 1, (20, 24)), atol=1e-9)
    np.testing.assert_allclose(ndc[..., 1], np.broadcast_to((2 * v - 1)[:, None], (20, 24)),
                               atol=1e-9)
    # clip w is the camera depth: the distance d times the cosine to the axis
    j, i = np.meshgrid(np.arange(20), np.arange(24), indexing="ij")
    xc, yc = (i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy
    np.testing.assert_allclose(clip[..., 3], d / np.sqrt(1 + xc * xc + yc * yc), rtol=1e-6)


def test_missing_depth_gives_no_point():
    cam = synth.axis_camera(8, 8)
    P, V = synth.clip_matrices(cam)
    d = np.full((8, 8), 2.0)
    d[0, 0], d[1, 1], d[2, 2] = 0.0, -1.0, np.inf
    clip = oracle.reproject(d, P, V, cam.campos, P, V)
    assert np.isnan(clip[0, 0]).all() and np.isnan(clip[1, 1]).all() and np.isnan(clip[2, 2]).all()
    assert np.isfinite(clip[3, 3]).all()


def test_sideways_move_gives_the_plane_disparity():
    cam = synth.axis_camera(40, 30)
    z0, b = 2.5, 0.04
    d = _plane_depth(cam, z0)
    new = _moved(cam, b)
    P, V = synth.clip_matrices(cam)
    P2, V2 = synth.clip_matrices(new)
    clip = oracle.reproject(d, P, V, cam.campos, P2, V2)
    px = (clip[..., 0] / clip[..., 3] + 1) * 0.5 * 40
    py = (clip[..., 1] / clip[..., 3] + 1) * 0.5 * 30
    j, i = np.meshgrid(np.arange(30), np.arange(40), indexing="ij")
    np.testing.assert_allclose(px, i + 0.5 - cam.fx * b / z0, atol=1e-6)
    np.testing.assert_allclose(py, j + 0.5, atol=1e-6)
    np.testing.assert_allclose(clip[..., 3], z0, rtol=1e-7)   # float32 matrices, far plane 100


def test_warp_of_an_unmoved_view_is_the_identity():
    cam = synth.axis_camera(16, 12)
    P, V = synth.clip_matrices(cam)
    rng = np.random.default_rng(5)
    rgba = rng.uniform(size=(4, 12, 16))
    d = _plane_depth(cam, 3.0)
    d[5, 7] = 0.0
    out, src, flags = oracle.reproject_warp(rgba, d, P, V, cam.campos, P, V, 16, 12)
    assert not flags.any()
    expect = np.arange(12 * 16).reshape(12, 16)
    expect[5, 7] = -1
    np.testing.assert_array_equal(src, expect)
    keep = expect >= 0
    np.testing.assert_array_equal(out[:, keep], rgba[:, keep])
    assert (out[:, 5, 7] == 0).all()


def test_warp_near_layer_slides_over_far_layer():
    """Left half at camera depth 2, right half at 4; the camera moves left so
    the near half shifts 4 px right and the far half 2 px: output columns 18
    and 19 receive both and keep the near pixels; columns 0-3 open up."""
    W, H = 32, 4
    cam = synth.axis_camera(W, H, fov_x_deg=90.0)
    b = -8.0 / cam.fx                                      # fx * |b| = 8 px at depth 1
    d = np.where(np.arange(W)[None, :] < 16, _plane_depth(cam, 2.0), _plane_depth(cam, 4.0))
    P, V = synth.clip_matrices(cam)
    P2, V2 = synth.clip_matrices(_moved(cam, b))
    rgba = np.arange(4 * H * W, dtype=np.float64).reshape(4, H, W)
    out, src, flags = oracle.reproject_warp(rgba, d, P, V, cam.campos, P2, V2, W, H)
    assert not flags.any()
    row = src[1] - 1 * W                                   # source columns of output row 1
    assert (src[1, :4] == -1).all()                        # disocclusion at the left edge
    np.testing.assert_array_equal(row[4:20], np.arange(0, 16))      # near: column i -> i + 4
    np.testing.assert_array_equal(row[20:32], np.arange(18, 30))    # far: column i -> i + 2
    np.testing.assert_array_equal(out[:, 1, 18], rgba[:, 1, 14])
