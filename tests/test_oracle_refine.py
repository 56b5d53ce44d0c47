"""Pins of the oracle's continual-refinement pieces (Method, "Periphery Model
Training"): the Eq. (1) view-selection rule, Gaussian visibility and the
visibility-masked Adam.  Every expected value here is derived by hand from the
geometry or from Adam's closed form, not by re-running the oracle's code."""
import math

import numpy as np

import oracle
import synth

F = lambda x: float(np.float32(x))  # noqa: E731  (the library takes float32 thresholds)


def _cam_at(x, yaw_deg=0.0, z=0.0):
    """Camera at (x, 0, z) looking along (sin yaw, 0, cos yaw)."""
    a = math.radians(yaw_deg)
    c = np.array([x, 0.0, z])
    return synth.look_at_camera(c, c + np.array([math.sin(a), 0.0, math.cos(a)]), 32, 32)


def test_view_pose_is_centre_and_forward_axis():
    cam = synth.look_at_camera([0.0, 0.0, -3.0], [0.0, 0.0, 0.0], 32, 32)
    c, d = oracle.view_pose(cam)
    np.testing.assert_allclose(c, [0.0, 0.0, -3.0])
    np.testing.assert_allclose(d, [0.0, 0.0, 1.0], atol=1e-7)
    cam = synth.look_at_camera([3.0, 0.0, 0.0], [0.0, 0.0, 0.0], 32, 32)
    np.testing.assert_allclose(oracle.view_pose(cam)[1], [-1.0, 0.0, 0.0], atol=1e-7)


def test_first_view_joins_an_empty_set_and_a_duplicate_does_not():
    a = _cam_at(0.0)
    assert oracle.select_views([], [a, _cam_at(0.0)]) == [True, False]


def test_views_along_a_line_keep_every_other_one():
    # centres 0.03 apart along x, same direction: 0 kept; 0.03 is 0.03 from it
    # (rejected); 0.06 is 0.06 from 0 (kept); 0.09 is 0.03 from 0.06; ...
    cands = [_cam_at(0.03 * k) for k in range(7)]
    assert oracle.select_views([], cands) == [True, False, True, False, True, False, True]


def test_distance_test_is_strict():
    # centres exactly delta_pos apart (the same float32 value) are not novel
    d = F(0.05)
    assert oracle.select_views([_cam_at(0.0)], [_cam_at(d)], delta_pos=d) == [False]
    assert oracle.select_views([_cam_at(0.0)], [_cam_at(d)], delta_pos=F(0.0499)) == [True]


def test_rotation_alone_is_novel_beyond_theta():
    kept = [_cam_at(0.0)]
    assert oracle.select_views(kept, [_cam_at(0.0, 4.0)]) == [False]
    assert oracle.select_views(kept, [_cam_at(0.0, 6.0)]) == [True]
    assert oracle.select_views(kept, [_cam_at(0.0, -6.0)]) == [True]
    # theta_view is a parameter: 10 degrees makes the 6 degree turn redundant
    assert oracle.select_views(kept, [_cam_at(0.0, 6.0)], theta_view_deg=10.0) == [False]


def test_either_condition_suffices_and_both_must_fail_to_reject():
    kept = [_cam_at(0.0)]
    assert oracle.select_views(kept, [_cam_at(0.04, 4.0)]) == [False]
    assert oracle.select_views(kept, [_cam_at(0.04, 6.0)]) == [True]
    assert oracle.select_views(kept, [_cam_at(0.06, 4.0)]) == [True]


def test_novelty_is_required_against_every_kept_view():
    kept = [_cam_at(0.0), _cam_at(0.2)]
    # 0.10 from both: novel; 0.17 is novel against the first view but only
    # 0.03 from the second
    assert oracle.select_views(kept, [_cam_at(0.17)]) == [False]
    assert oracle.select_views(kept, [_cam_at(0.10)]) == [True]
    # the accepted candidate joins the set before the next one is tested
    assert oracle.select_views(kept, [_cam_at(0.10), _cam_at(0.12)]) == [True, False]


def test_visibility_in_front_behind_and_outside():
    P = synth.random_gaussians(4, seed=5)
    P[0:3, 0] = [0.0, 0.0, 0.0]        # at the origin, in view
    P[0:3, 1] = [0.0, 0.0, -5.0]       # behind the camera
    P[0:3, 2] = [50.0, 0.0, 0.0]       # far outside the frustum
    P[0:3, 3] = [0.3, -0.2, 0.5]       # in view
    cam = synth.axis_camera(64, 64)
    assert oracle.visibility(P, [cam]).tolist() == [True, False, False, True]
    # a second view that sees the second Gaussian makes it visible
    back = synth.look_at_camera([0.0, 0.0, -8.0], [0.0, 0.0, -5.0], 64, 64)
    assert oracle.visibility(P, [cam, back]).tolist() == [True, True, False, True]


def _state(C, n, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(C, n)), rng.normal(size=(C, n)), np.zeros((C, n)), np.zeros((C, n)))


def test_masked_adam_first_step_closed_form():
    """t = 1 from zero moments: a visible element moves by -lr * sign(g) with
    m = (1 - b1) g and v = (1 - b2) g^2; hidden columns keep every value."""
    C, n = 5, 7
    p, g, m, v = _state(C, n, 1)
    p0 = p.copy()
    lr = np.array([1e-3, 2e-3, 3e-3, 4e-3, 5e-3])
    vis = np.array([1, 0, 1, 1, 0, 0, 1], bool)
    oracle.adam_masked(p, g, m, v, 1, vis, lr=lr, eps=0.0)
    for c in range(C):
        for i in range(n):
            if vis[i]:
                assert math.isclose(p[c, i], p0[c, i] - lr[c] * math.copysign(1.0, g[c, i]),
                                    rel_tol=0, abs_tol=1e-15)
                assert math.isclose(m[c, i], 0.1 * g[c, i], rel_tol=1e-15)
                assert math.isclose(v[c, i], 0.001 * g[c, i] ** 2, rel_tol=1e-12)
            else:
                assert p[c, i] == p0[c, i] and m[c, i] == 0.0 and v[c, i] == 0.0


def test_masked_adam_skipped_step_keeps_moments_and_global_step():
    """A Gaussian visible at t = 1 and 3 but hidden at t = 2 under a constant
    gradient: m3 = (1 - b1^2) g, v3 = (1 - b2^2) g^2, bias correction with t = 3."""
    b1, b2, lr, g0 = 0.9, 0.999, 1e-2, 0.5
    p = np.array([[1.0, 1.0]])
    g = np.array([[g0, g0]])
    m, v = np.zeros_like(p), np.zeros_like(p)
    oracle.adam_masked(p, g, m, v, 1, [True, True], lr=lr, eps=0.0)
    p1 = p[0, 0]
    oracle.adam_masked(p, g, m, v, 2, [False, True], lr=lr, eps=0.0)
    assert p[0, 0] == p1 and m[0, 0] == (1 - b1) * g0
    oracle.adam_masked(p, g, m, v, 3, [True, True], lr=lr, eps=0.0)
    m3, v3 = (1 - b1 ** 2) * g0, (1 - b2 ** 2) * g0 ** 2
    mh, vh = m3 / (1 - b1 ** 3), v3 / (1 - b2 ** 3)
    assert math.isclose(m[0, 0], m3, rel_tol=1e-14)
    assert math.isclose(v[0, 0], v3, rel_tol=1e-12)   # 1 - b2^2 cancels digits
    assert math.isclose(p[0, 0], p1 - lr * mh / math.sqrt(vh), rel_tol=1e-12)
    # the always-visible column took three full steps: under a constant gradient
    # every bias-corrected step is exactly -lr
    assert math.isclose(p[0, 1], 1.0 - 3 * lr, rel_tol=1e-14)


def test_masked_adam_all_visible_is_the_dense_update_and_none_visible_is_a_no_op():
    C, n = 4, 9
    p, g, m, v = _state(C, n, 2)
    p2, m2, v2 = p.copy(), m.copy(), v.copy()
    lr = np.array([1e-3, 1.5e-3, 1e-3, 2e-3])
    oracle.adam_masked(p, g, m, v, 1, np.ones(n, bool), lr=lr)
    oracle.adam(p2, g, m2, v2, 1, lr=np.repeat(lr[:, None], n, axis=1))
    np.testing.assert_array_equal(p, p2)
    np.testing.assert_array_equal(m, m2)
    q, mq, vq = p.copy(), m.copy(), v.copy()
    oracle.adam_masked(p, g, m, v, 2, np.zeros(n, bool), lr=lr)
    np.testing.assert_array_equal(p, q)
    np.testing.assert_array_equal(m, mq)
    np.testing.assert_array_equal(v, vq)
