"""Host logic of the continual refinement: the library's Eq. (1) view selection
(gsf_view_select, host code, no GPU needed) against the oracle, its argument
checks, and the per-plane learning rates of the initial fit."""
import math

import numpy as np
import pytest

import oracle
import synth

pytest.importorskip("torch")
gs = pytest.importorskip("paper_2601_22026_amd")

F = lambda x: float(np.float32(x))  # noqa: E731


def _cam_at(x, yaw_deg=0.0):
    a = math.radians(yaw_deg)
    c = np.array([x, 0.0, 0.0])
    return synth.look_at_camera(c, c + np.array([math.sin(a), 0.0, math.cos(a)]), 32, 32)


def test_library_selection_on_a_line_and_rotations():
    assert gs.select_views([], [_cam_at(0.03 * k) for k in range(7)]) == \
        [True, False, True, False, True, False, True]
    kept = [_cam_at(0.0)]
    assert gs.select_views(kept, [_cam_at(0.0, 4.0), _cam_at(0.0, 6.0)]) == [False, True]
    assert gs.select_views(kept, [_cam_at(F(0.05))], delta_pos=F(0.05)) == [False]
    assert gs.select_views(kept, []) == []


@pytest.mark.parametrize("delta,theta", [(0.05, 5.0), (0.02, 2.0), (0.1, 10.0), (0.0, 0.0)])
def test_library_selection_matches_oracle_on_a_head_path(delta, theta):
    stream = synth.view_stream(80)
    init = synth.sphere_cameras([(64, 64)] * 3)
    got = gs.select_views(init, stream, delta, theta)
    ref = oracle.select_views(init, stream, F(delta), F(theta))
    assert got == ref
    if (delta, theta) == (0.05, 5.0):     # the stream mixes novel and redundant views
        assert 10 < sum(got) < 70, sum(got)


def test_library_selection_rejects_bad_arguments():
    cam = _cam_at(0.0)
    for d, t in [(-0.1, 5.0), (0.05, -1.0), (0.05, 181.0), (float("nan"), 5.0)]:
        with pytest.raises(gs.GsfError):
            gs.select_views([cam], [cam], d, t)
    flat = synth.Camera(**{**cam.__dict__, "R": np.zeros((3, 3), np.float32)})
    with pytest.raises(gs.GsfError):
        gs.select_views([cam], [flat])
    with pytest.raises(gs.GsfError):
        gs.select_views([flat], [cam])


def test_plane_learning_rates_raise_scale_opacity_and_colour():
    lr = gs.plane_learning_rates(0, 1e-3, 1.5)
    assert len(lr) == 14
    for c in range(14):
        boosted = c in (3, 4, 5) or c >= 10
        assert lr[c] == pytest.approx(1.5e-3 if boosted else 1e-3, rel=1e-12), c
    lr3 = gs.plane_learning_rates(3, 2e-3, 1.5)
    assert len(lr3) == 59 and lr3[0] == 2e-3 and lr3[6] == 2e-3 and lr3[58] == pytest.approx(3e-3)
    assert gs.plane_learning_rates(0, list(range(14)), 1.0) == [float(x) for x in range(14)]
    with pytest.raises(ValueError):
        gs.plane_learning_rates(0, [1e-3] * 13)
