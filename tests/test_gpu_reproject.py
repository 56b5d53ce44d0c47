"""GPU tests of the depth-guided reprojection (Method, "Real-time Viewer",
Eqs. (2)-(4)) through the C ABI, against the FP64 oracle: clip coordinates
per pixel, and the nearest-wins forward warp of the foveal image (bit-exact
winners wherever FP32 rounding cannot change them)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_common import DEV, log  # noqa: E402


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_22026_amd
    return paper_2601_22026_amd


@pytest.fixture(scope="module")
def ctx(gs):
    return gs.Context(0)


def _head_motion(w, h, fov=40.0):
    """A foveal view of a unit sphere and the pose a few tens of ms later:
    3-4 cm of head translation and about a degree of rotation."""
    old = synth.look_at_camera([0.2, -0.1, -2.5], [0.0, 0.0, 0.0], w, h, fov)
    new = synth.look_at_camera([0.23, -0.09, -2.52], [0.03, 0.02, 0.0], w, h, fov)
    depth = synth.sphere_depth(old, radius=1.0)
    depth[::7, ::11] = 0.0          # a sparse grid of pixels without a first hit
    return old, new, depth


def _mats(old, new):
    P0, V0 = synth.clip_matrices(old)
    P1, V1 = synth.clip_matrices(new)
    return P0, V0, old.campos, P1, V1


@pytest.mark.parametrize("w,h", [(200, 150), (257, 96), (512, 512)])
def test_clip_coordinates_match_oracle(gs, ctx, w, h):
    old, new, depth = _head_motion(w, h)
    mats = _mats(old, new)
    clip = gs.reproject(ctx, torch.from_numpy(depth).to(DEV), *mats).cpu().numpy()
    ref = oracle.reproject(depth, *mats)
    miss = ~(depth > 0)
    assert miss.any() and not miss.all()
    assert np.isnan(clip[:, miss]).all()
    got = np.moveaxis(clip, 0, -1)[~miss]
    want = ref[~miss]
    scale = np.abs(want).max(axis=1, keepdims=True) + 1.0
    err = np.abs(got - want) / scale
    log(f"[reproject] {w}x{h}: max scaled clip error {err.max():.2e}")
    assert err.max() <= 5e-6      # ~20 float32 operations on values of the scale of |clip|


@pytest.mark.parametrize("w,h,ow,oh", [(200, 150, 200, 150), (160, 120, 96, 80), (512, 512, 512, 512)])
def test_warp_matches_oracle(gs, ctx, w, h, ow, oh):
    old, new, depth = _head_motion(w, h)
    mats = _mats(old, new)
    rng = np.random.default_rng(7)
    rgba = rng.uniform(size=(4, h, w)).astype(np.float32)
    out, src = gs.reproject_warp(ctx, torch.from_numpy(rgba).to(DEV),
                                 torch.from_numpy(depth).to(DEV), *mats, ow, oh)
    out, src = out.cpu().numpy(), src.cpu().numpy()
    ref_out, ref_src, flags = oracle.reproject_warp(rgba, depth, *mats, ow, oh)
    sure = ~flags
    mism = (src != ref_src) & sure
    log(f"[warp] {w}x{h} -> {ow}x{oh}: landed {int((ref_src >= 0).sum())}, "
        f"flagged {int(flags.sum())}, mismatched {int(mism.sum())}")
    assert not mism.any()
    assert (src >= 0).sum() > 0.3 * ow * oh
    # every output pixel carries its winner's values bit for bit
    flat = rgba.reshape(4, -1)
    hit = src >= 0
    np.testing.assert_array_equal(out[:, hit], flat[:, src[hit]])
    assert (out[:, ~hit] == 0).all()
    # flagged pixels: the GPU winner is still a point that lands on or beside them
    clip = oracle.reproject(depth, *mats).reshape(-1, 4)
    for t in np.argwhere(flags & (src >= 0))[:200]:
        s = src[t[0], t[1]]
        x = (clip[s, 0] / clip[s, 3] + 1) * 0.5 * ow
        y = (clip[s, 1] / clip[s, 3] + 1) * 0.5 * oh
        assert abs(np.floor(x) - t[1]) <= 1 and abs(np.floor(y) - t[0]) <= 1


def test_unmoved_warp_is_the_identity(gs, ctx):
    old, _, depth = _head_motion(96, 64)
    mats = _mats(old, old)
    rgba = np.random.default_rng(9).uniform(size=(4, 64, 96)).astype(np.float32)
    out, src = gs.reproject_warp(ctx, torch.from_numpy(rgba).to(DEV),
                                 torch.from_numpy(depth).to(DEV), *mats, 96, 64)
    src = src.cpu().numpy()
    expect = np.where(depth > 0, np.arange(96 * 64).reshape(64, 96), -1)
    assert (expect >= 0).any() and (expect < 0).any()
    np.testing.assert_array_equal(src, expect)


def test_reproject_rejects_bad_arguments(gs, ctx):
    old, new, depth = _head_motion(16, 16)
    P0, V0, c, P1, V1 = _mats(old, new)
    d = torch.from_numpy(depth).to(DEV)
    with pytest.raises(gs.GsfError):
        gs.reproject(ctx, d, np.zeros((4, 4)), V0, c, P1, V1)     # singular P_old V_old
    bad = P1.copy()
    bad[0, 0] = np.inf
    with pytest.raises(gs.GsfError):
        gs.reproject(ctx, d, P0, V0, c, bad, V1)
    with pytest.raises(gs.GsfError):
        gs.reproject_warp(ctx, torch.zeros((4, 16, 16), device=DEV), d, P0, V0, c, P1, V1, 0, 16)
