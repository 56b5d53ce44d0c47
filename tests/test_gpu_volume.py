"""The steps that read the CT volume on the device: seeding Gaussians from it
(bit-exact against the input generator's definition) and the FP32
emission-absorption ray march (against the FP64 C definition)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import DEV, log  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_22026_amd as gs
    return gs.Context(0)


def _vol_dev(vol):
    return torch.from_numpy(np.ascontiguousarray(vol).view(np.int16)).to(DEV)


@pytest.mark.parametrize("n,cap_frac", [(64, 1 / 3), (64, 2.0), (96, 0.5)])
def test_seed_volume_matches_generator(ctx, n, cap_frac):
    import paper_2601_22026_amd as gs
    vol = synth.phantom(n, seed=3)
    cand = int((vol > synth.TF_THRESHOLD).sum())
    cap = max(1, int(cand * cap_frac))
    ref = synth.seed_from_volume(vol, cap=cap, seed=4)
    got = gs.seed_volume(ctx, _vol_dev(vol), cap=cap, seed=4).cpu().numpy()
    log(f"[seed] n {n}: {cand} candidates, cap {cap}, kept {got.shape[1]}")
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_raymarch_matches_c_definition(ctx):
    """FP32 on the device against the FP64 C march.  Per-sample errors are a
    few float32 ulps and accumulate over at most ~2n samples; the stop at
    T < 1e-4 may land one sample apart, changing a pixel by < 1e-4 of its
    colour.  Bound: 3e-4 absolute per channel."""
    import paper_2601_22026_amd as gs
    vol = synth.phantom(64, seed=3)
    cams = [synth.look_at_camera([0.5, -0.8, -2.8], width=96, height=80, bg=(0.2, 0.1, 0.3)),
            synth.look_at_camera(3.0 * synth.sphere_directions(1, seed=2)[0], width=72, height=64)]
    out = gs.raymarch(ctx, _vol_dev(vol), cams).cpu().numpy()
    off = 0
    for c in cams:
        got = out[4 * off:4 * (off + c.npix)].reshape(4, c.height, c.width)
        ref = synth.raymarch_volume(vol, c)
        err = np.abs(got.astype(np.float64) - ref)
        log(f"[march] {c.width}x{c.height}: worst {err.max():.2e}, mean alpha {ref[3].mean():.3f}")
        assert ref[3].max() > 0.5
        assert err.max() <= 3e-4
        off += c.npix
