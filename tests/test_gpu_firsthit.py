"""GPU tests of the first-hit point cloud (Method, "Volumetric Path Tracing")
through the C ABI, against the FP64 oracle: which rays hit (bit-exact away from
the hit threshold), where and with which colour, and the capped selection."""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_common import DEV, log  # noqa: E402

KW = dict(step=0.01, extinction=40.0, threshold=synth.TF_THRESHOLD, range_=synth.TF_RANGE,
          lo=synth.TF_LO, hi=synth.TF_HI)
Y00 = 0.5 / math.sqrt(math.pi)


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_22026_amd
    return paper_2601_22026_amd


@pytest.fixture(scope="module")
def ctx(gs):
    return gs.Context(0)


def _run(gs, ctx, vol, cams, cap, seed, hit_alpha=0.5):
    v = torch.from_numpy(vol.astype(np.int16, copy=False).view(np.int16)).to(DEV)
    P, ids = gs.seed_first_hits(ctx, v, cams, cap, seed, hit_alpha=hit_alpha, **KW)
    return P.cpu().numpy(), ids.cpu().numpy()


@pytest.mark.parametrize("n,views,size,hit_alpha", [(48, 3, (40, 32), 0.5), (64, 4, (48, 40), 0.2),
                                                    (128, 8, (128, 128), 0.5)])
def test_hits_match_oracle(gs, ctx, n, views, size, hit_alpha):
    vol = synth.phantom(n, seed=synth.SEED_VOLUME)
    cams = synth.sphere_cameras([size] * views)
    P, ids = _run(gs, ctx, vol, cams, cap=10**7, seed=3, hit_alpha=hit_alpha)
    h = oracle.first_hits(vol, cams, hit_alpha=hit_alpha, **KW)
    flagged = h["margin"] < 1e-4
    ref_ids = np.nonzero(h["hit"])[0]
    sure_gpu = ids[~flagged[ids]]
    sure_ref = ref_ids[~flagged[ref_ids]]
    log(f"[firsthit] n={n} rays={h['hit'].size} hits gpu {ids.size} oracle {ref_ids.size} "
        f"flagged {int(flagged.sum())}")
    np.testing.assert_array_equal(sure_gpu, sure_ref)
    assert (np.diff(ids) > 0).all()
    assert ref_ids.size > 0.1 * h["hit"].size
    # positions and colours of the common rays
    common, gi, ri = np.intersect1d(ids, ref_ids, return_indices=True)
    pos_err = np.abs(P[0:3, gi].T - h["pos"][common]).max()
    col = P[11:14, gi].T * Y00 + 0.5
    col_err = (np.abs(col - h["col"][common]) / np.maximum(np.abs(h["col"][common]), 1e-3)).max()
    log(f"[firsthit] max position error {pos_err:.2e}, max relative colour error {col_err:.2e}")
    assert pos_err <= 5e-6        # float march: ~1e-7 per segment on unit coordinates
    assert col_err <= 2e-4        # eight float exp and blend steps, then a division
    np.testing.assert_allclose(P[3:6], math.log(2.0 / n), rtol=1e-6)
    assert (P[6] == 1).all() and (P[7:10] == 0).all()
    np.testing.assert_allclose(P[10], math.log(0.1 / 0.9), rtol=1e-6)


def test_cap_keeps_the_oracle_selection(gs, ctx):
    vol = synth.phantom(64, seed=synth.SEED_VOLUME)
    cams = synth.sphere_cameras([(48, 48)] * 4)
    _, all_ids = _run(gs, ctx, vol, cams, cap=10**7, seed=9)
    cap = all_ids.size // 3
    P, ids = _run(gs, ctx, vol, cams, cap=cap, seed=9)
    Pr, ref_ids, flagged = oracle.seed_first_hits(vol, cams, cap, 9, **KW)
    log(f"[firsthit] cap {cap}: gpu {ids.size}, oracle {ref_ids.size}, flagged {flagged.size}")
    assert ids.size == ref_ids.size == cap
    if flagged.size == 0:
        np.testing.assert_array_equal(ids, ref_ids)
    else:   # a flagged ray may enter or leave the candidates and shift the cut by one each
        assert np.setxor1d(ids, ref_ids).size <= 2 * flagged.size


def test_first_hits_reject_bad_arguments(gs, ctx):
    vol = torch.zeros((8, 8, 8), dtype=torch.int16, device=DEV)
    cams = synth.sphere_cameras([(8, 8)])
    for kw in [dict(hit_alpha=0.0), dict(hit_alpha=1.0), dict(step=0.0), dict(color_steps=0),
               dict(opacity=1.0)]:
        args = dict(step=0.01, hit_alpha=0.5, color_steps=8, opacity=0.1)
        args.update(kw)
        with pytest.raises(gs.GsfError):
            gs.seed_first_hits(ctx, vol, cams, 10, 1, **args)
    with pytest.raises(gs.GsfError):
        gs.seed_first_hits(ctx, vol, cams, 0, 1, step=0.01)
    # an empty volume gives no points
    P, ids = gs.seed_first_hits(ctx, vol, cams, 10, 1, step=0.01)
    assert P.shape == (14, 0) and ids.numel() == 0
