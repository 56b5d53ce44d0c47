"""The benchmark workloads at their full sizes, in the launch configuration the
benchmark times (one fused device-sized plan over all views, tile 16, LDS
batch 64), against the FP64 oracle on sampled pixels: the image at those
pixels and the gradient of a loss that lives only on them."""
import numpy as np
import pytest

import oracle
from paper_2601_22026_amd import _abi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from gpu_common import GpuScene, grads_close, image_close, log  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_22026_amd as gs
    return gs.Context(0)


def _key_count(ctx, P, cams, tile):
    probe = GpuScene(ctx, P, cams, tile=tile, host_sized=True)
    probe.forward()
    _, m = probe.plan.poll()
    probe.plan.close()
    return m


def _sampled_parity(ctx, P, cams, t_mode, per_view, seed, tile=16, batch=64):
    m = _key_count(ctx, P, cams, tile)
    sc = GpuScene(ctx, P, cams, tile=tile, batch=batch, host_sized=False, t_mode=t_mode,
                  key_capacity=int(m * 1.2) + 4096)
    imgs = sc.forward()
    flags, m2 = sc.plan.poll()
    assert flags == 0 and m2 == m
    rng = np.random.default_rng(seed)
    dls, G = [], np.zeros_like(P, dtype=np.float64)
    for v, (cam, img) in enumerate(zip(cams, imgs)):
        covered = np.nonzero(img[3] > 0.05)[0]
        k = min(3 * per_view // 4, covered.size)
        pix = np.sort(np.unique(np.concatenate([rng.choice(covered, k, replace=False),
                                                rng.choice(cam.npix, per_view - k, replace=False)])))
        ref = oracle.render(P, cam, pixels=pix)
        nbad, worst, nflag = image_close(img[:, pix], ref.rgba, ref.flags)
        log(f"[full]   view {v} {cam.width}x{cam.height}: {pix.size} px, worst {worst:.2e}, flagged {nflag}")
        assert nbad == 0, (v, worst)
        keep = pix[ref.flags == 0]
        d_sub = rng.normal(size=(4, keep.size))
        d = np.zeros((4, cam.npix))
        d[:, keep] = d_sub
        dls.append(d)
        G += oracle.backward(P, cam, d_sub.astype(np.float32).astype(np.float64), pixels=keep)
    g = sc.backward(dls)
    rep = grads_close(g, G)
    log(f"[full]   gradient groups {rep}")
    assert all(nb == 0 for _, nb, _ in rep), rep
    return sc


@pytest.mark.parametrize("t_mode", [1, 2])
def test_phantom_workload(ctx, t_mode):
    import bench
    wl = bench.build_workload("phantom")
    log(f"[full] phantom: {wl.P.shape[1]} Gaussians, 1024x1024, t_mode {t_mode}")
    sc = _sampled_parity(ctx, wl.P, wl.cams, t_mode, per_view=512, seed=11)
    _check_order(sc)


def test_batched_uneven_workload(ctx):
    import bench
    wl = bench.build_workload("batched")
    log(f"[full] batched: {wl.P.shape[1]} SH3 Gaussians, views "
        f"{[(c.width, c.height) for c in wl.cams]}")
    sc = _sampled_parity(ctx, wl.P, wl.cams, 1, per_view=64, seed=12)
    _check_order(sc)


def _check_order(sc):
    """The compositing order is a permutation of the tiles, heavier key-count
    classes (floor(log2(count)), empty last) before lighter ones."""
    T = sc.plan.total_tiles
    ranges = sc.debug(_abi.GSF_DBG_RANGES, np.uint32, 2 * T).reshape(-1, 2).astype(np.int64)
    assert (np.diff(ranges[:, 0]) >= 0).all()
    order = sc.debug(_abi.GSF_DBG_ORDER, np.uint32, T).astype(np.int64)
    np.testing.assert_array_equal(np.sort(order), np.arange(T))
    n = ranges[:, 1] - ranges[:, 0]
    cls = np.where(n > 0, np.floor(np.log2(np.maximum(n, 1))).astype(np.int64) + 1, 0)
    assert (np.diff(cls[order]) <= 0).all()


def test_stereo_workload(ctx):
    import bench
    wl = bench.build_workload("stereo")
    log(f"[full] stereo: {wl.P.shape[1]} SH3 Gaussians, two eyes 2064x2208")
    sc = _sampled_parity(ctx, wl.P, wl.cams, 1, per_view=96, seed=13)
    _check_order(sc)
