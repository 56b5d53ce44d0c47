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


_FOVEAL = {}


def _foveal():
    if not _FOVEAL:
        import bench
        wl = bench.build_workload("foveal")
        rng = np.random.default_rng(14)
        # seeded stand-in targets: only the sign of (image - target) enters the loss
        tgt = np.concatenate([rng.uniform(0.0, 1.0, size=3 * c.npix).astype(np.float32)
                              for c in wl.cams])
        _FOVEAL.update(wl=wl, tgt=tgt)
    return _FOVEAL["wl"], _FOVEAL["tgt"]


@pytest.mark.parametrize("t_mode", [0, 1])
def test_foveal_workload(ctx, t_mode):
    """The foveal refinement workload (500,000 Gaussians from the 256^3
    phantom, 16 views of 1920^2, loss masked to a fovea of radius 0.2 W per
    view) in the benchmark's launch configuration: one fused device-sized plan,
    fovea-culled, tile 16, LDS batch 64, the step captured and replayed, with
    either adjoint transmittance mode the autotuner picks between.  Sampled
    in-fovea pixels match the oracle's image; the step's masked L1 equals the
    oracle's loss of the same image; and the gradient of the step's own
    dL/dRGBA restricted to the sampled pixels matches the oracle's."""
    import paper_2601_22026_amd as gs
    wl, tgt = _foveal()
    P, cams, gaze = wl.P, wl.cams, wl.gaze
    log(f"[full] foveal: {P.shape[1]} Gaussians, 16 x 1920^2, culled, t_mode {t_mode}")
    dev = "cuda:0"
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        cfg = gs.FitConfig(lr=0.0, tile=16, lds_batch=64, t_mode=t_mode, fovea_cull=True)
        params = torch.from_numpy(np.ascontiguousarray(P)).to(dev)
        fs = gs.FitStep(ctx, params, cams, torch.from_numpy(tgt).to(dev),
                        torch.from_numpy(np.ascontiguousarray(gaze)).to(dev), cfg=cfg, fused=True)
        fs.capture()
        fs.replay()
        flags, m = fs.poll()
        assert flags == 0, flags
        torch.cuda.synchronize()
        rgba = fs.rgba.cpu().numpy()
        dl_step = fs.dl.cpu().numpy()
        loss = float(fs.loss.item())
    log(f"[full]   keys {m}, loss {loss:.6f}")
    rng = np.random.default_rng(15 + t_mode)
    imgs, tgts, dls = [], [], []
    G = np.zeros_like(P, dtype=np.float64)
    off = 0
    for v, cam in enumerate(cams):
        npx = cam.npix
        img = rgba[4 * off:4 * (off + npx)].reshape(4, npx)
        ys, xs = np.divmod(np.arange(npx), cam.width)
        inside = np.nonzero((xs + 0.5 - gaze[v][0]) ** 2 + (ys + 0.5 - gaze[v][1]) ** 2
                            <= (0.2 * cam.width) ** 2)[0]
        covered = inside[img[3, inside] > 0.05]
        pix = np.sort(rng.choice(covered if covered.size >= 24 else inside, 24, replace=False))
        ref = oracle.render(P, cam, pixels=pix)
        nbad, worst, nflag = image_close(img[:, pix], ref.rgba, ref.flags)
        log(f"[full]   view {v}: {pix.size} in-fovea px ({covered.size} covered), worst {worst:.2e}, "
            f"flagged {nflag}")
        if nbad:
            bad = np.nonzero((np.abs(img[:, pix] - ref.rgba) > 1e-4 * np.abs(ref.rgba) + 1e-6).any(axis=0)
                             & (ref.flags == 0))[0]
            for b in bad:
                log(f"[full]     pixel {pix[b]} (x {pix[b] % cam.width}, y {pix[b] // cam.width}): "
                    f"gpu {img[:, pix[b]]} oracle {ref.rgba[:, b]}")
        assert nbad == 0, (v, worst)
        keep = pix[ref.flags == 0]
        d = np.zeros((4, npx), np.float32)
        d[:, keep] = dl_step[4 * off:4 * (off + npx)].reshape(4, npx)[:, keep]
        dls.append(d)
        G += oracle.backward(P, cam, d[:, keep].astype(np.float64), pixels=keep)
        imgs.append(img.astype(np.float64))
        tgts.append(tgt[3 * off:3 * (off + npx)].astype(np.float64))
        off += npx
    L, _ = oracle.loss_l1(imgs, tgts, cams, gazes=gaze.astype(np.float64), radius_frac=0.2)
    log(f"[full]   loss {loss:.7f} vs oracle {L:.7f}")
    assert abs(loss - L) <= 1e-5 * L
    with torch.cuda.stream(stream):
        dl_dev = torch.from_numpy(np.concatenate([d.reshape(-1) for d in dls])).to(dev)
        g = torch.zeros_like(params)
        fs.plan.backward(params, params.shape[1], fs.cams_dev, dl_dev, g)
        torch.cuda.synchronize()
        g = g.cpu().numpy()
    rep = grads_close(g, G)
    log(f"[full]   gradient groups {rep}")
    assert all(nb == 0 for _, nb, _ in rep), rep
    fs.close()
