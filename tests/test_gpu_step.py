"""GPU tests of the whole step: Adam, graph replay, multi-step fit, autograd,
autotuning, failure paths and edge cases."""
import os

import numpy as np
import pytest

import oracle
import synth
from paper_2601_22026_amd import _abi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_common import DEV, GpuScene, grads_close, image_close, log  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_22026_amd
    return paper_2601_22026_amd


@pytest.fixture(scope="module")
def ctx(gs):
    return gs.Context(0)


def _cfg1_target():
    return np.load(os.path.join(GOLDEN, "cfg1_target_128.npy"))[:3]


def test_adam_matches_oracle_given_identical_inputs(gs, ctx):
    rng = np.random.default_rng(0)
    n = 1003                                   # not a multiple of 4: exercises the tail
    p = rng.normal(size=n).astype(np.float32)
    m = np.zeros(n, np.float32)
    v = np.zeros(n, np.float32)
    seg_off = [0, 300, 301, 1003]
    seg_lr = [1e-3, 2.5e-3, 1.5e-3]
    lr_el = np.repeat(seg_lr, np.diff(seg_off))
    tp, tm, tv = (torch.from_numpy(a.copy()).to(DEV) for a in (p, m, v))
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    pd, md, vd = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        # both sides start each step from the same float32 state
        pd, md, vd = (tp.cpu().numpy().astype(np.float64), tm.cpu().numpy().astype(np.float64),
                      tv.cpu().numpy().astype(np.float64))
        gs.adam(ctx, tp, torch.from_numpy(g).to(DEV), tm, tv, step, seg_off, seg_lr)
        torch.cuda.synchronize()
        # identical inputs: the kernel receives the hyper-parameters as float32
        f32 = lambda x: float(np.float32(x))  # noqa: E731
        oracle.adam(pd, g.astype(np.float64), md, vd, t,
                    lr=np.asarray([f32(x) for x in lr_el]), betas=(f32(0.9), f32(0.999)),
                    eps=f32(1e-15))
        np.testing.assert_allclose(tm.cpu().numpy(), md, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(tv.cpu().numpy(), vd, rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(tp.cpu().numpy(), pd, rtol=1e-6, atol=1e-7)
    assert int(step.item()) == 3


def test_graph_replay_equals_eager(gs, ctx):
    """Every replay of the captured step gives the eager image bits and
    gradients within tolerance (lr = 0 keeps the parameters fixed); eager work
    and synchronisations run between the replays."""
    P = synth.random_gaussians(1000, seed=0)
    cam = synth.axis_camera(128, 128)
    tgt = torch.from_numpy(_cfg1_target().reshape(-1).copy()).to(DEV)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        cfg = gs.FitConfig(lr=0.0)
        eager = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), [cam], tgt, cfg=cfg)
        eager.step()
        torch.cuda.synchronize()
        img0, g0, l0 = eager.rgba.cpu().numpy(), eager.grads.cpu().numpy(), eager.loss.item()
        cap = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), [cam], tgt, cfg=cfg)
        cap.capture()
        for k in range(4):
            cap.rgba.zero_()
            cap.grads.zero_()
            cap.replay()
            torch.cuda.synchronize()
            _ = (eager.params * 2).sum().item()           # unrelated eager work in between
            np.testing.assert_array_equal(cap.rgba.cpu().numpy().view(np.uint32), img0.view(np.uint32))
            assert cap.loss.item() == l0
            rep = grads_close(cap.grads.cpu().numpy(), g0.astype(np.float64))
            assert all(nb == 0 for _, nb, _ in rep), (k, rep)
        assert int(cap.step_dev.item()) == 4
        flags, m = cap.poll()
        assert flags == 0 and m > 0


def test_culled_step_replays_are_bitwise_identical(gs, ctx):
    """The fovea-culled multi-view step is deterministic: four replays of the
    captured step (lr = 0, the image buffer refilled between them) give the
    eager step's bits in every masked-in pixel, its loss, and gradients equal
    to each other bit for bit."""
    P = synth.random_gaussians(20000, seed=23, logscale_mean=synth.scaled_logscale_mean(20000))
    cams = [synth.look_at_camera([0.2, -0.3, -3.0], width=512, height=384),
            synth.look_at_camera([-2.0, 1.2, -2.0], width=384, height=448),
            synth.look_at_camera([2.4, 0.5, 1.6], width=448, height=448)]
    gaze = synth.gaze_points(cams, seed=10)
    gz = torch.from_numpy(np.ascontiguousarray(gaze)).to(DEV)
    rng = np.random.default_rng(9)
    tgt = torch.from_numpy(np.concatenate([rng.uniform(0, 1, size=3 * c.npix)
                                           for c in cams]).astype(np.float32)).to(DEV)
    masks = []
    for v, c in enumerate(cams):
        ys, xs = np.divmod(np.arange(c.npix), c.width)
        dx = (xs + np.float32(0.5) - gaze[v][0]).astype(np.float32)
        dy = (ys + np.float32(0.5) - gaze[v][1]).astype(np.float32)
        r = np.float32(0.2) * np.float32(c.width)
        masks.append(np.tile(dx * dx + dy * dy <= r * r, 4))
    inside = np.concatenate(masks)
    cfg = gs.FitConfig(lr=0.0, tile=16, lds_batch=64, t_mode=0, fovea_cull=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eager = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), cams, tgt, gz, cfg=cfg, fused=True)
        eager.step()
        torch.cuda.synchronize()
        img0, l0 = eager.rgba.cpu().numpy(), eager.loss.item()
        eager.close()
        cap = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), cams, tgt, gz, cfg=cfg, fused=True)
        cap.capture()
        g_first = None
        for k in range(4):
            cap.rgba.fill_(float(k + 3))
            cap.replay()
            torch.cuda.synchronize()
            img = cap.rgba.cpu().numpy()
            np.testing.assert_array_equal(img[inside].view(np.uint32), img0[inside].view(np.uint32))
            assert cap.loss.item() == l0
            g = cap.grads.cpu().numpy()
            if g_first is None:
                g_first = g
            np.testing.assert_array_equal(g.view(np.uint32), g_first.view(np.uint32))
        flags, m = cap.poll()
        assert flags == 0 and m > 0
        log(f"[cull] 4 replays bitwise equal, keys {m}, loss {l0:.7f}")
        cap.close()


def test_fit_loss_curve_matches_oracle(gs, ctx):
    """Ten fit steps of the 1,000-Gaussian single-view workload: the GPU loss
    curve follows the FP64 oracle's within 1e-3 relative."""
    P = synth.random_gaussians(1000, seed=0)
    cam = synth.axis_camera(128, 128)
    target = _cfg1_target()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        fs = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), [cam],
                        torch.from_numpy(target.reshape(-1).copy()).to(DEV),
                        cfg=gs.FitConfig(lr=1e-3))
        gpu_losses = []
        for _ in range(10):
            fs.step()
            gpu_losses.append(fs.loss.item())
    Pd = P.astype(np.float64)
    m, v = np.zeros_like(Pd), np.zeros_like(Pd)
    ref = [oracle.fit_step(Pd, m, v, t, [cam], [target.reshape(3, -1).astype(np.float64)])
           for t in range(1, 11)]
    log(f"[step] losses gpu {np.round(gpu_losses, 6)} oracle {np.round(ref, 6)}")
    np.testing.assert_allclose(gpu_losses, ref, rtol=1e-3)
    assert ref[-1] < ref[0]


def test_autograd_function_matches_direct_call_and_fd(gs, ctx):
    P = synth.random_gaussians(60, seed=4, logscale_mean=-2.2)
    cam = synth.look_at_camera([0.5, -0.3, -3.0], width=48, height=40, bg=(0.2, 0.2, 0.2))
    plan = gs.Plan(ctx, P.shape[1], [(cam.width, cam.height)], 0, 16, 64, host_sized=True)
    cams = gs.cameras_to_device([cam], DEV)
    w = torch.from_numpy(np.random.default_rng(1).normal(size=4 * cam.npix).astype(np.float32)).to(DEV)
    prm = torch.from_numpy(P).to(DEV).requires_grad_(True)
    img = gs.rasterize(prm, plan, cams)
    (img * w).sum().backward()
    G = prm.grad.cpu().numpy()
    ref = oracle.render(P, cam)
    assert image_close(img.detach().cpu().numpy().reshape(4, -1), ref.rgba, ref.flags)[0] == 0
    Gref = oracle.backward(P, cam, w.cpu().numpy().astype(np.float64).reshape(4, -1))
    rep = grads_close(G, Gref)
    assert all(nb == 0 for _, nb, _ in rep), rep
    # float32 central differences through the same autograd op.  Only colour
    # coefficients: they enter the image linearly, whereas moving geometry or
    # opacity by a finite step also moves pixels across the 1/255 cutoff, a
    # jump the exact derivative excludes by definition (geometry is pinned by
    # the oracle comparison above and the oracle's own FP64 differences).
    rng = np.random.default_rng(5)
    checked = 0
    with torch.no_grad():
        for _ in range(24):
            c, i = int(rng.integers(11, 14)), int(rng.integers(0, P.shape[1]))
            if abs(G[c, i]) < 1e-2 * np.abs(G[c]).max():
                continue
            h = 2e-3 * max(1.0, abs(float(P[c, i])))
            pp, pm = prm.detach().clone(), prm.detach().clone()
            pp[c, i] += h
            pm[c, i] -= h
            fd = ((gs.rasterize(pp, plan, cams) * w).sum() - (gs.rasterize(pm, plan, cams) * w).sum()).item() / (2 * h)
            assert abs(fd - G[c, i]) <= 0.01 * abs(G[c, i]) + 1e-3 * np.abs(G[c]).max(), (c, i, fd, G[c, i])
            checked += 1
    assert checked >= 8


def test_key_capacity_overflow_is_reported(gs, ctx):
    P = synth.random_gaussians(500, seed=1)
    cam = synth.axis_camera(64, 64)
    sc = GpuScene(ctx, P, [cam], key_capacity=100, host_sized=True)
    with pytest.raises(gs.GsfError) as e:
        sc.plan.forward(sc.params, sc.n, sc.cams_dev, sc.rgba)
    assert e.value.status == _abi.GSF_E_CAPACITY
    torch.cuda.synchronize()
    np.testing.assert_array_equal(sc.rgba.cpu().numpy().reshape(4, -1)[3], 0.0)   # background only
    flags, m = sc.plan.poll()
    assert flags & _abi.GSF_FLAG_CAPACITY and m > 100
    dev_sized = GpuScene(ctx, P, [cam], key_capacity=100, host_sized=False)
    dev_sized.forward()
    flags, _ = dev_sized.plan.poll()
    assert flags & _abi.GSF_FLAG_CAPACITY
    assert dev_sized.plan.poll()[0] == 0      # flags are cleared by the poll
    # nothing was listed, so the adjoint passes no gradient: the per-record sum
    # writes zeros without reading a key position
    dl = np.random.default_rng(3).normal(size=(4, cam.npix))
    g = dev_sized.backward([dl])
    assert np.isfinite(g).all() and not g.any()
    R = dev_sized.n
    g2d = dev_sized.debug(_abi.GSF_DBG_G2D, np.float32, 9 * R)
    assert not g2d.any()


def test_nonfinite_loss_is_flagged(gs, ctx):
    P = synth.random_gaussians(200, seed=2)
    cam = synth.axis_camera(32, 32)
    sc = GpuScene(ctx, P, [cam])
    sc.forward()
    tgt = np.zeros((3, cam.npix), np.float32)
    tgt[1, 17] = np.nan
    loss = torch.zeros(1, device=DEV)
    dl = torch.zeros(4 * cam.npix, device=DEV)
    sc.plan.loss_l1(sc.rgba, torch.from_numpy(tgt.reshape(-1)).to(DEV), loss, dl)
    flags, _ = sc.plan.poll()
    assert flags & _abi.GSF_FLAG_NONFINITE


def test_invalid_arguments_are_rejected(gs, ctx):
    P = synth.random_gaussians(10, seed=2)
    cam = synth.axis_camera(16, 16)
    with pytest.raises(gs.GsfError) as e:
        gs.Plan(ctx, 10, [(16, 16)], 0, tile=12)
    assert e.value.status == _abi.GSF_E_INVALID
    with pytest.raises(gs.GsfError):
        gs.Plan(ctx, 10, [(16, 16)], 4)
    sc = GpuScene(ctx, P, [cam])
    with pytest.raises(gs.GsfError) as e:
        sc.plan.backward(sc.params, 10, sc.cams_dev, torch.zeros(4 * 256, device=DEV),
                         torch.zeros_like(sc.params))
    assert e.value.status == _abi.GSF_E_STATE
    with pytest.raises(gs.GsfError) as e:
        sc.plan.forward(sc.params, 11, sc.cams_dev, sc.rgba)
    assert e.value.status == _abi.GSF_E_INVALID


def test_edge_cases(gs, ctx):
    # one Gaussian; one pixel; everything behind the camera; a huge Gaussian
    one = synth.random_gaussians(1, seed=3, logscale_mean=-1.0)
    one[0:3, 0] = 0.0
    for cam in (synth.axis_camera(1, 1), synth.axis_camera(37, 29, bg=(0.5, 0.25, 0.125))):
        sc = GpuScene(ctx, one, [cam])
        img = sc.forward()[0]
        ref = oracle.render(one, cam)
        assert image_close(img, ref.rgba, ref.flags)[0] == 0
    behind = synth.random_gaussians(50, seed=4)
    behind[2] = -4.0                                  # camera at z = -3 looks along +z
    cam = synth.axis_camera(40, 24, bg=(0.1, 0.2, 0.3))
    sc = GpuScene(ctx, behind, [cam])
    img = sc.forward()[0]
    np.testing.assert_array_equal(img[:3], np.repeat(cam.bg[:, None], cam.npix, 1))
    np.testing.assert_array_equal(img[3], 0.0)
    assert sc.debug(_abi.GSF_DBG_KEYS, np.uint32, 16).size == 0
    g = sc.backward([np.ones((4, cam.npix))])
    np.testing.assert_array_equal(g, 0.0)
    huge = synth.random_gaussians(3, seed=5, logscale_mean=0.5)
    cam = synth.axis_camera(96, 64)
    for t_mode in (0, 1, 2):
        sc = GpuScene(ctx, huge, [cam], t_mode=t_mode, batch=64)
        img = sc.forward()[0]
        ref = oracle.render(huge, cam)
        assert image_close(img, ref.rgba, ref.flags)[0] == 0
        dl = np.random.default_rng(0).normal(size=(4, cam.npix))
        dl[:, ref.flags != 0] = 0
        rep = grads_close(sc.backward([dl]), oracle.backward(huge, cam, dl.astype(np.float32).astype(np.float64)))
        assert all(nb == 0 for _, nb, _ in rep), rep


def test_autotune_sweeps_and_candidates_render_identically(gs, ctx):
    """The autotuner times every (tile, LDS batch, transmittance mode)
    candidate of the captured step and returns the fastest; every candidate
    renders the same image bits (the per-pixel arithmetic does not depend on
    them) and is a valid plan."""
    P = synth.random_gaussians(1000, seed=0)
    cam = synth.axis_camera(128, 128)
    tgt = torch.from_numpy(np.ascontiguousarray(_cfg1_target().reshape(-1))).to(DEV)
    Pd = torch.from_numpy(P).to(DEV)
    best, times = gs.autotune(ctx, Pd, [cam], tgt, tiles=(8, 16, 32), batches=(64, 256),
                              t_modes=(0, 1, 2), warmup=1, reps=2)
    assert set(times) == {(t, b, m) for t in (8, 16, 32) for b in (64, 256) for m in (0, 1, 2)}
    assert best == min(times, key=times.get) and all(v > 0 for v in times.values())
    imgs = []
    for (t, b, m) in [best, (8, 64, 2), (32, 256, 1)]:
        fs = gs.FitStep(ctx, Pd.clone(), [cam], tgt, cfg=gs.FitConfig(tile=t, lds_batch=b, t_mode=m))
        fs.plan.forward(fs.params, fs.n, fs.cams_dev, fs.rgba)
        torch.cuda.synchronize()
        imgs.append(fs.rgba.cpu().numpy())
        fs.plan.close()
    for img in imgs[1:]:
        np.testing.assert_array_equal(imgs[0].view(np.uint32), img.view(np.uint32))


def _fovea_tile_live(g, radius_frac, cam, tile, tx, ty):
    """Tile (tx, ty) can hold a pixel of the fovea disk: the nearest point of
    its rectangle of pixel centres within the radius plus one pixel of the gaze
    point, in the kernels' FP32 arithmetic."""
    f = np.float32
    r = f(radius_frac) * f(cam.width) + f(1)
    gx, gy = f(g[0]), f(g[1])
    x0, x1 = f(tx * tile) + f(0.5), f(min((tx + 1) * tile, cam.width)) - f(0.5)
    y0, y1 = f(ty * tile) + f(0.5), f(min((ty + 1) * tile, cam.height)) - f(0.5)
    dx = max(max(x0 - gx, gx - x1), f(0))
    dy = max(max(y0 - gy, gy - y1), f(0))
    return bool(dx * dx + dy * dy <= r * r)


def test_fovea_culling_composites_only_the_disk(gs, ctx):
    """A fovea-culled step composites the pixels of the fovea disk only: over a
    view whose fovea box holds far more tiles than the disk, the tiles whose
    pixel centres all lie more than the radius plus two pixels from the gaze
    point (the box's corners) keep what the image buffer held, every masked-in
    pixel is written, and the other pixels of the tiles composited are the
    camera background with alpha 0.  Pair counting covers the same pixels: it
    visits fewer pairs than over the full frame."""
    P = synth.random_gaussians(6000, seed=22)
    cams = [synth.look_at_camera([0.2, -0.3, -3.0], width=512, height=384),
            synth.look_at_camera([-2.0, 1.2, -2.0], width=384, height=448)]
    gaze = synth.gaze_points(cams, seed=9)
    rng = np.random.default_rng(8)
    tgt = np.concatenate([rng.uniform(0, 1, size=3 * c.npix) for c in cams]).astype(np.float32)
    gz = torch.from_numpy(np.ascontiguousarray(gaze)).to(DEV)
    sentinel = np.float32(7.0)
    pairs = {}
    for cull in (True, False):
        cfg = gs.FitConfig(lr=0.0, tile=16, lds_batch=64, fovea_cull=cull)
        fs = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), cams, torch.from_numpy(tgt).to(DEV), gz,
                        cfg=cfg, fused=True)
        fs.rgba.fill_(float(sentinel))
        fs.step()
        torch.cuda.synchronize()
        assert fs.poll()[0] == 0
        pairs[cull] = fs.plan.count_pairs()
        if cull:
            img = fs.rgba.cpu().numpy()
        fs.plan.close()
    log(f"[cull] pairs culled {pairs[True]} vs full frame {pairs[False]}")
    assert pairs[True]["visited_fwd"] < pairs[False]["visited_fwd"]
    off, skipped = 0, 0
    for v, c in enumerate(cams):
        a = img[4 * off:4 * (off + c.npix)].reshape(4, c.height, c.width)
        ys, xs = np.mgrid[0:c.height, 0:c.width]
        d2 = (xs + 0.5 - np.float64(gaze[v][0])) ** 2 + (ys + 0.5 - np.float64(gaze[v][1])) ** 2
        r = 0.2 * c.width
        inside = d2 <= r * r
        written = ~(a == sentinel).all(axis=0)
        assert written[inside].all()
        for ty in range(0, c.height, 16):
            for tx in range(0, c.width, 16):
                t = (slice(ty, ty + 16), slice(tx, tx + 16))
                if np.sqrt(d2[t].min()) > r + 2.0:      # no pixel centre near the disk
                    skipped += 1
                    assert not written[t].any(), (v, tx, ty)
                elif written[t].any():                   # composited: the disk, else background
                    out = ~inside[t]
                    np.testing.assert_array_equal(a[3][t][out], 0.0)
                    for ch in range(3):
                        np.testing.assert_array_equal(a[ch][t][out], np.float32(c.bg[ch]))
        off += c.npix
    log(f"[cull] tiles left untouched: {skipped}")
    assert skipped > 0


@pytest.mark.parametrize("tile,t_mode", [(16, 0), (8, 1), (32, 0)])
def test_fovea_culling_matches_full_frame(gs, ctx, tile, t_mode):
    """Fovea culling composites only the fovea disks' pixels: in-mask pixels
    keep their bits, the masked loss and the gradient equal the full-frame
    step's, with fewer keys; the loss also equals the oracle's on the same
    image.  Tiles of 8, 16 and 32 pixels, recomputed and checkpointed
    transmittance."""
    P = synth.random_gaussians(3000, seed=21)
    cams = [synth.look_at_camera([0.3, -0.2, -3.0], width=224, height=160),
            synth.look_at_camera([2.5, 1.0, 1.0], width=160, height=208)]
    gaze = synth.gaze_points(cams, seed=6)
    rng = np.random.default_rng(5)
    tgt = np.concatenate([rng.uniform(0, 1, size=3 * c.npix) for c in cams]).astype(np.float32)
    tgt_dev = torch.from_numpy(tgt).to(DEV)
    gz = torch.from_numpy(np.ascontiguousarray(gaze)).to(DEV)
    runs, lists = {}, {}
    for cull in (False, True):
        cfg = gs.FitConfig(lr=0.0, tile=tile, lds_batch=64, t_mode=t_mode, fovea_cull=cull)
        fs = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), cams, tgt_dev, gz, cfg=cfg, fused=True)
        fs.step()
        torch.cuda.synchronize()
        runs[cull] = (fs.loss.item(), fs.rgba.cpu().numpy(), fs.grads.cpu().numpy(), fs.poll()[1])
        T, M = fs.plan.total_tiles, runs[cull][3]
        lists[cull] = (fs.plan.debug(_abi.GSF_DBG_RANGES, np.uint32, 2 * T).reshape(-1, 2).astype(np.int64),
                       fs.plan.debug(_abi.GSF_DBG_KEYS, np.uint32, M).astype(np.int64),
                       fs.plan.debug(_abi.GSF_DBG_VALS, np.uint32, M).astype(np.int64),
                       fs.plan.debug(_abi.GSF_DBG_ORDER, np.uint32, T).astype(np.int64))
        fs.plan.close()
    (l0, img0, g0, m0), (l1, img1, g1, m1) = runs[False], runs[True]
    # the culled step sorts, ranges and composites compact fovea-box tiles; mapped
    # back to global tiles its lists are the full frame's lists of those tiles
    (r0, k0, v0, o0), (r1, k1, v1, o1) = lists[False], lists[True]
    T = r0.shape[0]
    assert (np.diff(k1) >= 0).all() and k1.size == m1
    np.testing.assert_array_equal(r1[:, 0], np.searchsorted(k1, np.arange(T), "left"))
    np.testing.assert_array_equal(r1[:, 1], np.searchsorted(k1, np.arange(T), "right"))
    assert np.unique(o1).size == o1.size and set(np.unique(k1)) <= set(o1.tolist())
    assert o1.size < T
    # a launch tile that can hold a pixel of the disk lists what the full frame
    # lists there; the box's other tiles list nothing
    tile_off = np.cumsum([0] + [((c.width + tile - 1) // tile) * ((c.height + tile - 1) // tile)
                                for c in cams])
    live_tiles = 0
    for t in o1:
        v = int(np.searchsorted(tile_off, t, "right") - 1)
        c = cams[v]
        ty, tx = divmod(int(t - tile_off[v]), (c.width + tile - 1) // tile)
        if _fovea_tile_live(gaze[v], 0.2, c, tile, tx, ty):
            live_tiles += 1
            np.testing.assert_array_equal(v1[r1[t, 0]:r1[t, 1]], v0[r0[t, 0]:r0[t, 1]])
        else:
            assert r1[t, 0] == r1[t, 1], (v, tx, ty)
    assert 0 < live_tiles < o1.size
    log(f"[cull] loss {l0:.7f} vs {l1:.7f}, keys {m0} -> {m1}")
    assert m1 < m0
    assert abs(l1 - l0) <= 1e-6 * abs(l0)
    off = 0
    imgs = []
    for v, c in enumerate(cams):
        a = img0[4 * off:4 * (off + c.npix)].reshape(4, c.npix)
        b = img1[4 * off:4 * (off + c.npix)].reshape(4, c.npix)
        ys, xs = np.divmod(np.arange(c.npix), c.width)
        inside = (xs + 0.5 - gaze[v][0]) ** 2 + (ys + 0.5 - gaze[v][1]) ** 2 <= (0.2 * c.width) ** 2
        assert inside.sum() > 100
        np.testing.assert_array_equal(a[:, inside].view(np.uint32), b[:, inside].view(np.uint32))
        imgs.append(a.astype(np.float64))
        off += c.npix
    rep = grads_close(g1, g0.astype(np.float64))
    assert all(nb == 0 for _, nb, _ in rep), rep
    tg, off = [], 0
    for c in cams:
        tg.append(tgt[3 * off:3 * (off + c.npix)].astype(np.float64))
        off += c.npix
    L, _ = oracle.loss_l1(imgs, tg, cams, gazes=gaze.astype(np.float64), radius_frac=0.2)
    assert abs(l1 - L) <= 1e-5 * L


def _rgba_targets(cams):
    Pt = synth.random_gaussians(300, seed=synth.SEED_TARGET_SET)
    return [oracle.render(Pt, c).rgba for c in cams]


def test_rgba_loss_over_background_matches_oracle(gs, ctx):
    P = synth.random_gaussians(300, seed=31)
    cams = [synth.look_at_camera([0.3, -0.2, -3.0], width=80, height=64),
            synth.look_at_camera([2.0, 1.0, 1.5], width=56, height=72)]
    sc = GpuScene(ctx, P, cams)
    imgs = sc.forward()
    tg = _rgba_targets(cams)
    bg = np.array([[0.9, 0.1, 0.4], [0.2, 0.7, 0.5]], np.float32)
    gaze = synth.gaze_points(cams, seed=6)
    for alpha in (True, False):
        for gz in (None, gaze):
            loss = torch.zeros(1, device=DEV)
            dl = torch.zeros(4 * sum(c.npix for c in cams), device=DEV)
            t = torch.from_numpy(np.concatenate([x.astype(np.float32).reshape(-1) for x in tg])).to(DEV)
            sc.plan.loss_l1_rgba(sc.rgba, t, loss, dl, bg=torch.from_numpy(bg).to(DEV), alpha=alpha,
                                 gaze=None if gz is None else torch.from_numpy(gz).to(DEV),
                                 radius_frac=0.2 if gz is not None else 0.0)
            torch.cuda.synchronize()
            L, dls = oracle.loss_l1_rgba([i.astype(np.float64) for i in imgs],
                                         [x.astype(np.float32).astype(np.float64) for x in tg], cams,
                                         bgs=bg.astype(np.float64), alpha=alpha,
                                         gazes=None if gz is None else gz.astype(np.float64),
                                         radius_frac=0.2)
            assert abs(loss.item() - L) <= 1e-5 * L
            np.testing.assert_allclose(dl.cpu().numpy(), np.concatenate([d.reshape(-1) for d in dls]),
                                       rtol=1e-6, atol=0)


def test_alpha_training_with_random_backgrounds(gs, ctx):
    """The fused step with alpha training over random backgrounds: the drawn
    backgrounds are the SplitMix64 values of the step number, and loss and
    gradient equal the oracle's for the scene rendered over them; captured
    replays draw each step's own backgrounds."""
    P = synth.random_gaussians(400, seed=32)
    P[10] -= 1.0      # lower opacities: no pixel near a threshold (checked below), so every
    #                   pixel's sign gradient can be compared as is
    cams = [synth.look_at_camera([0.3, -0.2, -3.0], width=96, height=80),
            synth.look_at_camera([2.5, 1.0, 1.0], width=64, height=48)]
    tg = _rgba_targets(cams)
    tgt = torch.from_numpy(np.concatenate([x.astype(np.float32).reshape(-1) for x in tg])).to(DEV)
    seed = 0x5EED1234ABCD
    cfg = gs.FitConfig(lr=0.0, tile=16, lds_batch=64, alpha_loss=True, random_bg=True, bg_seed=seed)
    fs = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), cams, tgt, cfg=cfg, fused=True)
    for step in range(2):
        fs.step()
        torch.cuda.synchronize()
        bg = fs.backgrounds()
        expect = oracle.background_draw(seed, step, len(cams))
        np.testing.assert_array_equal(bg.astype(np.float64), expect)
        ocams = [synth.Camera(**{**c.__dict__, "bg": expect[v].astype(np.float32)})
                 for v, c in enumerate(cams)]
        refs = [oracle.render(P, c) for c in ocams]
        L, dls = oracle.loss_l1_rgba([r.rgba for r in refs],
                                     [x.astype(np.float32).astype(np.float64) for x in tg], ocams,
                                     bgs=expect, alpha=True)
        log(f"[alpha] step {step}: bg {bg.tolist()}, loss {fs.loss.item():.6f} vs {L:.6f}")
        assert abs(fs.loss.item() - L) <= 1e-5 * L
        assert all((r.flags == 0).all() for r in refs)
        G = sum(oracle.backward(P, c, d) for c, d in zip(ocams, dls))
        rep = grads_close(fs.grads.cpu().numpy(), G)
        assert all(nb == 0 for _, nb, _ in rep), rep
    # captured (on a stream of its own): each replay draws its own step's backgrounds
    with torch.cuda.stream(torch.cuda.Stream()):
        fs.capture()
        for step in range(2, 5):
            fs.replay()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(fs.backgrounds().astype(np.float64),
                                          oracle.background_draw(seed, step, len(cams)))
    fs.plan.close()


def test_capacity_overflow_skips_the_update_and_replans(gs, ctx):
    """A captured step whose keys overflow the capacity leaves parameters, Adam
    moments and the step counter untouched; ensure_capacity re-plans, recaptures
    and the repeated step matches a step planned with room from the start."""
    P = synth.random_gaussians(1000, seed=0)
    cam = synth.axis_camera(128, 128)
    tgt = torch.from_numpy(_cfg1_target().reshape(-1).copy()).to(DEV)
    with torch.cuda.stream(torch.cuda.Stream()):
        fs = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), [cam], tgt,
                        cfg=gs.FitConfig(lr=1e-2, key_capacity=100))
        fs.capture()
        p0 = fs.params.clone()
        fs.replay()
        fs.replay()
        torch.cuda.synchronize()
        assert torch.equal(fs.params, p0)
        assert int(fs.step_dev.item()) == 0 and not fs.m.any().item() and not fs.v.any().item()
        assert fs.ensure_capacity() is True
        assert fs.key_capacity >= 200
        fs.replay()
        assert fs.ensure_capacity() is False
        assert int(fs.step_dev.item()) == 1 and not torch.equal(fs.params, p0)
        ref = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), [cam], tgt, cfg=gs.FitConfig(lr=1e-2))
        ref.step()
        torch.cuda.synchronize()
        assert abs(fs.loss.item() - ref.loss.item()) <= 1e-6 * ref.loss.item()
        rep = grads_close(fs.grads.cpu().numpy(), ref.grads.cpu().numpy().astype(np.float64),
                          rtol=1e-5)
        assert all(nb == 0 for _, nb, _ in rep), rep


@pytest.mark.parametrize("masked", [False, True])
def test_plain_step_equals_fused_step(gs, ctx, masked):
    """One plain step (a host-synchronised plan per view; the library divides
    each view's L1 by the entry count over all views and adds the views' losses
    and gradients) against one fused step over 3 uneven views, with and without
    a fovea mask and fovea culling: the same image bits (in the fovea when
    masked), the same loss, gradients within the parity tolerance, and every
    parameter whose gradient is not tiny moved by Adam to within 1e-6 of the
    fused step's value."""
    P = synth.random_gaussians(2500, seed=31)
    cams = [synth.look_at_camera([0.3, -0.2, -3.0], width=160, height=96),
            synth.look_at_camera([2.5, 1.0, 1.0], width=112, height=144),
            synth.look_at_camera([-1.0, 2.6, 1.2], width=128, height=128)]
    gaze = synth.gaze_points(cams, seed=6) if masked else None
    gz = torch.from_numpy(np.ascontiguousarray(gaze)).to(DEV) if masked else None
    rng = np.random.default_rng(32)
    tgt = torch.from_numpy(np.concatenate([rng.uniform(0, 1, size=3 * c.npix)
                                           for c in cams]).astype(np.float32)).to(DEV)
    log(f"[plain] 3 uneven views, masked {masked}: plain step vs fused step")
    runs = {}
    for fused in (True, False):
        cfg = gs.FitConfig(lr=1e-3, tile=16, lds_batch=64, t_mode=1, fovea_cull=masked)
        fs = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), cams, tgt, gz, cfg=cfg, fused=fused)
        fs.step()
        torch.cuda.synchronize()
        runs[fused] = (fs.loss.item(), fs.rgba.cpu().numpy(), fs.grads.cpu().numpy(),
                       fs.params.cpu().numpy())
        fs.close()
    (lf, imf, gf, pf), (lp, imp, gp, pp) = runs[True], runs[False]
    log(f"[plain]   loss fused {lf:.8f} plain {lp:.8f}")
    assert abs(lp - lf) <= 1e-6 * abs(lf)
    off = 0
    for v, c in enumerate(cams):
        a = imf[4 * off:4 * (off + c.npix)].reshape(4, c.npix)
        b = imp[4 * off:4 * (off + c.npix)].reshape(4, c.npix)
        keep = np.ones(c.npix, bool)
        if masked:
            ys, xs = np.divmod(np.arange(c.npix), c.width)
            keep = (xs + 0.5 - gaze[v][0]) ** 2 + (ys + 0.5 - gaze[v][1]) ** 2 <= (0.2 * c.width) ** 2
        np.testing.assert_array_equal(a[:, keep].view(np.uint32), b[:, keep].view(np.uint32))
        off += c.npix
    rep = grads_close(gp, gf.astype(np.float64))
    log(f"[plain]   gradient groups {rep}")
    assert all(nb == 0 for _, nb, _ in rep), rep
    big = np.abs(gf) > 1e-3 * np.abs(gf).max()
    assert big.sum() > 100
    assert np.abs(pp - pf)[big].max() <= 1e-6
