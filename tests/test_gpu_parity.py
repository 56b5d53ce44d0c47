"""GPU (HIP path through the C ABI) vs the FP64 oracle, stage by stage."""
import numpy as np
import pytest

import oracle
import synth
from paper_2601_22026_amd import _abi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_22026_amd as gs
    return gs.Context(0)


from gpu_common import GpuScene, grads_close, image_close, log  # noqa: E402


def _cfg1():
    return synth.random_gaussians(1000, seed=0), synth.axis_camera(128, 128)


def test_projection_matches_oracle(ctx):
    P, cam = _cfg1()
    log("[parity] projection cfg1 1000 Gaussians 128x128")
    sc = GpuScene(ctx, P, [cam])
    sc.forward()
    pr = sc.proj()
    ref = oracle.project(P, cam)
    valid = ref["valid"] != 0
    near = ref["flags"] != 0
    assert ((pr[:, 10] != 0) == valid)[~near].all()
    v = valid & ~near
    for j, k in enumerate(["mx", "my", "A", "B", "C", "o", "r", "g", "b", "tz"]):
        g, r = pr[v, j].astype(np.float64), ref[k][v]
        scale = np.abs(r).max()
        err = np.abs(g - r)
        assert (err <= 1e-4 * np.abs(r) + 1e-6 * scale).all(), (k, err.max())


def _discrete_scenes():
    yield "3 uneven views", synth.random_gaussians(600, seed=3), [
        synth.axis_camera(128, 96), synth.look_at_camera([2.0, -1.0, 2.0], width=77, height=53),
        synth.look_at_camera([0.0, 3.0, 0.2], width=40, height=64)]
    # boxes of tens of tile rows (over 32 at 8-pixel tiles), listed row by row
    yield "512^2 + 480x400 with near splats", \
        synth.with_near_splats(synth.random_gaussians(300, seed=12), 8, seed=12), [
            synth.axis_camera(512, 512), synth.look_at_camera([1.2, -0.8, -2.6], width=480,
                                                               height=400)]


def _depth_sort_passes(sc, R):
    """Passes the library's depth sort takes for the last forward: three when
    the depth keys of the records that list a tile lie below 2^24 above the
    smallest with its low 8 bits cleared, else four (its documented rule)."""
    count = sc.debug(_abi.GSF_DBG_COUNT, np.uint32, R)
    depth = sc.debug(_abi.GSF_DBG_DEPTH, np.uint32, R)[count > 0].astype(np.int64)
    if depth.size == 0:
        return 3
    return 3 if depth.max() - (depth.min() & ~0xFF) < (1 << 24) else 4


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_discrete_stage_bit_exact(ctx, tile):
    """Keys, values and ranges against the oracle, bit for bit.  Records the
    oracle flags (a box edge or depth tie within rounding) are removed from both
    key lists; ranges are compared on every tile no flagged record is listed in
    on either side (as that tile's list of records), and the GPU's ranges are
    checked to be the lower and upper bounds of its own sorted keys everywhere.
    The scenes take both forms of the depth sort: three passes (depths within
    about two binades) and four (near splats)."""
    passes = set()
    for name, P, cams in _discrete_scenes():
        log(f"[parity] discrete stage tile {tile}, {name}")
        sc = GpuScene(ctx, P, cams, tile=tile)
        sc.forward()
        d = oracle.discrete(P, cams, tile)
        flagged = np.nonzero(d.rflags != 0)[0]
        R = sc.n * len(cams)
        M = d.m
        count = sc.debug(_abi.GSF_DBG_COUNT, np.uint32, R)
        Mg = int(count.sum())
        keys = sc.debug(_abi.GSF_DBG_KEYS, np.uint32, Mg).astype(np.int64)
        vals = sc.debug(_abi.GSF_DBG_VALS, np.uint32, Mg).astype(np.int64)
        tiles = d.ranges.shape[0]
        ranges = sc.debug(_abi.GSF_DBG_RANGES, np.uint32, 2 * tiles).reshape(-1, 2).astype(np.int64)
        assert keys.size == Mg
        # remove the keys of records whose box or depth order is legitimately ambiguous
        drop_g = np.isin(vals, flagged)
        drop_o = np.isin(d.vals, flagged)
        np.testing.assert_array_equal(keys[~drop_g], d.keys[~drop_o])
        np.testing.assert_array_equal(vals[~drop_g], d.vals[~drop_o])
        # ranges: the GPU's own bounds everywhere ...
        assert (np.diff(keys) >= 0).all()
        np.testing.assert_array_equal(ranges[:, 0], np.searchsorted(keys, np.arange(tiles), "left"))
        np.testing.assert_array_equal(ranges[:, 1], np.searchsorted(keys, np.arange(tiles), "right"))
        # ... and the oracle's lists on every tile untouched by a flagged record
        touched = np.zeros(tiles, bool)
        touched[keys[drop_g]] = True
        touched[d.keys[drop_o]] = True
        for t in np.nonzero(~touched)[0]:
            np.testing.assert_array_equal(vals[ranges[t, 0]:ranges[t, 1]],
                                          d.vals[d.ranges[t, 0]:d.ranges[t, 1]])
        if flagged.size == 0:
            assert Mg == M
            np.testing.assert_array_equal(ranges, d.ranges)
        passes.add(_depth_sort_passes(sc, R))
        log(f"[parity]   keys {M}, flagged records {flagged.size}, tiles compared "
            f"{int((~touched).sum())} of {tiles}, depth-sort passes {_depth_sort_passes(sc, R)}")
    assert passes == {3, 4}, passes


def test_discrete_stage_with_saturated_counts(ctx):
    """A plan of over 2^23 records, so that a depth-sort value keeps only 8 bits
    for the record's tile count above its entry index: near splats list more
    tiles than that (the emission then reads their count from the entry).  All
    but 308 of the 4.2M Gaussians lie behind the cameras; the visible ones sit
    at spread indices, and the keys, values and ranges equal the oracle's for
    them alone (record ids mapped to the full plan), bit for bit."""
    n = (1 << 22) + 1000
    vis = synth.with_near_splats(synth.random_gaussians(300, seed=14), 8, seed=14)
    rng = np.random.default_rng(14)
    idx = np.sort(rng.choice(n, size=vis.shape[1], replace=False))
    P = np.repeat(vis[:, :1], n, axis=1)
    P[0:3] = [[0.0], [0.0], [-10.0]]   # every other Gaussian behind both cameras (negative view depth)
    P[:, idx] = vis
    cams = [synth.axis_camera(256, 256), synth.look_at_camera([0.4, -0.3, -2.8], width=224, height=200)]
    log(f"[parity] saturated counts: {n} Gaussians x 2 views, {vis.shape[1]} visible, tile 8")
    sc = GpuScene(ctx, P, cams, tile=8)
    sc.forward()
    d = oracle.discrete(vis, cams, 8)
    nv = vis.shape[1]
    full = lambda r: (r // nv) * n + idx[r % nv]   # subset record id -> plan record id
    count = sc.debug(_abi.GSF_DBG_COUNT, np.uint32, 2 * n).astype(np.int64)
    Mg = int(count.sum())
    assert count.max() > 255, count.max()   # counts that do not fit the value's 8 bits
    keys = sc.debug(_abi.GSF_DBG_KEYS, np.uint32, Mg).astype(np.int64)
    vals = sc.debug(_abi.GSF_DBG_VALS, np.uint32, Mg).astype(np.int64)
    tiles = d.ranges.shape[0]
    ranges = sc.debug(_abi.GSF_DBG_RANGES, np.uint32, 2 * tiles).reshape(-1, 2).astype(np.int64)
    flagged = full(np.nonzero(d.rflags != 0)[0])
    dvals = full(d.vals)
    drop_g, drop_o = np.isin(vals, flagged), np.isin(dvals, flagged)
    np.testing.assert_array_equal(keys[~drop_g], d.keys[~drop_o])
    np.testing.assert_array_equal(vals[~drop_g], dvals[~drop_o])
    assert (np.diff(keys) >= 0).all()
    np.testing.assert_array_equal(ranges[:, 0], np.searchsorted(keys, np.arange(tiles), "left"))
    np.testing.assert_array_equal(ranges[:, 1], np.searchsorted(keys, np.arange(tiles), "right"))
    log(f"[parity]   keys {Mg}, largest count {count.max()}, flagged records {flagged.size}")


@pytest.mark.parametrize("planes", [1, 3])
def test_equal_depths_keep_record_order(ctx, planes):
    """Means on one or three planes of constant camera depth, so most depths tie
    exactly: every tile's list is in (depth bits, record) order, for lists ranked
    in one step (at most 256 keys), sorted by radix passes in LDS (up to 1024)
    and on global scratch (longer).  The oracle flags such ties as ambiguous under
    rounding; this checks the order the GPU defines on its own depth keys."""
    P = synth.random_gaussians(12000, seed=11)
    P[2] = np.float32([-0.25, 0.0, 0.4])[np.arange(P.shape[1]) % planes]
    cams = [synth.axis_camera(96, 64)]
    log(f"[parity] equal depths on {planes} plane(s), 12000 Gaussians, tile 16")
    sc = GpuScene(ctx, P, cams, tile=16)
    sc.forward()
    count = sc.debug(_abi.GSF_DBG_COUNT, np.uint32, sc.n).astype(np.int64)
    M = int(count.sum())
    keys = sc.debug(_abi.GSF_DBG_KEYS, np.uint32, M).astype(np.int64)
    vals = sc.debug(_abi.GSF_DBG_VALS, np.uint32, M).astype(np.int64)
    depth = sc.debug(_abi.GSF_DBG_DEPTH, np.uint32, sc.n).astype(np.int64)
    ranges = sc.debug(_abi.GSF_DBG_RANGES, np.uint32, 2 * 24).reshape(-1, 2).astype(np.int64)
    lens = ranges[:, 1] - ranges[:, 0]
    assert lens.sum() == M, lens
    for lo, hi in [(2, 256), (257, 1024), (1025, M)]:
        assert ((lens >= lo) & (lens <= hi)).any(), (lo, hi, lens)
    want = np.lexsort((vals, depth[vals], keys))
    np.testing.assert_array_equal(want, np.arange(M))
    # each record appears once per tile it was counted for
    np.testing.assert_array_equal(np.bincount(vals, minlength=sc.n), count)
    ties = np.count_nonzero((np.diff(keys) == 0) & (np.diff(depth[vals]) == 0))
    assert ties > M // 2, ties


def test_image_matches_oracle_cfg1(ctx):
    P, cam = _cfg1()
    sc = GpuScene(ctx, P, [cam])
    img = sc.forward()[0]
    ref = oracle.render(P, cam)
    nbad, worst, nflag = image_close(img, ref.rgba, ref.flags)
    log(f"[parity] cfg1 image worst abs err {worst:.2e}, flagged px {nflag}")
    assert nbad == 0, worst
    # transmittance and last contributor
    tf = sc.debug(_abi.GSF_DBG_TFINAL, np.float32, cam.npix)
    ok = ref.flags == 0
    assert np.allclose(tf[ok], ref.tfinal[ok], rtol=1e-4, atol=1e-6)
    nc = sc.debug(_abi.GSF_DBG_NCONTRIB, np.uint32, cam.npix).astype(np.int64)
    ranges = sc.debug(_abi.GSF_DBG_RANGES, np.uint32, 2 * 64).reshape(-1, 2).astype(np.int64)
    vals = sc.debug(_abi.GSF_DBG_VALS, np.uint32, 10 ** 6).astype(np.int64)
    px = np.arange(cam.npix)
    tid = (px // 128) // 16 * 8 + (px % 128) // 16
    last_gpu = np.where(nc > 0, vals[np.clip(ranges[tid, 0] + nc - 1, 0, None)], -1)
    np.testing.assert_array_equal(last_gpu[ok], ref.last[ok])


@pytest.mark.parametrize("deg,t_mode,batch", [(0, 0, 128), (3, 0, 128), (0, 1, 64), (3, 1, 128),
                                               (0, 2, 64), (3, 2, 256)])
def test_multiview_image_and_gradient(ctx, deg, t_mode, batch):
    P = synth.random_gaussians(400, seed=5, sh_degree=deg)
    cams = [synth.look_at_camera([0.3, -0.2, -3.0], width=96, height=80, bg=(0.1, 0.2, 0.3)),
            synth.look_at_camera([2.5, 1.0, 1.0], width=61, height=47)]
    log(f"[parity] 2 views, SH degree {deg}, t_mode {t_mode}, batch {batch}: image + gradient")
    sc = GpuScene(ctx, P, cams, batch=batch, t_mode=t_mode)
    imgs = sc.forward()
    refs = [oracle.render(P, c) for c in cams]
    for img, ref in zip(imgs, refs):
        nbad, worst, _ = image_close(img, ref.rgba, ref.flags)
        assert nbad == 0, worst
    rng = np.random.default_rng(0)
    dls = [rng.normal(size=(4, c.npix)) for c in cams]
    for dl, ref in zip(dls, refs):
        dl[:, ref.flags != 0] = 0.0      # no upstream gradient on ambiguous pixels
    g = sc.backward(dls)
    G = sum(oracle.backward(P, c, dl.astype(np.float32).astype(np.float64)) for c, dl in zip(cams, dls))
    rep = grads_close(g, G)
    log(f"[parity]   gradient groups {rep}")
    assert all(nb == 0 for _, nb, _ in rep), rep


@pytest.mark.parametrize("tile,batch", [(8, 64), (8, 256), (16, 64), (16, 256), (32, 128), (32, 256)])
def test_image_bitwise_invariant_over_tile_and_batch(ctx, tile, batch):
    P, cam = _cfg1()
    base = GpuScene(ctx, P, [cam], tile=16, batch=128).forward()[0]
    other = GpuScene(ctx, P, [cam], tile=tile, batch=batch).forward()[0]
    np.testing.assert_array_equal(base.view(np.uint32), other.view(np.uint32))


def test_device_sized_equals_host_sized(ctx):
    P, cam = _cfg1()
    a = GpuScene(ctx, P, [cam], host_sized=True).forward()[0]
    b = GpuScene(ctx, P, [cam], host_sized=False).forward()[0]
    np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


def test_loss_and_dl_match_oracle(ctx):
    P, cam = _cfg1()
    target = np.load(__import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                                "cfg1_target_128.npy"))[:3].reshape(3, -1)
    sc = GpuScene(ctx, P, [cam])
    img = sc.forward()[0]
    loss = torch.zeros(1, device="cuda:0")
    dl = torch.zeros(4 * cam.npix, device="cuda:0")
    sc.plan.loss_l1(sc.rgba, torch.from_numpy(np.ascontiguousarray(target)).to("cuda:0"), loss, dl)
    torch.cuda.synchronize()
    # the oracle's loss on the GPU image (same inputs, float64 arithmetic)
    L, dls = oracle.loss_l1([img.astype(np.float64)], [target.astype(np.float64)], [cam])
    assert abs(loss.item() - L) <= 1e-5 * L
    np.testing.assert_allclose(dl.cpu().numpy().reshape(4, -1), dls[0], rtol=1e-6, atol=0)


@pytest.mark.parametrize("radius_frac", [0.05, 0.2, 0.9])
def test_loss_mask_count_is_exact(ctx, radius_frac):
    """The masked entry count (one thread per row: the row's mask is an
    interval whose ends a binary search finds) equals the oracle's
    pixel-by-pixel count, which takes the same single-precision test, on
    uneven views with gaze points inside, on a corner of, on the edge of and
    outside the image; the fovea windows (radius 0.05, 0.2) and the whole
    frames (0.9) are both counted.  The loss then divides by it."""
    sizes = [(1920, 1920), (333, 217), (64, 48), (1000, 700), (517, 901)]
    cams = [synth.axis_camera(w, h) for w, h in sizes]
    rng = np.random.default_rng(11)
    gaze = np.array([[rng.uniform(0, w), rng.uniform(0, h)] for w, h in sizes], np.float32)
    gaze[1] = (0.0, 0.0)
    gaze[2] = (-5.0, 24.0)
    gaze[3] = (999.7, 700.0)
    sc = GpuScene(ctx, synth.random_gaussians(10, seed=1), cams)
    gz = torch.from_numpy(gaze).to("cuda:0")
    got = sc.plan.loss_count(gz, radius_frac)
    imgs = sc.forward()
    tgts = [np.random.default_rng(12 + v).uniform(size=(3, c.npix)).astype(np.float32)
            for v, c in enumerate(cams)]
    want = 0
    for v, c in enumerate(cams):
        _, cnt, _ = oracle.loss_l1_view(imgs[v].astype(np.float64), tgts[v].astype(np.float64), c,
                                        gaze[v].astype(np.float64),
                                        oracle.fovea_radius(radius_frac, c.width))
        want += cnt
    log(f"[parity] mask count radius {radius_frac}: {got} (oracle {want})")
    assert got == want
    loss = torch.zeros(1, device="cuda:0")
    dl = torch.zeros(4 * sum(c.npix for c in cams), device="cuda:0")
    tgt = torch.from_numpy(np.concatenate([t.reshape(-1) for t in tgts])).to("cuda:0")
    sc.plan.loss_l1(sc.rgba, tgt, loss, dl, gaze=gz, radius_frac=radius_frac)
    torch.cuda.synchronize()
    L, dls = oracle.loss_l1([i.astype(np.float64) for i in imgs], [t.astype(np.float64) for t in tgts],
                            cams, gazes=gaze.astype(np.float64), radius_frac=radius_frac)
    assert abs(loss.item() - L) <= 1e-5 * L
    np.testing.assert_allclose(dl.cpu().numpy(), np.concatenate([d.reshape(-1) for d in dls]),
                               rtol=1e-6, atol=0)


@pytest.mark.parametrize("tile,batch", [(8, 64), (16, 64), (16, 128), (32, 64)])
def test_transmittance_modes_agree(ctx, tile, batch):
    """Recomputed, checkpointed and stored transmittance: same image bits,
    gradients equal within tolerance."""
    P = synth.random_gaussians(1500, seed=8)
    cam = synth.look_at_camera([0.2, 0.4, -3.0], width=112, height=90, bg=(0.3, 0.1, 0.2))
    scenes = [GpuScene(ctx, P, [cam], tile=tile, batch=batch, t_mode=m) for m in (0, 1, 2)]
    imgs = [sc.forward()[0] for sc in scenes]
    for img in imgs[1:]:
        np.testing.assert_array_equal(imgs[0].view(np.uint32), img.view(np.uint32))
    dl = [np.random.default_rng(2).normal(size=(4, cam.npix))]
    grads = [sc.backward(dl) for sc in scenes]
    for m in (1, 2):
        rep = grads_close(grads[m], grads[0].astype(np.float64))
        log(f"[parity] tile {tile} batch {batch}: t_mode {m} vs recompute {rep}")
        assert all(nb == 0 for _, nb, _ in rep), rep
    a = scenes[0]
    ranges = a.debug(_abi.GSF_DBG_RANGES, np.uint32, 2 * a.plan.total_tiles).reshape(-1, 2)
    assert (ranges[:, 1] - ranges[:, 0]).max() > 2 * batch   # several batches per tile exercised


def test_checkpointed_adjoint_with_empty_tiles(ctx):
    """A dense cluster plus a few scattered Gaussians in two views: most tiles
    hold no key, empty and full tiles interleave, some tiles span several LDS
    batches, and the checkpointed adjoint must still find every unit."""
    P = np.concatenate([synth.random_gaussians(300, seed=12, mean_range=0.12, logscale_mean=-4.0),
                        synth.random_gaussians(30, seed=13, logscale_mean=-4.0)], axis=1)
    cams = [synth.look_at_camera([0.2, 0.4, -3.0], width=320, height=256),
            synth.look_at_camera([2.5, 1.0, 1.0], width=192, height=144)]
    a = GpuScene(ctx, P, cams, tile=16, batch=64, t_mode=0)
    b = GpuScene(ctx, P, cams, tile=16, batch=64, t_mode=1)
    c = GpuScene(ctx, P, cams, tile=16, batch=64, t_mode=2)
    ia, ib, ic = a.forward(), b.forward(), c.forward()
    for x, y, z in zip(ia, ib, ic):
        np.testing.assert_array_equal(x.view(np.uint32), y.view(np.uint32))
        np.testing.assert_array_equal(x.view(np.uint32), z.view(np.uint32))
    ranges = b.debug(_abi.GSF_DBG_RANGES, np.uint32, 2 * b.plan.total_tiles).reshape(-1, 2)
    empty = ranges[:, 1] == ranges[:, 0]
    assert empty.sum() > ranges.shape[0] // 2 and (~empty[:-1] & empty[1:]).any()
    assert (ranges[:, 1] - ranges[:, 0]).max() > 2 * 64
    rng = np.random.default_rng(4)
    dls = [rng.normal(size=(4, c.npix)) for c in cams]
    ga, gb, gc = a.backward(dls), b.backward(dls), c.backward(dls)
    for g in (gb, gc):
        rep = grads_close(g, ga.astype(np.float64))
        log(f"[parity] sparse scene mode vs recompute {rep}")
        assert all(nb == 0 for _, nb, _ in rep), rep
    refs = [oracle.render(P, c) for c in cams]
    for dl, ref in zip(dls, refs):
        dl[:, ref.flags != 0] = 0.0
    G = sum(oracle.backward(P, c, dl.astype(np.float32).astype(np.float64)) for c, dl in zip(cams, dls))
    rep = grads_close(b.backward(dls), G)
    assert all(nb == 0 for _, nb, _ in rep), rep


@pytest.mark.parametrize("t_mode", [0, 1])
def test_gradient_of_wide_splats_is_exact_and_reproducible(ctx, t_mode):
    """A few wide Gaussians over a field of small ones, tile 8: records with
    hundreds of tile keys next to records with one or two, so the per-record
    sum of the per-key gradients crosses many 64-key steps within one record
    and many records within one step.  Gradients match the oracle and two
    adjoints of one forward agree bit for bit."""
    P = np.concatenate([synth.random_gaussians(300, seed=21, logscale_mean=-4.0),
                        synth.random_gaussians(6, seed=22, logscale_mean=-1.2, logscale_std=0.2,
                                               mean_range=0.3)], axis=1)
    cam = synth.look_at_camera([0.2, -0.3, -3.0], width=192, height=160, bg=(0.2, 0.1, 0.3))
    log(f"[parity] wide splats, tile 8, t_mode {t_mode}: gradient vs oracle, reproducibility")
    sc = GpuScene(ctx, P, [cam], tile=8, batch=64, t_mode=t_mode)
    img = sc.forward()[0]
    ref = oracle.render(P, cam)
    nbad, worst, _ = image_close(img, ref.rgba, ref.flags)
    assert nbad == 0, worst
    count = sc.debug(_abi.GSF_DBG_COUNT, np.uint32, sc.n)
    log(f"[parity]   keys per record: max {int(count.max())}, median {int(np.median(count))}")
    assert count.max() > 3 * 64 and (count <= 2).sum() > 50
    dl = np.random.default_rng(6).normal(size=(4, cam.npix))
    dl[:, ref.flags != 0] = 0.0
    g1 = sc.backward([dl])
    g2 = sc.backward([dl])
    np.testing.assert_array_equal(g1.view(np.uint32), g2.view(np.uint32))
    G = oracle.backward(P, cam, dl.astype(np.float32).astype(np.float64))
    rep = grads_close(g1, G)
    log(f"[parity]   gradient groups {rep}")
    assert all(nb == 0 for _, nb, _ in rep), rep


@pytest.mark.parametrize("tile,t_mode", [(8, 0), (8, 1), (16, 2)])
def test_tall_boxes_image_and_gradient_match_oracle(ctx, tile, t_mode):
    """Near splats whose support boxes are tens of tile rows tall (over 32 at
    8-pixel tiles) over a field of small ones in a 512^2 view: every box is
    listed row by row, the adjoint finds each key's slot through the record's
    row table, and image and gradient match the oracle."""
    P = synth.with_near_splats(synth.random_gaussians(300, seed=12), 8, seed=12)
    cam = synth.axis_camera(512, 512, bg=(0.1, 0.2, 0.3))
    log(f"[parity] tall boxes 512^2, tile {tile}, t_mode {t_mode}: image and gradient vs oracle")
    sc = GpuScene(ctx, P, [cam], tile=tile, batch=64, t_mode=t_mode)
    img = sc.forward()[0]
    rect = sc.debug(_abi.GSF_DBG_RECT, np.uint32, 2 * sc.n).reshape(-1, 2)
    rows = (rect[:, 1] >> 16) - (rect[:, 0] >> 16) + 1
    assert rows.max() > 32 if tile == 8 else rows.max() > 16, rows.max()
    ref = oracle.render(P, cam)
    nbad, worst, nflag = image_close(img, ref.rgba, ref.flags)
    assert nbad == 0, worst
    dl = np.random.default_rng(8).normal(size=(4, cam.npix))
    dl[:, ref.flags != 0] = 0.0
    g = sc.backward([dl])
    G = oracle.backward(P, cam, dl.astype(np.float32).astype(np.float64))
    rep = grads_close(g, G)
    log(f"[parity]   tallest box {int(rows.max())} tile rows, flagged px {nflag}, groups {rep}")
    assert all(nb == 0 for _, nb, _ in rep), rep
