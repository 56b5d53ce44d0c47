"""GPU tests of the continual-refinement pieces (Method, "Periphery Model
Training"): the visibility-masked Adam (standalone and inside the fused step),
the optimiser restart, and the Refiner loop (Eq. (1) view selection, restart
from the current Gaussians with the optimiser state discarded)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from gpu_common import DEV, grads_close, log  # noqa: E402

F = lambda x: float(np.float32(x))  # noqa: E731


@pytest.fixture(scope="module")
def gs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_22026_amd
    return paper_2601_22026_amd


@pytest.fixture(scope="module")
def ctx(gs):
    return gs.Context(0)


def test_masked_adam_matches_oracle_given_identical_inputs(gs, ctx):
    """Three steps with a new gradient and a new visibility mask each step: the
    visible columns match the oracle to 1e-6 from the same float32 state, the
    hidden columns keep their bits."""
    rng = np.random.default_rng(11)
    C, n = 14, 1001
    lr = [1e-3] * 3 + [1.5e-3] * 3 + [1e-3] * 4 + [1.5e-3] * 4
    tp = torch.from_numpy(rng.normal(size=(C, n)).astype(np.float32)).to(DEV)
    tm = torch.zeros_like(tp)
    tv = torch.zeros_like(tp)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    for t in range(1, 4):
        g = rng.normal(size=(C, n)).astype(np.float32)
        vis = (rng.random(n) < 0.6).astype(np.uint8)
        before = [x.cpu().numpy() for x in (tp, tm, tv)]
        pd, md, vd = (x.astype(np.float64) for x in before)
        gs.adam_masked(ctx, tp, torch.from_numpy(g).to(DEV), tm, tv, step, lr,
                       torch.from_numpy(vis).to(DEV))
        torch.cuda.synchronize()
        oracle.adam_masked(pd, g.astype(np.float64), md, vd, t, vis.astype(bool),
                           lr=np.array([F(x) for x in lr]), betas=(F(0.9), F(0.999)), eps=F(1e-15))
        after = [x.cpu().numpy() for x in (tp, tm, tv)]
        hid = vis == 0
        for a, b in zip(after, before):
            np.testing.assert_array_equal(a[:, hid].view(np.uint32), b[:, hid].view(np.uint32))
        np.testing.assert_allclose(after[0], pd, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(after[1], md, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(after[2], vd, rtol=1e-6, atol=1e-9)
    assert int(step.item()) == 3


def test_adam_reset_zeroes_moments_and_step(gs, ctx):
    n = 4099                                           # a ragged tail after the float4 body
    m = torch.randn(n, device=DEV)
    v = torch.rand(n, device=DEV)
    step = torch.full((1,), 7, dtype=torch.int32, device=DEV)
    gs.adam_reset(ctx, m, v, step)
    torch.cuda.synchronize()
    assert not m.any().item() and not v.any().item() and int(step.item()) == 0
    # the reset is an ordinary kernel: it can sit in a captured graph and replay
    m.fill_(1.0)
    v.fill_(2.0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            gs.adam_reset(ctx, m, v, step)
    for _ in range(3):
        m.fill_(3.0)
        step.fill_(5)
        g.replay()
        torch.cuda.synchronize()
        assert not m.any().item() and int(step.item()) == 0


def _scene():
    P = synth.random_gaussians(300, seed=41)
    P[10] -= 1.0
    wide = synth.look_at_camera([0.0, 0.0, -3.0], width=96, height=96, fov_x_deg=60.0)
    narrow = synth.look_at_camera([0.4, 0.3, -3.0], width=96, height=96, fov_x_deg=15.0)
    rng = np.random.default_rng(42)
    tg = [rng.uniform(0.0, 1.0, size=(3, 96 * 96)) for _ in range(2)]
    return P, wide, narrow, tg


def _colour_only_lr(C, lr=1e-2):
    # geometry and opacity fixed, so the visible set of each view is that of the
    # initial Gaussians on both sides
    return [0.0] * 11 + [lr] * (C - 11)


@pytest.mark.parametrize("masked", [True, False])
def test_masked_step_against_oracle(gs, ctx, masked):
    """Step 1 through a wide view, step 2 through a narrow one.  The fused
    step's visibility equals the oracle's bit for bit; after step 1 every
    parameter matches the oracle's masked step; in step 2 the Gaussians the
    narrow view misses keep parameters and moments (masked) or still move by
    their momentum (dense)."""
    P, wide, narrow, tg = _scene()
    C, n = P.shape
    lr = _colour_only_lr(C)
    cfg = gs.FitConfig(lr=lr, tile=16, lds_batch=64, key_capacity=1 << 20, masked_adam=masked)
    tgt = torch.from_numpy(tg[0].astype(np.float32).reshape(-1).copy()).to(DEV)
    fs = gs.FitStep(ctx, torch.from_numpy(P).to(DEV), [wide], tgt, cfg=cfg, fused=True)
    vis_w = oracle.visibility(P, [wide])
    vis_n = oracle.visibility(P, [narrow])
    assert vis_w.all() or vis_w.sum() > 250
    hidden2 = vis_w & ~vis_n
    assert hidden2.sum() > 50, hidden2.sum()
    # oracle, step 1 (its own float64 state from the same inputs)
    Pd = P.astype(np.float64)
    md, vd = np.zeros_like(Pd), np.zeros_like(Pd)
    ref = oracle.render(P, wide)
    L1, dls = oracle.loss_l1([ref.rgba], [tg[0].astype(np.float32).astype(np.float64)], [wide])
    G1 = oracle.backward(P, wide, dls[0])
    oracle.adam_masked(Pd, G1, md, vd, 1, vis_w, lr=np.array([F(x) for x in lr]))
    fs.step()
    torch.cuda.synchronize()
    assert fs.poll()[0] == 0
    if masked:
        np.testing.assert_array_equal(fs.visibility().astype(bool), vis_w)
    g1 = fs.grads.cpu().numpy()
    rep = grads_close(g1, G1)
    assert all(nb == 0 for _, nb, _ in rep), rep
    p1 = fs.params.cpu().numpy()
    # t = 1: each updated element moves by -lr sign(g); where the gradient is
    # tiny its sign may differ (at most 2 lr apart), elsewhere 1e-6
    tiny = np.abs(G1) < 1e-2 * np.abs(G1[11:]).max()
    diff = np.abs(p1 - Pd)
    assert (diff[~tiny] <= 1e-6).all(), diff[~tiny].max()
    assert (diff[tiny] <= 2 * 1e-2 + 1e-6).all()
    assert abs(fs.loss.item() - L1) <= 1e-4 * L1
    # step 2 through the narrow view
    state1 = [x.cpu().numpy().copy() for x in (fs.params, fs.m, fs.v)]
    fs.cams_dev.copy_(gs.cameras_to_device([narrow], DEV))
    fs.targets.copy_(torch.from_numpy(tg[1].astype(np.float32).reshape(-1)))
    fs.step()
    torch.cuda.synchronize()
    assert fs.poll()[0] == 0
    state2 = [x.cpu().numpy() for x in (fs.params, fs.m, fs.v)]
    if masked:
        np.testing.assert_array_equal(fs.visibility().astype(bool), vis_n)
        for a, b in zip(state2, state1):
            np.testing.assert_array_equal(a[:, ~vis_n].view(np.uint32), b[:, ~vis_n].view(np.uint32))
    else:
        # dense Adam: hidden Gaussians with momentum from step 1 still move
        moved = np.abs(state2[0][11:, hidden2] - state1[0][11:, hidden2]) > 0
        assert moved.mean() > 0.5, moved.mean()
    log(f"[refine] masked={masked}: hidden at step 2 {int(hidden2.sum())}, "
        f"visible {int(vis_n.sum())}")


def test_refiner_selects_views_and_restarts(gs, ctx):
    """Refiner: offered views are kept exactly when the oracle's Eq. (1) keeps
    them; a restart fits all kept views from the current Gaussians with zeroed
    optimiser state, and its loss curve follows the oracle's."""
    P = synth.random_gaussians(400, seed=51)
    init = synth.sphere_cameras([(64, 64), (64, 48)])
    stream = synth.view_stream(10, width=48, height=48)
    rng = np.random.default_rng(52)
    targets = {id(c): rng.uniform(0.0, 1.0, size=(3, c.width * c.height)) for c in init + stream}
    t_dev = lambda c: torch.from_numpy(targets[id(c)].astype(np.float32).reshape(-1)).to(DEV)  # noqa: E731
    params = torch.from_numpy(P).to(DEV)
    cfg = gs.FitConfig(lr=1e-3, lr_boost=1.5, tile=16, lds_batch=64)
    with torch.cuda.stream(torch.cuda.Stream()):
        ref = gs.Refiner(ctx, params, init, [t_dev(c) for c in init], cfg=cfg)
        kept = [ref.offer(c, t_dev(c)) for c in stream]
        assert kept == oracle.select_views(init, stream, F(0.05), F(5.0))
        assert 2 <= sum(kept) < len(stream), kept
        fit = ref.restart()
        assert int(fit.step_dev.item()) == 0 and not fit.m.any().item()
        losses = []
        for _ in range(3):
            ref.run(1)
            losses.append(fit.loss.item())
        torch.cuda.synchronize()
        assert fit.poll()[0] == 0
        # the oracle fits the same views from the same Gaussians with fresh state
        cams = init + [c for c, k in zip(stream, kept) if k]
        Pd = P.astype(np.float64)
        md, vd = np.zeros_like(Pd), np.zeros_like(Pd)
        lr = np.array([F(x) for x in gs.plane_learning_rates(0, 1e-3, 1.5)])[:, None]
        want = [oracle.fit_step(Pd, md, vd, t, cams,
                                [targets[id(c)].astype(np.float32).astype(np.float64) for c in cams],
                                lr=np.broadcast_to(lr, Pd.shape).copy())
                for t in range(1, 4)]
        log(f"[refine] {len(cams)} views, losses {np.round(losses, 6)} oracle {np.round(want, 6)}")
        np.testing.assert_allclose(losses, want, rtol=1e-3)
        # a later restart keeps the Gaussians and discards the optimiser state
        p_before = params.cpu().numpy().copy()
        more = synth.view_stream(6, seed=77, width=48, height=48)
        for c in more:
            targets[id(c)] = rng.uniform(0.0, 1.0, size=(3, c.width * c.height))
            ref.offer(c, t_dev(c))
        fit2 = ref.restart()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(params.cpu().numpy(), p_before)
        assert int(fit2.step_dev.item()) == 0 and not fit2.v.any().item()
        ref.run(2)
        torch.cuda.synchronize()
        assert int(fit2.step_dev.item()) == 2 and fit2.poll()[0] == 0
