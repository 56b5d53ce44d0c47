"""The warp entry point that allocates nothing (gsf_reproject_warp_noalloc,
whose z-buffer is the library's device-resident array) against the warp with
a caller-given z-buffer (gsf_reproject_warp), through the C ABI: two calls in
a row, the second smaller, must give the same outputs bit for bit."""
import ctypes as ct

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"


def _case(w, h, ow, oh, seed):
    old = synth.look_at_camera([0.2, -0.1, -2.5], [0.0, 0.0, 0.0], w, h, 40.0)
    new = synth.look_at_camera([0.23, -0.09, -2.52], [0.03, 0.02, 0.0], ow, oh, 40.0)
    depth = synth.sphere_depth(old, radius=1.0)
    depth[::7, ::11] = 0.0
    rgba = np.random.default_rng(seed).uniform(size=(4, h, w)).astype(np.float32)
    P0, V0 = synth.clip_matrices(old)
    P1, V1 = synth.clip_matrices(new)
    return rgba, depth, (P0, V0, old.campos, P1, V1)


def test_noalloc_warp_equals_warp_with_caller_zbuf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_22026_amd as gs
    ctx = gs.Context(0)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for (w, h, ow, oh, seed) in [(512, 512, 512, 512, 1), (200, 150, 160, 120, 2)]:
            print(f"[no-alloc] warp {w}x{h} -> {ow}x{oh}", flush=True)
            rgba, depth, mats = _case(w, h, ow, oh, seed)
            c_dev = torch.from_numpy(rgba).to(DEV)
            d_dev = torch.from_numpy(depth).to(DEV)
            ref_out, ref_src = gs.reproject_warp(ctx, c_dev, d_dev, *mats, ow, oh)
            out = torch.full((4, oh, ow), float("nan"), dtype=torch.float32, device=DEV)
            src = torch.full((oh, ow), -7, dtype=torch.int32, device=DEV)
            gs.reproject_warp_noalloc(ctx, c_dev, d_dev, *mats, out, src)
            torch.cuda.synchronize()
            a, b = ref_out.cpu().numpy(), out.cpu().numpy()
            np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))
            np.testing.assert_array_equal(ref_src.cpu().numpy(), src.cpu().numpy())
            landed = int((src >= 0).sum().item())
            print(f"[no-alloc]   equal; landed {landed} of {ow * oh}", flush=True)
            assert landed > ow * oh // 4
        # an output beyond the device z-buffer is refused on the host
        one = torch.zeros(1, dtype=torch.float32, device=DEV)
        idx = torch.zeros(1, dtype=torch.int32, device=DEV)
        m = (ct.c_float * 16)(*np.eye(4, dtype=np.float32).reshape(-1))
        pos = (ct.c_float * 3)(0.0, 0.0, 0.0)
        st = gs.lib().gsf_reproject_warp_noalloc(
            ctx.handle, ct.c_void_p(one.data_ptr()), ct.c_void_p(one.data_ptr()), 1, 1, m, m, pos,
            m, m, 2048, 2305, ct.c_void_p(one.data_ptr()), ct.c_void_p(idx.data_ptr()))
        assert st == gs._abi.GSF_E_INVALID
        assert b"exceeds" in gs.lib().gsf_last_error(ctx.handle)
