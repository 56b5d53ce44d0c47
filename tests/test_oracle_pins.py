"""Pins of the FP64 oracle against facts fixed by the mathematics.

None of these compare the oracle with itself: each checks a closed form, an
invariant, a special case with a known answer, finite differences, an
independent autograd re-statement, or a library routine.
"""
import math

import numpy as np
import pytest

import oracle
import synth

C0 = 0.5 / math.sqrt(math.pi)


def _gaussian_planes(mu, logscale, quat, logit, rgb, sh_rest=None, deg=0):
    n = len(mu)
    P = np.zeros((synth.n_planes(deg), n), np.float64)
    P[0:3] = np.asarray(mu, np.float64).T
    P[3:6] = np.asarray(logscale, np.float64).T
    P[6:10] = np.asarray(quat, np.float64).T
    P[10] = logit
    P[11:14] = ((np.asarray(rgb, np.float64) - 0.5) / C0).T
    if sh_rest is not None:
        P[14:] = sh_rest
    return P.astype(np.float32).astype(np.float64)


def _pixel_centres(cam):
    jj, ii = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    return (ii + 0.5).reshape(-1), (jj + 0.5).reshape(-1)


def _logit(p):
    return math.log(p / (1 - p))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("scale,opac,bg", [(0.02, 0.7, (0, 0, 0)), (0.05, 0.995, (0.2, 0.3, 0.4)),
                                          (0.004, 0.3, (1, 1, 1))])
def test_isotropic_on_axis_footprint(scale, opac, bg):
    """Isotropic Gaussian on the optical axis: image = c a + bg (1 - a) with
    a = min(0.99, o exp(-r^2 / (2 s'^2))), s'^2 = (f s / z)^2 + 0.3, cut at 1/255."""
    cam = synth.axis_camera(64, 48, distance=3.0, bg=bg)
    rgb = (0.9, 0.5, 0.1)
    logit = float(np.float32(_logit(opac)))
    ls = float(np.float32(math.log(scale)))
    P = _gaussian_planes([[0, 0, 0]], [[ls] * 3], [[1, 0, 0, 0]], logit, [rgb])
    r = oracle.render(P, cam)
    s = math.exp(ls)
    o = 1 / (1 + math.exp(-logit))
    var = (cam.fx * s / 3.0) ** 2 + 0.3
    px, py = _pixel_centres(cam)
    rr = (px - cam.cx) ** 2 + (py - cam.cy) ** 2
    ae = o * np.exp(-rr / (2 * var))
    a = np.where(ae < 1 / 255, 0.0, np.minimum(0.99, ae))
    col = np.asarray(rgb, np.float64)[:, None].astype(np.float32).astype(np.float64)
    rgb_rec = (np.asarray(P[11:14, 0]) * C0 + 0.5)[:, None]
    expect = rgb_rec * a + cam.bg.astype(np.float64)[:, None] * (1 - a)
    assert np.allclose(col, rgb_rec, atol=1e-7)
    np.testing.assert_allclose(r.rgba[:3], expect, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(r.rgba[3], a, rtol=1e-12, atol=1e-13)
    assert (r.ncontrib == (a > 0)).all()


def test_rotated_anisotropic_footprint_general_camera():
    """Anisotropic rotated Gaussian at the look-at point of a rotated camera:
    Sigma' = (f / z)^2 (W Sigma W^T)_{xy} + 0.3 I (up to the float32 rounding of
    the camera translation, ~1e-7)."""
    cam = synth.look_at_camera([1.2, -2.0, 2.1], width=80, height=60)
    q = np.array([0.8, 0.3, -0.4, 0.2])
    q /= np.linalg.norm(q)
    ls = np.log([0.06, 0.02, 0.03])
    P = _gaussian_planes([[0, 0, 0]], [ls], [q], _logit(0.8), [(0.3, 0.6, 0.9)])
    r = oracle.render(P, cam)
    # closed form with numpy linear algebra (rotation from the Euler-Rodrigues formula)
    qq = P[6:10, 0] / np.linalg.norm(P[6:10, 0])
    w, x, y, z = qq
    K = np.array([[0, -z, y], [z, 0, -x], [-y, x, 0]])
    Rg = np.eye(3) + 2 * w * K + 2 * K @ K
    S = Rg @ np.diag(np.exp(P[3:6, 0]) ** 2) @ Rg.T
    W = cam.R.astype(np.float64)
    dist = np.linalg.norm(cam.campos.astype(np.float64))
    Sp = (cam.fx / dist) ** 2 * (W @ S @ W.T)[:2, :2] + 0.3 * np.eye(2)
    Q = np.linalg.inv(Sp)
    px, py = _pixel_centres(cam)
    d = np.stack([px - cam.cx, py - cam.cy])
    power = -0.5 * np.einsum("ip,ij,jp->p", d, Q, d)
    o = 1 / (1 + np.exp(-P[10, 0]))
    ae = o * np.exp(power)
    a = np.where(ae < 1 / 255, 0.0, np.minimum(0.99, ae))
    col = P[11:14, 0] * C0 + 0.5
    keep = np.abs(ae * 255 - 1) > 1e-3
    np.testing.assert_allclose(r.rgba[3][keep], a[keep], atol=2e-5)
    np.testing.assert_allclose(r.rgba[:3][:, keep], (col[:, None] * a)[:, keep], atol=2e-5)
    assert a.max() > 0.5


# ---------------------------------------------------------------- invariants

def test_transmittance_invariant_white_scene():
    """With every colour 1 and bg 0, RGB = A = sum_i a_i T_i = 1 - T_final, and
    with bg 1 as well the image is exactly white."""
    P = synth.random_gaussians(300, seed=11).astype(np.float64)
    P[11:14] = 0.5 / C0
    cam = synth.axis_camera(64, 64)
    r = oracle.render(P, cam)
    for c in range(3):
        np.testing.assert_allclose(r.rgba[c], r.rgba[3], atol=1e-12)
    np.testing.assert_allclose(1 - r.rgba[3], r.tfinal, atol=1e-15)
    cam1 = synth.axis_camera(64, 64, bg=(1, 1, 1))
    r1 = oracle.render(P, cam1)
    np.testing.assert_allclose(r1.rgba[:3], 1.0, atol=1e-12)
    assert r.rgba[3].max() > 0.9   # the scene is not trivially empty


def test_transmittance_product_matches_contributors():
    """1 - A = prod over included Gaussians of (1 - alpha_i), recomputed from the
    projection records for a few pixels."""
    P = synth.random_gaussians(200, seed=5).astype(np.float64)
    cam = synth.axis_camera(32, 32)
    rec = oracle.project(P, cam)
    pix = np.array([0, 100, 528, 700, 1023])
    r = oracle.render(P, cam, pixels=pix)
    order = sorted([i for i in range(P.shape[1]) if rec["valid"][i]],
                   key=lambda i: (np.float32(rec["tz"][i]).view(np.uint32), i))
    for k, p in enumerate(pix):
        px, py = p % 32 + 0.5, p // 32 + 0.5
        T, prod, n = 1.0, 1.0, 0
        for i in order:
            dx, dy = px - rec["mx"][i], py - rec["my"][i]
            pw = -0.5 * (rec["A"][i] * dx * dx + rec["C"][i] * dy * dy) - rec["B"][i] * dx * dy
            if pw > 0:
                continue
            a = min(0.99, rec["o"][i] * math.exp(pw))
            if a < 1 / 255:
                continue
            if T * (1 - a) < 1e-4:
                break
            T *= 1 - a
            prod *= 1 - a
            n += 1
        assert n == r.ncontrib[k]
        assert abs((1 - r.rgba[3, k]) - prod) < 1e-14


def _alpha_at(rec, i, px, py):
    dx, dy = px - rec["mx"][i], py - rec["my"][i]
    pw = -0.5 * (rec["A"][i] * dx * dx + rec["C"][i] * dy * dy) - rec["B"][i] * dx * dy
    return min(0.99, rec["o"][i] * math.exp(pw))


def test_depth_order_two_gaussians():
    """Two equal Gaussians at depths z1 < z2: C = c1 a1 + c2 a2 (1 - a1); swapping
    the depths swaps the roles."""
    cam = synth.axis_camera(34, 34)
    c1, c2 = (0.9, 0.1, 0.1), (0.1, 0.1, 0.9)
    ls = [[math.log(0.05)] * 3] * 2
    quat = [[1, 0, 0, 0]] * 2
    P = _gaussian_planes([[0, 0, -0.5], [0, 0, 0.5]], ls, quat, _logit(0.6), [c1, c2])
    centre = np.array([16 * 34 + 16])
    cc1 = P[11:14, 0] * C0 + 0.5
    cc2 = P[11:14, 1] * C0 + 0.5
    r = oracle.render(P, cam, pixels=centre)
    rec = oracle.project(P, cam)
    a1, a2 = _alpha_at(rec, 0, 16.5, 16.5), _alpha_at(rec, 1, 16.5, 16.5)
    assert 0.05 < a2 < a1 < 0.6
    np.testing.assert_allclose(r.rgba[:3, 0], cc1 * a1 + cc2 * a2 * (1 - a1), atol=1e-14)
    # swap the depths: the second Gaussian is now in front
    P2 = P.copy()
    P2[2, 0], P2[2, 1] = P[2, 1], P[2, 0]
    r2 = oracle.render(P2, cam, pixels=centre)
    rec2 = oracle.project(P2, cam)
    b0, b1 = _alpha_at(rec2, 0, 16.5, 16.5), _alpha_at(rec2, 1, 16.5, 16.5)
    assert abs(b1 - a1) < 1e-12 and abs(b0 - a2) < 1e-12
    np.testing.assert_allclose(r2.rgba[:3, 0], cc2 * b1 + cc1 * b0 * (1 - b1), atol=1e-14)
    assert r.last[0] == 1 and r2.last[0] == 0


def test_early_stop_alpha_08_stack():
    """Identical-alpha stack with a = 0.8 at the centre pixel (the pixel centre sits
    on the projected means): 0.2^5 >= 1e-4 > 0.2^6, so exactly five Gaussians are
    included."""
    cam = synth.axis_camera(17, 17)
    n = 8
    zs = [float(np.float32(z)) for z in np.linspace(-0.4, 0.4, n)]
    ls = float(np.float32(math.log(0.08)))
    P = _gaussian_planes([[0.0, 0.0, z] for z in zs], [[ls] * 3] * n, [[1, 0, 0, 0]] * n, 0.0,
                         [(1, 1, 1)] * n)
    P[10] = math.log(0.8 / 0.2)                 # float64 logit: alpha = 0.8 to 1e-16
    r = oracle.render(P, cam, pixels=np.array([8 * 17 + 8]))
    assert r.ncontrib[0] == 5
    np.testing.assert_allclose(r.rgba[3, 0], 1 - 0.2 ** 5, rtol=1e-12)
    assert r.last[0] == 4
    # one Gaussian fewer in front changes nothing about the count rule
    r6 = oracle.render(P[:, :6], cam, pixels=np.array([8 * 17 + 8]))
    assert r6.ncontrib[0] == 5


def test_skip_below_1_over_255():
    """A Gaussian whose alpha at a pixel is just below 1/255 leaves it untouched."""
    cam = synth.axis_camera(9, 9)
    P = _gaussian_planes([[0, 0, 0]], [[math.log(0.02)] * 3], [[1, 0, 0, 0]], 0.0, [(1, 1, 1)])
    rec = oracle.project(P, cam)
    var_inv = rec["A"][0]
    o = rec["o"][0]
    r = oracle.render(P, cam)
    px, py = _pixel_centres(cam)
    ae = o * np.exp(-0.5 * var_inv * ((px - 4.5) ** 2 + (py - 4.5) ** 2))
    assert ((ae < 1 / 255) == (r.rgba[3] == 0)).all()
    assert (ae < 1 / 255).any() and (ae >= 1 / 255).any()


# ---------------------------------------------------------------- SH basis

def _real_sh_scipy(deg, dirs):
    from scipy.special import sph_harm_y
    x, y, z = dirs.T
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.mod(np.arctan2(y, x), 2 * np.pi)
    out = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            Yc = sph_harm_y(l, abs(m), theta, phi)
            if m < 0:
                out.append(math.sqrt(2) * Yc.imag)
            elif m == 0:
                out.append(Yc.real)
            else:
                out.append(math.sqrt(2) * Yc.real)
    return np.stack(out, axis=1)


def test_sh_basis_matches_scipy_real_harmonics():
    """Real SH (Condon-Shortley phase kept, k = l^2 + l + m) equal scipy's complex
    harmonics combined into real form."""
    d = np.random.default_rng(0).normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    np.testing.assert_allclose(oracle.sh_basis(3, d), _real_sh_scipy(3, d), atol=1e-13)


def test_sh_basis_orthonormal_by_quadrature():
    """int Y_j Y_k d omega = delta_jk (Gauss-Legendre in cos(theta) x uniform phi)."""
    nt, nphi = 24, 48
    xg, wg = np.polynomial.legendre.leggauss(nt)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    Y = oracle.sh_basis(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


# ---------------------------------------------------------------- gradients

def _tiny_scene(seed, n=6, deg=0, size=16, bg=(0.1, 0.2, 0.3)):
    rng = np.random.default_rng(seed)
    P = np.zeros((synth.n_planes(deg), n))
    P[0:3] = rng.uniform(-0.6, 0.6, size=(3, n))
    P[3:6] = rng.normal(-1.3, 0.3, size=(3, n))
    q = rng.normal(size=(4, n))
    P[6:10] = q / np.linalg.norm(q, axis=0)
    P[10] = rng.normal(0.5, 1.0, size=n)
    P[11:14] = (rng.uniform(0.1, 0.9, size=(3, n)) - 0.5) / C0
    if deg > 0:
        P[14:] = rng.normal(0, 0.1, size=P[14:].shape)
    P = P.astype(np.float32).astype(np.float64)
    cam = synth.look_at_camera(3.0 * np.array([0.3, -0.2, 0.93]) / np.linalg.norm([0.3, -0.2, 0.93]),
                               width=size, height=size, bg=bg)
    return P, cam


def _clean_scenes(count, **kw):
    out, seed = [], 0
    while len(out) < count:
        P, cam = _tiny_scene(seed, **kw)
        r = oracle.render(P, cam)
        rec = oracle.project(P, cam)
        if not r.flags.any() and not rec["flags"].any() and r.ncontrib.sum() > 20:
            out.append((seed, P, cam))
        seed += 1
        assert seed < 200
    return out


@pytest.mark.parametrize("deg", [0, 3])
def test_adjoint_matches_central_differences(deg):
    """Analytic FP64 adjoint vs central differences (h = 1e-6 max(1, |x|)) of
    L = sum w * RGBA on tiny scenes with no near-threshold pair."""
    for seed, P, cam in _clean_scenes(2, deg=deg):
        w = np.random.default_rng(100 + seed).normal(size=(4, cam.npix))
        G = oracle.backward(P, cam, w)

        def L(Pp):
            return float(np.sum(oracle.render(Pp, cam).rgba * w))

        fd = np.zeros_like(P)
        for c in range(P.shape[0]):
            for i in range(P.shape[1]):
                h = 1e-6 * max(1.0, abs(P[c, i]))
                Pp, Pm = P.copy(), P.copy()
                Pp[c, i] += h
                Pm[c, i] -= h
                fd[c, i] = (L(Pp) - L(Pm)) / (2 * h)
        scale = np.abs(G).max()
        assert scale > 1e-3
        np.testing.assert_allclose(G, fd, rtol=1e-5, atol=1e-7 * scale)


def test_adjoint_through_jacobian_and_alpha_clamps():
    """A Gaussian beyond the 1.3 tan(fov/2) Jacobian clamp whose footprint still
    reaches the image, and one saturating the 0.99 alpha clamp: FD still agrees."""
    cam = synth.axis_camera(24, 24, bg=(0.5, 0.5, 0.5))
    # tan(30 deg) * 1.3 * 3 = 2.25 world units off axis at depth 3
    mus = [[2.5, 0.1, 0.0], [0.05, -0.1, 0.3], [-0.2, 0.15, -0.2]]
    ls = [[0.0, -0.3, -0.2], [-1.2, -1.0, -1.4], [-1.6, -1.5, -1.3]]
    quat = [[0.9, 0.1, 0.2, 0.1], [0.7, -0.2, 0.1, 0.3], [1, 0, 0, 0]]
    P = _gaussian_planes(mus, ls, quat, 0.0, [(0.8, 0.2, 0.3), (0.1, 0.7, 0.2), (0.3, 0.3, 0.9)])
    P[10] = [1.0, 7.0, 0.3]
    r = oracle.render(P, cam)
    rec = oracle.project(P, cam)
    assert abs(rec["tx"][0] / rec["tz"][0]) > 1.3 * cam.tanx
    assert not r.flags.any() and not rec["flags"].any()
    w = np.random.default_rng(3).normal(size=(4, cam.npix))
    G = oracle.backward(P, cam, w)

    def L(Pp):
        return float(np.sum(oracle.render(Pp, cam).rgba * w))

    fd = np.zeros_like(P)
    for c in range(P.shape[0]):
        for i in range(P.shape[1]):
            h = 1e-6 * max(1.0, abs(P[c, i]))
            Pp, Pm = P.copy(), P.copy()
            Pp[c, i] += h
            Pm[c, i] -= h
            fd[c, i] = (L(Pp) - L(Pm)) / (2 * h)
    np.testing.assert_allclose(G, fd, rtol=1e-5, atol=1e-7 * np.abs(G).max())
    assert np.abs(G[:, 0]).max() > 1e-4    # the clamped Gaussian does get gradient


def _torch_render(P, cam, order):
    """Differentiable float64 re-statement of the forward map for tiny scenes."""
    import torch
    t = torch
    n = P.shape[1]
    deg = oracle.sh_degree_of(P.detach().numpy())
    mu, s = P[0:3], t.exp(P[3:6])
    q = P[6:10] / t.linalg.norm(P[6:10], dim=0, keepdim=True)
    w, x, y, z = q
    Rg = t.stack([t.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
                  t.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
                  t.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)])])
    Rg = Rg.permute(2, 0, 1)                                   # [n,3,3]
    Sig = Rg @ t.diag_embed(s.T ** 2) @ Rg.transpose(1, 2)
    W = t.tensor(cam.R, dtype=t.float64)
    tv = t.tensor(cam.t, dtype=t.float64)
    tc = (W @ mu).T + tv                                       # [n,3]
    tz = tc[:, 2]
    limx, limy = 1.3 * cam.tanx, 1.3 * cam.tany
    txc = tz * t.clamp(tc[:, 0] / tz, -limx, limx)
    tyc = tz * t.clamp(tc[:, 1] / tz, -limy, limy)
    zero = t.zeros_like(tz)
    J = t.stack([t.stack([cam.fx / tz, zero, -cam.fx * txc / tz ** 2]),
                 t.stack([zero, cam.fy / tz, -cam.fy * tyc / tz ** 2])]).permute(2, 0, 1)
    M = J @ W
    Sp = M @ Sig @ M.transpose(1, 2) + 0.3 * t.eye(2, dtype=t.float64)
    Q = t.linalg.inv(Sp)
    mx = cam.fx * tc[:, 0] / tz + cam.cx
    my = cam.fy * tc[:, 1] / tz + cam.cy
    o = t.sigmoid(P[10])
    u = mu.T - t.tensor(cam.campos, dtype=t.float64)
    d = u / t.linalg.norm(u, dim=1, keepdim=True)
    dx_, dy_, dz_ = d.T
    Y = _torch_sh(deg, dx_, dy_, dz_)                          # [K][n]
    K = (deg + 1) ** 2
    sh = P[11:11 + 3 * K].reshape(K, 3, n)
    col = t.clamp(t.einsum("kcn,kn->cn", sh, Y) + 0.5, min=0.0)
    jj, ii = np.meshgrid(np.arange(cam.height), np.arange(cam.width), indexing="ij")
    px = t.tensor(ii.reshape(-1) + 0.5, dtype=t.float64)
    py = t.tensor(jj.reshape(-1) + 0.5, dtype=t.float64)
    T = t.ones_like(px)
    C = t.zeros(3, px.shape[0], dtype=t.float64)
    active = t.ones_like(px, dtype=t.bool)
    for i in order:
        ddx, ddy = px - mx[i], py - my[i]
        pw = -0.5 * (Q[i, 0, 0] * ddx * ddx + Q[i, 1, 1] * ddy * ddy) - Q[i, 0, 1] * ddx * ddy
        ae = o[i] * t.exp(pw)
        a = t.clamp(ae, max=0.99)
        skip = (pw > 0) | (ae < 1 / 255)
        Tn = T * (1 - a)
        stop = active & ~skip & (Tn < 1e-4)
        inc = active & ~skip & ~stop
        C = C + t.where(inc, col[:, i:i + 1] * a * T, t.zeros_like(C))
        T = t.where(inc, Tn, T)
        active = active & ~stop
    bg = t.tensor(cam.bg, dtype=t.float64)[:, None]
    return t.cat([C + T * bg, (1 - T)[None]], 0)


def _torch_sh(deg, x, y, z):
    import torch
    pi = math.pi
    out = [torch.full_like(x, 0.5 / math.sqrt(pi))]
    if deg >= 1:
        c1 = math.sqrt(3 / (4 * pi))
        out += [-c1 * y, c1 * z, -c1 * x]
    if deg >= 2:
        a, b, c = 0.5 * math.sqrt(15 / pi), 0.25 * math.sqrt(5 / pi), 0.25 * math.sqrt(15 / pi)
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, c * (x * x - y * y)]
    if deg >= 3:
        c33, c32 = 0.25 * math.sqrt(35 / (2 * pi)), 0.5 * math.sqrt(105 / pi)
        c31, c30, c32b = 0.25 * math.sqrt(21 / (2 * pi)), 0.25 * math.sqrt(7 / pi), 0.25 * math.sqrt(105 / pi)
        out += [-c33 * y * (3 * x * x - y * y), c32 * x * y * z, -c31 * y * (4 * z * z - x * x - y * y),
                c30 * z * (2 * z * z - 3 * x * x - 3 * y * y), -c31 * x * (4 * z * z - x * x - y * y),
                c32b * z * (x * x - y * y), -c33 * x * (x * x - 3 * y * y)]
    return torch.stack(out)


@pytest.mark.parametrize("deg", [0, 3])
def test_adjoint_matches_torch_autograd(deg):
    """The analytic adjoint equals float64 autograd through an independent torch
    re-statement of the forward map (1e-10)."""
    import torch
    for seed, P, cam in _clean_scenes(2, deg=deg):
        rec = oracle.project(P, cam)
        order = sorted([i for i in range(P.shape[1]) if rec["valid"][i]],
                       key=lambda i: (np.float32(rec["tz"][i]).view(np.uint32), i))
        Pt = torch.tensor(P, dtype=torch.float64, requires_grad=True)
        img = _torch_render(Pt, cam, order)
        np.testing.assert_allclose(img.detach().numpy(), oracle.render(P, cam).rgba, atol=1e-12)
        w = np.random.default_rng(7 + seed).normal(size=(4, cam.npix))
        (img * torch.tensor(w)).sum().backward()
        G = oracle.backward(P, cam, w)
        np.testing.assert_allclose(G, Pt.grad.numpy(), rtol=1e-10, atol=1e-12 * np.abs(G).max())


def test_backward_pixel_subset_equals_masked_full():
    """Backward over a pixel subset equals the full backward with dl zero elsewhere."""
    P = synth.random_gaussians(200, seed=9).astype(np.float64)
    cam = synth.axis_camera(40, 40)
    rng = np.random.default_rng(1)
    pix = np.sort(rng.choice(cam.npix, 150, replace=False))
    dl_sub = rng.normal(size=(4, pix.size))
    dl_full = np.zeros((4, cam.npix))
    dl_full[:, pix] = dl_sub
    G1 = oracle.backward(P, cam, dl_sub, pixels=pix)
    G2 = oracle.backward(P, cam, dl_full)
    np.testing.assert_allclose(G1, G2, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- discrete stage

def test_discrete_stage_is_conservative_sorted_and_ranged():
    """Every pixel with alpha >= 1/255 for Gaussian i lies in a tile listed for i;
    keys ascend by (tile, depth, record); ranges are lower bounds."""
    P = synth.random_gaussians(400, seed=2).astype(np.float64)
    cams = [synth.axis_camera(48, 40), synth.look_at_camera([0, 3, 0.3], width=37, height=29)]
    for T in (8, 16, 32):
        d = oracle.discrete(P, cams, T)
        tile_base = 0
        listed = {}
        for k, v in zip(d.keys, d.vals):
            listed.setdefault(int(v), set()).add(int(k))
        for vi, cam in enumerate(cams):
            rec = oracle.project(P, cam)
            tw = (cam.width + T - 1) // T
            px, py = _pixel_centres(cam)
            for i in range(P.shape[1]):
                if not rec["valid"][i]:
                    continue
                dx, dy = px - rec["mx"][i], py - rec["my"][i]
                pw = -0.5 * (rec["A"][i] * dx * dx + rec["C"][i] * dy * dy) - rec["B"][i] * dx * dy
                hit = (pw <= 0) & (rec["o"][i] * np.exp(pw) >= 1 / 255)
                need = {tile_base + int(y) // T * tw + int(x) // T
                        for x, y in zip(px[hit] - 0.5, py[hit] - 0.5)}
                assert need <= listed.get(vi * P.shape[1] + i, set())
            tile_base += tw * ((cam.height + T - 1) // T)
        # ordering by (tile, depth bits, record)
        n = P.shape[1]
        dep = {}
        for vi, cam in enumerate(cams):
            tz = oracle.project(P, cam)["tz"]
            for i in range(n):
                dep[vi * n + i] = int(np.float32(tz[i]).view(np.uint32))
        tup = [(int(k), dep[int(v)], int(v)) for k, v in zip(d.keys, d.vals)]
        assert tup == sorted(tup)
        lo = np.searchsorted(d.keys, np.arange(tile_base), side="left")
        hi = np.searchsorted(d.keys, np.arange(tile_base), side="right")
        np.testing.assert_array_equal(d.ranges[:, 0], lo)
        np.testing.assert_array_equal(d.ranges[:, 1], hi)


def _tile_span(e0, e1, size, T):
    lo, hi = max(0, math.ceil(e0)), min(size - 1, math.floor(e1))
    return (lo // T, hi // T) if lo <= hi else None


def _band_columns(rec, i, ty, T, W, H, cols, nsamp=20001):
    """Brute force of one tile row's list: the tile columns whose pixel-centre
    columns lie within 1/64 px of the x extent of the padded support ellipse
    A x^2 + 2 B x y + C y^2 <= 2 ln(255 o) (1 + 1e-4)^2 over the row's band of
    pixel-centre rows (clamped to the ellipse's rows).  The extent is the
    max / min of the ellipse's chord ends, solved from the conic at nsamp
    evenly spaced band offsets.  Returns ((c0, c1) or None, distance of the
    nearest pixel-centre column threshold from either end of the extent)."""
    A, B, C = rec["A"][i], rec["B"][i], rec["C"][i]
    mx, my = rec["mx"][i], rec["my"][i]
    Kp = 2.0 * math.log(255.0 * rec["o"][i]) * (1.0 + 1e-4) ** 2
    ey = math.sqrt(A * Kp / (A * C - B * B))
    ja, jb = ty * T, min(ty * T + T, H) - 1
    ya, yb = ja + 0.5 - my, jb + 0.5 - my
    lo, hi = max(ya, -ey), min(yb, ey)
    if lo > hi:
        lo = hi = ey if ya > ey else -ey
    d = np.linspace(lo, hi, nsamp)
    root = np.sqrt(np.maximum(B * B * d * d - A * (C * d * d - Kp), 0.0))
    xr = ((-B * d + root) / A).max() + 1.0 / 64
    xl = ((-B * d - root) / A).min() - 1.0 / 64
    ul, ur = mx + xl - 0.5, mx + xr - 0.5          # column i is in when ul <= i <= ur
    margin = min(abs(ul - round(ul)), abs(ur - round(ur)))
    a, b = max(math.ceil(ul), 0), min(math.floor(ur), W - 1)
    if a > b:
        return None, margin
    c0, c1 = max(a // T, cols[0]), min(b // T, cols[1])
    return ((c0, c1) if c0 <= c1 else None), margin


@pytest.mark.parametrize("T", [8, 16, 32])
def test_tile_lists_equal_brute_force_band_extents(T):
    """Every record's listed tiles, row by row, equal the brute-force band
    extents of its padded support ellipse, for boxes of every height: a 512^2
    view holding large near splats whose boxes are tens of tile rows tall, and
    an oblique view of the same set.  Rows whose extent ends within 1e-4 px of a
    pixel-centre column (where sampling can decide either way) are skipped and
    counted."""
    P = synth.with_near_splats(synth.random_gaussians(150, seed=11), 8, seed=11).astype(np.float64)
    cams = [synth.axis_camera(512, 512), synth.look_at_camera([1.2, -0.8, -2.6], width=480,
                                                               height=400)]
    d = oracle.discrete(P, cams, T)
    n = P.shape[1]
    listed = {}
    for k, v in zip(d.keys, d.vals):
        listed.setdefault(int(v), set()).add(int(k))
    tile_base, tallest, rows, skipped = 0, 0, 0, 0
    for vi, cam in enumerate(cams):
        rec = oracle.project(P, cam)
        W, H = cam.width, cam.height
        tw = (W + T - 1) // T
        for i in range(n):
            r = vi * n + i
            if not rec["valid"][i] or d.rflags[r] & oracle.F_NEAR_BOX:
                continue
            cs = _tile_span(rec["ex0"][i], rec["ex1"][i], W, T)
            rs = _tile_span(rec["ey0"][i], rec["ey1"][i], H, T)
            if cs is None or rs is None:
                assert r not in listed
                continue
            tallest = max(tallest, rs[1] - rs[0] + 1)
            got = listed.get(r, set())
            for ty in range(rs[0], rs[1] + 1):
                want, margin = _band_columns(rec, i, ty, T, W, H, cs)
                row = {t - tile_base - ty * tw for t in got if (t - tile_base) // tw == ty}
                if margin < 1e-4:
                    skipped += 1
                    continue
                rows += 1
                expect = set() if want is None else set(range(want[0], want[1] + 1))
                assert row == expect, (vi, i, ty, sorted(row), want)
            assert all(rs[0] <= (t - tile_base) // tw <= rs[1] for t in got)
        tile_base += tw * ((H + T - 1) // T)
    assert tallest > 32 if T == 8 else tallest > 8
    assert skipped <= 0.01 * rows, (skipped, rows)


# ---------------------------------------------------------------- loss and Adam

def test_l1_loss_and_sign_gradient():
    rng = np.random.default_rng(0)
    cam = synth.axis_camera(20, 10)
    rgba = rng.uniform(size=(4, cam.npix))
    tgt = rng.uniform(size=(3, cam.npix))
    tgt[:, :5] = rgba[:3, :5]             # exact ties give zero gradient
    loss, dls = oracle.loss_l1([rgba], [tgt], [cam])
    assert abs(loss - np.mean(np.abs(rgba[:3] - tgt))) < 1e-14
    np.testing.assert_array_equal(dls[0][:3], np.sign(rgba[:3] - tgt) / (3 * cam.npix))
    assert (dls[0][3] == 0).all() and (dls[0][:, :5] == 0).all()
    # fovea mask: pixel centres within the radius of the gaze point (inclusive)
    g = np.array([[7.5, 4.5]])
    loss_m, dlm = oracle.loss_l1([rgba], [tgt], [cam], gazes=g, radius_frac=0.15)
    px, py = _pixel_centres(cam)
    m = (px - 7.5) ** 2 + (py - 4.5) ** 2 <= (0.15 * 20) ** 2
    assert abs(loss_m - np.mean(np.abs(rgba[:3, m] - tgt[:, m]))) < 1e-14
    assert (dlm[0][:, ~m] == 0).all()


def test_fovea_mask_counts_the_lattice_points_of_the_disk():
    """Gaze on a pixel centre and an integer radius: the mask holds the
    integer points of a closed disk, whose number the Gauss circle problem
    gives as 1 + 4 floor(r) + 4 sum_{i=1}^{floor(r)} floor(sqrt(r^2 - i^2));
    known values N(1..10) = 5, 13, 29, 49, 81, 113, 149, 197, 253, 317."""
    known = [5, 13, 29, 49, 81, 113, 149, 197, 253, 317]
    cam = synth.axis_camera(64, 64)
    z, t = np.zeros((4, cam.npix)), np.ones((3, cam.npix))
    for r, n in zip(range(1, 11), known):
        closed = 1 + 4 * r + 4 * sum(int(np.floor(np.sqrt(r * r - i * i))) for i in range(1, r + 1))
        assert closed == n
        _, cnt, _ = oracle.loss_l1_view(z, t, cam, np.array([32.5, 31.5]),
                                        oracle.fovea_radius(r / 64, 64))
        assert cnt == 3 * n, (r, cnt)


def test_rgba_loss_reduces_to_rgb_loss_and_hand_values():
    rng = np.random.default_rng(3)
    cam = synth.axis_camera(12, 9)
    rgba = rng.uniform(size=(4, cam.npix))
    tgt = rng.uniform(size=(4, cam.npix))
    # black background, no alpha term: the RGB loss
    L0, d0 = oracle.loss_l1([rgba], [tgt[:3]], [cam])
    L1, d1 = oracle.loss_l1_rgba([rgba], [tgt], [cam], bgs=None, alpha=False)
    assert abs(L0 - L1) < 1e-15
    np.testing.assert_array_equal(d0[0], d1[0])
    # one pixel by hand: target (0.3, 0.1, 0.2, A 0.5) over bg (1, 0.5, 0) is
    # (0.8, 0.35, 0.2); prediction (0.5, 0.2, 0.9, 0.6)
    one = synth.axis_camera(1, 1)
    L, d = oracle.loss_l1_rgba([np.array([0.5, 0.2, 0.9, 0.6])], [np.array([0.3, 0.1, 0.2, 0.5])],
                               [one], bgs=[np.array([1.0, 0.5, 0.0])], alpha=True)
    assert abs(L - (0.3 + 0.15 + 0.7 + 0.1) / 4) < 1e-15
    np.testing.assert_array_equal(d[0][:, 0], np.array([-1.0, -1.0, 1.0, 1.0]) / 4)


def test_target_over_background_is_the_renderers_own_compositing():
    """Rendering a scene over bg equals its render over black composited as
    target_rgb + (1 - target_alpha) bg - the rule the RGBA loss applies to
    the target - so a model that reproduces the target over black reproduces
    it over every background."""
    P = synth.random_gaussians(40, seed=4)
    bg = (0.7, 0.2, 0.4)
    black = synth.axis_camera(24, 20)
    coloured = synth.axis_camera(24, 20, bg=bg)
    r0 = oracle.render(P, black)
    r1 = oracle.render(P, coloured)
    over = r0.rgba[:3] + (1.0 - r0.rgba[3]) * coloured.bg.astype(np.float64)[:, None]
    np.testing.assert_allclose(r1.rgba[:3], over, rtol=0, atol=1e-12)
    L, _ = oracle.loss_l1_rgba([r1.rgba], [r0.rgba], [coloured], bgs=[coloured.bg], alpha=True)
    assert L < 1e-12


def test_splitmix64_published_first_output_and_background_range():
    # first output of SplitMix64 from state 0, as published with the generator
    assert oracle.splitmix64(0, 1) == 0xE220A8397B1DCDAF
    bg = oracle.background_draw(7, 3, 5)
    assert bg.shape == (5, 3) and (bg >= 0).all() and (bg < 1).all()
    assert (bg.astype(np.float32).astype(np.float64) == bg).all()
    assert not np.array_equal(bg, oracle.background_draw(7, 4, 5))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    p0 = p.copy()
    m, v = np.zeros(100), np.zeros(100)
    oracle.adam(p, g, m, v, 1, lr=1e-3)
    np.testing.assert_allclose(p - p0, -1e-3 * g / (np.abs(g) + 1e-15), rtol=1e-12)


def test_adam_matches_torch_optim_float64():
    import torch
    rng = np.random.default_rng(1)
    p = rng.normal(size=64)
    m, v = np.zeros(64), np.zeros(64)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=2e-3, betas=(0.9, 0.999), eps=1e-15)
    for step in range(1, 11):
        g = rng.normal(size=64)
        oracle.adam(p, g, m, v, step, lr=2e-3)
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_per_segment_learning_rate():
    rng = np.random.default_rng(2)
    p = rng.normal(size=30)
    g = rng.normal(size=30)
    lr = np.repeat([1e-3, 1.5e-3, 3e-3], 10)
    m, v = np.zeros(30), np.zeros(30)
    p0 = p.copy()
    oracle.adam(p, g, m, v, 1, lr=lr)
    np.testing.assert_allclose(p - p0, -lr * np.sign(g), rtol=1e-12)


def test_discrete_stage_lists_only_tiles_the_ellipse_reaches():
    """A thin splat along the image diagonal: its box spans many tiles, but only
    the tiles near the diagonal are listed, and each listed tile's band of pixel
    centres (widened by one pixel) meets the padded support ellipse."""
    P = synth.random_gaussians(1, seed=3).astype(np.float64)
    P[0:3, 0] = [0.0, 0.0, 0.0]
    P[3:6, 0] = [np.log(0.6), np.log(0.01), np.log(0.01)]       # long along x
    c, s = np.cos(np.pi / 8), np.sin(np.pi / 8)                   # 45 degrees about z
    P[6:10, 0] = [c, 0.0, 0.0, s]
    P[10, 0] = 3.0
    cam = synth.axis_camera(128, 128)
    T = 8
    d = oracle.discrete(P, [cam], T)
    rec = oracle.project(P, cam)
    assert rec["valid"][0] and d.rflags[0] == 0
    tw = 128 // T
    x0, x1 = int(max(0, np.ceil(rec["ex0"][0]))) // T, int(min(127, np.floor(rec["ex1"][0]))) // T
    y0, y1 = int(max(0, np.ceil(rec["ey0"][0]))) // T, int(min(127, np.floor(rec["ey1"][0]))) // T
    area = (x1 - x0 + 1) * (y1 - y0 + 1)
    assert d.m < 0.5 * area, (d.m, area)
    Kp = 2 * np.log(255 * rec["o"][0]) * (1 + 1e-4) ** 2
    for t in d.keys:
        ty, tx = divmod(int(t), tw)
        xs = np.linspace(tx * T - 1.0, tx * T + T, 64) + 0.5 - rec["mx"][0]
        ys = np.linspace(ty * T, ty * T + T - 1, 32) + 0.5 - rec["my"][0]
        X, Y = np.meshgrid(xs, ys)
        q = rec["A"][0] * X * X + 2 * rec["B"][0] * X * Y + rec["C"][0] * Y * Y
        assert q.min() <= Kp, (tx, ty)
