"""CPU pins of the feature-pass adjoint oracle (oracle/feature_adjoint.py) and of the oracle
render's reverse mode with respect to the feature values:
  * the matrix-form forward equals the loop-form C oracle (g, k, V, gmax, H at the first scale);
  * each matrix is the clamped operator of its definition (a ramp, a constant, an impulse);
  * the adjoint equals FP64 central differences of the C oracle's forward, along a random
    direction and voxel by voxel (corners, faces, interior);
  * dL/d(g, k, V, gmax) of the render equal central differences of the C oracle's render;
  * end to end, dL/dI through the TF lookup plus through the features equals central differences
    of render(I, features(I))."""
import numpy as np
import pytest

import oracle
import phantoms
from oracle import feature_adjoint as fa

SP = (1.0, 0.8, 1.3)
SIGMAS = [0.9, 1.5]
FR = dict(alpha=0.5, beta=0.5, c=0.08)


def _tube_volume(shape, seed):
    """A bright tilted tube plus a blob and noise: V > 0 on many voxels, |g| with a unique max."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) * SP[2], np.arange(ny) * SP[1], np.arange(nx) * SP[0], indexing="ij")
    c = np.array([(nx - 1) * SP[0], (ny - 1) * SP[1], (nz - 1) * SP[2]]) / 2
    d = np.array([0.9, 0.3, 0.3])
    d /= np.linalg.norm(d)
    p = np.stack([x - c[0], y - c[1], z - c[2]], -1)
    r2 = (p * p).sum(-1) - (p @ d) ** 2
    vol = 0.7 * np.exp(-r2 / (2 * 1.3 ** 2)) + 0.3 * np.exp(-((x - 1) ** 2 + (y - 2) ** 2 + (z - 1.5) ** 2) / 3.0)
    return vol + rng.normal(0, 0.02, shape)


def _loss_features(I, gb, kb, Vb, gmb):
    f = oracle.features(I, SP, SIGMAS, **FR)
    return float((gb * f["g"]).sum() + (kb * f["kappa"]).sum() + (Vb * f["V"]).sum() + gmb * f["gmax"])


def _upstream(shape, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(3,) + shape), rng.normal(size=shape), rng.normal(size=shape) * 5.0, 0.7)


def test_matrix_forward_matches_loop_oracle():
    I = _tube_volume((9, 11, 13), 3)
    f = oracle.features(I, SP, SIGMAS, want_H0=True, **FR)
    m = fa.forward(I, SP, SIGMAS, **FR)
    for k in ("g", "kappa", "V"):
        np.testing.assert_allclose(m[k], f[k], rtol=0, atol=1e-12 * max(np.abs(f[k]).max(), 1e-300))
    np.testing.assert_allclose(m["H"][0], f["H0"], rtol=0, atol=1e-12 * np.abs(f["H0"]).max())
    assert m["gmax"] == pytest.approx(f["gmax"], rel=1e-14)
    assert (m["V"] > 0).mean() > 0.1  # the tube makes the Frangi branch active


def test_matrices_are_the_clamped_operators():
    n, h = 9, 0.7
    ramp = np.arange(n) * 2.0
    D1 = fa.d1_matrix(n, h)
    exp = np.full(n, 2.0 / h)
    exp[0] = exp[-1] = 1.0 / h  # one-sided halves at the faces
    np.testing.assert_allclose(D1 @ ramp, exp, rtol=1e-15)
    np.testing.assert_allclose(fa.d2_matrix(n, h) @ (np.arange(n) ** 2.0), np.r_[1.0, [2.0] * (n - 2), -(2 * n - 3.0)] / h ** 2,
                               rtol=1e-14)
    G = fa.gauss_matrix(n, 1.2)
    np.testing.assert_allclose(G.sum(1), 1.0, rtol=1e-15)  # constants are kept (clamped rows too)
    imp = np.zeros(n)
    imp[4] = 1.0
    r = 4  # floor(3 * 1.2 + 1/2)
    w = np.exp(-np.arange(-r, r + 1) ** 2 / (2 * 1.44))
    np.testing.assert_allclose(G @ imp, w / w.sum(), rtol=1e-14)  # the interior row is the kernel


def test_feature_vjp_matches_central_differences():
    shape = (7, 8, 9)
    I = _tube_volume(shape, 5)
    gb, kb, Vb, gmb = _upstream(shape, 6)
    dI = fa.vjp(I, SP, SIGMAS, FR["alpha"], FR["beta"], FR["c"], gb, kb, Vb, gmb)
    rng = np.random.default_rng(7)
    eps = 1e-6
    for _ in range(2):
        dirn = rng.normal(size=shape)
        fd = (_loss_features(I + eps * dirn, gb, kb, Vb, gmb) - _loss_features(I - eps * dirn, gb, kb, Vb, gmb)) / (2 * eps)
        assert abs(fd - (dI * dirn).sum()) <= 1e-6 * abs(fd)
    for idx in [(0, 0, 0), (6, 7, 8), (0, 7, 4), (3, 0, 8), (3, 4, 4), (1, 1, 1), (5, 6, 0), (2, 3, 7)]:
        p, m = I.copy(), I.copy()
        p[idx] += eps
        m[idx] -= eps
        fd = (_loss_features(p, gb, kb, Vb, gmb) - _loss_features(m, gb, kb, Vb, gmb)) / (2 * eps)
        assert abs(fd - dI[idx]) <= 1e-6 * np.abs(dI).max(), idx


def test_feature_vjp_terms_separately():
    """Each upstream alone (so a term that cancels another cannot hide): gradient, curvature,
    vesselness, gmax."""
    shape = (6, 7, 8)
    I = _tube_volume(shape, 8)
    gb, kb, Vb, gmb = _upstream(shape, 9)
    z3, z1 = np.zeros((3,) + shape), np.zeros(shape)
    rng = np.random.default_rng(10)
    eps = 1e-6
    for up in [(gb, z1, z1, 0.0), (z3, kb, z1, 0.0), (z3, z1, Vb, 0.0), (z3, z1, z1, gmb)]:
        dI = fa.vjp(I, SP, SIGMAS, FR["alpha"], FR["beta"], FR["c"], *up)
        dirn = rng.normal(size=shape)
        fd = (_loss_features(I + eps * dirn, *up) - _loss_features(I - eps * dirn, *up)) / (2 * eps)
        assert np.abs(dI).max() > 0
        assert abs(fd - (dI * dirn).sum()) <= 1e-6 * max(abs(fd), 1e-8), up[3]


def _render_setup(seed, dims=(7, 6, 5)):
    sp = (1.0, 0.9, 1.1)
    vol = phantoms.small_random(seed, dims, lo=0.05, hi=0.95)
    f = oracle.features(vol, sp, [1.0], c=0.05)
    knots = np.array([0.0, 0.31, 0.57, 0.83, 1.0])
    rng = np.random.default_rng(seed)
    rgba = np.concatenate([rng.uniform(0, 1, (5, 3)), rng.uniform(0.1, 1.5, (5, 1))], 1)
    prm = phantoms.render_params(lambda_g=0.7, lambda_k=0.4, kappa0=0.05, lambda_v=1.2, step_vox=0.5)
    cams = [phantoms.ortho_camera(dims, sp, 25.0, 15.0, 4, 4), phantoms.persp_camera(dims, sp, 160.0, 30.0, 4, 4)]
    dout = rng.normal(size=(2, 4, 4, 4))
    return vol, f, sp, knots, rgba, prm, cams, dout


def test_render_feature_grads_match_central_differences():
    vol, f, sp, knots, rgba, prm, cams, dout = _render_setup(41)
    _, _, fg = oracle.render_vjp(vol, f, f["gmax"], sp, knots, rgba, prm, cams, dout, want_features=True)

    def L(ff, gmax):
        return float((oracle.render(vol, ff, gmax, sp, knots, rgba, prm, cams)["rgba"] * dout).sum())

    eps = 1e-6
    rng = np.random.default_rng(2)
    for key in ("g", "kappa", "V"):
        assert np.abs(fg[key]).max() > 0, key
        dirn = rng.normal(size=f[key].shape)
        p = dict(f, **{key: f[key] + eps * dirn})
        m = dict(f, **{key: f[key] - eps * dirn})
        fd = (L(p, f["gmax"]) - L(m, f["gmax"])) / (2 * eps)
        assert abs(fd - (fg[key] * dirn).sum()) <= 1e-6 * abs(fd), key
    fd = (L(f, f["gmax"] + eps) - L(f, f["gmax"] - eps)) / (2 * eps)
    assert fg["gmax"] != 0 and abs(fd - fg["gmax"]) <= 1e-6 * abs(fd)


def test_end_to_end_gradient_through_the_features():
    """dL/dI = (TF-lookup path) + feature adjoint of dL/d(g, k, V, gmax), against central
    differences of L(I) = <dout, render(I, features(I))>."""
    dims = (7, 6, 5)
    vol, _, sp, knots, rgba, prm, cams, dout = _render_setup(43, dims)
    sig, fr = [1.0, 1.4], dict(alpha=0.5, beta=0.5, c=0.05)

    def L(I):
        f = oracle.features(I, sp, sig, **fr)
        return float((oracle.render(I, f, f["gmax"], sp, knots, rgba, prm, cams)["rgba"] * dout).sum())

    f = oracle.features(vol, sp, sig, **fr)
    _, dI_tf, fg = oracle.render_vjp(vol, f, f["gmax"], sp, knots, rgba, prm, cams, dout, want_features=True)
    dI_feat = fa.vjp(vol, sp, sig, fr["alpha"], fr["beta"], fr["c"], fg["g"], fg["kappa"], fg["V"], fg["gmax"])
    dI = dI_tf + dI_feat
    assert np.linalg.norm(dI_feat) > 0.05 * np.linalg.norm(dI_tf)  # the morphology terms matter
    eps = 1e-6
    rng = np.random.default_rng(4)
    for _ in range(2):
        dirn = rng.normal(size=vol.shape)
        fd = (L(vol + eps * dirn) - L(vol - eps * dirn)) / (2 * eps)
        assert abs(fd - (dI * dirn).sum()) <= 1e-5 * abs(fd)


def test_near_knot_mask_matches_brute_force():
    """The oracle's near-knot corner mask (the tolerated set of dL/dI comparisons) equals the one
    found by brute force (face-clipped rays, map_coordinates samples)."""
    from tests import bruteforce as bf
    vol, f, sp, knots, rgba, prm, cams, dout = _render_setup(41)
    eps = 2e-2  # wide, so that the mask is not empty on this small scene
    *_, mask = oracle.render_vjp(vol, f, f["gmax"], sp, knots, rgba, prm, cams, dout, near_knot_eps=eps)
    ref = bf.near_knot_voxels(vol.shape, sp, vol, knots, prm, cams, eps=eps)
    assert mask.any() and not mask.all()
    np.testing.assert_array_equal(mask, ref)
