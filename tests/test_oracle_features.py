"""CPU pins of the oracle's feature pass (gradient, scale space, Hessian, curvature, eigenvalues,
vesselness) against closed forms, library special cases and brute force."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import phantoms
from tests import bruteforce as bf


def _interior(arr, m):
    return arr[..., m:-m, m:-m, m:-m]


# ---------------------------------------------------------------- gradient (Sec. 2.3 Eq. 2)

@pytest.mark.parametrize("spacing", [(1.0, 1.0, 1.0), (0.7, 1.3, 3.5)])
def test_ramp_gradient_exact(spacing):
    """P1: a linear ramp has the constant gradient (a, b, c) on interior voxels; a face voxel
    gets half of it (clamped one-sided difference over 2h)."""
    dims = (12, 10, 9)
    X, Y, Z = phantoms.grid_mm(dims, spacing)
    a, b, c = 0.3, -1.7, 0.45
    I = a * X + b * Y + c * Z + 2.0
    g, gmax = oracle.gradient(I, spacing)
    inner = g[:, 1:-1, 1:-1, 1:-1]
    np.testing.assert_allclose(inner[0], a, rtol=0, atol=1e-12)
    np.testing.assert_allclose(inner[1], b, rtol=0, atol=1e-12)
    np.testing.assert_allclose(inner[2], c, rtol=0, atol=1e-12)
    np.testing.assert_allclose(g[0][1:-1, 1:-1, 0], a / 2, atol=1e-12)
    np.testing.assert_allclose(g[0][1:-1, 1:-1, -1], a / 2, atol=1e-12)
    np.testing.assert_allclose(g[1][1:-1, 0, 1:-1], b / 2, atol=1e-12)
    np.testing.assert_allclose(g[2][-1, 1:-1, 1:-1], c / 2, atol=1e-12)
    assert gmax == pytest.approx(math.sqrt(a * a + b * b + c * c), rel=1e-12)


def test_gradient_linear_and_flip():
    """P12: gradient is linear in I; flipping x negates g_x and mirrors the field; swapping the
    x and y axes swaps g_x and g_y."""
    A = phantoms.small_random(1, (9, 8, 7))
    B = phantoms.small_random(2, (9, 8, 7))
    sp = (1.0, 1.0, 1.0)
    gA, _ = oracle.gradient(A, sp)
    gB, _ = oracle.gradient(B, sp)
    gAB, _ = oracle.gradient(2.5 * A - 0.5 * B, sp)
    np.testing.assert_allclose(gAB, 2.5 * gA - 0.5 * gB, atol=1e-13)
    gF, _ = oracle.gradient(A[:, :, ::-1], sp)
    np.testing.assert_allclose(gF[0], -gA[0][:, :, ::-1], atol=1e-14)
    np.testing.assert_allclose(gF[1], gA[1][:, :, ::-1], atol=1e-14)
    C = phantoms.small_random(3, (8, 8, 7))
    gC, _ = oracle.gradient(C, sp)
    gT, _ = oracle.gradient(np.swapaxes(C, 1, 2).copy(), sp)
    np.testing.assert_allclose(gT[0], np.swapaxes(gC[1], 1, 2), atol=1e-14)
    np.testing.assert_allclose(gT[1], np.swapaxes(gC[0], 1, 2), atol=1e-14)


# ---------------------------------------------------------------- Gaussian scale space

@pytest.mark.parametrize("sig", [(1.0, 1.0, 1.0), (1.0 / 0.7, 2.0, 0.3), (0.5, 0.26, 3.0)])
def test_smooth_matches_scipy(sig):
    """P5: the separable clamped smoothing equals scipy.ndimage.gaussian_filter with
    mode='nearest' and the same radius floor(3 sigma + 1/2)."""
    vol = phantoms.small_random(5, (17, 14, 13))
    s = oracle.smooth(vol, sig)
    radius = [oracle.gauss_radius(sig[2]), oracle.gauss_radius(sig[1]), oracle.gauss_radius(sig[0])]
    ref = ndi.gaussian_filter(vol, sigma=(sig[2], sig[1], sig[0]), mode="nearest", radius=radius)
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e-13)


def test_gauss_radius_rule():
    """scipy's radius rule int(3 sigma + 0.5); at least 1."""
    assert oracle.gauss_radius(1.0) == 3
    assert oracle.gauss_radius(2.0) == 6
    assert oracle.gauss_radius(3.0) == 9
    assert oracle.gauss_radius(1 / 0.7) == 4
    assert oracle.gauss_radius(0.2) == 1
    assert oracle.gauss_radius(0.1) == 1


def test_smooth_nonseparable_bruteforce():
    """P10: separable passes equal one non-separable 3-D convolution with edge padding."""
    vol = phantoms.small_random(7, (9, 8, 6))
    sig = (1.2, 0.8, 0.6)
    np.testing.assert_allclose(oracle.smooth(vol, sig), bf.smooth_nonseparable(vol, sig), atol=1e-13)


def test_hessian_bruteforce():
    """Hessian second differences (clamped) vs an edge-padded NumPy stencil, anisotropic h."""
    vol = phantoms.small_random(8, (9, 8, 7))
    sp = (0.8, 1.1, 2.5)
    np.testing.assert_allclose(oracle.hessian(vol, sp), bf.hessian_np(vol, sp), atol=1e-12)


# ---------------------------------------------------------------- quadratic bowl (Eq. 2-3)

@pytest.mark.parametrize("spacing", [(1.0, 1.0, 1.0), (0.8, 1.2, 1.5)])
def test_bowl_closed_form(spacing):
    """P3: for I = 1/2 (x-x0)^T A (x-x0): g = A (x-x0) exactly in the interior (central
    differences are exact on quadratics); smoothing only adds a constant, so H = A exactly away
    from the faces; k = (x^T A^3 x) / (x^T A^2 x); eigenvalues of sigma^2 H are sigma^2 eig(A)."""
    dims = (24, 22, 20)
    X, Y, Z = phantoms.grid_mm(dims, spacing)
    x0 = np.array([11.3, 10.1, 9.7]) * np.array(spacing)
    A = np.array([[-0.9, 0.2, -0.1], [0.2, -0.5, 0.15], [-0.1, 0.15, 0.3]])
    R = np.stack([X - x0[0], Y - x0[1], Z - x0[2]])
    I = 0.5 * np.einsum("a...,ab,b...->...", R, A, R)
    sigma = 1.0
    f = oracle.features(I, spacing, [sigma], c=0.3, want_H0=True, want_lam=True)
    gref = np.einsum("ab,b...->a...", A, R)
    np.testing.assert_allclose(f["g"][:, 1:-1, 1:-1, 1:-1], gref[:, 1:-1, 1:-1, 1:-1], atol=1e-11)
    r = max(oracle.gauss_radius(sigma / h) for h in spacing)
    m = r + 2
    H = f["H0"]
    for e, (a, b) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
        np.testing.assert_allclose(_interior(H[e], m), A[a, b], atol=1e-10)
    A2, A3 = A @ A, A @ A @ A
    num = np.einsum("a...,ab,b...->...", R, A3, R)
    den = np.einsum("a...,ab,b...->...", R, A2, R)
    kref = num / den
    np.testing.assert_allclose(_interior(f["kappa"], m), _interior(kref, m), rtol=1e-9, atol=1e-10)
    ev = np.linalg.eigvalsh(sigma * sigma * A)
    ev = ev[np.lexsort((ev, np.abs(ev)))]
    lam = f["lam"][0]
    for e in range(3):
        np.testing.assert_allclose(_interior(lam[e], m), ev[e], atol=1e-10)


def test_curvature_zero_where_gradient_zero():
    """k = 0 exactly where g = 0 (a constant volume; and the centre of a symmetric bowl)."""
    dims = (11, 11, 11)
    X, Y, Z = phantoms.grid_mm(dims, (1.0, 1.0, 1.0))
    I = -((X - 5) ** 2 + 2 * (Y - 5) ** 2 + 3 * (Z - 5) ** 2)
    f = oracle.features(I, (1, 1, 1), [1.0], c=0.5)
    assert f["kappa"][5, 5, 5] == 0.0
    assert np.all(f["g"][:, 5, 5, 5] == 0.0)
    f0 = oracle.features(np.full((5, 6, 7), 0.3), (1, 1, 1), [1.0], c=0.5)
    assert np.all(f0["kappa"] == 0.0) and np.all(f0["V"] == 0.0) and f0["gmax"] == 0.0


def test_ramp_hessian_zero():
    """P2: the linear ramp has H = 0 (so k = 0 and V = 0) away from the faces."""
    dims = (20, 18, 17)
    X, Y, Z = phantoms.grid_mm(dims, (1.0, 1.0, 1.0))
    I = 0.3 * X - 0.2 * Y + 0.1 * Z
    f = oracle.features(I, (1, 1, 1), [1.0, 2.0], c=0.1, want_H0=True)
    m = 6 + 2
    np.testing.assert_allclose(_interior(f["H0"], 3 + 2), 0.0, atol=1e-12)
    np.testing.assert_allclose(_interior(f["kappa"], 3 + 2), 0.0, atol=1e-12)
    np.testing.assert_allclose(_interior(f["V"], m), 0.0, atol=1e-12)


# ---------------------------------------------------------------- eigenvalues, vesselness

def test_eig_matches_lapack():
    """P6: every voxel's sorted eigenvalues of sigma^2 H equal numpy.linalg.eigvalsh (LAPACK)."""
    vol = phantoms.small_random(11, (10, 9, 8))
    sigmas = [1.0, 1.5]
    f = oracle.features(vol, (1.0, 0.9, 1.2), sigmas, c=0.2, want_lam=True)
    for sc, sg in enumerate(sigmas):
        s = oracle.smooth(vol, (sg / 1.0, sg / 0.9, sg / 1.2))
        H = oracle.hessian(s, (1.0, 0.9, 1.2)) * sg * sg
        M = np.empty(vol.shape + (3, 3))
        idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
        for e, (a, b) in enumerate(idx):
            M[..., a, b] = H[e]
            M[..., b, a] = H[e]
        ev = np.linalg.eigvalsh(M)
        order = np.lexsort((ev, np.abs(ev)), axis=-1)
        ev = np.take_along_axis(ev, order, -1)
        scale = np.abs(ev).max()
        np.testing.assert_allclose(np.moveaxis(f["lam"][sc], 0, -1), ev, atol=1e-13 * max(scale, 1))


def test_eig_degenerate_and_ties():
    """Repeated eigenvalues, diagonal and zero matrices; the (|l|, l) order puts the negative
    one first at an exact magnitude tie."""
    np.testing.assert_allclose(oracle.eig3([2, 2, 2, 0, 0, 0]), [2, 2, 2])
    np.testing.assert_allclose(oracle.eig3([0, 0, 0, 0, 0, 0]), [0, 0, 0])
    np.testing.assert_allclose(oracle.eig3([1, -1, 3, 0, 0, 0]), [-1, 1, 3])
    lam = oracle.eig3([1.0, 1.0, -2.0, 1.0, 0.0, 0.0])  # eig of [[1,1],[1,1]] = 0, 2; plus -2
    np.testing.assert_allclose(lam, [0.0, -2.0, 2.0], atol=1e-14)


def test_vesselness_branches():
    """Frangi bright-tube rule: V = 0 unless l2 < 0 and l3 < 0; an ideal line (l1 = 0,
    l2 = l3 = -s) gives (1 - e^-2)(1 - exp(-s^2/c^2)) with alpha = beta = 1/2; a blob
    (l1 = l2 = l3 = -s) gives (1 - e^-2) e^-2 (1 - exp(-3 s^2 / 2 c^2))."""
    c = 0.3
    assert oracle.vesselness([0.0, 0.5, -0.7], 0.5, 0.5, c) == 0.0
    assert oracle.vesselness([0.0, -0.5, 0.7], 0.5, 0.5, c) == 0.0
    assert oracle.vesselness([0.0, 0.0, -0.7], 0.5, 0.5, c) == 0.0
    s = 0.4
    v = oracle.vesselness([0.0, -s, -s], 0.5, 0.5, c)
    assert v == pytest.approx((1 - math.exp(-2)) * (1 - math.exp(-s * s / (c * c))), rel=1e-14)
    v = oracle.vesselness([-s, -s, -s], 0.5, 0.5, c)
    assert v == pytest.approx((1 - math.exp(-2)) * math.exp(-2) * (1 - math.exp(-1.5 * s * s / (c * c))), rel=1e-14)
    # plate-like (l1 = l2 = 0, l3 < 0): R_A = 0 -> V = 0
    assert oracle.vesselness([0.0, 0.0, -s], 0.5, 0.5, c) == 0.0


def test_tube_vesselness_on_axis():
    """P4: a Gaussian tube along x through voxel centres.  On the axis H_xx = 0, H_yy = H_zz and
    the off-diagonals vanish, so l1 = 0, l2 = l3 = sigma^2 H_yy and
    V = (1 - e^-2)(1 - exp(-sigma^4 H_yy^2 / c^2)); the axis is the argmax of V over each
    cross-section; smoothing is exact in x so H_xx = H_xy = H_xz = 0 everywhere."""
    dims = (16, 21, 21)
    X, Y, Z = phantoms.grid_mm(dims, (1.0, 1.0, 1.0))
    R = 2.0
    I = np.exp(-((Y - 10) ** 2 + (Z - 10) ** 2) / (2 * R * R))
    sigma, c = 1.5, 0.2
    f = oracle.features(I, (1, 1, 1), [sigma], c=c, want_H0=True, want_lam=True)
    H = f["H0"]
    np.testing.assert_allclose(H[0], 0.0, atol=1e-14)
    np.testing.assert_allclose(H[3], 0.0, atol=1e-14)
    np.testing.assert_allclose(H[4], 0.0, atol=1e-14)
    ax = (10, 10, slice(None))
    np.testing.assert_allclose(H[1][ax], H[2][ax], rtol=1e-13)
    np.testing.assert_allclose(H[5][ax], 0.0, atol=1e-15)
    hyy = H[1][ax]
    assert np.all(hyy < 0)
    vref = (1 - math.exp(-2)) * (1 - np.exp(-(sigma ** 4) * hyy ** 2 / c ** 2))
    np.testing.assert_allclose(f["V"][ax], vref, rtol=1e-12)
    np.testing.assert_allclose(f["lam"][0, 0][ax], 0.0, atol=1e-14)
    # independent value of H_yy on the axis: scipy smoothing + second difference
    s = ndi.gaussian_filter(I, sigma, mode="nearest", radius=oracle.gauss_radius(sigma))
    np.testing.assert_allclose(hyy, s[10, 11, :] - 2 * s[10, 10, :] + s[10, 9, :], rtol=1e-12)
    V = f["V"]
    for x in range(dims[0]):
        sl = V[:, :, x]
        assert np.unravel_index(np.argmax(sl), sl.shape) == (10, 10)


def test_tube_scale_selection():
    """Continuum sanity check: sigma^2 |l2| on the axis peaks near sigma = R (within 15 %)."""
    dims = (8, 41, 41)
    X, Y, Z = phantoms.grid_mm(dims, (1.0, 1.0, 1.0))
    R = 3.0
    I = np.exp(-((Y - 20) ** 2 + (Z - 20) ** 2) / (2 * R * R))
    sig = np.linspace(1.5, 5.0, 15)
    resp = []
    for s in sig:
        f = oracle.features(I, (1, 1, 1), [s], c=1.0, want_lam=True)
        resp.append(abs(f["lam"][0, 1][20, 20, 4]))
    best = sig[int(np.argmax(resp))]
    assert abs(best - R) / R < 0.15


def test_vesselness_max_over_scales_and_c_rule():
    """V is the max of the per-scale responses; c <= 0 gives 1/2 max |sigma^2 H|_F over voxels
    and scales (checked on the bowl, whose interior Hessian is A at every scale)."""
    vol = phantoms.small_random(13, (12, 11, 10))
    f = oracle.features(vol, (1, 1, 1), [1.0, 1.7], c=0.05, want_Vs=True)
    np.testing.assert_array_equal(f["V"], np.maximum(f["Vs"][0], f["Vs"][1]))
    f1 = oracle.features(vol, (1, 1, 1), [1.0], c=-1.0, want_H0=True)
    H = f1["H0"]
    fro = np.sqrt(H[0] ** 2 + H[1] ** 2 + H[2] ** 2 + 2 * (H[3] ** 2 + H[4] ** 2 + H[5] ** 2))
    assert f1["c"] == pytest.approx(0.5 * fro.max(), rel=1e-14)


def test_feature_invariance_axis_swap_and_flip():
    """P12: swapping x and y (isotropic grid) or flipping x leaves k and V invariant as fields."""
    vol = phantoms.small_random(17, (10, 10, 8))
    f = oracle.features(vol, (1, 1, 1), [1.0], c=0.1)
    fs = oracle.features(np.swapaxes(vol, 1, 2).copy(), (1, 1, 1), [1.0], c=0.1)
    np.testing.assert_allclose(fs["kappa"], np.swapaxes(f["kappa"], 1, 2), atol=1e-12)
    np.testing.assert_allclose(fs["V"], np.swapaxes(f["V"], 1, 2), atol=1e-12)
    ff = oracle.features(vol[:, :, ::-1].copy(), (1, 1, 1), [1.0], c=0.1)
    np.testing.assert_allclose(ff["kappa"], f["kappa"][:, :, ::-1], atol=1e-12)
    np.testing.assert_allclose(ff["V"], f["V"][:, :, ::-1], atol=1e-12)


def test_normalize():
    """Eq. 1: (I - min)/(max - min); a constant volume maps to 0."""
    raw = np.array([[[3.0, 7.0], [5.0, 11.0]]])
    out, mn, mx = oracle.normalize(raw)
    np.testing.assert_allclose(out, (raw - 3.0) / 8.0)
    assert (mn, mx) == (3.0, 11.0)
    out, _, _ = oracle.normalize(np.full((2, 2, 2), 4.0))
    assert np.all(out == 0.0)
