"""CPU pins of the oracle's reverse mode: FP64 central finite differences (h = 1e-4) and the
closed form of a homogeneous column."""
import math

import numpy as np

import oracle
import phantoms


def _loss_and_grad(vol, f, sp, knots, rgba, prm, cams, target):
    r = oracle.render(vol, f, f["gmax"], sp, knots, rgba, prm, cams)
    diff = r["rgba"] - target
    L = 0.5 * float(np.sum(diff * diff))
    dtf, dI = oracle.render_vjp(vol, f, f["gmax"], sp, knots, rgba, prm, cams, diff)
    return L, dtf, dI, r


def _loss(vol, f, sp, knots, rgba, prm, cams, target):
    r = oracle.render(vol, f, f["gmax"], sp, knots, rgba, prm, cams)
    d = r["rgba"] - target
    return 0.5 * float(np.sum(d * d))


def _setup(seed):
    dims, sp = (7, 6, 5), (1.0, 0.9, 1.1)
    vol = phantoms.small_random(seed, dims, lo=0.05, hi=0.95)
    f = oracle.features(vol, sp, [1.0], c=0.05)
    knots = np.array([0.0, 0.31, 0.57, 0.83, 1.0])
    rng = np.random.default_rng(seed)
    rgba = np.concatenate([rng.uniform(0, 1, (5, 3)), rng.uniform(0.1, 1.5, (5, 1))], 1)
    prm = phantoms.render_params(lambda_g=0.7, lambda_k=0.4, kappa0=0.05, lambda_v=1.2, step_vox=0.5)
    cams = [phantoms.ortho_camera(dims, sp, 25.0, 15.0, 4, 4), phantoms.persp_camera(dims, sp, 160.0, 30.0, 4, 4)]
    target = rng.uniform(0, 1, (2, 4, 4, 4))
    return vol, f, sp, knots, rgba, prm, cams, target


def _min_knot_distance(vol, f, sp, knots, prm, cams):
    """Smallest |I(sample) - knot| over all samples: central differences of step h are valid only
    when no sample sits within h of a knot (the TF is piecewise linear)."""
    from tests import bruteforce as bf
    import scipy.ndimage as ndi
    nz, ny, nx = vol.shape
    h = np.asarray(sp)
    hi = np.array([(nx - 1) * h[0], (ny - 1) * h[1], (nz - 1) * h[2]])
    best = np.inf
    for cam in cams:
        pk = cam.packed()
        for j in range(cam.height):
            for i in range(cam.width):
                o, d = bf.ray_of(pk, i, j)
                cl = bf.clip_faces(o, d, hi)
                if cl is None:
                    continue
                delta = prm["step_vox"] * h.min()
                L = cl[1] - cl[0]
                N = int(math.ceil(L / delta))
                dks = np.full(N, delta)
                dks[-1] = L - (N - 1) * delta
                tk = cl[0] + np.arange(N) * delta + 0.5 * dks
                Q = np.clip((o[None] + tk[:, None] * d[None]) / h, 0, [nx - 1, ny - 1, nz - 1])
                I = ndi.map_coordinates(vol, np.stack([Q[:, 2], Q[:, 1], Q[:, 0]]), order=1, mode="nearest")
                best = min(best, np.abs(I[:, None] - knots[None]).min())
    return best


def test_vjp_matches_central_fd():
    """P11: the reverse mode equals FP64 central differences (h = 1e-4) for every TF value and
    every voxel intensity (features held constant), normwise to 1e-6."""
    vol, f, sp, knots, rgba, prm, cams, target = _setup(41)
    assert _min_knot_distance(vol, f, sp, knots, prm, cams) > 3e-4
    L, dtf, dI, _ = _loss_and_grad(vol, f, sp, knots, rgba, prm, cams, target)
    h = 1e-4
    fd_tf = np.zeros_like(rgba)
    for k in range(rgba.shape[0]):
        for ch in range(4):
            p, m = rgba.copy(), rgba.copy()
            p[k, ch] += h
            m[k, ch] -= h
            fd_tf[k, ch] = (_loss(vol, f, sp, knots, p, prm, cams, target) -
                            _loss(vol, f, sp, knots, m, prm, cams, target)) / (2 * h)
    assert np.linalg.norm(dtf - fd_tf) <= 1e-6 * np.linalg.norm(fd_tf)
    fd_I = np.zeros_like(vol)
    for idx in np.ndindex(vol.shape):
        p, m = vol.copy(), vol.copy()
        p[idx] += h
        m[idx] -= h
        fd_I[idx] = (_loss(p, f, sp, knots, rgba, prm, cams, target) -
                     _loss(m, f, sp, knots, rgba, prm, cams, target)) / (2 * h)
    assert np.linalg.norm(fd_I) > 1e-3
    assert np.linalg.norm(dI - fd_I) <= 1e-6 * np.linalg.norm(fd_I)


def test_vjp_homogeneous_column_closed_form():
    """One homogeneous column with a constant TF (colour c, extinction tau): C = c (1 - e^{-tau L}),
    so dC/dtau = c L e^{-tau L}; with a linear TF in two knots the knot adjoints split by
    (1 - t, t) at the constant intensity."""
    dims, sp = (5, 5, 9), (1.0, 1.0, 1.0)
    vol = np.full(dims[::-1], 0.25)
    feats = dict(g=np.zeros((3,) + vol.shape), kappa=np.zeros(vol.shape), V=np.zeros(vol.shape))
    knots = np.array([0.0, 1.0])
    tau, col = 0.3, np.array([0.5, 0.2, 0.9])
    rgba = np.array([[*col, tau], [*col, tau]])
    prm = phantoms.render_params(lambda_g=0.0, lambda_k=0.0, lambda_v=0.0, step_vox=0.5)
    cam = phantoms.Camera(0, 1, 1, np.array([2.0, 2.0, -3.0], np.float32), np.array([0, 0, 1], np.float32),
                          np.array([0.1, 0, 0], np.float32), np.array([0, 0.1, 0], np.float32))
    L = (dims[2] - 1) * sp[2]
    r = oracle.render(vol, feats, 1.0, sp, knots, rgba, prm, [cam])
    np.testing.assert_allclose(r["rgba"][0, 0, 0, :3], col * (1 - math.exp(-tau * L)), rtol=1e-14)
    # upstream gradient only on the red channel: dL/dtau_total = c_r L e^{-tau L}
    dout = np.zeros((1, 1, 1, 4))
    dout[..., 0] = 1.0
    dtf, dI = oracle.render_vjp(vol, feats, 1.0, sp, knots, rgba, prm, [cam], dout)
    total = dtf[0, 3] + dtf[1, 3]
    np.testing.assert_allclose(total, col[0] * L * math.exp(-tau * L), rtol=1e-12)
    np.testing.assert_allclose(dtf[1, 3] / total, 0.25, rtol=1e-12)
    np.testing.assert_allclose(dtf[0, 0] + dtf[1, 0], 1 - math.exp(-tau * L), rtol=1e-12)
    # flat TF: no dependence on I
    np.testing.assert_allclose(dI, 0.0, atol=1e-15)
