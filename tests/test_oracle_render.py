"""CPU pins of the oracle's raymarcher (Sec. 2.4 Eq. 4-6) against closed forms (Beer-Lambert,
partial-volume slab), NumPy/SciPy brute force on tiny volumes, and invariants."""
import math

import numpy as np
import pytest

import oracle
import phantoms
from tests import bruteforce as bf


def _feats_const(vol):
    return dict(g=np.zeros((3,) + vol.shape), kappa=np.zeros(vol.shape), V=np.zeros(vol.shape))


def _axis_cam(dims, spacing, axis, sign, W, H, offset=(0.37, 0.41)):
    """Orthographic camera looking along +/- axis with pixel centres on a regular lattice."""
    nx, ny, nz = dims
    ext = np.array([(nx - 1) * spacing[0], (ny - 1) * spacing[1], (nz - 1) * spacing[2]])
    a1, a2 = [b for b in range(3) if b != axis]
    d0 = np.zeros(3)
    d0[axis] = sign
    du = np.zeros(3)
    dv = np.zeros(3)
    du[a1] = ext[a1] / W
    dv[a2] = ext[a2] / H
    o = np.zeros(3)
    o[axis] = -5.0 if sign > 0 else ext[axis] + 5.0
    o[a1] = -0.5 * du[a1] + offset[0] * du[a1]
    o[a2] = -0.5 * dv[a2] + offset[1] * dv[a2]
    return phantoms.Camera(0, W, H, o.astype(np.float32), d0.astype(np.float32), du.astype(np.float32),
                           dv.astype(np.float32))


def test_beer_lambert_homogeneous():
    """P8: homogeneous volume, constant TF (colour c, extinction s), lambda's = 0:
    A = 1 - exp(-s L) and C = c (1 - exp(-s L)) for the chord length L, for any step."""
    dims, sp = (9, 8, 7), (1.0, 1.2, 0.9)
    vol = np.full(dims[::-1], 0.5)
    knots = np.array([0.0, 1.0])
    col = np.array([0.2, 0.7, 0.9])
    s = 0.13
    rgba = np.array([[*col, s], [*col, s]])
    cams = [phantoms.ortho_camera(dims, sp, 33.0, 17.0, 8, 8), phantoms.persp_camera(dims, sp, 200.0, -25.0, 8, 8)]
    hi = np.array([(n - 1) * h for n, h in zip(dims, sp)])
    for step in (0.5, 0.37, 1.3):
        prm = phantoms.render_params(lambda_g=0.0, lambda_k=0.0, lambda_v=0.0, step_vox=step)
        r = oracle.render(vol, _feats_const(vol), 1.0, sp, knots, rgba, prm, cams)
        for ci, cam in enumerate(cams):
            pk = cam.packed()
            for j in range(8):
                for i in range(8):
                    o, d = bf.ray_of(pk, i, j)
                    cl = bf.clip_faces(o, d, hi)
                    L = 0.0 if cl is None else cl[1] - cl[0]
                    A = 1 - math.exp(-s * L)
                    np.testing.assert_allclose(r["rgba"][ci, j, i, 3], A, atol=1e-13)
                    np.testing.assert_allclose(r["rgba"][ci, j, i, :3], col * A, atol=1e-13)


def test_partial_volume_slab():
    """P9: node-aligned slab of ones (planes k0..k1), axis-parallel rays, step dividing h,
    extinction linear in I (tau = s I): each trilinear ramp adds h/2, so A = 1 - exp(-s (L + h))
    with L = (k1 - k0) h."""
    dims, sp = (6, 5, 20), (1.0, 1.0, 0.8)
    vol = np.zeros(dims[::-1])
    k0, k1 = 6, 13
    vol[k0:k1 + 1] = 1.0
    knots = np.array([0.0, 1.0])
    s = 0.21
    rgba = np.array([[1.0, 1.0, 1.0, 0.0], [1.0, 1.0, 1.0, s]])
    prm = phantoms.render_params(lambda_g=0.0, lambda_k=0.0, lambda_v=0.0, step_vox=0.25)
    cams = [_axis_cam(dims, sp, 2, +1, 4, 3), _axis_cam(dims, sp, 2, -1, 4, 3)]
    r = oracle.render(vol, _feats_const(vol), 1.0, sp, knots, rgba, prm, cams)
    L = (k1 - k0) * sp[2]
    np.testing.assert_allclose(r["rgba"][..., 3], 1 - math.exp(-s * (L + sp[2])), atol=1e-13)


def test_opposite_views_same_alpha():
    """P12: two opposite axis-aligned orthographic views sample the same midpoints in reverse
    order (L / delta is an integer), so A = 1 - prod(1 - a_k) agrees."""
    dims, sp = (7, 6, 11), (1.0, 1.0, 1.0)
    vol = phantoms.small_random(21, dims)
    f = oracle.features(vol, sp, [1.0], c=0.1)
    knots, rgba = phantoms.tf_c1()
    prm = phantoms.render_params(lambda_v=0.7)
    cams = [_axis_cam(dims, sp, 2, +1, 5, 4), _axis_cam(dims, sp, 2, -1, 5, 4)]
    r = oracle.render(vol, f, f["gmax"], sp, knots, rgba, prm, cams)
    np.testing.assert_allclose(r["rgba"][0, ..., 3], r["rgba"][1, ..., 3], atol=1e-14)
    assert np.any(r["rgba"][0, ..., 3] > 0.05)


def _tiny_scene(seed, dims, sp):
    vol = phantoms.small_random(seed, dims)
    f = oracle.features(vol, sp, [1.0, 1.6], c=0.05)
    return vol, f


@pytest.mark.parametrize("case", range(4))
def test_bruteforce_tiny(case):
    """P10: oracle images equal an explicit-product NumPy/SciPy render on tiny volumes, for
    orthographic and perspective cameras, all Eq. 4 factors on, with and without early
    termination."""
    dims = [(6, 5, 4), (5, 6, 6), (6, 6, 5), (4, 5, 6)][case]
    sp = [(1.0, 1.0, 1.0), (0.9, 1.1, 1.3), (1.0, 0.8, 1.0), (1.2, 1.0, 0.7)][case]
    vol, f = _tiny_scene(30 + case, dims, sp)
    knots = np.array([0.1, 0.35, 0.6, 0.9])
    rgba = np.array([[0.1, 0.2, 0.3, 0.4], [0.9, 0.1, 0.5, 1.5], [0.3, 0.8, 0.2, 0.2], [0.6, 0.6, 0.9, 2.5]])
    et = [0.0, 0.9, 0.0, 0.6][case]
    prm = phantoms.render_params(lambda_g=0.8, lambda_k=0.6, kappa0=0.07, lambda_v=1.5, step_vox=0.45, et_alpha=et)
    cams = [phantoms.ortho_camera(dims, sp, 30.0 + 50 * case, 20.0, 4, 4),
            phantoms.persp_camera(dims, sp, 110.0 + 40 * case, -10.0, 4, 4, dist_diag=1.5, fov_y_deg=40.0)]
    r = oracle.render(vol, f, f["gmax"], sp, knots, rgba, prm, cams)
    hit = 0
    for ci, cam in enumerate(cams):
        for j in range(4):
            for i in range(4):
                ref, ns = bf.render_pixel(vol, f["g"], f["kappa"], f["V"], f["gmax"], sp, knots, rgba, prm,
                                          cam.packed(), i, j)
                np.testing.assert_allclose(r["rgba"][ci, j, i], ref, atol=1e-12)
                assert r["k_last"][ci, j, i] == ns - 1
                hit += ns > 0
    assert hit > 8


def test_early_termination_state():
    """Early termination stops right after the first sample with T <= 1 - a_ET; T_last is the
    transmittance before that sample; a miss has k_last = -1 and zero colour."""
    dims, sp = (8, 8, 8), (1.0, 1.0, 1.0)
    vol = np.full(dims[::-1], 0.9)
    knots = np.array([0.0, 1.0])
    rgba = np.array([[1, 1, 1, 2.0], [1, 1, 1, 2.0]])
    prm = phantoms.render_params(lambda_g=0.0, lambda_k=0.0, lambda_v=0.0, step_vox=0.5, et_alpha=0.99)
    cam = _axis_cam(dims, sp, 0, +1, 3, 3)
    r = oracle.render(vol, _feats_const(vol), 1.0, sp, knots, rgba, prm, [cam])
    x = 2.0 * 0.5
    # T after k+1 samples = exp(-(k+1) x) <= 0.01  ->  k+1 = ceil(ln(100)/x)
    n = math.ceil(math.log(100.0) / x)
    assert np.all(r["k_last"] == n - 1)
    np.testing.assert_allclose(r["T_last"], math.exp(-(n - 1) * x), rtol=1e-13)
    np.testing.assert_allclose(r["rgba"][..., 3], 1 - math.exp(-n * x), rtol=1e-13)
    miss = phantoms.Camera(0, 2, 2, np.array([-5, -5, -5], np.float32), np.array([0, 0, 1], np.float32),
                           np.array([1, 0, 0], np.float32), np.array([0, 1, 0], np.float32))
    r = oracle.render(vol, _feats_const(vol), 1.0, sp, knots, rgba, prm, [miss])
    assert np.all(r["k_last"] == -1) and np.all(r["rgba"] == 0.0)


def test_pixel_subset_matches_full():
    """Rendering a list of pixels gives the same values as the full image at those pixels."""
    w = phantoms.c1(32, 32)
    f = oracle.features(w.vol, w.spacing, w.sigmas, c=w.c)
    full = oracle.render(w.vol, f, f["gmax"], w.spacing, w.tf_knots, w.tf_rgba, w.params, w.cams)
    pix = np.array([[0, 3, 5], [0, 31, 0], [0, 16, 16], [0, 0, 31]], np.int32)
    sub = oracle.render(w.vol, f, f["gmax"], w.spacing, w.tf_knots, w.tf_rgba, w.params, w.cams, pix=pix)
    for p, (c, i, j) in enumerate(pix):
        np.testing.assert_array_equal(sub["rgba"][p], full["rgba"][c, j, i])


def test_ray_split_composites_over():
    """P12: a ray split at a node plane (segment boundary) gives (C1, T1) for the front slab and
    (C2, T2) for the back one, and "over", (C1 + T1 C2, T1 T2), reproduces the full ray; the two
    slabs share the plane's voxels, and the features and gmax are those of the whole volume."""
    rng = np.random.default_rng(12)
    dims, sp = (6, 5, 9), (1.0, 1.0, 1.0)
    vol = rng.uniform(0.05, 0.95, dims[::-1])
    f = oracle.features(vol, sp, [1.0], c=0.1)
    knots = np.array([0.0, 0.3, 0.6, 1.0])
    rgba = np.concatenate([rng.uniform(0, 1, (4, 3)), rng.uniform(0.1, 1.0, (4, 1))], 1)
    prm = phantoms.render_params(lambda_g=0.6, lambda_k=0.4, kappa0=0.05, lambda_v=1.0, step_vox=0.5)
    cam = _axis_cam(dims, sp, 2, 1, 4, 3)
    full = oracle.render(vol, f, f["gmax"], sp, knots, rgba, prm, [cam])["rgba"]
    m = 4  # split at the node plane z = 4 (8 segments of 0.5 on each side)

    def part(z0, z1, dz):
        sub = dict(g=f["g"][:, z0:z1], kappa=f["kappa"][z0:z1], V=f["V"][z0:z1])
        c = phantoms.Camera(0, cam.width, cam.height, (cam.o - np.array([0, 0, dz], np.float32)).astype(np.float32),
                            cam.d0, cam.du, cam.dv)
        return oracle.render(vol[z0:z1], sub, f["gmax"], sp, knots, rgba, prm, [c])["rgba"]

    a = part(0, m + 1, 0.0)
    b = part(m, dims[2], float(m))
    T1, T2 = 1.0 - a[..., 3], 1.0 - b[..., 3]
    over = np.concatenate([a[..., :3] + T1[..., None] * b[..., :3], (1.0 - T1 * T2)[..., None]], -1)
    assert (full[..., 3] > 0.1).all()
    np.testing.assert_allclose(over, full, rtol=1e-12, atol=1e-15)
