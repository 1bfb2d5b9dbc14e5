"""GPU parity of the feature pass (dvr_features) against the FP64 oracle.

Bar: for every output array, max|gpu - oracle| / max|oracle| <= 1e-5 in FP32 storage (gradient,
curvature, vesselness); |grad I|_max to 1e-6.  Vesselness excludes voxels at an opposite-sign
magnitude tie of lambda1/lambda2 (V is discontinuous there; both sides are correct), and the
count of such voxels is checked to be small (< 0.2 %)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_19737_amd as dvr
import phantoms
from paper_2605_19737_amd import _abi as abi
from tests.gpu_common import feats_np, f32, fmt_rates, rel_err, sp32, to_dev, vessel_tie_mask

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _compare(vol, spacing, sigmas, c, eig_gap=1e-3, dtype=torch.float32, layout=abi.DVR_PLANAR, tol=TOL, label=""):
    print(f"[features] {label} shape={vol.shape} spacing={spacing} sigmas={sigmas} c={c}", flush=True)
    sp = sp32(spacing)
    sg = [f32(s) for s in sigmas]
    dv = to_dev(vol)
    f = dvr.features(dv, spacing, sigmas, c=c, eig_gap=eig_gap, dtype=dtype, layout=layout)
    got = feats_np(f)
    ref = oracle.features(dv.cpu().numpy().astype(np.float64), sp, sg, c=f32(c) if c > 0 else c, want_lam=True)
    e_g = rel_err(got["g"], ref["g"])
    e_k = rel_err(got["kappa"], ref["kappa"])
    tie = vessel_tie_mask(ref["lam"])
    e_v = rel_err(got["V"][~tie], ref["V"][~tie])
    e_m = abs(got["gmax"] - ref["gmax"]) / ref["gmax"]
    rates = fmt_rates([("g", got["g"], ref["g"]), ("kappa", got["kappa"], ref["kappa"]),
                       ("V", got["V"][~tie], ref["V"][~tie])])
    print(f"  err g={e_g:.2e} kappa={e_k:.2e} V={e_v:.2e} gmax={e_m:.2e} ties={int(tie.sum())}; "
          f"floor rates {rates}", flush=True)
    assert tie.mean() < 2e-3
    assert e_g <= tol and e_k <= tol and e_v <= tol
    assert e_m <= 1e-6
    return got, ref


def test_features_c1():
    """64^3 nested ellipsoids, sigma = 1 voxel (the plain-method workload)."""
    w = phantoms.c1(8, 8)
    _compare(w.vol, w.spacing, w.sigmas, w.c, label="c1")


def test_features_multiscale_ragged_anisotropic():
    """Several 64 x 8 tiles with ragged tails on every axis, anisotropic spacing, two scales."""
    vol = phantoms.small_random(101, (150, 37, 23), lo=0.0, hi=1.0)
    _compare(vol, (0.9, 1.1, 1.3), [1.0, 2.0], 0.1, label="ragged")


def test_features_frangi_auto_c():
    """c <= 0 selects Frangi's rule c = 1/2 max |sigma^2 H|_F (a reduction pass on the device)."""
    w = phantoms.c1(8, 8)
    _compare(w.vol[:40, :50, :60], w.spacing, [1.0, 1.5], -1.0, label="auto-c")


@pytest.mark.parametrize("layout", [abi.DVR_PLANAR, abi.DVR_SPLIT])
def test_features_every_fixed_radius(layout):
    """Each stencil radius of the fixed-radius kernels (2..10, sigma = r/3 mm at 1 mm spacing for
    r = 1..9, one scale per call so that kappa checks that radius's Hessian everywhere) on a crop
    of the head with vessels that spans several 64 x 8 tiles with ragged tails."""
    w = phantoms.c2(8, 8, views=[0])
    vol = w.vol[60:97, 70:140, 40:130]
    for r in range(1, 10):
        _compare(vol, (1.0, 1.0, 1.0), [r / 3.0], w.c, layout=layout, label=f"radius {r + 1}")


def test_features_head_three_scales():
    """The 181x217x181 head phantom with vessels at sigma = {1, 2, 3} (the benchmarked workload)."""
    w = phantoms.c2(8, 8, views=[0])
    _compare(w.vol, w.spacing, w.sigmas, w.c, label="head")


def test_features_batched_volume_anisotropic():
    """A batched-set volume: thick slices (sigma_z ~ 0.25 voxel, radius 1) and sub-mm in-plane."""
    w = phantoms.c4_volume(3, 8, 8, views=[0])
    _compare(w.vol, w.spacing, w.sigmas, w.c, label="c4_3")


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 2, 5), (2, 9, 3), (65, 2, 2)])
def test_features_tiny_grids(dims):
    """Degenerate grids: two voxels along an axis (both faces at once), one-tile and one-row cases."""
    vol = phantoms.small_random(7, dims)
    _compare(vol, (1.0, 0.8, 1.2), [1.0], 0.1, label=f"tiny{dims}")


def test_features_layouts_agree():
    """The interleaved record (I, g, k, V) holds bitwise the planar values."""
    w = phantoms.c1(8, 8)
    dv = to_dev(w.vol[:30, :40, :50])
    a = feats_np(dvr.features(dv, w.spacing, [1.0, 2.0], c=0.1))
    b = feats_np(dvr.features(dv, w.spacing, [1.0, 2.0], c=0.1, layout=abi.DVR_INTERLEAVED))
    for k in ("g", "kappa", "V"):
        np.testing.assert_array_equal(a[k], b[k])
    np.testing.assert_array_equal(b["I"], dv.cpu().numpy())
    assert a["gmax"] == b["gmax"]


@pytest.mark.parametrize("layout", [abi.DVR_PLANAR, abi.DVR_INTERLEAVED])
def test_features_fp16_storage(layout):
    """FP16 storage of an FP16 volume: compared with the oracle on the same FP16-rounded input, each
    output is within its FP16 rounding (2^-11 relative to the element, so <= 2^-11 of the range)
    plus the FP32 compute bound."""
    w = phantoms.c1(8, 8)
    v16 = torch.from_numpy(w.vol).half().cuda()
    f = dvr.features(v16, w.spacing, w.sigmas, c=w.c, dtype=torch.float16, layout=layout)
    got = feats_np(f)
    ref = oracle.features(v16.float().cpu().numpy().astype(np.float64), sp32(w.spacing), [f32(s) for s in w.sigmas],
                          c=f32(w.c), want_lam=True)
    tie = vessel_tie_mask(ref["lam"])
    bound = 2.0 ** -11 + TOL
    errs = dict(g=rel_err(got["g"], ref["g"]), kappa=rel_err(got["kappa"], ref["kappa"]),
                V=rel_err(got["V"][~tie], ref["V"][~tie]))
    print("  fp16 storage errors", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= bound, (k, v)
    if layout == abi.DVR_INTERLEAVED:
        np.testing.assert_array_equal(got["I"], v16.float().cpu().numpy())
