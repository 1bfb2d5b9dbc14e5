"""GPU parity of the denoise pre-pass (Sec. 5.3) against the oracle (oracle/denoise.py): the 3x3x3
median bit-exact (it selects one of the inputs), the separable Gaussian within 1e-6 of the range in
FP32 and within one FP16 ulp of the FP64 value rounded to FP16."""
import numpy as np
import pytest
import torch

import oracle.denoise as od
import paper_2605_19737_amd as dvr
import phantoms
from tests.gpu_common import rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(2, 2, 2), (3, 2, 5), (17, 23, 29), (64, 9, 130)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_median3_exact(shape, dtype):
    rng = np.random.default_rng(sum(shape))
    v = rng.random(shape).astype(np.float32)
    v[..., ::3] = np.round(v[..., ::3] * 4) / 4  # many ties
    dv = to_dev(v, dtype)
    got = dvr.denoise(dv, (1.0, 1.0, 1.0), "median3").float().cpu().numpy()
    ref = od.median3(dv.float().cpu().numpy())
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("spacing,sigma", [((1.0, 1.0, 1.0), 1.0), ((0.7, 1.1, 3.0), 1.5), ((1.0, 1.0, 1.0), 3.0)])
def test_gauss_fp32(spacing, sigma):
    rng = np.random.default_rng(4)
    v = rng.random((21, 34, 47)).astype(np.float32)
    got = dvr.denoise(to_dev(v), spacing, "gauss", sigma).cpu().numpy()
    ref = od.gauss(v, tuple(float(np.float32(h)) for h in spacing), float(np.float32(sigma)))
    assert rel_err(got, ref) <= 1e-6


def test_gauss_fp16_and_pipeline():
    w = phantoms.c1(64, 64)
    v16 = to_dev(w.vol, torch.float16)
    got = dvr.denoise(v16, w.spacing, "gauss", 1.0).float().cpu().numpy().astype(np.float64)
    ref = od.gauss(v16.float().cpu().numpy(), w.spacing, 1.0)
    r16 = ref.astype(np.float16).astype(np.float64)
    assert np.all(np.abs(got - r16) <= np.spacing(np.abs(r16).astype(np.float16)).astype(np.float64))
    # the denoised volume feeds the feature pass and the raymarch like any other
    d32 = dvr.denoise(to_dev(w.vol), w.spacing, "median3")
    f = dvr.features(d32, w.spacing, w.sigmas, c=w.c)
    img, _, _ = dvr.render(d32, f, to_dev(w.tf_knots), to_dev(w.tf_rgba), w.params,
                           [dvr.camera_struct(c) for c in w.cams], want_state=False)
    assert torch.isfinite(img).all() and img[..., 3].max() > 0
