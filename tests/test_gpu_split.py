"""The split feature layout (I and V planes, a (gx, gy, gz, k) record) holds the same values as the
planar one and renders the same bits: the features are computed by the same arithmetic, and the
raymarch interpolates the same corner values in the same order.  The adjoint matches to the
rounding of its atomic sums (their order is not fixed)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_19737_amd as dvr
import phantoms
from paper_2605_19737_amd import _abi as abi
from tests.gpu_common import f32, feats_np, oracle_params, rel_err, sp32, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_split_features_equal_planar(dtype):
    w = phantoms.c2(64, 64, nviews=1)
    v = to_dev(w.vol, dtype)
    fp = dvr.features(v, w.spacing, w.sigmas, c=w.c, dtype=dtype, layout=abi.DVR_PLANAR)
    fs = dvr.features(v, w.spacing, w.sigmas, c=w.c, dtype=dtype, layout=abi.DVR_SPLIT)
    a, b = feats_np(fp), feats_np(fs)
    for k in ("g", "kappa", "V"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["gmax"] == b["gmax"]
    np.testing.assert_array_equal(fp.brick_minmax().cpu().numpy(), fs.brick_minmax().cpu().numpy())


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_split_render_equals_planar_and_oracle(dtype):
    w = phantoms.c2(128, 96, nviews=3)
    v = to_dev(w.vol, dtype)
    cams = [dvr.camera_struct(c) for c in w.cams]
    kn, tf = to_dev(w.tf_knots), to_dev(w.tf_rgba)
    fp = dvr.features(v, w.spacing, [1.0, 2.0], c=w.c, dtype=dtype, layout=abi.DVR_PLANAR)
    fs = dvr.features(v, w.spacing, [1.0, 2.0], c=w.c, dtype=dtype, layout=abi.DVR_SPLIT)
    for skip in (True, False):
        a = dvr.render(v, fp if skip else fp.without_bricks(), kn, tf, w.params, cams)
        b = dvr.render(v, fs if skip else fs.without_bricks(), kn, tf, w.params, cams)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    if dtype == torch.float32:
        img = b[0].cpu().numpy()
        fsn = feats_np(fs)
        ref = oracle.render(v.cpu().numpy().astype(np.float64), fsn, fsn["gmax"], sp32(w.spacing), w.tf_knots,
                            w.tf_rgba, oracle_params(w.params), w.cams)
        et = f32(w.params["et_alpha"])
        T = ref["T_last"]
        excl = np.abs(T - (1 - et)) <= 1e-5 * (1 - et)
        for ch in range(4):
            assert rel_err(img[..., ch][~excl], ref["rgba"][..., ch][~excl]) <= 1e-5


def test_split_adjoint_matches_planar():
    w = phantoms.c3(96, 96)
    v = to_dev(w.vol)
    cams = [dvr.camera_struct(c) for c in w.cams[:3]]
    kn, tf = to_dev(w.tf_knots), to_dev(w.tf_rgba)
    tgt = to_dev(w.extra["target_tf_rgba"])
    out = []
    for lay in (abi.DVR_PLANAR, abi.DVR_SPLIT):
        f = dvr.features(v, w.spacing, w.sigmas, c=w.c, layout=lay)
        img, T, k = dvr.render(v, f, kn, tf, w.params, cams)
        target, _, _ = dvr.render(v, f, kn, tgt, w.params, cams, want_state=False)
        dtf, dI = dvr.render_backward(v, f, kn, tf, w.params, cams, T, k, img - target)
        out.append((dtf.cpu().numpy(), dI.cpu().numpy()))
    (a1, b1), (a2, b2) = out
    assert np.linalg.norm(a1 - a2) <= 1e-6 * np.linalg.norm(a1)
    assert np.linalg.norm(b1 - b2) <= 1e-6 * np.linalg.norm(b1)
