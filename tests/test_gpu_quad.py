"""The quad feature layout (the split records; V and the intensity as per-voxel (y, z) quads) holds
the split layout's values, its quads are the shifted fields with zeros past the last row and slice,
and it renders the split layout's bits: the raymarch interpolates the same corner values in the same
order.  The adjoint, with and without the feature gradients, matches the split layout's to the
rounding of its atomic sums."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_19737_amd as dvr
import phantoms
from paper_2605_19737_amd import _abi as abi
from tests.gpu_common import f32, feats_np, oracle_params, rel_err, sp32, to_dev

pytestmark = pytest.mark.gpu


def _quads(a):
    """Reference quads of a [nz][ny][nx] array: (a(y,z), a(y+1,z), a(y,z+1), a(y+1,z+1)), 0 outside."""
    nz, ny, nx = a.shape
    p = np.zeros((nz + 1, ny + 1, nx), a.dtype)
    p[:nz, :ny] = a
    return np.stack([p[:nz, :ny], p[:nz, 1:], p[1:, :ny], p[1:, 1:]], -1)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_quad_features_equal_split(dtype):
    w = phantoms.c2(64, 64, nviews=1)
    v = to_dev(w.vol, dtype)
    fs = dvr.features(v, w.spacing, w.sigmas, c=w.c, dtype=dtype, layout=abi.DVR_SPLIT)
    fq = dvr.features(v, w.spacing, w.sigmas, c=w.c, dtype=dtype, layout=abi.DVR_QUAD)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(fs.grad.cpu().numpy(), fq.grad.cpu().numpy())
    assert fs.gmax.item() == fq.gmax.item()
    # bit copies: compare the raw element bits
    it = np.uint32 if dtype == torch.float32 else np.uint16
    vb = fs.ves.cpu().numpy().view(it)
    np.testing.assert_array_equal(fq.ves.cpu().numpy().view(it), _quads(vb))
    np.testing.assert_array_equal(fq.iquad.cpu().numpy().view(it), _quads(v.cpu().numpy().view(it)))
    np.testing.assert_array_equal(fs.brick_minmax().cpu().numpy(), fq.brick_minmax().cpu().numpy())


def test_quad_features_odd_small_grid():
    """A 2x3x5 grid: every voxel sits on a last row or slice or next to one."""
    rng = np.random.default_rng(5)
    vol = rng.uniform(0, 1, (5, 3, 2))
    v = to_dev(vol)
    fs = dvr.features(v, (1.0, 1.0, 1.0), [1.0], c=0.1, layout=abi.DVR_SPLIT)
    fq = dvr.features(v, (1.0, 1.0, 1.0), [1.0], c=0.1, layout=abi.DVR_QUAD)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(fq.ves.cpu().numpy(), _quads(fs.ves.cpu().numpy()))
    np.testing.assert_array_equal(fq.iquad.cpu().numpy(), _quads(v.cpu().numpy()))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_quad_render_equals_split_and_oracle(dtype):
    w = phantoms.c2(128, 96, nviews=3)
    v = to_dev(w.vol, dtype)
    cams = [dvr.camera_struct(c) for c in w.cams]
    kn, tf = to_dev(w.tf_knots), to_dev(w.tf_rgba)
    fs = dvr.features(v, w.spacing, [1.0, 2.0], c=w.c, dtype=dtype, layout=abi.DVR_SPLIT)
    fq = dvr.features(v, w.spacing, [1.0, 2.0], c=w.c, dtype=dtype, layout=abi.DVR_QUAD)
    for skip in (True, False):
        a = dvr.render(v, fs if skip else fs.without_bricks(), kn, tf, w.params, cams)
        # the quad layout reads its own intensity copy: the volume argument is not sampled
        b = dvr.render(torch.zeros_like(v), fq if skip else fq.without_bricks(), kn, tf, w.params, cams)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    if dtype == torch.float32:
        img = b[0].cpu().numpy()
        fsn = feats_np(fq)
        ref = oracle.render(v.cpu().numpy().astype(np.float64), fsn, fsn["gmax"], sp32(w.spacing), w.tf_knots,
                            w.tf_rgba, oracle_params(w.params), w.cams)
        et = f32(w.params["et_alpha"])
        T = ref["T_last"]
        excl = np.abs(T - (1 - et)) <= 1e-5 * (1 - et)
        for ch in range(4):
            assert rel_err(img[..., ch][~excl], ref["rgba"][..., ch][~excl]) <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_quad_adjoint_matches_split(dtype):
    w = phantoms.c3(96, 96)
    v = to_dev(w.vol, dtype)
    cams = [dvr.camera_struct(c) for c in w.cams[:3]]
    kn, tf = to_dev(w.tf_knots), to_dev(w.tf_rgba)
    tgt = to_dev(w.extra["target_tf_rgba"])
    out = []
    for lay in (abi.DVR_SPLIT, abi.DVR_QUAD):
        f = dvr.features(v, w.spacing, w.sigmas, c=w.c, dtype=dtype, layout=lay)
        img, T, k = dvr.render(v, f, kn, tf, w.params, cams)
        target, _, _ = dvr.render(v, f, kn, tgt, w.params, cams, want_state=False)
        dtf, dI = dvr.render_backward(v, f, kn, tf, w.params, cams, T, k, img - target)
        dtf2, dI2, fg = dvr.render_backward(v, f, kn, tf, w.params, cams, T, k, img - target, want_features=True)
        out.append([x.cpu().numpy().astype(np.float64) for x in (img, dtf, dI, dtf2, dI2, fg["packed"], fg["gmax"])])
    for i, (a, b) in enumerate(zip(*out)):
        if i == 0:
            np.testing.assert_array_equal(a, b)
        else:
            assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(a), i
    print(f"[quad] {dtype}: adjoint |dI| {np.linalg.norm(out[1][2]):.3e}, feature grads "
          f"|dfeat| {np.linalg.norm(out[1][5]):.3e} match the split layout", flush=True)


def test_quad_needs_matching_volume_dtype():
    w = phantoms.c1(32, 32)
    v = to_dev(w.vol)
    with pytest.raises(abi.DVRError):
        dvr.features(v, w.spacing, w.sigmas, c=w.c, dtype=torch.float16, layout=abi.DVR_QUAD)


@pytest.mark.parametrize("dims", [(2, 3, 5), (2, 2, 2), (7, 2, 3)])
def test_quad_render_tiny_grids(dims):
    """Grids where every cell touches a last row or slice (the quads' zero padding sits under the
    weight-0 corners of samples on the faces): the same bits as the split layout, and the oracle."""
    sp = (1.0, 0.9, 1.2)
    vol = phantoms.small_random(11, dims, sp, lo=0.05, hi=0.95)
    v = to_dev(vol)
    knots = np.float32([0.0, 0.3, 0.6, 1.0]).astype(np.float64)
    rgba = np.float32([[0.2, 0.4, 0.6, 0.5], [0.9, 0.3, 0.1, 1.2], [0.1, 0.8, 0.3, 0.8],
                       [0.7, 0.7, 0.9, 1.5]]).astype(np.float64)
    kn, tf = to_dev(knots), to_dev(rgba)
    prm = phantoms.render_params(lambda_g=0.6, lambda_k=0.4, kappa0=0.05, lambda_v=1.0, step_vox=0.25)
    cams = [phantoms.ortho_camera(dims, sp, 30.0, 20.0, 24, 20), phantoms.persp_camera(dims, sp, 200.0, -35.0, 24, 20)]
    cs = [dvr.camera_struct(c) for c in cams]
    fs = dvr.features(v, sp, [1.0], c=0.1, layout=abi.DVR_SPLIT).without_bricks()
    fq = dvr.features(v, sp, [1.0], c=0.1, layout=abi.DVR_QUAD).without_bricks()
    a = dvr.render(v, fs, kn, tf, prm, cs)
    b = dvr.render(v, fq, kn, tf, prm, cs)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    fn = feats_np(fq)
    ref = oracle.render(v.cpu().numpy().astype(np.float64), fn, fn["gmax"], sp32(sp), knots, rgba,
                        oracle_params(prm), cams)
    img = b[0].cpu().numpy()
    assert ref["rgba"][..., 3].max() > 0.05
    for ch in range(4):
        assert rel_err(img[..., ch], ref["rgba"][..., ch]) <= 1e-5


def test_head_fp16_quad_full_size_sampled():
    """The FP16 leg as the benchmark times it: the head with FP16 quad-layout features (no brick
    table), 1024^2 perspective views, against the oracle fed the same stored FP16 values (intensity
    from the quads, g, k from the records, V from the V quads) on 4000 sampled pixels."""
    w = phantoms.c2(1024, 1024, views=[0, 120, 250])
    v16 = to_dev(w.vol, torch.float16)
    f = dvr.features(v16, w.spacing, w.sigmas, c=w.c, dtype=torch.float16, layout=abi.DVR_QUAD).without_bricks()
    kn, tf = to_dev(w.tf_knots), to_dev(w.tf_rgba)
    img, T, k = dvr.render(None, f, kn, tf, w.params, [dvr.camera_struct(c) for c in w.cams])
    torch.cuda.synchronize()
    rec = f.grad.float().cpu().numpy().astype(np.float64)
    feats = dict(g=np.ascontiguousarray(np.moveaxis(rec[..., 0:3], -1, 0)), kappa=rec[..., 3].copy(),
                 V=f.ves.float().cpu().numpy().astype(np.float64)[..., 0].copy())
    vin = f.iquad.float().cpu().numpy().astype(np.float64)[..., 0].copy()
    np.testing.assert_array_equal(vin, v16.float().cpu().numpy())
    rng = np.random.default_rng(16)
    M = 4000
    pix = np.stack([rng.integers(0, 3, M), rng.integers(0, 1024, M), rng.integers(0, 1024, M)], 1).astype(np.int32)
    ref = oracle.render(vin, feats, float(f.gmax.item()), sp32(w.spacing), w.tf_knots, w.tf_rgba,
                        oracle_params(w.params), w.cams, pix=pix)
    got = img.cpu().numpy()[pix[:, 0], pix[:, 2], pix[:, 1]].astype(np.float64)
    et = f32(w.params["et_alpha"])
    excl = np.abs(ref["T_last"] - (1 - et)) <= 1e-5 * (1 - et)
    eb = [rel_err(got[~excl, ch], ref["rgba"][~excl, ch]) for ch in range(4)]
    print(f"[quad fp16 head 1024^2] compute error vs oracle on the stored values: {['%.2e' % e for e in eb]}, "
          f"ET-boundary rays excluded {int(excl.sum())}/{M}", flush=True)
    assert max(eb) <= 1e-5 and excl.mean() < 1e-3
