"""Exact empty-space skipping: the brick table holds each brick's intensity (min, max) exactly, and a
raymarch that steps over bricks mapping onto zero extinction returns the same bits (image, ray state
and sample counts) as one that visits every sample.  The parity of skipping renders against the FP64
oracle is covered by every other render test, since the binding builds the brick table by default."""
import numpy as np
import pytest
import torch

import paper_2605_19737_amd as dvr
import phantoms
from paper_2605_19737_amd import _abi as abi
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu


def _brick_ref(I):
    """(nbz, nby, nbx, 2) min/max over the voxels [4b, min(4b + 4, n - 1)] of each axis."""
    B = abi.DVR_BRICK
    nz, ny, nx = I.shape
    nb = [(n - 1 + B - 1) // B for n in I.shape]
    out = np.empty((*nb, 2), np.float32)
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                blk = I[bz * B:min(bz * B + B, nz - 1) + 1, by * B:min(by * B + B, ny - 1) + 1,
                        bx * B:min(bx * B + B, nx - 1) + 1]
                out[bz, by, bx] = (blk.min(), blk.max())
    return out


@pytest.mark.parametrize("layout,dtype", [(abi.DVR_PLANAR, torch.float32), (abi.DVR_INTERLEAVED, torch.float16),
                                          (abi.DVR_INTERLEAVED, torch.float32), (abi.DVR_PLANAR, torch.float16)])
def test_brick_table_exact(layout, dtype):
    rng = np.random.default_rng(3)
    for shape in [(13, 18, 21), (2, 2, 2), (9, 5, 17)]:
        vol = rng.random(shape).astype(np.float32)
        dv = to_dev(vol, dtype)
        f = dvr.features(dv, (1.0, 0.8, 1.3), [1.0], c=0.2, dtype=dtype, layout=layout)
        torch.cuda.synchronize()
        # the intensity the raymarcher samples: the volume (planar) or the records' I (interleaved)
        I = dv.float().cpu().numpy() if layout == abi.DVR_PLANAR else f.grad[..., 0].float().cpu().numpy()
        np.testing.assert_array_equal(f.brick_minmax().cpu().numpy(), _brick_ref(I))


def _both(dv, f, knots, rgba, params, cams):
    """(image, T_last, k_last, counters) with and without the brick table."""
    out = []
    for ff in (f, f.without_bricks()):
        cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
        img, T, k = dvr.render(dv if f.layout == abi.DVR_PLANAR else None, ff, knots, rgba, params, cams,
                               counters=cnt)
        torch.cuda.synchronize()
        out.append((img.cpu().numpy(), T.cpu().numpy(), k.cpu().numpy(), cnt.cpu().numpy()))
    return out


def _assert_same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def _zero_band_tf(lo, hi):
    """8 knots with zero extinction on [lo, hi] (and below), colour everywhere."""
    knots = np.array([0.0, lo, hi, hi + 0.05, 0.5, 0.7, 0.85, 1.0], np.float32)
    rgba = np.array([[0.1, 0.1, 0.1, 0.0], [0.2, 0.3, 0.4, 0.0], [0.5, 0.4, 0.3, 0.0], [0.6, 0.5, 0.2, 0.3],
                     [0.9, 0.6, 0.5, 0.6], [1.0, 0.9, 0.8, 0.2], [0.8, 0.3, 0.2, 1.5], [1.0, 0.2, 0.1, 3.0]],
                    np.float32)
    return to_dev(knots), to_dev(rgba)


@pytest.mark.parametrize("et", [0.0, 0.99])
@pytest.mark.parametrize("step", [0.5, 0.37])
def test_skip_bit_exact_head(et, step):
    """Head phantom (background noise in the zero-extinction band), perspective and orthographic
    views, with and without early termination, two step sizes."""
    w = phantoms.c2(160, 128, nviews=4)
    dv = to_dev(w.vol)
    f = dvr.features(dv, w.spacing, [1.0], c=w.c)
    kn, tf = _zero_band_tf(0.1, 0.15)
    params = dict(w.params, et_alpha=et, step_vox=step)
    cams = [dvr.camera_struct(c) for c in w.cams]
    cams += [dvr.camera_struct(phantoms.ortho_camera((181, 217, 181), (1.0, 1.0, 1.0), a, 25.0, 160, 128))
             for a in (10.0, 100.0)]
    a, b = _both(dv, f, kn, tf, params, cams[:4])
    _assert_same(a, b)
    a, b = _both(dv, f, kn, tf, params, cams[4:])
    _assert_same(a, b)
    mm = f.brick_minmax().cpu().numpy()
    assert (mm[..., 1] < 0.1).mean() > 0.1  # some bricks really are skipped


def test_skip_bit_exact_fp16_records_and_extremes():
    """FP16 records; a TF with zero extinction everywhere (every brick empty: transparent image, the
    last sample reached on every ray) and one with none."""
    w = phantoms.c1(96, 96)
    dv = to_dev(w.vol, torch.float16)
    f = dvr.features(dv, w.spacing, w.sigmas, c=w.c, dtype=torch.float16, layout=abi.DVR_INTERLEAVED)
    cams = [dvr.camera_struct(c) for c in w.cams]
    cams += [dvr.camera_struct(phantoms.persp_camera((64, 64, 64), (1.0, 1.0, 1.0), 33.0, -12.0, 96, 96))]
    cams = cams[:1] + cams[-1:]
    for kn, tf in [_zero_band_tf(0.1, 0.15), _zero_band_tf(0.3, 0.5)]:
        a, b = _both(dv, f, kn, tf, w.params, cams)
        _assert_same(a, b)
    kn = to_dev(np.array([0.0, 1.0], np.float32))
    zero = to_dev(np.array([[0.5, 0.5, 0.5, 0.0], [1.0, 1.0, 1.0, 0.0]], np.float32))
    a, b = _both(dv, f, kn, zero, w.params, cams)
    _assert_same(a, b)
    img, T, k, cnt = a
    assert not img.any() and np.all(T[k >= 0] == 1.0)
    full = to_dev(np.array([[0.5, 0.5, 0.5, 0.05], [1.0, 1.0, 1.0, 0.2]], np.float32))
    a, b = _both(dv, f, kn, full, w.params, cams)
    _assert_same(a, b)
