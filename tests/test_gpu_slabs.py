"""The one-GPU part of a z-slab decomposition over several GPUs, on the head workload:
  * the feature pass of one slab with an input halo of R slices (R the largest stencil radius)
    gives the same bits as the whole volume on the slab's own slices (a voxel reads only voxels
    within R of it, through the same code);
  * the raymarch of two slabs that meet at a node plane, composited with "over",
    (C1 + T1 C2, T1 T2), equals the raymarch of the whole volume (axis-parallel orthographic rays
    whose segments end on the plane; the features and gmax of the whole volume)."""
import numpy as np
import pytest
import torch

import paper_2605_19737_amd as dvr
import phantoms
from paper_2605_19737_amd import _abi as abi
from tests.gpu_common import tf_dev, to_dev

pytestmark = pytest.mark.gpu


def test_feature_slab_with_halo_is_bit_exact():
    w = phantoms.c2(8, 8, views=[0])
    dv = to_dev(w.vol)
    full = dvr.features(dv, w.spacing, w.sigmas, c=w.c, layout=abi.DVR_SPLIT)
    R = max(int(np.floor(3.0 * s / h + 0.5)) + 1 for s in w.sigmas for h in w.spacing)
    z0, z1 = 60, 120
    sub = dv[z0 - R:z1 + R].clone()
    part = dvr.features(sub, w.spacing, w.sigmas, c=w.c, layout=abi.DVR_SPLIT)
    torch.cuda.synchronize()
    a = full.grad[z0:z1].cpu().numpy()
    b = part.grad[R:R + (z1 - z0)].cpu().numpy()
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(full.ves[z0:z1].cpu().numpy(), part.ves[R:R + (z1 - z0)].cpu().numpy())
    print(f"[slabs] features of slices {z0}..{z1} with a {R}-slice halo: bit-identical (g, k, V)", flush=True)


def test_slab_renders_composite_over():
    w = phantoms.c2(8, 8, views=[0])
    dv = to_dev(w.vol)
    f = dvr.features(dv, w.spacing, w.sigmas, c=w.c, layout=abi.DVR_SPLIT)
    kn, rg = tf_dev(w)
    nz, ny, nx = dv.shape
    # orthographic rays along +z through the whole (x, y) extent, pixel centres off the nodes
    W, H = 128, 160
    du = np.array([(nx - 1) / W, 0, 0], np.float32)
    dvv = np.array([0, (ny - 1) / H, 0], np.float32)
    cam = phantoms.Camera(0, W, H, np.array([-0.5 * du[0] + 0.37 * du[0], -0.5 * dvv[1] + 0.41 * dvv[1], -4.0],
                                             np.float32), np.array([0, 0, 1], np.float32), du, dvv)
    params = dict(w.params, et_alpha=0.0)  # no early termination: each slab marches to its face
    full, _, _ = dvr.render(dv, f, kn, rg, params, [cam], want_state=False)
    m = 90  # node plane; 0.5-voxel segments end on it from both sides

    def slab(z0, z1):
        g = f.grad[z0:z1].clone()
        v = f.ves[z0:z1].clone()
        fs = dvr.Features(grad=g, kappa=None, ves=v, gmax=f.gmax, layout=f.layout, shape=tuple(v.shape),
                          spacing=f.spacing, bricks=None)
        c = phantoms.Camera(0, W, H, (cam.o - np.array([0, 0, z0], np.float32)).astype(np.float32), cam.d0, cam.du,
                            cam.dv)
        img, _, _ = dvr.render(dv[z0:z1].clone(), fs, kn, rg, params, [c], want_state=False)
        return img.cpu().numpy().astype(np.float64)

    a = slab(0, m + 1)
    b = slab(m, nz)
    T1, T2 = 1.0 - a[..., 3], 1.0 - b[..., 3]
    over = np.concatenate([a[..., :3] + T1[..., None] * b[..., :3], (1.0 - T1 * T2)[..., None]], -1)
    ref = full.cpu().numpy().astype(np.float64)
    err = np.abs(over - ref).max() / np.abs(ref).max()
    print(f"[slabs] two slabs composited over vs the whole volume: max err {err:.2e} of the range; "
          f"mean A {ref[..., 3].mean():.3f}", flush=True)
    assert ref[..., 3].max() > 0.5 and err <= 1e-5
