"""CPU pin of the oracle's reverse mode at the differentiable-render workload's stated scope: the
32^3 crop [48, 80)^3 of the 128^3 phantom with its features taken from the pass over the whole
volume, 8 orthographic views at 64^2, L2 loss against the image of the perturbed 16-knot TF.
Every one of the 64 TF values and every one of the 32,768 crop voxels is compared with FP64 central
differences (h = 1e-4); voxels whose perturbation can move a sample across a TF knot (a sample
within w h of a knot, w the voxel's trilinear weight in it: the loss has a kink there and a central
difference is not the derivative) are excluded and counted."""
import numpy as np
import pytest

import oracle
from tests import fd_common as fc


@pytest.fixture(scope="module")
def crop():
    s = fc.CropScene()
    of = s.oracle_features()
    target = s.target(of)
    base = s.render(of)
    dtf, dI, kink = oracle.render_vjp(s.vol, of, of["gmax"], s.spacing, s.knots, s.tf, s.params, s.cams,
                                      base["rgba"] - target, near_knot_eps=fc.H_FD, near_knot_weighted=True)
    return s, of, target, dtf, dI, kink


def test_footprint_covers_every_changed_pixel(crop):
    """The pixel footprint of a voxel holds every pixel whose loss changes when that voxel changes
    (checked against whole-image renders at interior, face, edge and corner voxels)."""
    s, of, target, _, _, _ = crop
    l0 = fc.pixel_losses(s.render(of)["rgba"], target)
    for v in [(15, 16, 24), (30, 1, 4), (0, 0, 0), (31, 31, 31), (16, 0, 31), (0, 17, 9)]:
        vol = s.vol.copy()
        vol[v[2], v[1], v[0]] += 1e-3
        l1 = fc.pixel_losses(s.render(of, vol=vol)["rgba"], target)
        changed = {tuple(c) for c in np.argwhere(l1 != l0).tolist()}
        pix = s.footprint(v)
        inset = {(int(c), int(j), int(i)) for c, i, j in pix}
        assert changed and changed <= inset, v


def test_tf_gradient_against_fd(crop):
    s, of, target, dtf, _, _ = crop
    fd = fc.fd_tf(s, of, target)
    e = np.linalg.norm(dtf - fd) / np.linalg.norm(fd)
    print(f"[oracle-fd crop] dTF err {e:.2e} over {fd.size} values", flush=True)
    assert e <= 1e-6


def test_voxel_gradient_against_fd_every_voxel(crop):
    s, of, target, _, dI, kink = crop
    fd, onesided = fc.fd_voxels(s, of, target)
    keep = ~kink
    e = np.linalg.norm(dI[keep] - fd[keep]) / np.linalg.norm(fd[keep])
    print(f"[oracle-fd crop] dI err {e:.2e} over {int(keep.sum())} voxels; {int(kink.sum())} ({kink.mean():.2%}) "
          f"have a sample within w h of a TF knot; one-sided differences disagree on {int(onesided.sum())}, "
          f"{int((onesided & keep).sum())} of them kept", flush=True)
    assert kink.mean() < 0.5
    assert e <= 1e-6
