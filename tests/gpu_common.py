"""Helpers shared by the GPU parity tests: device inputs from the seeded phantoms, conversion of
the HIP path's outputs to NumPy, and the error measures the parity bar is stated in."""
from __future__ import annotations

import numpy as np
import torch

import paper_2605_19737_amd as dvr
from paper_2605_19737_amd import _abi as abi

DEV = "cuda"


def f32(x):
    """The float32 value the C ABI sees, as a Python float (what the oracle must be given)."""
    return float(np.float32(x))


def sp32(spacing):
    return tuple(f32(h) for h in spacing)


def rel_err(x, r):
    """max |x - r| / max |r| over an output array (the parity measure)."""
    x = np.asarray(x, np.float64)
    r = np.asarray(r, np.float64)
    den = np.abs(r).max()
    return float(np.abs(x - r).max() / den) if den > 0 else float(np.abs(x - r).max())


def to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype).contiguous()


def feats_np(f: dvr.Features):
    """(g [3][...], kappa, V, gmax, I or None) as float64 NumPy arrays."""
    torch.cuda.synchronize()
    if f.layout == abi.DVR_PLANAR:
        g = f.grad.float().cpu().numpy().astype(np.float64)
        k = f.kappa.float().cpu().numpy().astype(np.float64)
        V = f.ves.float().cpu().numpy().astype(np.float64)
        I = None
    elif f.layout in (abi.DVR_SPLIT, abi.DVR_QUAD):
        rec = f.grad.float().cpu().numpy().astype(np.float64)
        g = np.moveaxis(rec[..., 0:3], -1, 0)
        k = rec[..., 3]
        V = f.ves.float().cpu().numpy().astype(np.float64)
        if f.layout == abi.DVR_QUAD:
            V = V[..., 0]
        I = None
    else:
        rec = f.grad.float().cpu().numpy().astype(np.float64)
        g = np.moveaxis(rec[..., 1:4], -1, 0)
        k, V, I = rec[..., 4], rec[..., 5], rec[..., 0]
    return dict(g=g, kappa=k, V=V, gmax=float(f.gmax.item()), I=I)


def vessel_tie_mask(lam, tol=1e-5):
    """Voxels where |l1| and |l2| nearly tie with opposite signs at some scale: Frangi's V jumps
    there, so either side of the tie is a correct result (excluded from the V comparison)."""
    l1, l2, l3 = lam[:, 0], lam[:, 1], lam[:, 2]
    tie = (l1 * l2 < 0) & (np.abs(np.abs(l1) - np.abs(l2)) < tol * np.abs(l3))
    return tie.any(axis=0)


def tf_dev(w):
    return to_dev(w.tf_knots), to_dev(w.tf_rgba)


def oracle_params(params):
    return {k: f32(v) for k, v in params.items()}
