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


def floor_rate(x, r, tol=1e-5):
    """Elementwise rate with a floor: the share of elements where |x - r| > tol (|r| + 1e-3 max|r|).
    It shows large relative errors on small elements that max|x - r| / max|r| alone can hide."""
    x = np.asarray(x, np.float64)
    r = np.asarray(r, np.float64)
    if r.size == 0:
        return 0.0, 0
    bad = np.abs(x - r) > tol * (np.abs(r) + 1e-3 * np.abs(r).max())
    return float(bad.mean()), int(bad.sum())


def fmt_rates(pairs):
    """'name=rate (count)' for a list of (name, x, r)."""
    out = []
    for name, x, r in pairs:
        fr, n = floor_rate(x, r)
        out.append(f"{name}={fr:.1e} ({n})")
    return " ".join(out)


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


def vessel_tie_mask(lam, tol=1e-5, tol_vol=1e-6):
    """Voxels where |l1| and |l2| nearly tie with opposite signs at some scale: Frangi's V jumps
    there, so either side of the tie is a correct result (excluded from the V comparison).  Near
    tie: ||l1| - |l2|| below tol |l3| (the voxel's own scale) or below tol_vol times the largest |l|
    of that scale over the volume: the FP32 stencils' error in sigma^2 H is absolute, set by the
    data's magnitude, so on voxels with small eigenvalues a tie can flip well inside tol |l3|'s reach
    of the volume's scale (seen at ~3e-7 of it on a thick-slice volume)."""
    l1, l2, l3 = lam[:, 0], lam[:, 1], lam[:, 2]
    vmax = np.abs(lam).reshape(lam.shape[0], -1).max(axis=1).reshape((-1,) + (1,) * (lam.ndim - 2))
    d = np.abs(np.abs(l1) - np.abs(l2))
    tie = (l1 * l2 < 0) & ((d < tol * np.abs(l3)) | (d < tol_vol * vmax))
    return tie.any(axis=0)


def tf_dev(w):
    return to_dev(w.tf_knots), to_dev(w.tf_rgba)


def oracle_params(params):
    return {k: f32(v) for k, v in params.items()}


def compare_images(got, T_got, k_got, ref, et, label, pix=None, tol=1e-5):
    """Per-channel image parity with the early-termination boundary exclusion: rays whose oracle
    transmittance at the stop sample lies within 1e-5 (relative) of 1 - et may take one sample more
    or less (excluded, counted, < 0.1 %).  RGBA and T_last within tol of each output's range, k_last
    equal; the floor rate of every output is printed."""
    img = got.cpu().numpy().astype(np.float64)
    Tg = T_got.cpu().numpy()
    kg = k_got.cpu().numpy()
    if pix is not None:
        img = img[pix[:, 0], pix[:, 2], pix[:, 1]]
        Tg = Tg[pix[:, 0], pix[:, 2], pix[:, 1]]
        kg = kg[pix[:, 0], pix[:, 2], pix[:, 1]]
    r = ref["rgba"].reshape(img.shape)
    rk = ref["k_last"].reshape(kg.shape)
    rT = ref["T_last"].reshape(Tg.shape)
    excl = np.zeros(kg.shape, bool)
    if et > 0:
        # oracle T after the stop sample near 1 - et: either side is a correct stop
        Tend = 1.0 - r[..., 3]
        excl = np.abs(Tend - (1.0 - et)) <= 1e-5 * (1.0 - et)
        excl |= np.abs(rT - (1.0 - et)) <= 1e-5 * (1.0 - et)
    errs = [rel_err(img[..., ch][~excl], r[..., ch][~excl]) for ch in range(4)]
    keep = ~excl & ((1.0 - r[..., 3]) > 1e-6)
    # T before the last sample: defined where both sides stop at the same sample (k_last compared
    # below); misses carry no T
    hit = keep & (rk >= 0)
    e_T = rel_err(Tg[hit], rT[hit]) if hit.any() else 0.0
    rates = fmt_rates([(n, img[..., ch][~excl], r[..., ch][~excl]) for ch, n in enumerate("RGBA")] +
                      [("T_last", Tg[hit], rT[hit])])
    print(f"[render] {label}: err R={errs[0]:.2e} G={errs[1]:.2e} B={errs[2]:.2e} A={errs[3]:.2e} "
          f"T_last={e_T:.2e} excluded={int(excl.sum())}/{excl.size}; floor rates {rates}", flush=True)
    assert excl.mean() < 1e-3
    assert max(errs) <= tol
    assert e_T <= tol, f"T_last err {e_T:.2e}"
    mism = (kg != rk) & keep
    assert np.all(kg[rk < 0] == -1)
    assert mism.sum() == 0, f"k_last differs on {int(mism.sum())} rays"


def compare_features(got, ref, label, tol=1e-5):
    """Feature parity against the oracle (ref from oracle.features(..., want_lam=True)): g, kappa
    and V within tol of each output's range (V without Frangi's opposite-sign magnitude ties, < 0.2 %
    of the voxels), |g|_max to 1e-6; floor rates printed.  Returns the errors."""
    e_g = rel_err(got["g"], ref["g"])
    e_k = rel_err(got["kappa"], ref["kappa"])
    tie = vessel_tie_mask(ref["lam"])
    e_v = rel_err(got["V"][~tie], ref["V"][~tie])
    e_m = abs(got["gmax"] - ref["gmax"]) / ref["gmax"]
    rates = fmt_rates([("g", got["g"], ref["g"]), ("kappa", got["kappa"], ref["kappa"]),
                       ("V", got["V"][~tie], ref["V"][~tie])])
    print(f"[features] {label}: err g={e_g:.2e} kappa={e_k:.2e} V={e_v:.2e} gmax={e_m:.2e} ties={int(tie.sum())}; "
          f"floor rates {rates}", flush=True)
    assert tie.mean() < 2e-3
    assert e_g <= tol and e_k <= tol and e_v <= tol
    assert e_m <= 1e-6
    return dict(g=e_g, kappa=e_k, V=e_v, gmax=e_m)

