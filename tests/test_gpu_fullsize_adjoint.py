"""Full-size parity of the gradients on the benchmarked workload (181x217x181 head, 3 scales, FP32
quad layout, perspective views at 1024^2), through the C ABI:
  * dvr_render_backward_features on four whole 1024^2 views: dL/dTF, dL/dI through the TF lookup
    (corners of samples within 1e-6 of a TF knot left out, counted) and dL/d(g, k, V, gmax) against
    the oracle render's reverse mode fed the GPU's own feature values (normwise <= 1e-4);
  * dvr_features_backward at sampled voxels: the oracle's feature adjoint is exact on a crop of
    half-width 2R + 1 around a voxel (R the largest stencil radius): dL/dI there depends on dL/dH
    within R and H within R of that, and the crop's clamped faces only change values within R of
    them; crops that reach the volume's faces keep its own clamping.  The gmax term is left out here
    (the arg-max is global; it is covered on whole volumes elsewhere), and voxels where two scales'
    V tie to 1e-4 get no V upstream."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_19737_amd as dvr
import phantoms
from oracle import feature_adjoint as fa
from paper_2605_19737_amd import _abi as abi
from tests.gpu_common import f32, feats_np, oracle_params, sp32, tf_dev, to_dev

pytestmark = pytest.mark.gpu


def _nerr(x, r):
    x = np.asarray(x, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.linalg.norm(x - r) / np.linalg.norm(r))


def test_head_full_size_gradients():
    w = phantoms.c2(1024, 1024, views=[0, 90, 200, 300])
    print("[full-size adjoint] head 181x217x181, sigma {1,2,3}, 4 views 1024^2, quad FP32", flush=True)
    dv = to_dev(w.vol)
    f = dvr.features(dv, w.spacing, w.sigmas, c=w.c, layout=abi.DVR_QUAD)
    kn, rg = tf_dev(w)
    img, T, k = dvr.render(dv, f, kn, rg, w.params, w.cams)
    rng = np.random.default_rng(21)
    dout = to_dev(0.1 * rng.normal(size=tuple(img.shape)))
    dtf, dvol, fg = dvr.render_backward(dv, f, kn, rg, w.params, w.cams, T, k, dout, want_features=True)
    torch.cuda.synchronize()
    fn = feats_np(f)
    I = dv.cpu().numpy().astype(np.float64)
    sp = sp32(w.spacing)
    rtf, rI, rfg, near = oracle.render_vjp(I, fn, fn["gmax"], sp, w.tf_knots, w.tf_rgba, oracle_params(w.params),
                                           w.cams, dout.cpu().numpy(), want_features=True, near_knot_eps=1e-6)
    errs = {key: _nerr(fg[key].cpu().numpy(), rfg[key]) for key in ("g", "kappa", "V")}
    errs["gmax"] = abs(float(fg["gmax"].item()) - rfg["gmax"]) / abs(rfg["gmax"])
    errs["tf"] = _nerr(dtf.cpu().numpy(), rtf)
    # dL/dI through the TF lookup, leaving out the corners of samples within 1e-6 of a TF knot (the TF
    # slope jumps there, so FP32 and FP64 may take different segments); counted
    keep = ~near
    errs["I"] = _nerr(dvol.cpu().numpy()[keep], rI[keep])
    e_all = _nerr(dvol.cpu().numpy(), rI)
    print("[full-size adjoint] render: " + " ".join(f"{a}={b:.2e}" for a, b in errs.items())
          + f" (near-knot voxels left out of dI: {int(near.sum())}; with them {e_all:.2e})", flush=True)
    assert all(v <= 1e-4 for v in errs.values()), errs

    # feature-pass adjoint at sampled voxels
    sig = [f32(s) for s in w.sigmas]
    Rmax = max(int(np.floor(3.0 * s / h + 0.5)) + 1 for s in sig for h in sp)
    M = 2 * Rmax + 1
    nz, ny, nx = I.shape
    gb = fg["g"].cpu().numpy().astype(np.float64)
    kb = fg["kappa"].cpu().numpy().astype(np.float64)
    Vb = fg["V"].cpu().numpy().astype(np.float64).copy()
    pick = [tuple(rng.integers(0, n) for n in I.shape) for _ in range(10)]
    big = np.argsort(np.abs(Vb).ravel())[-3:]
    pick += [tuple(int(x) for x in np.unravel_index(b, I.shape)) for b in big]
    pick += [(0, ny // 2, nx // 2), (nz - 1, 3, nx - 2), (nz // 2, 0, 5)]
    crops = []
    for v in pick:
        lo = [max(0, c - M) for c in v]
        hi = [min(n, c + M + 1) for c, n in zip(v, I.shape)]
        sl = tuple(slice(a, b) for a, b in zip(lo, hi))
        m = fa.forward(I[sl], sp, sig, c=f32(w.c))
        Vs = np.sort(m["Vs"], axis=0)
        tie = (Vs[-1] - Vs[-2]) <= 1e-4 * Vs[-1]
        Vb[sl][tie] = 0.0
        crops.append((v, sl))
    up = dict(g=to_dev(gb), kappa=to_dev(kb), V=to_dev(Vb), gmax=torch.zeros(1, dtype=torch.float32, device="cuda"))
    dI = dvr.features_backward(dv, w.spacing, w.sigmas, up, c=w.c).cpu().numpy().astype(np.float64)
    got, ref = [], []
    for v, sl in crops:
        d = fa.vjp(I[sl], sp, sig, 0.5, 0.5, f32(w.c), np.float32(gb[(slice(None),) + sl]).astype(np.float64),
                   np.float32(kb[sl]).astype(np.float64), np.float32(Vb[sl]).astype(np.float64), 0.0)
        local = tuple(c - s.start for c, s in zip(v, sl))
        got.append(dI[v])
        ref.append(d[local])
    got, ref = np.array(got), np.array(ref)
    e = float(np.abs(got - ref).max() / np.abs(ref).max())
    print(f"[full-size adjoint] feature adjoint at {len(pick)} sampled voxels: max err {e:.2e} of max |dI| "
          f"{np.abs(ref).max():.3e}", flush=True)
    assert np.abs(ref).max() > 0 and e <= 1e-4
