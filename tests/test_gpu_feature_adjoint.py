"""GPU parity of the feature-pass adjoint (through the C ABI) against the oracle:
  * dvr_render_backward_features: dL/d(g, k, V, gmax) against the oracle render's reverse mode fed
    the GPU's own feature values, for every feature layout, normwise <= 1e-4;
  * dvr_features_backward: dL/dI for random upstream gradients against oracle/feature_adjoint.py
    on ragged, anisotropic, multi-scale volumes spanning several tiles, normwise <= 1e-4; voxels
    where two scales' V tie to 1e-4 (either scale is a correct choice of the derivative of the max)
    get no V upstream;
  * end to end: dL/dI through the TF lookup plus through the features, against the oracle's.
Voxels that are corners of a sample within 1e-6 of a TF knot are left out of the dL/dI comparisons
(the TF slope jumps there, so FP32 and FP64 may take different segments), and counted."""
import numpy as np
import pytest
import torch

import oracle
import paper_2605_19737_amd as dvr
import phantoms
from oracle import feature_adjoint as fa
from paper_2605_19737_amd import _abi as abi
from tests import bruteforce as bf
from tests.gpu_common import f32, feats_np, oracle_params, sp32, tf_dev, to_dev

pytestmark = pytest.mark.gpu


def _nerr(x, r):
    x = np.asarray(x, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.linalg.norm(x - r) / np.linalg.norm(r))


def _diff_scene(n=48):
    w = phantoms.c3(n, n, views=[0, 3])
    w.vol = w.vol[40:40 + n, 40:40 + n, 40:40 + n].copy()
    w.cams = [phantoms.ortho_camera(w.dims, w.spacing, 45.0 * k + 5, 20.0, n, n) for k in (0, 3)]
    return w


@pytest.mark.parametrize("layout,dtype,K", [(abi.DVR_PLANAR, torch.float32, 16), (abi.DVR_SPLIT, torch.float32, 16),
                                            (abi.DVR_INTERLEAVED, torch.float16, 16), (abi.DVR_SPLIT, torch.float16, 16),
                                            (abi.DVR_PLANAR, torch.float16, 16), (abi.DVR_SPLIT, torch.float32, 40),
                                            (abi.DVR_INTERLEAVED, torch.float32, 6)])
def test_render_feature_grads_match_oracle(layout, dtype, K):
    w = _diff_scene()
    if K != len(w.tf_knots):
        # a TF with K knots (the K <= 8 and K <= 64 kernel variants)
        rng = np.random.default_rng(K)
        w.tf_knots = np.sort(np.concatenate([[0.0, 1.0], rng.uniform(0.02, 0.98, K - 2)])).astype(np.float32)
        w.tf_rgba = np.concatenate([rng.uniform(0, 1, (K, 3)), rng.uniform(0.0, 0.2, (K, 1))], 1).astype(np.float32)
    print(f"[render feature grads] layout={layout} dtype={dtype} K={K}", flush=True)
    dv = to_dev(w.vol, dtype)
    f = dvr.features(dv, w.spacing, w.sigmas, c=w.c, dtype=dtype, layout=layout)
    kn, rg = tf_dev(w)
    vol_arg = dv if layout != abi.DVR_INTERLEAVED else None
    img, T, k = dvr.render(vol_arg, f, kn, rg, w.params, w.cams)
    rng = np.random.default_rng(11)
    dout = to_dev(rng.normal(size=tuple(img.shape)))
    dtf, dvol, fg = dvr.render_backward(vol_arg, f, kn, rg, w.params, w.cams, T, k, dout, want_features=True)
    dtf0, dvol0 = dvr.render_backward(vol_arg, f, kn, rg, w.params, w.cams, T, k, dout)
    torch.cuda.synchronize()
    fn = feats_np(f)
    I = fn["I"] if fn["I"] is not None else dv.float().cpu().numpy().astype(np.float64)
    rtf, rI, rfg = oracle.render_vjp(I, fn, fn["gmax"], sp32(w.spacing), w.tf_knots, w.tf_rgba,
                                     oracle_params(w.params), w.cams, dout.cpu().numpy(), want_features=True)
    errs = {key: _nerr(fg[key].cpu().numpy(), rfg[key]) for key in ("g", "kappa", "V")}
    errs["gmax"] = abs(float(fg["gmax"].item()) - rfg["gmax"]) / abs(rfg["gmax"])
    errs["tf"] = _nerr(dtf.cpu().numpy(), rtf)
    # samples within rounding of a TF knot may take the other segment (tolerated set, counted)
    near = bf.near_knot_voxels(I.shape, sp32(w.spacing), I, w.tf_knots, w.params, w.cams)
    keep = ~near
    errs["I"] = _nerr(dvol.cpu().numpy()[keep], rI[keep])
    print("[render feature grads] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items())
          + f" (near-knot voxels excluded from dI: {int(near.sum())})", flush=True)
    assert all(v <= 1e-4 for v in errs.values()), errs
    # the TF and intensity gradients are those of the plain adjoint
    assert _nerr(dtf.cpu().numpy(), dtf0.cpu().numpy()) <= 1e-6
    assert _nerr(dvol.cpu().numpy(), dvol0.cpu().numpy()) <= 1e-6


def test_render_feature_grads_ragged_quad():
    """Quad layout, perspective and orthographic views of 37 x 29 pixels: tiles and 2 x 2 lane quads
    cut by the image edge (lanes without a ray), against the oracle's reverse mode."""
    w = _diff_scene()
    w.cams = [phantoms.ortho_camera(w.dims, w.spacing, 50.0, 25.0, 37, 29),
              phantoms.persp_camera(w.dims, w.spacing, 200.0, -20.0, 37, 29)]
    dv = to_dev(w.vol)
    f = dvr.features(dv, w.spacing, w.sigmas, c=w.c, layout=abi.DVR_QUAD)
    kn, rg = tf_dev(w)
    img, T, k = dvr.render(dv, f, kn, rg, w.params, w.cams)
    rng = np.random.default_rng(12)
    dout = to_dev(rng.normal(size=tuple(img.shape)))
    dtf, dvol, fg = dvr.render_backward(dv, f, kn, rg, w.params, w.cams, T, k, dout, want_features=True)
    torch.cuda.synchronize()
    fn = feats_np(f)
    I = dv.cpu().numpy().astype(np.float64)
    rtf, rI, rfg = oracle.render_vjp(I, fn, fn["gmax"], sp32(w.spacing), w.tf_knots, w.tf_rgba,
                                     oracle_params(w.params), w.cams, dout.cpu().numpy(), want_features=True)
    errs = {key: _nerr(fg[key].cpu().numpy(), rfg[key]) for key in ("g", "kappa", "V")}
    errs["gmax"] = abs(float(fg["gmax"].item()) - rfg["gmax"]) / abs(rfg["gmax"])
    errs["tf"] = _nerr(dtf.cpu().numpy(), rtf)
    near = bf.near_knot_voxels(I.shape, sp32(w.spacing), I, w.tf_knots, w.params, w.cams)
    errs["I"] = _nerr(dvol.cpu().numpy()[~near], rI[~near])
    print("[render feature grads, ragged quad] " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    assert all(v <= 1e-4 for v in errs.values()), errs


def _tie_free_upstream(I, spacing, sigmas, fr, seed, tie=1e-4):
    """Random upstream gradients; no V upstream where two scales' V are within tie of each other
    (relative) or where V is 0; the |g| maximum made unique by the caller's input."""
    shape = I.shape
    rng = np.random.default_rng(seed)
    gb = rng.normal(size=(3,) + shape)
    kb = rng.normal(size=shape)
    Vb = rng.normal(size=shape) * 5.0
    m = fa.forward(I, spacing, sigmas, **fr)
    Vs = np.sort(m["Vs"], axis=0)
    if len(sigmas) > 1:
        close = (Vs[-1] - Vs[-2]) <= tie * Vs[-1]
        Vb[close] = 0.0
    Vb[m["V"] == 0.0] = 0.0
    return gb, kb, Vb, 0.8, m


def _vessel_crop(shape, seed):
    """A crop of the 128^3 phantom with vessel tubes (V > 0 on many voxels), plus one bright voxel
    that makes the |g| maximum unique."""
    w = phantoms.c3(32, 32, views=[0])
    nz, ny, nx = shape
    v = w.vol[30:30 + nz, 35:35 + ny, 28:28 + min(nx, 90)].astype(np.float64)
    # longer rows repeat the crop mirrored, so that rows span several x chunks of the adjoint kernels
    v = np.concatenate([v, v[:, :, ::-1]] * (1 + nx // 180), axis=2)[:, :, :nx].copy()
    v[nz // 2, ny // 3, nx // 4] += 0.6
    return v


@pytest.mark.parametrize("shape,spacing,sigmas,dtype", [
    ((23, 29, 37), (1.0, 0.8, 1.3), [1.0, 1.6], torch.float32),
    ((40, 70, 90), (0.9, 0.9, 1.2), [1.0, 2.0, 3.0], torch.float32),
    ((17, 19, 66), (0.7, 1.1, 2.5), [0.8], torch.float16),
    # rows of 530 voxels: several x chunks per row (236..252 outputs each at the radii 2..10)
    ((6, 9, 530), (1.0, 1.0, 1.0), [0.7, 1.5, 3.0], torch.float32),
    ((5, 6, 300), (1.0, 1.0, 1.0), [1.2], torch.float16),
    ((2, 3, 5), (1.0, 1.0, 1.0), [1.0, 1.5], torch.float32),
    ((2, 2, 2), (1.0, 1.0, 1.0), [1.0, 1.5], torch.float32),
    # eight scales (the most the ABI takes); radii up to 12 take the generic Hessian kernels
    ((9, 12, 70), (0.8, 0.8, 1.1), [0.6, 0.8, 1.0, 1.3, 1.6, 2.0, 2.4, 2.8], torch.float32),
])
def test_feature_adjoint_matches_oracle(shape, spacing, sigmas, dtype):
    print(f"[feature adjoint] shape={shape} spacing={spacing} sigmas={sigmas} dtype={dtype}", flush=True)
    fr = dict(alpha=0.5, beta=0.5, c=f32(0.08))
    vol = _vessel_crop(shape, 1) if min(shape) > 4 else np.random.default_rng(2).random(shape)
    dv = to_dev(vol, dtype)
    I = dv.float().cpu().numpy().astype(np.float64)
    sp, sg = sp32(spacing), [f32(s) for s in sigmas]
    gb, kb, Vb, gmb, m = _tie_free_upstream(I, sp, sg, fr, 3)
    gn = np.sqrt((m["g"] ** 2).sum(0)).ravel()
    top = np.sort(gn)[-2:]
    if top[1] - top[0] <= 1e-5 * top[1]:
        gmb = 0.0  # no unique maximum on this input: the gmax term is checked elsewhere
    fg = dict(g=to_dev(gb), kappa=to_dev(kb), V=to_dev(Vb), gmax=torch.tensor([gmb], dtype=torch.float32, device="cuda"))
    base = np.random.default_rng(4).normal(size=shape)
    dvol = dvr.features_backward(dv, spacing, sigmas, fg, dvol=to_dev(base), **fr)
    torch.cuda.synchronize()
    ref = fa.vjp(I, sp, sg, fr["alpha"], fr["beta"], fr["c"], np.float32(gb).astype(np.float64),
                 np.float32(kb).astype(np.float64), np.float32(Vb).astype(np.float64), float(np.float32(gmb)))
    got = dvol.cpu().numpy().astype(np.float64) - np.float32(base).astype(np.float64)
    e = _nerr(got, ref)
    print(f"[feature adjoint] err={e:.2e} |V>0|={(m['V'] > 0).mean():.2f} V upstream on "
          f"{(Vb != 0).mean():.2f}", flush=True)
    assert e <= 1e-4
    # each term on its own
    z3, z1 = np.zeros((3,) + shape), np.zeros(shape)
    for name, up in [("g", (gb, z1, z1, 0.0)), ("k", (z3, kb, z1, 0.0)), ("V", (z3, z1, Vb, 0.0)),
                     ("gmax", (z3, z1, z1, gmb))]:
        if not np.any(up[2]) and name == "V" or (name == "gmax" and gmb == 0.0):
            continue
        fgt = dict(g=to_dev(up[0]), kappa=to_dev(up[1]), V=to_dev(up[2]),
                   gmax=torch.tensor([up[3]], dtype=torch.float32, device="cuda"))
        d = dvr.features_backward(dv, spacing, sigmas, fgt, **fr).cpu().numpy()
        r = fa.vjp(I, sp, sg, fr["alpha"], fr["beta"], fr["c"], *[np.float32(u).astype(np.float64) for u in up[:3]],
                   float(np.float32(up[3])))
        et = _nerr(d, r)
        print(f"[feature adjoint]   term {name}: err={et:.2e}", flush=True)
        assert et <= 1e-4, name


def test_end_to_end_gradient():
    """L = <dout, render(I, features(I))>: GPU dL/dI (TF lookup + feature adjoint) against the
    oracle's, normwise <= 1e-4 (c given, V near-ties counted and reported)."""
    w = _diff_scene(40)
    w.sigmas = [1.0, 2.0]
    dv = to_dev(w.vol)
    f = dvr.features(dv, w.spacing, w.sigmas, c=w.c)
    kn, rg = tf_dev(w)
    img, T, k = dvr.render(dv, f, kn, rg, w.params, w.cams)
    rng = np.random.default_rng(12)
    dout = to_dev(rng.normal(size=tuple(img.shape)))
    _, dvol, fg = dvr.render_backward(dv, f, kn, rg, w.params, w.cams, T, k, dout, want_features=True)
    dvol = dvr.features_backward(dv, w.spacing, w.sigmas, fg, dvol=dvol, c=w.c)
    torch.cuda.synchronize()
    I = dv.cpu().numpy().astype(np.float64)
    sp, sg, c = sp32(w.spacing), [f32(s) for s in w.sigmas], f32(w.c)
    of = oracle.features(I, sp, sg, c=c)
    _, rI, rfg = oracle.render_vjp(I, of, of["gmax"], sp, w.tf_knots, w.tf_rgba, oracle_params(w.params), w.cams,
                                   dout.cpu().numpy(), want_features=True)
    rfeat = fa.vjp(I, sp, sg, 0.5, 0.5, c, rfg["g"], rfg["kappa"], rfg["V"], rfg["gmax"])
    ref = rI + rfeat
    keep = ~bf.near_knot_voxels(I.shape, sp, I, w.tf_knots, w.params, w.cams)
    e = _nerr(dvol.cpu().numpy()[keep], ref[keep])
    m = fa.forward(I, sp, sg, c=c)
    Vs = np.sort(m["Vs"], axis=0)
    ties = int(((Vs[-1] - Vs[-2]) <= 1e-4 * Vs[-1]).sum() - (Vs[-1] == 0).sum())
    print(f"[end to end] err={e:.2e} (TF part {np.linalg.norm(rI):.3e}, feature part {np.linalg.norm(rfeat):.3e}, "
          f"near-tie voxels {ties}, near-knot voxels {int((~keep).sum())})", flush=True)
    assert np.linalg.norm(rfeat) > 0.05 * np.linalg.norm(rI)
    assert e <= 1e-4


def test_feature_adjoint_flat_volume():
    """A constant volume: g = 0, k = 0, V = 0 and gmax = 0 everywhere, so only the transposed
    gradient of dL/dg remains (no curvature, vesselness or gmax term), against the oracle."""
    shape = (11, 13, 17)
    I = np.full(shape, 0.37)
    dv = to_dev(I)
    rng = np.random.default_rng(8)
    gb, kb, Vb = rng.normal(size=(3,) + shape), rng.normal(size=shape), rng.normal(size=shape)
    fg = dict(g=to_dev(gb), kappa=to_dev(kb), V=to_dev(Vb), gmax=torch.tensor([0.9], dtype=torch.float32, device="cuda"))
    sp = (1.0, 0.9, 1.2)
    d = dvr.features_backward(dv, sp, [1.0, 2.0], fg, c=0.1).cpu().numpy()
    I64 = dv.cpu().numpy().astype(np.float64)
    r = fa.vjp(I64, sp32(sp), [1.0, 2.0], 0.5, 0.5, f32(0.1), np.float32(gb).astype(np.float64),
               np.float32(kb).astype(np.float64), np.float32(Vb).astype(np.float64), float(np.float32(0.9)))
    only_g = fa.gradient_T(np.float32(gb).astype(np.float64), sp32(sp))
    np.testing.assert_allclose(r, only_g, rtol=0, atol=1e-12)
    e = _nerr(d, r)
    print(f"[feature adjoint] flat volume err={e:.2e}", flush=True)
    assert e <= 1e-5
