"""FP64 CPU oracle of the volume-rendering hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use
this package.  The product path (the HIP library and its binding) never imports it, and this
package never imports the product.  The computation lives in ``dvr_oracle.c`` (plain C, IEEE
double, no FMA contraction); this file only marshals NumPy arrays through ctypes.

Every function follows a passage of the paper (Beckley, "Decentralized Direct Volume Rendering"):
  normalize      Sec. 2.2 Eq. 1
  gradient       Sec. 2.3 Eq. 2 (and the |grad I|_max reduction of Eq. 4)
  smooth/hessian Sec. 1 "multi-scale Hessian analysis", Sec. 2.3 (Hessian H)
  eig3/vesselness  Sec. 1 "vesselness measures" (Frangi et al. 1998, named method)
  features       Sec. 2.3 Eq. 2-3 plus the above
  render         Sec. 2.4 Eq. 4-6
  render_vjp     reverse mode of render (TF values and voxel intensities)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dvr_oracle.c")
_LIB = os.path.join(_HERE, "libdvr_oracle.so")
_lib = None

PARAM_ORDER = ("lambda_g", "lambda_k", "kappa0", "lambda_v", "step_vox", "et_alpha")


def build():
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction, no fast-math)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                           "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp, ip, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        i, d, i64 = C.c_int, C.c_double, C.c_int64
        L.oracle_normalize.argtypes = [dp, i64, dp, dp, dp]
        L.oracle_gradient.argtypes = [dp, i, i, i, d, d, d, dp, dp]
        L.oracle_gauss_radius.argtypes = [d]
        L.oracle_smooth.argtypes = [dp, i, i, i, d, d, d, dp]
        L.oracle_hessian.argtypes = [dp, i, i, i, d, d, d, dp]
        L.oracle_eig3.argtypes = [dp, dp]
        L.oracle_eig3.restype = None
        L.oracle_vesselness.argtypes = [dp, d, d, d]
        L.oracle_vesselness.restype = d
        L.oracle_features.argtypes = [dp, i, i, i, d, d, d, i, dp, d, d, d, dp, dp, dp, dp, dp, dp, dp, dp]
        L.oracle_render.argtypes = [dp, dp, dp, dp, i, i, i, d, d, d, d, i, dp, dp, dp, dp, i, ip, i64,
                                    dp, dp, ip, i64p]
        L.oracle_render_vjp.argtypes = [dp, dp, dp, dp, i, i, i, d, d, d, d, i, dp, dp, dp, dp, i, ip, i64,
                                        dp, dp, dp, dp, dp, dp, dp, d, i, C.POINTER(C.c_uint8)]
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def _dims(vol):
    nz, ny, nx = vol.shape
    return nx, ny, nz


def normalize(raw):
    raw = _f64(raw)
    out = np.empty_like(raw)
    mn, mx = C.c_double(), C.c_double()
    rc = lib().oracle_normalize(_p(raw), raw.size, _p(out), C.byref(mn), C.byref(mx))
    assert rc == 0
    return out, mn.value, mx.value


def gradient(vol, spacing):
    vol = _f64(vol)
    g = np.empty((3,) + vol.shape)
    gmax = C.c_double()
    rc = lib().oracle_gradient(_p(vol), *_dims(vol), *map(float, spacing), _p(g), C.byref(gmax))
    assert rc == 0
    return g, gmax.value


def gauss_radius(sigma_vox):
    return lib().oracle_gauss_radius(float(sigma_vox))


def smooth(vol, sigma_vox):
    vol = _f64(vol)
    s = np.empty_like(vol)
    rc = lib().oracle_smooth(_p(vol), *_dims(vol), *map(float, sigma_vox), _p(s))
    assert rc == 0
    return s


def hessian(s, spacing):
    """[6][nz][ny][nx]: xx, yy, zz, xy, xz, yz of the (already smoothed) field s."""
    s = _f64(s)
    H = np.empty((6,) + s.shape)
    rc = lib().oracle_hessian(_p(s), *_dims(s), *map(float, spacing), _p(H))
    assert rc == 0
    return H


def eig3(A6):
    """Eigenvalues of one symmetric 3x3 (xx, yy, zz, xy, xz, yz), sorted by (|l|, l)."""
    A = _f64(A6)
    lam = np.empty(3)
    lib().oracle_eig3(_p(A), _p(lam))
    return lam


def vesselness(lam, alpha=0.5, beta=0.5, c=0.1):
    return lib().oracle_vesselness(_p(_f64(lam)), float(alpha), float(beta), float(c))


def features(vol, spacing, sigmas, alpha=0.5, beta=0.5, c=0.1, want_H0=False, want_lam=False, want_Vs=False):
    """Returns dict(g [3][nz][ny][nx], kappa, V, gmax, c, and optionally H0, lam, Vs)."""
    vol = _f64(vol)
    N = vol.size
    sig = _f64(sigmas)
    g = np.empty((3,) + vol.shape)
    kap = np.empty(vol.shape)
    V = np.empty(vol.shape)
    H0 = np.empty((6,) + vol.shape) if want_H0 else None
    lam = np.empty((len(sig), 3) + vol.shape) if want_lam else None
    Vs = np.empty((len(sig),) + vol.shape) if want_Vs else None
    gmax, c_used = C.c_double(), C.c_double()
    rc = lib().oracle_features(_p(vol), *_dims(vol), *map(float, spacing), len(sig), _p(sig),
                               float(alpha), float(beta), float(c), _p(g), _p(kap), _p(V),
                               C.byref(gmax), C.byref(c_used), _p(H0), _p(lam), _p(Vs))
    assert rc == 0, rc
    out = dict(g=g, kappa=kap, V=V, gmax=gmax.value, c=c_used.value)
    if want_H0:
        out["H0"] = H0
    if want_lam:
        out["lam"] = lam
    if want_Vs:
        out["Vs"] = Vs
    del N
    return out


def pack_cams(cams):
    arr = np.stack([c.packed() if hasattr(c, "packed") else _f64(c) for c in cams])
    return np.ascontiguousarray(arr, dtype=np.float64)


def pack_params(params):
    return np.array([float(params[k]) for k in PARAM_ORDER], np.float64)


def all_pixels(cams):
    out = []
    for ci, c in enumerate(cams):
        w, h = (int(c.width), int(c.height)) if hasattr(c, "width") else (int(c[1]), int(c[2]))
        jj, ii = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
        out.append(np.stack([np.full(w * h, ci), ii.ravel(), jj.ravel()], 1))
    return np.ascontiguousarray(np.concatenate(out), dtype=np.int32)


def _scene_args(vol, feats, gmax, spacing, knots, rgba, params):
    vol = _f64(vol)
    g, kap, V = _f64(feats["g"]), _f64(feats["kappa"]), _f64(feats["V"])
    assert g.shape == (3,) + vol.shape and kap.shape == vol.shape and V.shape == vol.shape
    knots, rgba = _f64(knots), _f64(rgba).reshape(-1, 4)
    keep = (vol, g, kap, V, knots, rgba, pack_params(params))
    args = [_p(vol), _p(g), _p(kap), _p(V), *_dims(vol), *map(float, spacing), float(gmax),
            len(knots), _p(keep[4]), _p(keep[5]), _p(keep[6])]
    return keep, args


def render(vol, feats, gmax, spacing, knots, rgba, params, cams, pix=None):
    """pix=None: full images -> dict(rgba [ncam][H][W][4], T_last [ncam][H][W], k_last, nsamp).
    pix = int32 [M][3] (camera, i, j): per-pixel arrays of length M instead."""
    camarr = pack_cams(cams)
    full = pix is None
    pix = all_pixels(cams) if full else np.ascontiguousarray(pix, dtype=np.int32)
    M = len(pix)
    out = np.empty((M, 4))
    T = np.empty(M)
    k = np.empty(M, np.int32)
    ns = C.c_int64()
    keep, args = _scene_args(vol, feats, gmax, spacing, knots, rgba, params)
    rc = lib().oracle_render(*args, _p(camarr), len(camarr), _p(pix, C.c_int32), M, _p(out), _p(T),
                             _p(k, C.c_int32), C.byref(ns))
    assert rc == 0
    del keep
    if full:
        H, W = int(camarr[0, 2]), int(camarr[0, 1])
        n = len(camarr)
        return dict(rgba=out.reshape(n, H, W, 4), T_last=T.reshape(n, H, W), k_last=k.reshape(n, H, W),
                    nsamp=ns.value)
    return dict(rgba=out, T_last=T, k_last=k, nsamp=ns.value)


def render_vjp(vol, feats, gmax, spacing, knots, rgba, params, cams, dout, pix=None, want_dI=True,
               want_features=False, near_knot_eps=None, near_knot_weighted=False):
    """dL/d(TF values) [K][4] and dL/dI [nz][ny][nx] for upstream dout (same layout as render).
    want_features: also dict(g [3][nz][ny][nx], kappa, V, gmax) of dL/d(feature values), returned
    as a third element.  near_knot_eps: also a bool [nz][ny][nx] mask of the corners of samples
    whose intensity lies within that distance of a TF knot, returned last; near_knot_weighted:
    within that distance times the corner's trilinear weight (the voxels whose change by
    +-near_knot_eps moves some sample across a knot)."""
    camarr = pack_cams(cams)
    pix = all_pixels(cams) if pix is None else np.ascontiguousarray(pix, dtype=np.int32)
    d = _f64(dout).reshape(-1, 4)
    assert len(d) == len(pix)
    keep, args = _scene_args(vol, feats, gmax, spacing, knots, rgba, params)
    K = len(keep[4])
    dtf = np.empty((K, 4))
    shape = keep[0].shape
    dI = np.empty(shape) if want_dI else None
    fg = dict(g=np.empty((3,) + shape), kappa=np.empty(shape), V=np.empty(shape)) if want_features else None
    dgm = C.c_double()
    nk = np.zeros(shape, np.uint8) if near_knot_eps is not None else None
    rc = lib().oracle_render_vjp(*args, _p(camarr), len(camarr), _p(pix, C.c_int32), len(pix), _p(d),
                                 _p(dtf), _p(dI), _p(fg["g"]) if fg else None, _p(fg["kappa"]) if fg else None,
                                 _p(fg["V"]) if fg else None, C.byref(dgm) if fg else None,
                                 float(near_knot_eps or 0.0), int(bool(near_knot_weighted)), _p(nk, C.c_uint8))
    assert rc == 0
    del keep
    out = [dtf, dI]
    if fg is not None:
        fg["gmax"] = dgm.value
        out.append(fg)
    if nk is not None:
        out.append(nk.astype(bool))
    return tuple(out)
