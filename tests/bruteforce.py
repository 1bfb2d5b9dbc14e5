"""Brute-force NumPy/SciPy references for tiny inputs (test-only; independent of the oracle).

These take the definitions the slow way so that a mistake in the oracle's structure shows up:
  * smoothing as one non-separable 3-D convolution with an explicit Gaussian kernel and
    edge-padded input (no separable passes);
  * ray/box clipping by enumerating the six face rectangles (not the slab method);
  * trilinear sampling with scipy.ndimage.map_coordinates(order=1, mode='nearest');
  * transfer-function lookup with numpy.interp;
  * compositing as explicit sums of alpha_k c_k prod_{j<k}(1 - alpha_j) (no running state).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.ndimage as ndi


def gauss1d(sigma_vox):
    r = max(1, int(math.floor(3.0 * sigma_vox + 0.5)))
    j = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-j * j / (2.0 * sigma_vox * sigma_vox))
    return w / w.sum(), r


def smooth_nonseparable(vol, sig_xyz):
    wx, rx = gauss1d(sig_xyz[0])
    wy, ry = gauss1d(sig_xyz[1])
    wz, rz = gauss1d(sig_xyz[2])
    ker = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
    pad = np.pad(vol, ((rz, rz), (ry, ry), (rx, rx)), mode="edge")
    nz, ny, nx = vol.shape
    out = np.zeros_like(vol, dtype=np.float64)
    for a in range(2 * rz + 1):
        for b in range(2 * ry + 1):
            for c in range(2 * rx + 1):
                out += ker[a, b, c] * pad[a:a + nz, b:b + ny, c:c + nx]
    return out


def hessian_np(s, spacing):
    """Second differences with edge clamping via np.pad(mode='edge')."""
    hx, hy, hz = spacing
    p = np.pad(s, 1, mode="edge")
    c = p[1:-1, 1:-1, 1:-1]
    sh = lambda dz, dy, dx: p[1 + dz:p.shape[0] - 1 + dz, 1 + dy:p.shape[1] - 1 + dy, 1 + dx:p.shape[2] - 1 + dx]
    Hxx = (sh(0, 0, 1) - 2 * c + sh(0, 0, -1)) / hx ** 2
    Hyy = (sh(0, 1, 0) - 2 * c + sh(0, -1, 0)) / hy ** 2
    Hzz = (sh(1, 0, 0) - 2 * c + sh(-1, 0, 0)) / hz ** 2
    Hxy = (sh(0, 1, 1) - sh(0, -1, 1) - sh(0, 1, -1) + sh(0, -1, -1)) / (4 * hx * hy)
    Hxz = (sh(1, 0, 1) - sh(-1, 0, 1) - sh(1, 0, -1) + sh(-1, 0, -1)) / (4 * hx * hz)
    Hyz = (sh(1, 1, 0) - sh(-1, 1, 0) - sh(1, -1, 0) + sh(-1, -1, 0)) / (4 * hy * hz)
    return np.stack([Hxx, Hyy, Hzz, Hxy, Hxz, Hyz])


def ray_of(cam, i, j):
    persp, o, d0, du, dv = int(cam[0]), cam[3:6], cam[6:9], cam[9:12], cam[12:15]
    if persp:
        d = d0 + (i + 0.5) * du + (j + 0.5) * dv
        return o.copy(), d / np.linalg.norm(d)
    return o + (i + 0.5) * du + (j + 0.5) * dv, d0.copy()


def clip_faces(o, d, hi):
    """Entry/exit parameters of the ray against the box [0, hi] by testing each face rectangle."""
    ts = []
    for a in range(3):
        if d[a] == 0.0:
            continue
        for plane in (0.0, hi[a]):
            t = (plane - o[a]) / d[a]
            p = o + t * d
            ok = all(-1e-12 * max(1.0, hi[b]) <= p[b] <= hi[b] * (1 + 1e-12) + 1e-12 for b in range(3) if b != a)
            if ok:
                ts.append(t)
    if len(ts) < 2:
        # ray along a face or grazing an edge/corner: inside test over the axis-parallel case
        inside = all(0.0 <= o[a] <= hi[a] for a in range(3) if d[a] == 0.0)
        if not inside or len(ts) == 0:
            return None
    t0, t1 = min(ts), max(ts)
    t0 = max(t0, 0.0)
    if t1 <= t0:
        return None
    return t0, t1


def render_pixel(vol, g, kap, ves, gmax, spacing, knots, rgba, prm, cam, i, j):
    """Returns (rgba[4], nsamp)."""
    h = np.asarray(spacing, np.float64)
    nz, ny, nx = vol.shape
    hi = np.array([(nx - 1) * h[0], (ny - 1) * h[1], (nz - 1) * h[2]])
    o, d = ray_of(cam, i, j)
    cl = clip_faces(o, d, hi)
    if cl is None:
        return np.zeros(4), 0
    tn, tf = cl
    delta = prm["step_vox"] * h.min()
    L = tf - tn
    N = int(math.ceil(L / delta))
    dks = np.full(N, delta)
    dks[-1] = L - (N - 1) * delta
    tk = tn + np.arange(N) * delta + 0.5 * dks
    P = o[None, :] + tk[:, None] * d[None, :]
    Q = np.clip(P / h[None, :], 0.0, np.array([nx - 1, ny - 1, nz - 1], np.float64)[None, :])
    coords = np.stack([Q[:, 2], Q[:, 1], Q[:, 0]])  # (z, y, x) for map_coordinates
    mc = lambda f: ndi.map_coordinates(f, coords, order=1, mode="nearest")
    I = mc(vol)
    gv = np.stack([mc(g[0]), mc(g[1]), mc(g[2])], 1)
    kk = mc(kap)
    vv = mc(ves)
    col = np.stack([np.interp(I, knots, rgba[:, ch]) for ch in range(4)], 1)
    gn = np.linalg.norm(gv, axis=1)
    lg, lk, k0, lv = prm["lambda_g"], prm["lambda_k"], prm["kappa0"], prm["lambda_v"]
    m = (1 - lg) + lg * np.minimum(gn / gmax, 1.0) if gmax > 0 else np.full(N, 1 - lg)
    w = (1 - lk) + lk * np.abs(kk) / (np.abs(kk) + k0)
    u = 1 + lv * vv
    x = col[:, 3] * m * w * u * dks
    a = 1.0 - np.exp(-x)
    keep = N
    if prm["et_alpha"] > 0:
        for k in range(N):
            if np.prod(1.0 - a[:k + 1]) <= 1.0 - prm["et_alpha"]:
                keep = k + 1
                break
    out = np.zeros(4)
    for k in range(keep):
        trans = np.prod(1.0 - a[:k])
        out[:3] += trans * a[k] * col[k, :3]
    out[3] = 1.0 - np.prod(1.0 - a[:keep])
    return out, keep


def near_knot_voxels(shape_zyx, spacing, I, knots, prm, cams, eps=1e-6):
    """Voxels that are trilinear corners of a sample whose intensity lies within eps of a TF knot.
    There the TF slope jumps, so FP32 and FP64 evaluations may take different segments and the
    intensity gradient of that one sample differs by O(1): a tolerated set for dL/dI comparisons."""
    nz, ny, nx = shape_zyx
    h = np.asarray(spacing, np.float64)
    hi = np.array([(nx - 1) * h[0], (ny - 1) * h[1], (nz - 1) * h[2]])
    mask = np.zeros(shape_zyx, bool)
    kn = np.asarray(knots, np.float64)
    delta = prm["step_vox"] * h.min()
    for cam in cams:
        pk = cam.packed()
        for j in range(cam.height):
            for i in range(cam.width):
                o, d = ray_of(pk, i, j)
                cl = clip_faces(o, d, hi)
                if cl is None:
                    continue
                L = cl[1] - cl[0]
                N = int(math.ceil(L / delta))
                dks = np.full(N, delta)
                dks[-1] = L - (N - 1) * delta
                tk = cl[0] + np.arange(N) * delta + 0.5 * dks
                Q = np.clip((o[None] + tk[:, None] * d[None]) / h, 0, [nx - 1, ny - 1, nz - 1])
                Iq = ndi.map_coordinates(I, np.stack([Q[:, 2], Q[:, 1], Q[:, 0]]), order=1, mode="nearest")
                near = np.abs(Iq[:, None] - kn[None]).min(1) < eps
                for q in Q[near]:
                    c = np.minimum(np.floor(q).astype(int), [nx - 2, ny - 2, nz - 2])
                    mask[c[2]:c[2] + 2, c[1]:c[1] + 2, c[0]:c[0] + 2] = True
    return mask
