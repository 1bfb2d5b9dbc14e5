"""Seeded synthetic inputs for the volume-rendering hot path.

This module only *draws inputs*: phantom volumes, camera frames, transfer-function
knots and render parameters.  It holds none of the method's arithmetic (no
gradient, smoothing, Hessian, eigenvalue, vesselness, sampling or compositing
step), so both the FP64 oracle tests and the HIP path can take their inputs
from here without sharing any of the computation under test.

The paper measured on BrainWeb, a Mendeley pathology set and a private clinical
cohort (Sec. 2.1); none is available, so the phantoms below stand in for them
with the shapes, spacings and tissue values of those workloads: nested
ellipsoid tissue shells whose values sit at the paper's normalized tissue peaks
(Sec. 3.1, Tables 1-2 give CSF/GM/WM peaks in the 0.05-0.31 range; the phantoms
use well separated values so that the transfer function has distinct bands),
bright tubes for contrast-enhanced vessels (Sec. 3.2, Fig. 2), and Gaussian or
Rician noise.

Recipe (fixed, so a phantom is reproducible from this description alone):
  * Grid: voxel (i, j, k) is at (i*hx, j*hy, k*hz) mm; arrays are C-order
    [nz][ny][nx] (x fastest).
  * A config's draws come from ``numpy.random.default_rng(seed)``: geometry
    first (jitters, tube lines and radii), then noise slab by slab along z in
    C order, then the cast to the storage type.
  * Seeds: config k uses 19737 + k; volume b of the batched config uses
    [19737, 4, b].
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 19737

# Frangi's structure sensitivity of the benchmarked workloads, c = 1/2 max over voxels and scales of
# |sigma^2 H|_F (Frangi's rule), computed once by the oracle (tests/golden/make_frangi_c.py writes
# tests/golden/frangi_c.json) and fixed here, so the timed feature passes are single-pass.  The
# batched set shares one value: half the largest norm over its 64 volumes.
FRANGI_C = {"c2": 0.414322618, "c3": 0.137696885, "c4": 0.0771826, "c5": 0.151685491}

# Tissue values of the simple phantom (background, CSF, GM, WM).
C1_VALUES = (0.0, 0.2, 0.55, 0.8)
# Semi-axes (x, y, z) in mm of the simple 64^3 phantom, outermost first.
C1_SEMI_MM = ((28.0, 25.0, 22.0), (24.0, 21.0, 18.0), (17.0, 14.0, 12.0))
# Head phantom: shells as fractions of the half-extent, outermost first, with values.
HEAD_SHELLS = ((0.95, 0.9), (0.88, 0.05), (0.82, 0.2), (0.76, 0.55), (0.55, 0.8))
HEAD_HALF_MM = (90.0, 108.0, 90.0)
# Vessel tubes are painted out to TUBE_CUT radii, where the Gaussian profile is below 1e-6 of its peak.
TUBE_CUT = 5.3


@dataclass
class Camera:
    """One view.  ortho: ray origin o + (i+.5) du + (j+.5) dv, direction d0 (unit).
    persp: origin o, direction normalize(d0 + (i+.5) du + (j+.5) dv).  Row j = 0 is the top."""
    persp: int
    width: int
    height: int
    o: np.ndarray
    d0: np.ndarray
    du: np.ndarray
    dv: np.ndarray

    def packed(self) -> np.ndarray:
        """16 float64: persp, width, height, o[3], d0[3], du[3], dv[3], 0 (the float32 values widened)."""
        v = np.zeros(16, np.float64)
        v[0], v[1], v[2] = self.persp, self.width, self.height
        v[3:6], v[6:9], v[9:12], v[12:15] = self.o, self.d0, self.du, self.dv
        return v


@dataclass
class Workload:
    name: str
    vol: np.ndarray                      # [nz][ny][nx] float32 (or uint16 raw for the FP16 config)
    spacing: tuple                       # (hx, hy, hz) mm
    sigmas: list                         # Gaussian scales in mm
    alpha: float = 0.5
    beta: float = 0.5
    c: float = 0.1
    tf_knots: np.ndarray = None          # float32 [K]
    tf_rgba: np.ndarray = None           # float32 [K][4]  (R, G, B non-premultiplied; A = extinction per mm)
    params: dict = field(default_factory=dict)
    cams: list = field(default_factory=list)
    extra: dict = field(default_factory=dict)

    @property
    def dims(self):
        nz, ny, nx = self.vol.shape
        return nx, ny, nz


# ----------------------------------------------------------------------------------------------
# geometry helpers (input drawing only)

def _axes_mm(shape_zyx, spacing):
    nz, ny, nx = shape_zyx
    hx, hy, hz = spacing
    return (np.arange(nx) * hx, np.arange(ny) * hy, np.arange(nz) * hz)


def _centre(shape_zyx, spacing):
    nz, ny, nx = shape_zyx
    hx, hy, hz = spacing
    return np.array([(nx - 1) * hx / 2, (ny - 1) * hy / 2, (nz - 1) * hz / 2])


def _paint_slab(out, z_mm, x_mm, y_mm, shells, centre, tubes, ventricles=()):
    """Paint shells (outermost first, innermost wins), then ventricles, then max-combine tubes."""
    Z = z_mm[:, None, None]
    Y = y_mm[None, :, None]
    X = x_mm[None, None, :]
    out[...] = 0.0
    for semi, val in shells:
        q = ((X - centre[0]) / semi[0]) ** 2 + ((Y - centre[1]) / semi[1]) ** 2 + ((Z - centre[2]) / semi[2]) ** 2
        out[np.broadcast_to(q <= 1.0, out.shape)] = val
    for cen, semi, val in ventricles:
        q = ((X - cen[0]) / semi[0]) ** 2 + ((Y - cen[1]) / semi[1]) ** 2 + ((Z - cen[2]) / semi[2]) ** 2
        out[np.broadcast_to(q <= 1.0, out.shape)] = val
    for p0, u, r_mm, peak in tubes:
        # the profile is below 1e-6 of its peak beyond TUBE_CUT * R: paint only the part of the slab
        # within that distance of the line (bounding box of the line's passage through the slab)
        reach = TUBE_CUT * r_mm
        zlo, zhi = z_mm[0] - reach, z_mm[-1] + reach
        if abs(u[2]) > 1e-9:
            ta, tb = (zlo - p0[2]) / u[2], (zhi - p0[2]) / u[2]
            t0, t1 = min(ta, tb), max(ta, tb)
            xs = (p0[0] + t0 * u[0], p0[0] + t1 * u[0])
            ys = (p0[1] + t0 * u[1], p0[1] + t1 * u[1])
            bx = (min(xs) - reach, max(xs) + reach)
            by = (min(ys) - reach, max(ys) + reach)
        else:
            if p0[2] < zlo or p0[2] > zhi:
                continue
            bx = (-np.inf, np.inf)
            by = (-np.inf, np.inf)
        ix = np.nonzero((x_mm >= bx[0]) & (x_mm <= bx[1]))[0]
        iy = np.nonzero((y_mm >= by[0]) & (y_mm <= by[1]))[0]
        if len(ix) == 0 or len(iy) == 0:
            continue
        sx, sy = slice(ix[0], ix[-1] + 1), slice(iy[0], iy[-1] + 1)
        dx, dy, dz = X[..., sx] - p0[0], Y[:, sy, :] - p0[1], Z - p0[2]
        along = dx * u[0] + dy * u[1] + dz * u[2]
        d2 = dx * dx + dy * dy + dz * dz - along * along
        prof = peak * np.exp(-np.maximum(d2, 0.0) / (2.0 * r_mm * r_mm))
        prof[d2 > reach * reach] = 0.0
        sub = out[:, sy, sx]
        np.maximum(sub, prof, out=sub)


def _draw_tubes(rng, n, r_lo, r_hi, centre, half, h_min):
    tubes = []
    for _ in range(n):
        p0 = centre + rng.uniform(-0.5, 0.5, 3) * np.asarray(half)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        r_vox = rng.uniform(r_lo, r_hi)
        tubes.append((p0, u, r_vox * h_min, 1.0))
    return tubes


def _render_volume(shape_zyx, spacing, shells, centre, tubes, ventricles, rng, noise, chunk=16):
    """Paint the clean phantom slab by slab, then add noise drawn slab by slab in C order.
    noise = ("gauss", s) adds N(0, s^2); ("rician", s) gives sqrt((I+s n1)^2 + (s n2)^2)."""
    nz, ny, nx = shape_zyx
    x_mm, y_mm, z_mm = _axes_mm(shape_zyx, spacing)
    out = np.empty(shape_zyx, np.float64)
    for z0 in range(0, nz, chunk):
        z1 = min(nz, z0 + chunk)
        _paint_slab(out[z0:z1], z_mm[z0:z1], x_mm, y_mm, shells, centre, tubes, ventricles)
    kind, s = noise
    for z0 in range(0, nz, chunk):
        z1 = min(nz, z0 + chunk)
        sl = out[z0:z1]
        if kind == "gauss":
            sl += s * rng.standard_normal(sl.shape)
        elif kind == "rician":
            n = rng.standard_normal((2,) + sl.shape)
            sl[...] = np.sqrt((sl + s * n[0]) ** 2 + (s * n[1]) ** 2)
        elif kind != "none":
            raise ValueError(kind)
    return out


# ----------------------------------------------------------------------------------------------
# cameras

def _view_frame(az_deg, el_deg):
    az, el = math.radians(az_deg), math.radians(el_deg)
    toward = np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    fwd = -toward
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    cam_up = np.cross(right, fwd)
    return fwd, right, cam_up


def box_diag(dims, spacing):
    return float(math.sqrt(sum(((n - 1) * h) ** 2 for n, h in zip(dims, spacing))))


def ortho_camera(dims, spacing, az_deg, el_deg, width, height, span=None):
    """Orthographic view of the box centre; the square image spans the box diagonal."""
    centre = _centre(dims[::-1], spacing)
    diag = box_diag(dims, spacing)
    span = diag if span is None else span
    fwd, right, cam_up = _view_frame(az_deg, el_deg)
    du = right * (span / width)
    dv = -cam_up * (span / height)
    o = centre - diag * fwd - 0.5 * width * du - 0.5 * height * dv
    f = lambda a: np.asarray(a, np.float32)
    return Camera(0, width, height, f(o), f(fwd), f(du), f(dv))


def persp_camera(dims, spacing, az_deg, el_deg, width, height, dist_diag=2.0, fov_y_deg=30.0):
    """Pinhole view of the box centre from dist_diag box diagonals away."""
    centre = _centre(dims[::-1], spacing)
    diag = box_diag(dims, spacing)
    fwd, right, cam_up = _view_frame(az_deg, el_deg)
    eye = centre - dist_diag * diag * fwd
    pix = 2.0 * math.tan(math.radians(fov_y_deg) / 2) / height
    du = right * pix
    dv = -cam_up * pix
    d0 = fwd - 0.5 * width * du - 0.5 * height * dv
    f = lambda a: np.asarray(a, np.float32)
    return Camera(1, width, height, f(eye), f(d0), f(du), f(dv))


# ----------------------------------------------------------------------------------------------
# transfer functions

def tf_c1():
    knots = np.array([0.0, 0.2, 0.55, 0.8], np.float32)
    rgba = np.array([[0, 0, 0, 0], [0.3, 0.5, 1.0, 0.02], [0.9, 0.6, 0.5, 0.08], [1.0, 0.95, 0.85, 0.3]], np.float32)
    return knots, rgba


def tf_head():
    """8 knots: background and skull (~0.05) clipped to zero extinction (the paper's implicit
    skull stripping by TF windows, Sec. 2.2), CSF/GM/WM bands, scalp fat (~0.9) suppressed,
    vessels (peak 1.0) bright and dense."""
    knots = np.array([0.0, 0.1, 0.2, 0.45, 0.7, 0.85, 0.92, 1.0], np.float32)
    rgba = np.array([
        [0.0, 0.0, 0.0, 0.0],
        [0.0, 0.0, 0.0, 0.0],
        [0.3, 0.5, 1.0, 0.08],
        [0.9, 0.6, 0.5, 0.25],
        [1.0, 0.95, 0.85, 0.5],
        [0.9, 0.9, 0.8, 0.15],
        [0.8, 0.2, 0.1, 0.4],
        [1.0, 0.1, 0.1, 3.0]], np.float32)
    return knots, rgba


def tf_random16(rng):
    knots = (np.arange(16) / 15.0).astype(np.float32)
    rgba = np.empty((16, 4), np.float64)
    rgba[:, :3] = rng.uniform(0.0, 1.0, (16, 3))
    rgba[:, 3] = rng.uniform(0.0, 0.2, 16)
    return knots, rgba.astype(np.float32)


def perturb_tf(rng, rgba, s=0.05):
    out = rgba.astype(np.float64) + s * rng.standard_normal(rgba.shape)
    out[:, :3] = np.clip(out[:, :3], 0.0, 1.0)
    out[:, 3] = np.maximum(out[:, 3], 0.0)
    return out.astype(np.float32)


def render_params(lambda_g=1.0, lambda_k=0.5, kappa0=0.05, lambda_v=0.0, step_vox=0.5, et_alpha=0.0):
    return dict(lambda_g=lambda_g, lambda_k=lambda_k, kappa0=kappa0, lambda_v=lambda_v,
                step_vox=step_vox, et_alpha=et_alpha)


# ----------------------------------------------------------------------------------------------
# the five workloads

def _c1_geometry(dims, spacing, scale=(1.0, 1.0, 1.0)):
    centre = _centre(dims[::-1], spacing)
    shells = [(tuple(a * s for a, s in zip(semi, scale)), val)
              for semi, val in zip(C1_SEMI_MM, C1_VALUES[1:])]
    return centre, shells


def c1(width=256, height=256):
    """64^3 at 1 mm: nested ellipsoids (CSF 0.2, GM 0.55, WM 0.8) + N(0, 0.01^2); sigma = 1 vox;
    one 256^2 orthographic view (az 30, el 20), 4-knot TF, no early termination."""
    rng = np.random.default_rng(SEED_BASE + 1)
    dims, h = (64, 64, 64), (1.0, 1.0, 1.0)
    centre, shells = _c1_geometry(dims, h)
    vol = _render_volume(dims[::-1], h, shells, centre, [], (), rng, ("gauss", 0.01)).astype(np.float32)
    knots, rgba = tf_c1()
    return Workload("c1", vol, h, [1.0], c=0.1, tf_knots=knots, tf_rgba=rgba,
                    params=render_params(lambda_v=0.0, et_alpha=0.0),
                    cams=[ortho_camera(dims, h, 30.0, 20.0, width, height)])


def _head(rng, dims, h, tube_r_vox=(1.0, 4.0), ntubes=24):
    centre = _centre(dims[::-1], h) + rng.uniform(-2.0, 2.0, 3)
    half = np.array([(n - 1) * s / 2 for n, s in zip(dims, h)])
    scale = half / np.array(HEAD_HALF_MM)
    shells = []
    for frac, val in HEAD_SHELLS:
        jit = rng.uniform(0.97, 1.03, 3)
        shells.append((tuple(frac * np.array(HEAD_HALF_MM) * scale * jit), val))
    vent = []
    for sx in (-1.0, 1.0):
        cen = centre + np.array([sx * 12.0, 8.0, 6.0]) * scale
        vent.append((cen, tuple(np.array([6.0, 22.0, 9.0]) * scale), 0.2))
    tubes = _draw_tubes(rng, ntubes, tube_r_vox[0], tube_r_vox[1], centre, half * 0.8, min(h))
    return centre, shells, vent, tubes


def c2(width=1024, height=1024, views=None, nviews=360):
    """181x217x181 at 1 mm head phantom with 24 vessel tubes and 3% Rician noise; sigma = {1,2,3};
    360 perspective orbit views (az = v deg, el 15, 2 box diagonals away, fov_y 30) at 1024^2,
    8-knot TF, early termination at alpha >= 0.99."""
    rng = np.random.default_rng(SEED_BASE + 2)
    dims, h = (181, 217, 181), (1.0, 1.0, 1.0)
    centre, shells, vent, tubes = _head(rng, dims, h)
    vol = _render_volume(dims[::-1], h, shells, centre, tubes, vent, rng, ("rician", 0.03)).astype(np.float32)
    knots, rgba = tf_head()
    views = range(nviews) if views is None else views
    cams = [persp_camera(dims, h, float(v), 15.0, width, height) for v in views]
    return Workload("c2", vol, h, [1.0, 2.0, 3.0], c=FRANGI_C["c2"], tf_knots=knots, tf_rgba=rgba,
                    params=render_params(lambda_g=0.5, lambda_v=2.0, et_alpha=0.99), cams=cams)


def c3(width=512, height=512, views=None):
    """128^3 at 1 mm: the simple phantom scaled x2 plus 6 tubes (R in [1.5, 3] vox) + N(0, 0.01^2);
    8 orthographic views (az k*45, el 20) at 512^2; 16-knot random TF and a perturbed target TF."""
    rng = np.random.default_rng(SEED_BASE + 3)
    dims, h = (128, 128, 128), (1.0, 1.0, 1.0)
    centre, shells = _c1_geometry(dims, h, (2.0, 2.0, 2.0))
    half = np.array([(n - 1) * s / 2 for n, s in zip(dims, h)])
    tubes = _draw_tubes(rng, 6, 1.5, 3.0, centre, half * 0.8, 1.0)
    knots, rgba = tf_random16(rng)
    target_rgba = perturb_tf(rng, rgba)
    vol = _render_volume(dims[::-1], h, shells, centre, tubes, (), rng, ("gauss", 0.01)).astype(np.float32)
    views = range(8) if views is None else views
    cams = [ortho_camera(dims, h, 45.0 * k, 20.0, width, height) for k in views]
    return Workload("c3", vol, h, [1.0], c=FRANGI_C["c3"], tf_knots=knots, tf_rgba=rgba,
                    params=render_params(lambda_v=0.5, et_alpha=0.0), cams=cams,
                    extra=dict(target_tf_rgba=target_rgba))


def c4_volume(b, width=512, height=512, views=None):
    """Volume b of the batched set: uneven shape (nx, ny in 96..256, nz in 40..180), in-plane
    spacing in [0.5, 1.2] mm, slice thickness in [3, 5] mm; the simple phantom in half-extent
    fractions + N(0, 0.01^2); 4 orthographic views (az k*90, el 15) at 512^2."""
    rng = np.random.default_rng([SEED_BASE, 4, b])
    nx, ny = (int(v) for v in rng.integers(96, 257, 2))
    nz = int(rng.integers(40, 181))
    hxy = float(rng.uniform(0.5, 1.2))
    hz = float(rng.uniform(3.0, 5.0))
    dims, h = (nx, ny, nz), (hxy, hxy, hz)
    half = np.array([(n - 1) * s / 2 for n, s in zip(dims, h)])
    scale = half / 31.5
    centre, shells = _c1_geometry(dims, h, tuple(scale))
    vol = _render_volume(dims[::-1], h, shells, centre, [], (), rng, ("gauss", 0.01)).astype(np.float32)
    knots, rgba = tf_c1()
    views = range(4) if views is None else views
    cams = [ortho_camera(dims, h, 90.0 * k, 15.0, width, height) for k in views]
    return Workload(f"c4_{b}", vol, h, [1.0], c=FRANGI_C["c4"], tf_knots=knots, tf_rgba=rgba,
                    params=render_params(lambda_v=0.0, et_alpha=0.99), cams=cams)


def c4_shapes(nvol=64):
    """Shapes and spacings of the batched set without painting the volumes."""
    out = []
    for b in range(nvol):
        rng = np.random.default_rng([SEED_BASE, 4, b])
        nx, ny = (int(v) for v in rng.integers(96, 257, 2))
        nz = int(rng.integers(40, 181))
        hxy = float(rng.uniform(0.5, 1.2))
        hz = float(rng.uniform(3.0, 5.0))
        out.append(((nx, ny, nz), (hxy, hxy, hz)))
    return out


def c5(width=2048, height=2048, views=None, dims=(512, 512, 400), spacing=(0.5, 0.5, 0.5)):
    """512x512x400 at 0.5 mm: the head phantom scaled, x60000 + N(0, 600^2), rounded to nearest
    and clipped to uint16 (raw scanner-like counts; normalized on the device); sigma = 0.5 mm;
    8 orthographic views (az k*45, el 20) at 2048^2, early termination 0.99, C3-style loss."""
    rng = np.random.default_rng(SEED_BASE + 5)
    h = spacing
    centre, shells, vent, tubes = _head(rng, dims, h)
    knots, rgba = tf_head()
    target_rgba = perturb_tf(rng, rgba)
    clean = _render_volume(dims[::-1], h, shells, centre, tubes, vent, rng, ("none", 0.0))
    nz = dims[2]
    raw = np.empty(dims[::-1], np.uint16)
    for z0 in range(0, nz, 16):
        z1 = min(nz, z0 + 16)
        sl = clean[z0:z1] * 60000.0 + 600.0 * rng.standard_normal(clean[z0:z1].shape)
        raw[z0:z1] = np.clip(np.rint(sl), 0, 65535).astype(np.uint16)
    del clean
    views = range(8) if views is None else views
    cams = [ortho_camera(dims, h, 45.0 * k, 20.0, width, height) for k in views]
    return Workload("c5", raw, h, [0.5], c=FRANGI_C["c5"], tf_knots=knots, tf_rgba=rgba,
                    params=render_params(lambda_g=0.5, lambda_v=2.0, et_alpha=0.99), cams=cams,
                    extra=dict(target_tf_rgba=target_rgba))


def small_random(seed, dims=(13, 11, 9), spacing=(1.0, 1.0, 1.0), lo=0.0, hi=1.0):
    """A small uniform-random volume for brute-force checks."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    return rng.uniform(lo, hi, (nz, ny, nx))


def grid_mm(dims, spacing):
    """Node positions X, Y, Z (mm), each [nz][ny][nx] float64, for closed-form test fields."""
    nx, ny, nz = dims
    hx, hy, hz = spacing
    Z, Y, X = np.meshgrid(np.arange(nz) * hz, np.arange(ny) * hy, np.arange(nx) * hx, indexing="ij")
    return X, Y, Z
