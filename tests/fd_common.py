"""FP64 central finite differences of the oracle's render loss on the differentiable-render workload's
32^3 crop, at its stated scope: every TF value and every crop voxel (CPU only; calls the oracle).

Scene: the 128^3 phantom's features (g, k, V and |g|_max) from the pass over the whole volume,
cropped to [48, 80)^3 together with the intensities; 8 orthographic views (azimuth k 45 deg,
elevation 20 deg) of the crop at 64^2; the loss L = 1/2 sum (rgba - target)^2 against the image the
oracle renders with the workload's perturbed 16-knot TF; early termination off.  The features are
constants of the loss (the adjoint under test holds them fixed).

Perturbing voxel v changes only samples whose trilinear cell has v as a corner, i.e. samples inside
the open box (v - 1, v + 1)^3 in index space.  An orthographic ray meets that box only if its pixel
lies in the box's projection, so each voxel's difference is taken over the pixels of that
projection (plus one pixel of margin) in every view: the other pixels' losses do not change, and
each pixel is rendered exactly as in a whole-image render.
"""
from __future__ import annotations

import numpy as np

import oracle
import phantoms

CROP = (48, 80)
RES = 64
H_FD = 1e-4


def f32(x):
    return float(np.float32(x))


class CropScene:
    def __init__(self, res=RES):
        w = phantoms.c3(res, res, views=[0])
        self.w = w
        lo, hi = CROP
        self.vol_full = w.vol
        self.vol = np.ascontiguousarray(w.vol[lo:hi, lo:hi, lo:hi]).astype(np.float64)
        self.spacing = tuple(f32(h) for h in w.spacing)
        self.sigmas = [f32(s) for s in w.sigmas]
        self.c = f32(w.c)
        dims = (hi - lo,) * 3
        self.cams = [phantoms.ortho_camera(dims, w.spacing, 45.0 * k, 20.0, res, res) for k in range(8)]
        self.params = {k: f32(v) for k, v in w.params.items()}
        assert self.params["et_alpha"] == 0.0
        self.knots = w.tf_knots
        self.tf = w.tf_rgba.astype(np.float64)
        self.tf_target = w.extra["target_tf_rgba"].astype(np.float64)
        self.res = res

    def oracle_features(self):
        """The full-volume oracle features cropped, and the full volume's |g|_max."""
        lo, hi = CROP
        of = oracle.features(self.vol_full.astype(np.float64), self.spacing, self.sigmas, c=self.c)
        return dict(g=np.ascontiguousarray(of["g"][:, lo:hi, lo:hi, lo:hi]),
                    kappa=np.ascontiguousarray(of["kappa"][lo:hi, lo:hi, lo:hi]),
                    V=np.ascontiguousarray(of["V"][lo:hi, lo:hi, lo:hi]), gmax=of["gmax"])

    def render(self, feats, vol=None, tf=None, pix=None):
        return oracle.render(self.vol if vol is None else vol, feats, feats["gmax"], self.spacing, self.knots,
                             self.tf if tf is None else tf, self.params, self.cams, pix=pix)

    def target(self, feats):
        return self.render(feats, tf=self.tf_target)["rgba"]

    def footprint(self, v):
        """int32 [M][3] (view, i, j) of the pixels whose rays may pass through the open box (v-1, v+1)^3
        around voxel v = (x, y, z) (index space), in every view."""
        h = np.array(self.spacing, np.float64)
        corners = np.array([[v[0] + sx, v[1] + sy, v[2] + sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)],
                           np.float64) * h
        out = []
        for ci, cam in enumerate(self.cams):
            assert cam.persp == 0
            M = np.stack([np.asarray(cam.du, np.float64), np.asarray(cam.dv, np.float64),
                          np.asarray(cam.d0, np.float64)], 1)
            ab = np.linalg.solve(M, (corners - np.asarray(cam.o, np.float64)).T)  # (u, w, t) per corner
            u, wv = ab[0], ab[1]
            i0 = max(int(np.floor(u.min() - 0.5)) - 1, 0)
            i1 = min(int(np.ceil(u.max() - 0.5)) + 1, cam.width - 1)
            j0 = max(int(np.floor(wv.min() - 0.5)) - 1, 0)
            j1 = min(int(np.ceil(wv.max() - 0.5)) + 1, cam.height - 1)
            if i0 > i1 or j0 > j1:
                continue
            jj, ii = np.meshgrid(np.arange(j0, j1 + 1), np.arange(i0, i1 + 1), indexing="ij")
            ii, jj = ii.ravel(), jj.ravel()
            # keep the pixels whose ray meets the box grown by 1e-3 voxel (slab test in FP64)
            org = (np.asarray(cam.o, np.float64)[None] + (ii[:, None] + 0.5) * np.asarray(cam.du, np.float64)[None]
                   + (jj[:, None] + 0.5) * np.asarray(cam.dv, np.float64)[None])
            d = np.asarray(cam.d0, np.float64)
            lo = (np.asarray(v, np.float64) - 1.001) * h
            hi = (np.asarray(v, np.float64) + 1.001) * h
            tn, tf_ = np.full(len(ii), -np.inf), np.full(len(ii), np.inf)
            ok = np.ones(len(ii), bool)
            for a in range(3):
                if d[a] == 0.0:
                    ok &= (org[:, a] > lo[a]) & (org[:, a] < hi[a])
                    continue
                t1, t2 = (lo[a] - org[:, a]) / d[a], (hi[a] - org[:, a]) / d[a]
                tn = np.maximum(tn, np.minimum(t1, t2))
                tf_ = np.minimum(tf_, np.maximum(t1, t2))
            ok &= tf_ > tn
            out.append(np.stack([np.full(int(ok.sum()), ci), ii[ok], jj[ok]], 1))
        if not out:
            return np.zeros((0, 3), np.int32)
        return np.ascontiguousarray(np.concatenate(out), dtype=np.int32)


def pixel_losses(rgba, target, pix=None):
    """1/2 |rgba - target|^2 per pixel; rgba [M][4] for a pixel list, or whole images."""
    if pix is not None:
        t = target[pix[:, 0], pix[:, 2], pix[:, 1]]
        d = rgba - t
    else:
        d = rgba - target
    return 0.5 * np.sum(d * d, axis=-1)


def fd_tf(scene, feats, target, h=H_FD):
    """Central differences of L with respect to every TF value (knot RGB and extinction), [K][4]."""
    fd = np.zeros_like(scene.tf)
    for k in range(scene.tf.shape[0]):
        for ch in range(4):
            p, m = scene.tf.copy(), scene.tf.copy()
            p[k, ch] += h
            m[k, ch] -= h
            lp = pixel_losses(scene.render(feats, tf=p)["rgba"], target)
            lm = pixel_losses(scene.render(feats, tf=m)["rgba"], target)
            fd[k, ch] = float(np.sum(lp - lm)) / (2 * h)
    return fd


def _fd_chunk(scene, feats, target, l0_img, h, todo):
    vol = scene.vol.copy()
    out = []
    for (x, y, z) in todo:
        pix = scene.footprint((x, y, z))
        if len(pix) == 0:
            out.append((0.0, False))
            continue
        l0 = l0_img[pix[:, 0], pix[:, 2], pix[:, 1]]
        v0 = vol[z, y, x]
        vol[z, y, x] = v0 + h
        lp = pixel_losses(scene.render(feats, vol=vol, pix=pix)["rgba"], target, pix)
        vol[z, y, x] = v0 - h
        lm = pixel_losses(scene.render(feats, vol=vol, pix=pix)["rgba"], target, pix)
        vol[z, y, x] = v0
        dp = float(np.sum(lp - l0)) / h
        dm = float(np.sum(l0 - lm)) / h
        out.append((float(np.sum(lp - lm)) / (2 * h), abs(dp - dm) > 1e-3 * max(abs(dp), abs(dm)) + 1e-9))
    return out


_W = {}


def _worker_init(scene, feats, target, l0_img, h):
    # one thread per worker process: the pool provides the parallelism (set before the oracle loads)
    import os
    os.environ["OMP_NUM_THREADS"] = "1"
    _W.update(scene=scene, feats=feats, target=target, l0=l0_img, h=h)


def _worker_run(todo):
    return _fd_chunk(_W["scene"], _W["feats"], _W["target"], _W["l0"], _W["h"], todo)


def fd_voxels(scene, feats, target, h=H_FD, voxels=None, workers=None):
    """Central differences of L with respect to each crop voxel's intensity.  Returns (fd [nz][ny][nx],
    kink mask): a voxel whose +-h moves a sample across a TF knot has one-sided differences that
    disagree beyond the smooth curvature term; the central difference is not the derivative there.
    workers > 1 spreads the voxels over that many spawned single-threaded processes."""
    import os
    base = scene.render(feats)
    l0_img = pixel_losses(base["rgba"], target)
    nz, ny, nx = scene.vol.shape
    fd = np.zeros(scene.vol.shape)
    kink = np.zeros(scene.vol.shape, bool)
    todo = voxels if voxels is not None else [(x, y, z) for z in range(nz) for y in range(ny) for x in range(nx)]
    workers = min(16, os.cpu_count() or 1) if workers is None else workers
    if workers <= 1:
        res = _fd_chunk(scene, feats, target, l0_img, h, todo)
    else:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        chunks = [todo[i::workers * 4] for i in range(workers * 4)]
        with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"), initializer=_worker_init,
                                 initargs=(scene, feats, target, l0_img, h)) as ex:
            parts = list(ex.map(_worker_run, chunks))
        res = [None] * len(todo)
        for i, part in enumerate(parts):
            res[i::workers * 4] = part
    for (x, y, z), (d, k) in zip(todo, res):
        fd[z, y, x] = d
        kink[z, y, x] = k
    return fd, kink
