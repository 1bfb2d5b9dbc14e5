"""Oracle of the optional denoise pre-pass (Sec. 5.3: in-shader spatial smoothing or median filtering
before the morphology pass) -- TEST INFRASTRUCTURE ONLY (same rules as the package).

  median3   3x3x3 median with clamp-to-edge indices: the 14th smallest of the 27 neighbours
  gauss     the sampled, normalized Gaussian of radius floor(3 sigma/h + 1/2) per axis with
            clamp-to-edge, applied along x, y and z (the oracle's own separable smoothing, FP64)
"""
from __future__ import annotations

import numpy as np

from oracle import smooth


def median3(vol):
    v = np.asarray(vol)
    p = np.pad(v, 1, mode="edge")
    nz, ny, nx = v.shape
    stack = [p[dz:dz + nz, dy:dy + ny, dx:dx + nx] for dz in range(3) for dy in range(3) for dx in range(3)]
    s = np.sort(np.stack(stack, 0), axis=0)
    return s[13]


def gauss(vol, spacing, sigma_mm):
    sv = tuple(float(sigma_mm) / float(h) for h in spacing)
    return smooth(np.asarray(vol, np.float64), sv)
