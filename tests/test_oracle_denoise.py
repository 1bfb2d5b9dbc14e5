"""Pins of the denoise oracle (CPU): the 3x3x3 median against scipy.ndimage.median_filter (mode
'nearest') and a per-voxel brute force; constant and linear volumes are fixed points of the median."""
import numpy as np
import scipy.ndimage as ndi

from oracle import denoise


def test_median3_library_and_brute_force():
    rng = np.random.default_rng(2)
    v = rng.random((7, 9, 11)).astype(np.float32)
    m = denoise.median3(v)
    np.testing.assert_array_equal(m, ndi.median_filter(v, size=3, mode="nearest"))
    nz, ny, nx = v.shape
    for (z, y, x) in [(0, 0, 0), (6, 8, 10), (3, 4, 5), (0, 8, 5), (6, 0, 10)]:
        nb = [v[min(max(z + a, 0), nz - 1), min(max(y + b, 0), ny - 1), min(max(x + c, 0), nx - 1)]
              for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
        assert m[z, y, x] == sorted(nb)[13]


def test_median3_fixed_points():
    c = np.full((5, 6, 7), 0.3, np.float32)
    np.testing.assert_array_equal(denoise.median3(c), c)
    z, y, x = np.meshgrid(np.arange(5), np.arange(6), np.arange(7), indexing="ij")
    lin = (x + 2 * y - 3 * z).astype(np.float32)  # exact: the 27 values are symmetric about the centre
    np.testing.assert_array_equal(denoise.median3(lin)[1:-1, 1:-1, 1:-1], lin[1:-1, 1:-1, 1:-1])
