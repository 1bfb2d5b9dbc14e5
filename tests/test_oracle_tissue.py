"""Pins of the tissue-window oracle (CPU).

* Sec. 3.1: Table 2's mean peaks and SDs are the per-class mean and sample SD (ddof = 1) of Table 1's
  three cohorts, and every Table 1 peak lies in its Table 2 window ("100 % within windows").
* The histogram against a brute-force per-value loop, the exact bin edges k/256, the top value 1.0,
  and the floor; the peak finder on closed-form histograms (three separated bumps, plateaus, the
  minimum separation, fewer than three maxima) and on a phantom with known tissue values.
* The synthesized TF: knots strictly increasing, zero extinction below the CSF window and at the
  peaks' colours/extinctions, for regular and degenerate peak sets."""
import json
import os

import numpy as np
import pytest

from oracle import tissue

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tissue_tables.json")


def test_table2_is_mean_and_sample_sd_of_table1():
    g = json.load(open(GOLDEN))
    P = [g["table1_peaks"][k] for k in ("A", "B", "C")]
    mean, sd, ok = tissue.aggregate(P)
    t2 = g["table2"]
    for c, name in enumerate(("CSF", "GM", "WM")):
        # Table 2 prints 3 decimals; the WM mean 0.2247 is printed as 0.224 (truncated), so the
        # comparison allows one unit in the third decimal
        assert abs(mean[c] - t2[name]["mean"]) <= 1e-3 + 1e-12, (name, mean[c])
        assert abs(sd[c] - t2[name]["sd"]) <= 5e-4 + 1e-12, (name, sd[c])
    np.testing.assert_allclose(mean, [0.075667, 0.141, 0.224667], atol=1e-6)
    np.testing.assert_allclose(sd, [0.030072, 0.022517, 0.073908], atol=1e-6)
    assert ok  # Sec. 3.1: 100 % of the extracted peaks within their windows
    # a sample SD (ddof = 1), not a population SD: the latter would give 0.0246 for CSF
    assert abs(np.std(np.asarray(P)[:, 0]) - 0.030) > 4e-3


def test_histogram_matches_brute_force_and_edges():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.random(5000), np.arange(257) / 256.0, [0.0, 1.0, 1.0, -0.0]]).astype(np.float32)
    h, used = tissue.histogram(x, floor=0.0)
    ref = np.zeros(256, np.int64)
    n = 0
    for v in x.astype(np.float64):
        if v > 0.0:
            b = min(int(np.floor(v * 256)), 255)
            ref[b] += 1
            n += 1
    np.testing.assert_array_equal(h, ref)
    assert used == n == h.sum()
    # k/256 falls in bin k (k < 256); 1.0 falls in the last bin
    h1, _ = tissue.histogram(np.array([3 / 256, 100 / 256, 1.0]), 0.0)
    assert h1[3] == 1 and h1[100] == 1 and h1[255] == 1
    h2, u2 = tissue.histogram(np.array([0.01, 0.02, 0.5]), floor=0.015)
    assert u2 == 2 and h2[int(0.02 * 256)] == 1 and h2[128] == 1


def _bumps(centres, widths, heights):
    b = np.arange(256)
    return np.round(sum(hh * np.exp(-0.5 * ((b - c) / w) ** 2) for c, w, hh in zip(centres, widths, heights))).astype(np.int64)


def test_peaks_closed_form():
    h = _bumps([20, 35, 50], [2.0, 2.5, 3.0], [5000, 9000, 7000])
    p = tissue.tissue_peaks(h)
    assert p["bin"] == [20, 35, 50]
    assert p["in_window"] == [True, True, True]  # 20.5/256 = 0.080, 35.5/256 = 0.139, 50.5/256 = 0.197
    # a flat top: the left end of the plateau
    h = np.zeros(256, np.int64)
    h[[30, 31, 32]] = 10
    h[[100, 101]] = 4
    h[200] = 2
    assert tissue.tissue_peaks(h)["bin"] == [31, 100, 200]
    # two maxima (of the smoothed counts) closer than min_sep: only the higher one is taken
    h = np.zeros(256, np.int64)
    h[40], h[43], h[90] = 100, 80, 50
    assert tissue.tissue_peaks(h, min_sep=4)["bin"] == [40, 90, -1]
    assert tissue.tissue_peaks(h, min_sep=2)["bin"] == [40, 43, 90]
    # spikes one bin apart merge under the [1, 2, 1] smoothing
    h[43], h[42] = 0, 80
    assert tissue.tissue_peaks(h, min_sep=1)["bin"] == [40, 90, -1]
    # nothing above zero
    p = tissue.tissue_peaks(np.zeros(256, np.int64))
    assert p["bin"] == [-1, -1, -1] and p["in_window"] == [False, False, False]


def test_peaks_of_a_phantom_with_known_tissues():
    """Three tissue classes at 0.08, 0.15, 0.22 (inside the three windows) with N(0, 0.004^2)
    noise and a zero background: the peaks fall on the bins holding the class values."""
    rng = np.random.default_rng(7)
    vals = np.concatenate([np.full(40000, 0.08), np.full(60000, 0.15), np.full(50000, 0.22)])
    I = np.concatenate([vals + rng.normal(0, 0.004, vals.size), np.zeros(30000)])
    h, used = tissue.histogram(I, floor=0.0)
    assert used == 150000
    p = tissue.tissue_peaks(h)
    for b, v in zip(p["bin"], (0.08, 0.15, 0.22)):
        assert abs(b - int(v * 256)) <= 1
    assert p["in_window"] == [True, True, True]


@pytest.mark.parametrize("bins", [[20, 35, 50], [-1, 35, -1], [250, 252, 255], [0, 1, 2], [-1, -1, -1]])
def test_synthesized_tf(bins):
    peaks = dict(bin=bins)
    cols = [(0.2, 0.4, 1.0), (0.9, 0.6, 0.5), (1.0, 0.95, 0.85)]
    taus = (0.1, 0.3, 0.6)
    kn, rgba = tissue.tissue_tf(peaks, cols, taus)
    assert kn.shape == (8,) and rgba.shape == (8, 4)
    assert np.all(np.diff(kn) > 0) and kn[0] == 0.0 and kn[-1] == 1.0
    assert rgba[0, 3] == 0.0 and rgba[1, 3] == 0.0 and kn[1] == 0.05
    np.testing.assert_array_equal(rgba[2:5, 3], taus)
    if bins == [20, 35, 50]:
        np.testing.assert_allclose(kn[2:5], [(b + 0.5) / 256 for b in bins])
        np.testing.assert_allclose(kn[5], 2 * kn[4] - kn[3])
