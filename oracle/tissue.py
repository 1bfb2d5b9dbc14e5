"""Oracle of the automatic tissue windows -- TEST INFRASTRUCTURE ONLY (same rules as the package).

Plain NumPy, written from the paper's description:
  histogram      Sec. 2.2: a 256-bin density analysis of I_norm over the used voxels
  tissue_peaks   Sec. 2.2: the three tissue peaks of the tri-modal histogram (CSF < GM < WM), each
                 then checked against its target window (Sec. 3.1, Table 2)
  tissue_tf      Sec. 2.2 / Sec. 3.2: a transfer function built from the peaks with zero extinction
                 below the CSF window (low-intensity bone and air clipped)
  aggregate      Sec. 3.1: per-class mean and sample SD of the peaks over cohorts (Table 1 -> Table 2)

Readings (the paper names these steps but not their arithmetic):
  * used voxels: I_norm > floor (floor = 0 drops the exact-zero background);
  * bin b = floor(256 I) clamped to [0, 255] (256 I is exact in binary floating point; I = 1 falls
    in the last bin);
  * peaks: local maxima of the [1, 2, 1]-smoothed counts S[b] = h[b-1] + 2 h[b] + h[b+1] (clamped
    ends, integer), a maximum being S[b] > S[b-1] and S[b] >= S[b+1] (the left end of a plateau);
    taken greedily by S descending (lower bin first on a tie), each at least min_sep bins from the
    ones taken, at most three, then ordered by bin; the peak intensity is the bin centre
    (b + 1/2) / 256; a missing peak has bin -1;
  * windows (Table 2): CSF [0.05, 0.12), GM [0.12, 0.18), WM (0.18, 1].
"""
from __future__ import annotations

import numpy as np

NBINS = 256
WINDOWS = ((0.05, 0.12), (0.12, 0.18), (0.18, 1.0))
# stand-in for a missing peak: the window centre (WM: its lower edge plus the GM window's width)
FALLBACK = (0.085, 0.15, 0.24)


def histogram(I, floor=0.0):
    """256-bin counts (int64) of the values I > floor (I in [0, 1]), and the number used."""
    x = np.asarray(I, np.float64).ravel()
    x = x[x > floor]
    b = np.clip(np.floor(x * NBINS), 0, NBINS - 1).astype(np.int64)
    return np.bincount(b, minlength=NBINS).astype(np.int64), int(x.size)


def smoothed(h):
    h = np.asarray(h, np.int64)
    left = np.concatenate([h[:1], h[:-1]])
    right = np.concatenate([h[1:], h[-1:]])
    return left + 2 * h + right


def in_window(c, peak):
    lo, hi = WINDOWS[c]
    if c < 2:
        return bool(lo <= peak < hi)
    return bool(lo < peak <= hi)


def tissue_peaks(h, min_sep=2):
    """dict(bin=[3], peak=[3], in_window=[3]) of the three tissue peaks (see the readings above)."""
    S = smoothed(h)
    cand = []
    for b in range(NBINS):
        left = S[b - 1] if b > 0 else -1
        right = S[b + 1] if b < NBINS - 1 else -1
        if S[b] > 0 and S[b] > left and S[b] >= right:
            cand.append(b)
    cand.sort(key=lambda b: (-S[b], b))
    taken = []
    for b in cand:
        if all(abs(b - t) >= min_sep for t in taken):
            taken.append(b)
        if len(taken) == 3:
            break
    taken.sort()
    bins = taken + [-1] * (3 - len(taken))
    peak = [(b + 0.5) / NBINS if b >= 0 else -1.0 for b in bins]
    return dict(bin=bins, peak=peak, in_window=[b >= 0 and in_window(c, p) for c, (b, p) in enumerate(zip(bins, peak))])


def tissue_tf(peaks, colours, taus, tau_hi=0.0, colour_hi=(1.0, 1.0, 1.0)):
    """8-knot TF from the peaks: knots (0, lo_CSF, m_CSF, m_GM, m_WM, u, u + 1/256, 1) with
    u = m_WM + (m_WM - m_GM) (the WM plateau mirrored about its peak), within [m_WM + 1/256,
    1 - 2/256].  A missing peak is replaced by FALLBACK; the knots are kept strictly increasing (at
    least one bin apart, the WM peak at most three bins below 1).  RGBA: zero extinction up to
    lo_CSF (bone and air clipped), the class colour and extinction at each peak (linear in between),
    the WM plateau up to u, then colour_hi / tau_hi (0 clips extracranial fat and enhancing tissue).
    Returns (knots float64 [8], rgba float64 [8][4])."""
    m = [(b + 0.5) / NBINS if b >= 0 else FALLBACK[c] for c, b in enumerate(peaks["bin"])]
    lo_csf = WINDOWS[0][0]
    s = 1.0 / NBINS
    # strictly increasing knots: each peak at least one bin above the previous knot, the WM peak at
    # most three bins below 1 (then the GM and CSF peaks at least one bin below the next)
    m[0] = max(m[0], lo_csf + s)
    m[1] = max(m[1], m[0] + s)
    m[2] = max(m[2], m[1] + s)
    m[2] = min(m[2], 1.0 - 3 * s)
    m[1] = min(m[1], m[2] - s)
    m[0] = min(m[0], m[1] - s)
    u = min(max(2 * m[2] - m[1], m[2] + s), 1.0 - 2 * s)
    knots = np.array([0.0, lo_csf, m[0], m[1], m[2], u, u + s, 1.0])
    cols = [colours[0], colours[0], colours[0], colours[1], colours[2], colours[2], colour_hi, colour_hi]
    tau = [0.0, 0.0, taus[0], taus[1], taus[2], taus[2], tau_hi, tau_hi]
    rgba = np.array([[*c, t] for c, t in zip(cols, tau)], np.float64)
    return knots, rgba


def aggregate(peaks_by_cohort):
    """Per-class (mean, sample SD with ddof = 1) over cohorts of (CSF, GM, WM) peaks, and whether
    every peak lies in its class window."""
    P = np.asarray(peaks_by_cohort, np.float64)
    mean = P.mean(axis=0)
    sd = P.std(axis=0, ddof=1)
    ok = all(in_window(c, p) for row in P for c, p in enumerate(row))
    return mean, sd, ok
