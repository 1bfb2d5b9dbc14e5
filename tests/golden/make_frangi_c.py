"""Writes frangi_c.json: Frangi's structure sensitivity c = 1/2 max over voxels (and scales) of the
Frobenius norm of sigma^2 H, computed by the oracle for each benchmarked workload (its automatic-c
rule), so that the timed feature passes run with c fixed to that value and stay single-pass.
The batched set shares one c: half the largest norm over all 64 volumes.

    python tests/golden/make_frangi_c.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import phantoms  # noqa: E402


def rule_c(vol, spacing, sigmas):
    sp = tuple(float(np.float32(h)) for h in spacing)
    return oracle.features(np.ascontiguousarray(vol, dtype=np.float64), sp, [float(np.float32(s)) for s in sigmas],
                           c=0.0)["c"]


def main():
    out = {}
    w = phantoms.c2(8, 8, views=[0])
    out["c2"] = rule_c(w.vol, w.spacing, w.sigmas)
    w = phantoms.c3(8, 8, views=[0])
    out["c3"] = rule_c(w.vol, w.spacing, w.sigmas)
    w = phantoms.c5(8, 8, views=[0])
    v = w.vol.astype(np.float64)
    v = (v - v.min()) / (v.max() - v.min())  # the normalized volume the feature pass reads (Eq. 1)
    out["c5"] = rule_c(v, w.spacing, w.sigmas)
    del v, w
    per = []
    for b in range(64):
        w = phantoms.c4_volume(b, 8, 8, views=[0])
        per.append(rule_c(w.vol, w.spacing, w.sigmas))
        print(f"c4 volume {b}: {per[-1]:.6g}", flush=True)
    out["c4_per_volume"] = per
    out["c4"] = max(per)
    for k in ("c2", "c3", "c5", "c4"):
        print(f"{k}: c = {out[k]:.9g}")
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "frangi_c.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
