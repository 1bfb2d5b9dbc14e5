"""Frangi's structure sensitivity by Frangi's rule, c = 1/2 max over voxels and scales of
|sigma^2 H|_F (the automatic c of the feature pass, Sec. 1's multi-scale vesselness): the oracle's
rule against a brute-force non-separable smoothing and NumPy Hessian, and the c stored for the
benchmarked workloads against the oracle's rule on their volumes."""
import json
import os

import numpy as np
import pytest

import oracle
import phantoms
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "frangi_c.json")


def _rule_bruteforce(vol, spacing, sigmas):
    fro = 0.0
    for s in sigmas:
        sm = bf.smooth_nonseparable(vol, tuple(s / h for h in spacing))
        H = bf.hessian_np(sm, spacing) * s * s
        f = np.sqrt(H[0] ** 2 + H[1] ** 2 + H[2] ** 2 + 2.0 * (H[3] ** 2 + H[4] ** 2 + H[5] ** 2))
        fro = max(fro, float(f.max()))
    return 0.5 * fro


def test_rule_against_bruteforce():
    vol = phantoms.small_random(21, (10, 9, 8))
    sp = (0.7, 1.1, 1.9)
    sig = [0.9, 1.6]
    c = oracle.features(vol, sp, sig, c=0.0)["c"]
    np.testing.assert_allclose(c, _rule_bruteforce(vol, sp, sig), rtol=1e-12)
    # one scale's rule is below the two-scale one unless that scale holds the maximum
    c1 = oracle.features(vol, sp, sig[:1], c=0.0)["c"]
    assert c1 <= c * (1 + 1e-15)


def test_flat_volume_takes_c_one():
    vol = np.full((6, 5, 4), 0.3)
    assert oracle.features(vol, (1.0, 1.0, 1.0), [1.0], c=0.0)["c"] == 1.0


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_stored_values_match_the_golden_file():
    d = _golden()
    for k in ("c2", "c3", "c4", "c5"):
        assert phantoms.FRANGI_C[k] == pytest.approx(d[k], rel=1e-8), k
    assert d["c4"] == max(d["c4_per_volume"]) and len(d["c4_per_volume"]) == 64


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_stored_c_is_the_rule_on_the_workload(name):
    w = getattr(phantoms, name)(8, 8, views=[0])
    sp = tuple(float(np.float32(h)) for h in w.spacing)
    c = oracle.features(w.vol.astype(np.float64), sp, [float(np.float32(s)) for s in w.sigmas], c=0.0)["c"]
    assert c == pytest.approx(phantoms.FRANGI_C[name], rel=1e-8)
    assert w.c == phantoms.FRANGI_C[name]


@pytest.mark.parametrize("b", [0, 29, 63])
def test_batched_volumes_rule(b):
    w = phantoms.c4_volume(b, 8, 8, views=[0])
    sp = tuple(float(np.float32(h)) for h in w.spacing)
    c = oracle.features(w.vol.astype(np.float64), sp, [float(np.float32(s)) for s in w.sigmas], c=0.0)["c"]
    d = _golden()
    assert c == pytest.approx(d["c4_per_volume"][b], rel=1e-12)
    assert c <= phantoms.FRANGI_C["c4"] * (1 + 1e-8) and w.c == phantoms.FRANGI_C["c4"]
