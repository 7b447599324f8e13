"""Seeded generators: determinism, achieved fractions, geometry rules."""
import hashlib

import numpy as np

from synth import batch_workload, circles2d, conductivity_grf, laminate, spheres, workload


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_spheres_deterministic_and_non_overlapping():
    p1, vf1, s1 = spheres(32, (3.0, 5.0), 0.3, seed=3)
    p2, vf2, s2 = spheres(32, (3.0, 5.0), 0.3, seed=3)
    assert _h(p1) == _h(p2) and vf1 == vf2
    assert vf1 >= 0.3 and abs(p1.mean() - vf1) < 1e-12
    c = np.array([s[:3] for s in s1])
    r = np.array([s[3] for s in s1])
    for i in range(len(r)):
        d = (c - c[i] + 16.0) % 32.0 - 16.0
        dist = np.sqrt((d * d).sum(axis=1))
        dist[i] = np.inf
        assert np.all(dist >= r + r[i])
    p3, _, _ = spheres(32, (3.0, 5.0), 0.3, seed=4)
    assert _h(p3) != _h(p1)


def test_circles_and_grf_and_laminate():
    a = circles2d(32, 8, (3, 6), seed=0)
    assert a.shape == (32, 32) and a.dtype == np.uint8 and 0 < a.mean() < 1
    k = conductivity_grf(32, 4.0, 1.5, 1e3, seed=1)
    assert k.max() / k.min() <= 1e3 * (1 + 1e-12)
    assert abs(np.log(k).std() - 1.5) < 0.3
    lam = laminate((4, 5, 6), 1, [0, 1, 1, 0, 1])
    assert lam.shape == (6, 5, 4) and np.all(lam[:, 1, :] == 1) and np.all(lam[:, 0, :] == 0)


def test_named_workloads():
    w = workload("conductivity2d_tri")
    assert w["phase"].shape == (32, 32) and w["n"] == (32, 32, 1)
    w = workload("elastic3d_spheres", n=32)
    assert w["phase"].shape == (32, 32, 32) and w["vf"] >= 0.3
    b = batch_workload(count=3)
    assert [x["n"][0] for x in b] == [x["n"][0] for x in batch_workload(count=3)]


def test_parallel_batch_workload_equals_serial():
    from synth.microstructure import batch_workload, batch_workload_parallel
    a = batch_workload(count=3, seed0=77, fixed_n=16)
    b = batch_workload_parallel(count=3, seed0=77, fixed_n=16, workers=2)
    for x, y in zip(a, b):
        assert np.array_equal(x["phase"], y["phase"]) and x["contrast"] == y["contrast"]
