"""GPU parity of the guaranteed eigenvalue bounds (Sec. 4.3) and of the
reference choice built on them, through the C-ABI, against the oracle's
oracle/bounds.py (itself pinned to dense generalized eigenvalues in
tests/test_oracle_pins.py).

Tolerances: the nodal bounds are extreme generalized eigenvalues of small
SPD pairs, computed on the host by Jacobi rotations (library) and LAPACK
(oracle); they agree to 1e-12 relative.  The min / max over nodes and the
condition-number bound follow to the same accuracy.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import bounds as ob
from oracle.assembly import Problem
from synth import isotropic_conductivity, isotropic_mandel, spheres
from tests.helpers_tensor import random_spd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fh():
    from paper_2203_02962_amd import fh as fhmod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    fhmod.load_library()
    return fhmod


def _case(elem, problem, n, kind, seed):
    rng = np.random.default_rng(seed)
    dim = len(n)
    m = dim * (dim + 1) // 2 if problem == "elastic" else dim
    wl = dict(dim=dim, n=tuple(n) + (1,) * (3 - dim), problem=problem, element=elem,
              loads=np.eye(m))
    if kind == "field":
        wl["kfield"] = np.exp(rng.uniform(-2, 2, size=n[::-1]))
        return wl, Problem(n, problem, elem, kfield=wl["kfield"])
    nphase = 3
    wl["phase"] = rng.integers(0, nphase, size=n[::-1]).astype(np.uint8)
    if kind == "iso" and problem == "elastic":
        wl["mat"] = np.stack([isotropic_mandel(1.0 + 20 * p, 0.15 + 0.12 * p, dim)
                              for p in range(nphase)])
    elif kind == "iso":
        wl["mat"] = np.stack([isotropic_conductivity(1.0 + 20 * p, dim) for p in range(nphase)])
    else:
        wl["mat"] = np.stack([random_spd(m, rng, 20.0) * (1 + 10 * p) for p in range(nphase)])
    return wl, Problem(n, problem, elem, phase=wl["phase"], mat=wl["mat"])


CASES = [
    ("hex8", "elastic", (12, 8, 9), "phase"),
    ("hex8", "elastic", (16, 16, 16), "iso"),
    ("hex8", "scalar", (12, 6, 9), "field"),
    ("hex8", "scalar", (8, 8, 8), "phase"),
    ("tri2", "scalar", (12, 18), "iso"),
    ("quad4", "elastic", (12, 8), "phase"),
]


def _ctx(wl):
    from paper_2203_02962_amd.runner import setup_context
    return setup_context(wl)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}-{'x'.join(map(str, c[2]))}-{c[3]}")
def test_nodal_bounds_match_oracle(fh, case):
    elem, problem, n, kind = case
    say("eigen bounds", case)
    wl, prob = _case(elem, problem, n, kind, seed=5)
    ctx = _ctx(wl)
    Cmean = oracle.mean_material(prob)
    rng = np.random.default_rng(1)
    Cother = random_spd(Cmean.shape[0], rng, 5.0) * np.abs(Cmean).max()
    for Cref, pass_ref in ((Cmean, False), (Cmean, True), (Cother, True)):
        lo = torch.full((prob.N,), np.nan, dtype=torch.float64, device="cuda")
        hi = torch.full((prob.N,), np.nan, dtype=torch.float64, device="cuda")
        b = ctx.eigen_bounds(Cref if pass_ref else None, 1e-6, lo, hi)
        lo_o, hi_o = ob.node_bounds(prob, Cref)
        assert _rel(lo.cpu().numpy(), lo_o) <= 1e-12
        assert _rel(hi.cpu().numpy(), hi_o) <= 1e-12
        assert abs(b["lambda_min"] - lo_o.min()) <= 1e-12 * lo_o.min()
        assert abs(b["lambda_max"] - hi_o.max()) <= 1e-12 * hi_o.max()
        kap = ob.kappa_bound(lo_o, hi_o)
        assert abs(b["kappa"] - kap) <= 1e-12 * kap
        assert b["predicted_iterations"] == ob.predicted_iterations(kap, 1e-6)
        # the same range without the nodal arrays
        b2 = ctx.eigen_bounds(Cref if pass_ref else None, 1e-6)
        assert abs(b2["kappa"] - kap) <= 1e-12 * kap
    ctx.close()


def test_solve_stays_within_the_bound(fh):
    """PCG on the 2-phase sphere workload at 24^3 needs no more iterations
    than the CG estimate from the guaranteed condition-number bound allows
    for the relative Kref^-1-norm of the residual, which can exceed the
    energy-norm error ratio by sqrt(kappa)."""
    n = 24
    phase, _, _ = spheres(n, (2.0, 3.5), 0.3, seed=4)
    mat = np.stack([isotropic_mandel(1.0, 0.3), isotropic_mandel(100.0, 0.3)])
    wl = dict(dim=3, n=(n, n, n), problem="elastic", element="hex8", phase=phase, mat=mat,
              loads=np.eye(6))
    ctx = _ctx(wl)
    eta = 1e-8
    b = ctx.eigen_bounds(None, eta)
    assert abs(b["kappa"] - 100.0) <= 1e-12 * 100.0  # same nu: E ratio
    rc, st = ctx.solve(eta=eta)
    assert rc == 0
    limit = math.ceil(0.5 * math.sqrt(b["kappa"]) * math.log(2.0 * math.sqrt(b["kappa"]) / eta))
    say("iterations", st["iterations"], "bound", limit)
    assert max(st["iterations"]) <= limit
    ctx.close()


def test_reference_choice(fh):
    """FH_REF_BEST picks the smallest bound among the mean, I_s and the
    kappa-optimal isotropic reference; each candidate's bound equals the
    oracle's for that reference, the choice becomes the solve's reference,
    and C_hom does not depend on it."""
    n = 16
    phase, _, _ = spheres(n, (2.0, 3.5), 0.3, seed=9)
    # bulk-to-shear ratios 0.1 and 10: the mean's ratio (about 0.5 at volume
    # fraction 0.3) is far from the best isotropic reference's
    def iso_kg(K, G):
        C = np.zeros((6, 6))
        C[:3, :3] = K - 2.0 * G / 3.0
        return C + 2.0 * G * np.eye(6)
    mat = np.stack([iso_kg(1.0, 10.0), iso_kg(10.0, 1.0)])
    wl = dict(dim=3, n=(n, n, n), problem="elastic", element="hex8", phase=phase, mat=mat,
              loads=np.eye(6))
    prob = Problem((n,) * 3, "elastic", "hex8", phase=phase, mat=mat)
    ctx = _ctx(wl)
    rc, st_mean = ctx.solve(eta=1e-10)
    H_mean = ctx.get_homogenized()
    kap, chosen = {}, {}
    for strat in (fh.FH_REF_MEAN, fh.FH_REF_IDENTITY, fh.FH_REF_BEST):
        C, b = ctx.choose_reference(strat)
        chosen[strat] = C
        k_o = ob.kappa_bound(*ob.node_bounds(prob, C))
        assert abs(b["kappa"] - k_o) <= 1e-12 * k_o
        kap[strat] = k_o
        if strat == fh.FH_REF_MEAN:
            assert _rel(C, oracle.mean_material(prob)) <= 1e-14
        if strat == fh.FH_REF_IDENTITY:
            assert np.array_equal(C, np.eye(6))
    say("kappa mean / I_s / best:", kap)
    assert kap[fh.FH_REF_BEST] <= min(kap[fh.FH_REF_MEAN], kap[fh.FH_REF_IDENTITY])
    assert kap[fh.FH_REF_BEST] < 0.9 * kap[fh.FH_REF_MEAN]
    rc, st_best = ctx.solve(eta=1e-10)
    assert rc == 0
    assert np.array_equal(ctx.get_reference(), chosen[fh.FH_REF_BEST])
    assert _rel(ctx.get_homogenized(), H_mean) <= 1e-9
    # a new reference makes the previous solution stale
    ctx.choose_reference(fh.FH_REF_MEAN)
    with pytest.raises(fh.FHError):
        ctx.get_homogenized()
    say("iterations mean", st_mean["iterations"], "best", st_best["iterations"])
    ctx.close()


def test_bounds_input_errors(fh):
    wl, prob = _case("hex8", "elastic", (6, 4, 4), "phase", seed=2)
    ctx = _ctx(wl)
    with pytest.raises(fh.FHError):
        ctx.eigen_bounds(-np.eye(6))            # not SPD
    with pytest.raises(fh.FHError):
        ctx.choose_reference(7)                 # unknown strategy
    b = ctx.eigen_bounds(None, 1e-6)            # context still usable
    assert b["kappa"] >= 1.0
    ctx.close()
