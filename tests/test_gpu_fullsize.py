"""GPU parity at the benchmark sizes, with the benchmark's launch shapes.

Workloads: 128^3 elasticity (spheres, two isotropic phases, 6 unit strains)
and 256^3 heat conduction (k = exp of a periodic Gaussian random field, 3 unit
gradients); the operator also at 256^3 elasticity, the largest grid.  These grids are too large for the assembled oracle, so:

- operator outputs are compared at 2000 sampled nodes with the oracle's
  per-node rows (the element sum of eq. lin_system written out node by node),
  to 1e-12 of the largest sampled entry;
- the preconditioner is compared element by element over the whole field with
  the oracle's FFT form (Alg. 2 symbol from the sparse impulse response,
  numpy FFT as the transform), to 1e-11 of the largest entry: the round-off of
  a 2^21- or 2^24-point transform, amplified by the low-frequency blocks of
  K^+;
- solves are checked through properties that hold at any size: the residual
  of the GPU solution in the oracle's own system (right-hand side and operator
  rows at sampled nodes) within 100 times the PCG tolerance (which bounds the
  residual in the preconditioner's norm, not over sampled rows), symmetry of
  C_hom, the Voigt and Reuss bounds, and FP64 against FP32-refined results.
"""
import os
import sys

import numpy as np
import pytest

from oracle.assembly import Problem, operator_rows, rhs
from oracle.homog import mean_material
from oracle.precond import FFTPreconditioner
from synth import workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NSAMPLE = 2000


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fh():
    from paper_2203_02962_amd import fh as fhmod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    fhmod.load_library()
    return fhmod


def _problem(wl):
    n = tuple(wl["n"][: wl["dim"]])
    if wl.get("phase") is not None:
        return Problem(n, wl["problem"], wl["element"], phase=wl["phase"], mat=wl["mat"])
    return Problem(n, wl["problem"], wl["element"], kfield=wl["kfield"])


_CACHE = {}


def _setup(fh, name):
    """(workload, oracle problem, context), generated once per module."""
    if name not in _CACHE:
        from paper_2203_02962_amd.runner import setup_context
        say("generate", name)
        if name == "elastic128":
            wl = workload("elastic3d_spheres", seed=0, n=128)
        elif name == "elastic256":  # the largest grid the library accepts
            wl = workload("elastic3d_spheres", seed=0, n=256)
        else:
            wl = workload("conduction3d_grf", seed=0)
        _CACHE[name] = (wl, _problem(wl), setup_context(wl))
    return _CACHE[name]


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _nodes(prob, seed):
    return np.random.default_rng(seed).choice(prob.N, NSAMPLE, replace=False)


@pytest.mark.parametrize("name", ["elastic128", "conduction256", "elastic256"])
def test_full_size_operator_rows(fh, name):
    wl, prob, ctx = _setup(fh, name)
    say("operator rows", name)
    u = np.random.default_rng(11).standard_normal(prob.ndof_node * prob.N)
    ud = torch.from_numpy(u).cuda()
    qd = torch.empty_like(ud)
    ctx.apply_operator(ud, qd)
    q = qd.cpu().numpy().reshape(prob.ndof_node, prob.N)
    nodes = _nodes(prob, 12)
    ref = operator_rows(prob, u, nodes)
    say("rel err", _rel(q[:, nodes], ref))
    assert _rel(q[:, nodes], ref) < 1e-12


@pytest.mark.parametrize("name", ["elastic128", "conduction256"])
def test_full_size_preconditioner(fh, name):
    wl, prob, ctx = _setup(fh, name)
    say("preconditioner", name)
    r = np.random.default_rng(13).standard_normal(prob.ndof_node * prob.N)
    rd = torch.from_numpy(r).cuda()
    zd = torch.empty_like(rd)
    ctx.apply_preconditioner(rd, zd)
    z = zd.cpu().numpy()
    say("oracle preconditioner", name)
    zo = FFTPreconditioner(prob, mean_material(prob)).apply(r)
    say("rel err", _rel(z, zo))
    assert _rel(z, zo) < 1e-11


def _residual_ratio(prob, E, u, nodes):
    """||b - K u|| / ||b|| over the sampled rows, in the oracle's system."""
    b = rhs(prob, E).reshape(prob.ndof_node, prob.N)[:, nodes]
    Ku = operator_rows(prob, u, nodes)
    return np.linalg.norm(b - Ku) / np.linalg.norm(b)


def _fields(ctx, prob, nload):
    out = []
    for j in range(nload):
        d = torch.empty(prob.ndof_node * prob.N, dtype=torch.float64, device="cuda")
        ctx.get_fluctuation(j, d)
        out.append(d.cpu().numpy())
    return out


def test_elastic_128_solution_solves_oracle_system(fh):
    """FP64 solve to 1e-10 at 128^3 (6 loads together): the fluctuation of
    every load satisfies the oracle's equations at the sampled nodes."""
    wl, prob, ctx = _setup(fh, "elastic128")
    say("solve 128^3 residual rows")
    rc, st = ctx.solve(eta=1e-10, rebuild=True)
    assert rc == 0
    nodes = _nodes(prob, 14)
    for j, u in enumerate(_fields(ctx, prob, 6)):
        rr = _residual_ratio(prob, wl["loads"][j], u, nodes)
        say("load", j, "residual ratio", rr)
        assert rr < 100 * 1e-10, j  # measured 2e-10


def test_conduction_256_solves(fh):
    """256^3 conduction to 1e-8, FP64 and FP32-refined (the benchmark's two
    solves): both solutions satisfy the oracle's equations at sampled nodes,
    C_hom is symmetric, lies between the Reuss and Voigt bounds, and the two
    precisions agree (C_hom is quadratic in the solver error)."""
    wl, prob, ctx = _setup(fh, "conduction256")
    k = np.asarray(wl["kfield"], dtype=float)
    voigt, reuss = k.mean(), 1.0 / (1.0 / k).mean()
    nodes = _nodes(prob, 15)
    H = {}
    for prec in (fh.FH_FP64, fh.FH_FP32_REFINED):
        say("solve 256^3 precision", prec)
        rc, st = ctx.solve(eta=1e-8, precision=prec, rebuild=True)
        assert rc == 0
        say("rel_res", st["rel_res"][:3], "iterations", st["iterations"][:3])
        assert max(st["rel_res"][:3]) <= 1e-8
        H[prec] = ctx.get_homogenized()
        for j, u in enumerate(_fields(ctx, prob, 3)):
            rr = _residual_ratio(prob, wl["loads"][j], u, nodes)
            say("load", j, "residual ratio", rr)
            assert rr < 100 * 1e-8, (prec, j)  # measured 6e-8
        C = H[prec]
        assert _rel(C, C.T) < 1e-12
        lam = np.linalg.eigvalsh(0.5 * (C + C.T))
        assert lam.min() > reuss * (1 - 1e-12) and lam.max() < voigt * (1 + 1e-12)
    say("C_hom FP32-refined vs FP64", _rel(H[fh.FH_FP32_REFINED], H[fh.FH_FP64]))
    assert _rel(H[fh.FH_FP32_REFINED], H[fh.FH_FP64]) < 1e-10


GOLDEN_256 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                          "conduction3d_grf_256_seed0.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN_256),
                    reason="stored oracle result for 256^3 conduction not written yet "
                           "(tests/golden/make_golden.py conduction3d_grf_256)")
def test_conduction_256_matches_stored_oracle(fh):
    """256^3 conduction against the CPU oracle's stored result (assembled CSR
    K, FFT-form preconditioner, PCG to 1e-8; tests/golden/make_golden.py):
    FP64 and FP32-refined C_hom element by element to 1e-10 of the largest
    entry, FP64 iteration counts to +-max(1, 1 %), and the fluctuation at
    the stored sample nodes to 1e-6 relative (both solutions are within
    about sqrt(kappa) eta = 3e-7 of the exact one at eta = 1e-8)."""
    import hashlib
    import json
    g = json.load(open(GOLDEN_256))
    wl, prob, ctx = _setup(fh, "conduction256")
    k = np.ascontiguousarray(np.asarray(wl["kfield"], dtype=np.float64))
    assert hashlib.sha256(k.tobytes()).hexdigest() == g["kfield_sha256"]
    Hg = np.array(g["C_hom"])
    nodes = np.array(g["sample_nodes"])
    for prec in (fh.FH_FP64, fh.FH_FP32_REFINED):
        rc, st = ctx.solve(eta=g["eta"], precision=prec, rebuild=True)
        assert rc == 0
        H = ctx.get_homogenized()
        say("C_hom vs stored oracle, precision", prec, _rel(H, Hg))
        assert _rel(H, Hg) <= 1e-10
        if prec == fh.FH_FP64:
            for a, b in zip(st["iterations"][:3], g["iterations"]):
                assert abs(a - b) <= max(1, 0.01 * b), (st["iterations"], g["iterations"])
        for j, u in enumerate(_fields(ctx, prob, 3)):
            us = np.asarray(g["u_samples"][j])
            assert np.linalg.norm(u[nodes] - us) <= 1e-6 * np.linalg.norm(us), (prec, j)


def test_batch_96_benchmark_workload(fh):
    """The benchmark's batch: 96 microstructures (n in {32, 48, 64, 96}) x 6
    unit strains in one FP32-refined call to 1e-6.  Every system's C_hom
    agrees with its own FP64 single solve to 1e-10 within 1e-8 (C_hom is
    quadratic in the 1e-6 solver error; measured 1.6e-9), and the fluctuation
    fields of one system per grid size satisfy the oracle's equations at
    sampled nodes to 1e-5 (ten times the tolerance, which bounds the residual
    in the preconditioner's norm, not the 2-norm; measured 1-2e-6)."""
    from paper_2203_02962_amd.runner import setup_context
    from synth import batch_workload_parallel
    say("batch: generate 96")
    wls = batch_workload_parallel(count=96, workers=16)
    devs = [(torch.from_numpy(w["phase"]).cuda(), w["n"], w["mat"]) for w in wls]
    pick = {}
    for i, w in enumerate(wls):
        pick.setdefault(w["n"][0], i)
    u_out = [None] * len(wls)
    for i in pick.values():
        u_out[i] = torch.empty(6 * 3 * int(np.prod(wls[i]["n"])), dtype=torch.float64,
                               device="cuda")
    ctx = fh.Context(0)
    say("batch: solve")
    rc, Hb, sts, rep = ctx.solve_batch(devs, np.eye(6), eta=1e-6,
                                       precision=fh.FH_FP32_REFINED, u_out=u_out)
    assert rc == 0
    worst = 0.0
    for i, w in enumerate(wls):
        wl = dict(dim=3, n=w["n"], problem="elastic", element="hex8", phase=w["phase"],
                  mat=w["mat"], loads=np.eye(6))
        c1 = setup_context(wl)
        c1.solve(eta=1e-10)
        worst = max(worst, _rel(Hb[i], c1.get_homogenized()))
        c1.close()
    say("batch: worst C_hom difference vs FP64 single solves", worst)
    assert worst < 1e-8
    for n, i in pick.items():
        w = wls[i]
        prob = Problem(tuple(w["n"]), "elastic", "hex8", phase=w["phase"], mat=w["mat"])
        u = u_out[i].cpu().numpy().reshape(6, -1)
        nodes = _nodes(prob, 16)
        for j in range(6):
            rr = _residual_ratio(prob, np.eye(6)[j], u[j], nodes)
            say("batch system", i, "n", n, "load", j, "residual ratio", rr)
            assert rr < 1e-5, (i, j)
