"""GPU parity: the HIP path through the C-ABI against the CPU FP64 oracle.

Tolerances (FP64): step-level results (operator, right-hand side, symbol,
preconditioner) agree element by element to 1e-12 relative to the largest
entry (round-off of sums of at most a few hundred terms); full solves agree on
the homogenized tensor to 1e-10 relative and on the PCG iteration count to
+-max(1, 1% of the count).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle.assembly import Problem, assemble_stiffness, rhs
from oracle.precond import Preconditioner
from synth import isotropic_conductivity, isotropic_mandel, laminate, spheres, workload
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


def _case(elem, problem, n, nphase=3, kind="phase", seed=0, l=None):
    rng = np.random.default_rng(seed)
    dim = len(n)
    m = dim * (dim + 1) // 2 if problem == "elastic" else dim
    wl = dict(dim=dim, n=tuple(n) + (1,) * (3 - dim), problem=problem, element=elem,
              loads=np.eye(m), l=l)
    if kind in ("phase", "iso"):
        wl["phase"] = rng.integers(0, nphase, size=n[::-1]).astype(np.uint8)
        if kind == "iso" and problem == "scalar":
            wl["mat"] = np.stack([isotropic_conductivity(1.0 + 20 * p, dim)
                                  for p in range(nphase)])
        elif kind == "iso":
            wl["mat"] = np.stack([isotropic_mandel(1.0 + 20 * p, 0.2 + 0.1 * p, dim)
                                  for p in range(nphase)])
        else:
            wl["mat"] = np.stack([random_spd(m, rng, 20.0) * (1 + 10 * p) for p in range(nphase)])
        prob = Problem(n, problem, elem, phase=wl["phase"], mat=wl["mat"], l=l)
    else:
        wl["kfield"] = np.exp(rng.uniform(-2, 2, size=n[::-1]))
        prob = Problem(n, problem, elem, kfield=wl["kfield"], l=l)
    return wl, prob


CASES = [
    ("hex8", "elastic", (24, 12, 18), "phase", (1.0, 0.8, 1.2)),
    ("hex8", "elastic", (32, 16, 16), "phase", None),
    ("hex8", "elastic", (6, 4, 6), "phase", None),
    ("hex8", "elastic", (24, 12, 18), "iso", (1.0, 0.8, 1.2)),
    ("hex8", "elastic", (36, 18, 24), "iso", None),
    ("hex8", "elastic", (4, 2, 2), "iso", None),
    # cubic voxels, z chunks of 8, 8 and 2: the carried face modes across a
    # partial last chunk
    ("hex8", "elastic", (12, 18, 18), "iso", None),
    ("hex8", "scalar", (12, 18, 6), "phase", None),
    ("hex8", "scalar", (12, 18, 6), "field", (0.5, 1.0, 1.5)),
    ("hex8", "scalar", (12, 18, 6), "iso", (1.0, 0.8, 1.2)),
    ("hex8", "scalar", (24, 12, 18), "iso", None),
    ("hex8", "scalar", (36, 18, 24), "field", None),
    # z lengths whose plans end in radix 8 and 4 (fused scalar z pass)
    ("hex8", "scalar", (6, 4, 64), "field", None),
    ("hex8", "scalar", (4, 6, 32), "iso", (1.0, 0.8, 1.2)),
    ("tri2", "scalar", (12, 18), "phase", None),
    ("tri2", "elastic", (12, 6), "phase", None),
    ("quad4", "elastic", (12, 8), "phase", (1.0, 0.7)),
    ("quad4", "scalar", (8, 6), "phase", None),
]


def _ids(c):
    return f"{c[0]}-{c[1]}-{'x'.join(map(str, c[2]))}-{c[3]}"


def _ctx(fh, wl):
    from paper_2203_02962_amd.runner import setup_context
    return setup_context(wl)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_operator_matches_oracle(fh, case):
    elem, problem, n, kind, l = case
    say("operator", _ids(case))
    wl, prob = _case(elem, problem, n, kind=kind, l=l)
    ctx = _ctx(fh, wl)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(prob.ndof_node * prob.N)
    ud = torch.from_numpy(u).cuda()
    qd = torch.empty_like(ud)
    ctx.apply_operator(ud, qd)
    ref = assemble_stiffness(prob) @ u
    assert _rel(qd.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_rhs_matches_oracle(fh, case):
    elem, problem, n, kind, l = case
    say("rhs", _ids(case))
    wl, prob = _case(elem, problem, n, kind=kind, l=l)
    ctx = _ctx(fh, wl)
    E = np.random.default_rng(2).standard_normal(wl["loads"].shape[1])
    bd = torch.empty(prob.ndof_node * prob.N, dtype=torch.float64, device="cuda")
    ctx.compute_rhs(E, bd)
    ref = rhs(prob, E)
    assert _rel(bd.cpu().numpy(), ref) < 1e-12


def _half_symbol(prob, Kplus):
    """oracle K^+ (N, nd, nd) -> [s][kx][ky][kz] half spectrum, / N."""
    nd = prob.ndof_node
    n = prob.n + (1,) * (3 - prob.dim)
    K = Kplus.reshape(n[2], n[1], n[0], nd, nd)[:, :, : n[0] // 2 + 1]
    K = np.transpose(K, (2, 1, 0, 3, 4)) / prob.N
    pairs = {3: [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)], 2: [(0, 0), (1, 1), (0, 1)],
             1: [(0, 0)]}[nd]
    return np.stack([K[..., a, b] for a, b in pairs])


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_symbol_and_preconditioner_match_oracle(fh, case):
    elem, problem, n, kind, l = case
    say("symbol+precond", _ids(case))
    wl, prob = _case(elem, problem, n, kind=kind, l=l)
    ctx = _ctx(fh, wl)
    Cref = oracle.mean_material(prob)
    M = Preconditioner(prob, Cref)
    nsym = prob.ndof_node * (prob.ndof_node + 1) // 2
    nf = (wl["n"][0] // 2 + 1) * wl["n"][1] * wl["n"][2]
    kd = torch.empty(nsym * nf, dtype=torch.float64, device="cuda")
    ctx.get_symbol(kd)
    ref = _half_symbol(prob, M.Kplus)
    assert np.abs(ref.imag).max() < 1e-12 * np.abs(ref).max()
    assert _rel(kd.cpu().numpy(), ref.real.ravel()) < 1e-12
    # the oracle sums the voxel tables pairwise, the library uses exact
    # per-phase counts: both are exact up to a few roundings
    assert _rel(ctx.get_reference(), Cref) < 1e-14
    r = np.random.default_rng(3).standard_normal(prob.ndof_node * prob.N)
    rd = torch.from_numpy(r).cuda()
    zd = torch.empty_like(rd)
    ctx.apply_preconditioner(rd, zd)
    assert _rel(zd.cpu().numpy(), M.apply(r)) < 1e-12


def _solve_both(fh, wl, prob, eta):
    from paper_2203_02962_amd.runner import fluctuations
    ctx = _ctx(fh, wl)
    rc, st = ctx.solve(eta=eta)
    H = ctx.get_homogenized()
    us = fluctuations(ctx)
    Ho, uo, res = oracle.homogenize(prob, wl["loads"], eta)
    return (rc, st, H, us), (Ho, uo, res)


SOLVE_CASES = [
    ("elastic-spheres-24", lambda: _spheres_case(24, (2.5, 4.5), 100.0, 0)),
    ("elastic-random-18x24x36", lambda: _spheres_box((18, 24, 36), 1)),
    ("conductivity2d-tri-32", lambda: _named("conductivity2d_tri")),
    ("scalar-hex8-field-16", lambda: _field_case(16)),
    ("elastic-laminate-x", lambda: _laminate_case()),
]


def _spheres_case(n, rr, contrast, seed):
    phase, _, _ = spheres(n, rr, 0.3, seed)
    mat = np.stack([isotropic_mandel(1.0, 0.3), isotropic_mandel(contrast, 0.3)])
    wl = dict(dim=3, n=(n, n, n), problem="elastic", element="hex8", phase=phase, mat=mat,
              loads=np.eye(6))
    return wl, Problem((n,) * 3, "elastic", "hex8", phase=phase, mat=mat)


def _spheres_box(n, seed):
    rng = np.random.default_rng(seed)
    phase = (rng.random(n[::-1]) < 0.3).astype(np.uint8)
    mat = np.stack([isotropic_mandel(1.0, 0.3), isotropic_mandel(30.0, 0.25)])
    wl = dict(dim=3, n=n, problem="elastic", element="hex8", phase=phase, mat=mat,
              loads=np.eye(6))
    return wl, Problem(n, "elastic", "hex8", phase=phase, mat=mat)


def _named(name):
    wl = workload(name)
    n = wl["n"][: wl["dim"]]
    return wl, Problem(n, wl["problem"], wl["element"], phase=wl["phase"], mat=wl["mat"])


def _field_case(n):
    from synth import conductivity_grf
    k = conductivity_grf(n, 2.0, 1.5, 1e3, seed=5)
    wl = dict(dim=3, n=(n, n, n), problem="scalar", element="hex8", kfield=k, loads=np.eye(3))
    return wl, Problem((n,) * 3, "scalar", "hex8", kfield=k)


def _laminate_case():
    n = (12, 6, 8)
    phase = laminate(n, 0, [0, 1, 1, 0, 1, 0, 0, 1, 1, 1, 0, 0])
    rng = np.random.default_rng(7)
    mat = np.stack([random_spd(6, rng, 5.0), 50 * random_spd(6, rng, 5.0)])
    wl = dict(dim=3, n=n, problem="elastic", element="hex8", phase=phase, mat=mat,
              loads=np.eye(6))
    return wl, Problem(n, "elastic", "hex8", phase=phase, mat=mat)


@pytest.mark.parametrize("name,make", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_solve_matches_oracle(fh, name, make):
    say("solve", name)
    wl, prob = make()
    (rc, st, H, us), (Ho, uo, res) = _solve_both(fh, wl, prob, 1e-10)
    assert rc == 0, st
    assert _rel(H, Ho) < 1e-10
    for j, r in enumerate(res):
        # the two FP64 runs sum in different orders; over long runs (high
        # contrast, a flat residual tail) the stop can move by about 1% of
        # the count, hence +-max(1, 1%)
        tol = max(1, int(0.01 * r.iterations))
        assert abs(st["iterations"][j] - r.iterations) <= tol, (st["iterations"], [x.iterations for x in res])
        # fluctuation: relative l2 error at most 1e-8 at eta = 1e-10 (the
        # field error of either solve is about sqrt(kappa) eta in norm)
        l2 = np.linalg.norm(us[j] - uo[j]) / max(np.linalg.norm(uo[j]), 1e-300)
        say("load", j, "u rel l2", l2)
        assert l2 < 1e-8, (j, l2)


def test_homogeneous_medium_zero_iterations(fh):
    say("homogeneous")
    n = (8, 6, 12)
    C0 = isotropic_mandel(3.0, 0.2)
    wl = dict(dim=3, n=n, problem="elastic", element="hex8",
              phase=np.zeros(n[::-1], np.uint8), mat=C0[None], loads=np.eye(6))
    ctx = _ctx(fh, wl)
    rc, st = ctx.solve(eta=1e-10)
    assert rc == 0 and st["iterations"] == [0] * 6
    assert _rel(ctx.get_homogenized(), C0) < 1e-14


def test_reference_equal_material_one_iteration(fh):
    say("C = Cref")
    n = (12, 8, 6)
    C = random_spd(6, np.random.default_rng(4))
    wl = dict(dim=3, n=n, problem="elastic", element="hex8",
              phase=np.zeros(n[::-1], np.uint8), mat=C[None], loads=np.eye(6))
    ctx = _ctx(fh, wl)
    b = np.random.default_rng(5).standard_normal((3, int(np.prod(n))))
    b -= b.mean(axis=1, keepdims=True)
    bd = torch.from_numpy(b.ravel()).cuda()
    ud = torch.empty_like(bd)
    rc, st = ctx.solve_rhs(bd, ud, eta=1e-12)
    assert rc == 0 and st["iterations"] == [1]


def test_solve_is_bitwise_deterministic(fh):
    say("determinism")
    from paper_2203_02962_amd.runner import fluctuations
    wl, prob = _spheres_case(16, (2.0, 3.5), 100.0, 3)
    ctx = _ctx(fh, wl)
    ctx.solve(eta=1e-8)
    H1, u1 = ctx.get_homogenized(), fluctuations(ctx)
    ctx.solve(eta=1e-8)
    H2, u2 = ctx.get_homogenized(), fluctuations(ctx)
    assert np.array_equal(H1, H2)
    assert all(np.array_equal(a, b) for a, b in zip(u1, u2))


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_graph_replay_matches_host_launches(fh, precision):
    """With FH_FLAG_GRAPH a single solve replays one captured PCG iteration
    from a hipGraph on the context's private stream; by default the host
    launches every kernel.  The kernels and their order are the same, so
    C_hom, the fluctuations, the iteration counts and the residual
    histories are bit for bit equal, over repeated solves in both orders."""
    say("graph replay vs eager", precision)
    from paper_2203_02962_amd.runner import fluctuations
    prec = fh.FH_FP64 if precision == "fp64" else fh.FH_FP32_REFINED
    wl, prob = _spheres_case(16, (2.0, 3.5), 100.0, 3)
    ctx = _ctx(fh, wl)
    runs = []
    for graph in (False, True, True, False):
        rc, st = ctx.solve(eta=1e-10, precision=prec, graph=graph, rebuild=True)
        assert rc == 0
        runs.append((st["iterations"], ctx.get_homogenized(), fluctuations(ctx),
                     [ctx.get_history(j) for j in range(6)]))
    it0, H0, u0, h0 = runs[0]
    for it, H, u, h in runs[1:]:
        assert it == it0
        assert np.array_equal(H, H0)
        assert all(np.array_equal(a, b) for a, b in zip(u, u0))
        assert all(np.array_equal(a, b) for a, b in zip(h, h0))
    ctx.close()


def test_kernel_timing_counts(fh):
    """Event timing of every launch, or of every 8th PCG iteration: the
    launch counts, timed counts and totals are consistent, and timing does
    not change the result."""
    say("kernel timing")
    wl, prob = _spheres_case(16, (2.0, 3.5), 100.0, 3)
    ctx = _ctx(fh, wl)
    rc0, st0 = ctx.solve(eta=1e-10)
    H0 = ctx.get_homogenized()
    rc1, st1 = ctx.solve(eta=1e-10, time_kernels=True, rebuild=True)
    rc2, st2 = ctx.solve(eta=1e-10, time_kernels=True, time_sampled=True, rebuild=True)
    # graph replay between the sampled iterations: the same counts
    rc3, st3 = ctx.solve(eta=1e-10, time_kernels=True, time_sampled=True, rebuild=True,
                         graph=True)
    assert rc3 == 0 and np.array_equal(ctx.get_homogenized(), H0)
    for key in ("iterations", "kernel_issued", "kernel_launches", "kernel_units"):
        assert st3[key] == st2[key], key
    assert rc0 == rc1 == rc2 == 0
    assert st0["iterations"] == st1["iterations"] == st2["iterations"]
    assert np.array_equal(ctx.get_homogenized(), H0)
    assert sum(st0["kernel_launches"]) == 0 and sum(st0["kernel_issued"]) == 0
    # every launch timed: issued == timed; one operator launch per iteration
    assert st1["kernel_issued"] == st1["kernel_launches"]
    n_op = st1["kernel_issued"][0]
    assert n_op >= max(st1["iterations"])
    # sampled: same launches issued, about an eighth of them timed
    assert st2["kernel_issued"] == st1["kernel_issued"]
    assert st2["kernel_launches"][0] == (n_op + 3) // 8   # loop iterations 4, 12, ...
    for k in range(7):
        if st2["kernel_launches"][k]:
            assert st2["kernel_ms"][k] > 0.0
    # load cases advanced by the timed launches: load j takes part in loop
    # iterations 0 .. iterations[j] - 1 of every pass
    its = st1["iterations"]
    for k in (0, 1, 2, 3, 4, 5):
        assert st1["kernel_units"][k] == sum(its)
        assert st2["kernel_units"][k] == sum((i + 3) // 8 for i in its)
    # the adaptive status poll stops within a few iterations of the last
    # load's convergence
    assert max(its) <= n_op <= max(its) + 3


def test_input_validation(fh):
    """Bad sizes, call order and inputs are rejected with an error code and
    a message before any kernel reads them; the context stays usable."""
    say("input validation")
    ctx = fh.Context(0)

    def rejects(code, fn, *a, **k):
        with pytest.raises(fh.FHError) as e:
            fn(*a, **k)
        assert e.value.code == code, e.value
        return str(e.value)

    for n in [(5, 4, 4), (512, 4, 4), (3, 4, 4), (4, 4, 1), (0, 4, 4)]:
        rejects(fh.FH_EINVAL, ctx.set_grid, n, "elastic", "hex8")
    ctx.set_grid((8, 6, 4), "elastic", "hex8")
    rejects(fh.FH_ESTATE, ctx.solve, eta=1e-8)          # no material, no loads
    mat = np.stack([isotropic_mandel(1.0, 0.3), isotropic_mandel(5.0, 0.3)])
    ph = np.zeros((4, 6, 8), dtype=np.uint8)
    ph[1, 2, 3] = 2                                       # id 2 with 2 tables
    ph_dev = torch.from_numpy(ph).cuda()
    msg = rejects(fh.FH_EINVAL, lambda: (ctx.set_phases(ph_dev, mat), ctx.set_load(np.eye(6)),
                                         ctx.solve(eta=1e-8)))
    assert "phase" in msg
    ph[1, 2, 3] = 1
    ctx.set_phases(torch.from_numpy(ph).cuda(), mat)
    rejects(fh.FH_EINVAL, ctx.set_load, np.zeros((0, 6)))
    rejects(fh.FH_EINVAL, ctx.set_load, np.ones((fh.FH_MAX_LOADS + 1, 6)))
    rejects(fh.FH_EINVAL, ctx.solve, eta=0.0)
    rejects(fh.FH_EINVAL, ctx.solve, eta=1e-8, itmax=0)
    # after the rejections the same context solves normally
    ctx.set_load(np.eye(6))
    rc, st = ctx.solve(eta=1e-8)
    assert rc == 0 and min(st["iterations"]) > 0
    ctx.close()


def test_reference_is_reset_when_the_grid_changes(fh):
    """A 6 x 6 reference set for elasticity must not survive a switch to a
    scalar problem: the next solve uses the 3 x 3 mean conductivity, and
    get_reference returns exactly that 3 x 3 matrix."""
    say("reference reset on set_grid")
    ctx = fh.Context(0)
    ctx.set_grid((8, 6, 4), "elastic", "hex8")
    ctx.set_reference(7.0 * isotropic_mandel(1.0, 0.3))
    ctx.set_grid((8, 6, 4), "scalar", "hex8")
    ph = (np.arange(8 * 6 * 4).reshape(4, 6, 8) % 3 == 0).astype(np.uint8)
    mat = np.stack([np.eye(3), 9.0 * np.eye(3)])
    ctx.set_phases(torch.from_numpy(ph).cuda(), mat)
    ctx.set_load(np.eye(3))
    rc, _ = ctx.solve(eta=1e-10)
    assert rc == 0
    C = ctx.get_reference()
    f = ph.mean()
    assert C.shape == (3, 3)
    assert np.abs(C - ((1 - f) * 1.0 + f * 9.0) * np.eye(3)).max() < 1e-14
    ctx.close()


def test_binding_rejects_bad_tensors(fh):
    """Each device argument is checked for dtype, size and device before the
    library is called: a wrong tensor raises TypeError and the context stays
    usable."""
    say("binding argument checks")
    wl, prob = _spheres_case(8, (1.5, 2.5), 10.0, 3)
    ctx = _ctx(fh, wl)
    N = prob.N
    bad = [
        lambda: ctx.set_phases(torch.zeros(N, dtype=torch.int32, device="cuda"), wl["mat"]),
        lambda: ctx.set_phases(torch.zeros(N - 1, dtype=torch.uint8, device="cuda"), wl["mat"]),
        lambda: ctx.get_fluctuation(0, torch.empty(3 * N - 1, dtype=torch.float64,
                                                   device="cuda")),
        lambda: ctx.get_fluctuation(0, torch.empty(3 * N, dtype=torch.float32, device="cuda")),
        lambda: ctx.apply_operator(torch.zeros(3 * N, dtype=torch.float64, device="cuda"),
                                   torch.empty(N, dtype=torch.float64, device="cuda")),
        lambda: ctx.solve(eta=1e-8, guess_dev=torch.zeros(3 * N, dtype=torch.float64,
                                                          device="cuda")),
        lambda: ctx.get_symbol(torch.empty(10, dtype=torch.float64, device="cuda")),
    ]
    for fn in bad:
        with pytest.raises(TypeError):
            fn()
    kf = Problem((8, 8, 8), "scalar", "hex8", kfield=np.ones((8, 8, 8)))
    ctx2 = fh.Context(0)
    ctx2.set_grid((8, 8, 8), "scalar", "hex8")
    with pytest.raises(TypeError):
        ctx2.set_conductivity_field(torch.ones(kf.N, dtype=torch.float32, device="cuda"))
    ctx2.close()
    rc, _ = ctx.solve(eta=1e-8)
    assert rc == 0
    ctx.close()


def test_conductivity_field_must_be_positive(fh):
    """A zero, negative or infinite voxel conductivity (App. A asks for a
    positive one) is an input error, found before any PCG iteration."""
    say("conductivity field validation")
    n = (8, 6, 4)
    for badv in (0.0, -1.0, np.inf, np.nan):
        k = np.ones(n[::-1])
        k[1, 2, 3] = badv
        ctx = fh.Context(0)
        ctx.set_grid(n, "scalar", "hex8")
        kd = torch.from_numpy(k).cuda()
        ctx.set_conductivity_field(kd)
        ctx.set_load(np.eye(3))
        with pytest.raises(fh.FHError) as e:
            ctx.solve(eta=1e-8)
        assert e.value.code == fh.FH_EINVAL, badv
        ctx.close()


@pytest.mark.parametrize("itmax", [1, 3, 7])
def test_refined_solve_respects_the_iteration_cap(fh, itmax):
    """FP32 refinement counts every inner iteration against it_max (Alg. 1):
    the summed inner iterations never exceed it, and a solve that cannot
    reach eta within it reports not-converged."""
    say("refined itmax", itmax)
    wl, prob = _spheres_case(16, (2.0, 3.5), 100.0, 6)
    ctx = _ctx(fh, wl)
    rc, st = ctx.solve(eta=1e-10, itmax=itmax, precision=fh.FH_FP32_REFINED)
    assert rc == fh.FH_NOT_CONVERGED
    assert max(st["iterations"]) <= itmax, st["iterations"]
    assert all(s == 1 for s in st["status"])
    ctx.close()


@pytest.mark.parametrize("nload", [1, 2, 4, 8])
def test_energy_products_for_any_load_count(fh, nload):
    """nload arbitrary macroscopic strains E (rows): the nload x nload result
    is E C_hom E^T with C_hom from the six unit strains (the energy form is
    bilinear in the loads), for every load count the pair-product kernel is
    specialised to."""
    say("energy products, loads", nload)
    wl, prob = _spheres_case(16, (2.0, 3.5), 50.0, 5)
    ctx = _ctx(fh, wl)
    rc, _ = ctx.solve(eta=1e-12)
    assert rc == 0
    C6 = ctx.get_homogenized()
    E = np.random.default_rng(40 + nload).standard_normal((nload, 6))
    ctx.set_load(E)
    nbytes = ctx.workspace_size()     # more loads than the bound workspace holds
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    ctx.bind_workspace(ws[off:off + nbytes])
    rc, _ = ctx.solve(eta=1e-12)
    assert rc == 0
    assert _rel(ctx.get_homogenized(), E @ C6 @ E.T) < 1e-10


@pytest.mark.parametrize("kind", ["field", "iso"])
@pytest.mark.parametrize("nload", [1, 2, 4, 5])
def test_refined_scalar_solves_for_any_load_count(fh, kind, nload):
    """The FP32 scalar hex8 operator applies the operator to up to three load
    cases per block (one, two or three by the load count; with 4 = 2 + 2 and
    5 = 3 + 2 the last group is partly empty): refined solves of nload
    arbitrary gradients give E C E^T, with C from the FP64 solve of the
    three unit gradients, for a conductivity field and a per-phase table,
    on a grid whose x and y tiles are ragged."""
    say("refined scalar, loads", kind, nload)
    wl, prob = _case("hex8", "scalar", (18, 12, 8), kind=kind, seed=3)
    ctx = _ctx(fh, wl)
    rc, _ = ctx.solve(eta=1e-12)
    assert rc == 0
    C3 = ctx.get_homogenized()
    E = np.random.default_rng(60 + nload).standard_normal((nload, 3))
    ctx.set_load(E)
    nbytes = ctx.workspace_size()
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    ctx.bind_workspace(ws[off:off + nbytes])
    rc, st = ctx.solve(eta=1e-12, precision=fh.FH_FP32_REFINED, eta_inner=1e-4)
    assert rc == 0, st
    assert _rel(ctx.get_homogenized(), E @ C3 @ E.T) < 1e-10
    ctx.close()


def test_breakdown_and_itmax_statuses(fh):
    say("statuses")
    wl, prob = _spheres_case(12, (1.5, 3.0), 100.0, 2)
    ctx = _ctx(fh, wl)
    rc, st = ctx.solve(eta=1e-12, itmax=3)
    assert rc == fh.FH_NOT_CONVERGED and st["status"] == [1] * 6 and st["iterations"] == [3] * 6
    # a negative-definite phase breaks PCG (p.q <= 0) -> FH_ENOTSPD
    bad = dict(wl)
    bad["mat"] = np.stack([wl["mat"][0], -wl["mat"][1]])
    from paper_2203_02962_amd.runner import setup_context
    with pytest.raises(fh.FHError) as e:
        c2 = setup_context(bad, Cref=wl["mat"][0])
        c2.solve(eta=1e-10)
    assert e.value.code == fh.FH_ENOTSPD


def test_full_size_128_matches_stored_oracle(fh):
    """128^3 elasticity at the benchmark's launch configuration (6 loads
    advanced together): C_hom against the oracle's stored result (written by
    tests/golden/make_golden.py, oracle only) and the same iteration counts."""
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "elastic3d_spheres_128_seed0.json")
    g = json.load(open(path))
    wl = workload("elastic3d_spheres", seed=0, n=128)
    assert hashlib.sha256(np.ascontiguousarray(wl["phase"]).tobytes()).hexdigest() == g["phase_sha256"]
    say("solve 128^3 vs stored oracle")
    ctx = _ctx(fh, wl)
    rc, st = ctx.solve(eta=g["eta"])
    assert rc == 0
    H = ctx.get_homogenized()
    Hg = np.array(g["C_hom"])
    assert _rel(H, Hg) < 1e-10
    # both means are exact up to a few roundings (GPU: integer phase counts;
    # oracle: pairwise voxel sum, error ~ eps log N)
    assert _rel(ctx.get_reference(), np.array(g["Cref"])) < 1e-14
    for a, b in zip(st["iterations"], g["iterations"]):
        assert abs(a - b) <= max(1, int(0.01 * b))


REFINED_CASES = [
    ("elastic-spheres-24", lambda: _spheres_case(24, (2.5, 4.5), 100.0, 0)),
    ("scalar-hex8-field-16", lambda: _field_case(16)),
    ("elastic-aniso-random-12x18x24", lambda: _case("hex8", "elastic", (12, 18, 24))),
]


@pytest.mark.parametrize("name,make", REFINED_CASES, ids=[c[0] for c in REFINED_CASES])
def test_fp32_refined_solve_reaches_fp64_accuracy(fh, name, make):
    """FP32 operator/FFT/solve inside FP64 refinement: the outer residual and
    its Kref^-1-norm are FP64, so the refined result meets the same stopping
    rule as the plain solve and C_hom agrees with the oracle to 1e-10."""
    say("fp32 refined", name)
    wl, prob = make()
    ctx = _ctx(fh, wl)
    rc, st = ctx.solve(eta=1e-10, precision=fh.FH_FP32_REFINED, eta_inner=1e-4)
    assert rc == 0, st
    H = ctx.get_homogenized()
    Ho, _, res = oracle.homogenize(prob, wl["loads"], 1e-10)
    assert _rel(H, Ho) < 1e-10
    assert all(o >= 2 for o in st["outer"])            # more than one sweep to 1e-10
    assert all(r <= 1e-10 for r in st["rel_res"])
    # plain FP64 to the same tolerance for reference: same answer
    rc2, st2 = ctx.solve(eta=1e-10)
    assert _rel(ctx.get_homogenized(), H) < 1e-10


def _same_batch(H, sts, rep, H2, sts2, rep2):
    """Two batch calls on the same systems agree: bit for bit when the tuner
    picked the same launch shapes for every group (the shapes set the
    partial-sum blocks of p.q and r.z, hence their rounding), else C_hom to
    1e-10 relative and iterations to +-1."""
    shapes = [(r["n"], r["kz"], r["zb"], r["kyb"], r["xrows"]) for r in rep]
    shapes2 = [(r["n"], r["kz"], r["zb"], r["kyb"], r["xrows"]) for r in rep2]
    if shapes == shapes2:
        assert np.array_equal(H, H2)
        assert [s["iterations"] for s in sts] == [s["iterations"] for s in sts2]
    else:
        assert np.abs(H - H2).max() <= 1e-10 * np.abs(H).max()
        for a, b in zip(sts, sts2):
            assert all(abs(x - y) <= 1 for x, y in zip(a["iterations"], b["iterations"]))


def _batch_systems(specs):
    """specs: list of (n, seed, contrast); isotropic two-phase spheres."""
    out = []
    for n, seed, contrast in specs:
        n3 = n if isinstance(n, tuple) else (n, n, n)
        rng = np.random.default_rng(seed)
        if n3[0] == n3[1] == n3[2]:
            ph, _, _ = spheres(n3[0], (1.5, 3.0), 0.25, seed)
        else:
            ph = (rng.random(n3[::-1]) < 0.3).astype(np.uint8)
        mat = np.stack([isotropic_mandel(1.0, 0.3), isotropic_mandel(contrast, 0.25)])
        out.append((ph, n3, mat))
    return out


def test_batch_takes_its_layouts_from_a_bound_workspace(fh):
    """With a workspace of fh_batch_workspace_size bytes bound to the
    context, the batch groups carve their fields, spectra and K^+ from it:
    the call writes into it and gives the same result as with library-owned
    memory, concurrently and group by group; one byte less is FH_ENOMEM and
    leaves the context usable."""
    say("batch workspace")
    specs = [(16, 1, 10.0), (24, 2, 100.0), (16, 3, 500.0), ((12, 18, 24), 4, 50.0)]
    sysl = _batch_systems(specs)
    ctx = fh.Context(0)
    devs = [(torch.from_numpy(ph).cuda(), n, m) for ph, n, m in sysl]
    E = np.eye(6)[:2]
    rc0, H0, st0, rep0 = ctx.solve_batch(devs, E, eta=1e-8)
    assert rc0 == 0
    need = ctx.batch_workspace_size(devs, 2)
    assert need > 3 * 16 ** 3 * 8 * 2 * 5      # at least x, r, p, q, b of the 16^3 systems
    ws = torch.full((need,), 0x5A, dtype=torch.uint8, device="cuda")
    ctx.bind_workspace(ws)
    for serial in (False, True):
        rc, H, st, rp = ctx.solve_batch(devs, E, eta=1e-8, serial=serial)
        assert rc == 0
        _same_batch(H0, st0, rep0, H, st, rp)
    torch.cuda.synchronize()
    assert int((ws != 0x5A).sum()) > need // 4   # the layouts went there
    small = torch.empty((need - 1,), dtype=torch.uint8, device="cuda")
    ctx.bind_workspace(small)
    with pytest.raises(fh.FHError):
        ctx.solve_batch(devs, E, eta=1e-8)
    ctx.bind_workspace(None)
    rc, H, st, rp = ctx.solve_batch(devs, E, eta=1e-8)
    assert rc == 0
    _same_batch(H0, st0, rep0, H, st, rp)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_batch_matches_single_solves_and_oracle(fh, precision):
    """Systems of three grid sizes (one with radix-3 FFTs, one non-cubic)
    solved in one batch call: every system's C_hom equals its own single
    solve (catches cross-system indexing or races in the batched launches
    and the graph replays) and, for one system, the oracle."""
    say("batch", precision)
    specs = [(16, 1, 10.0), (24, 2, 100.0), (16, 3, 500.0), ((12, 18, 24), 4, 50.0),
             (24, 5, 30.0), (16, 6, 1000.0)]
    sysl = _batch_systems(specs)
    from paper_2203_02962_amd.runner import setup_context
    ctx = fh.Context(0)
    devs = [(torch.from_numpy(ph).cuda(), n, m) for ph, n, m in sysl]
    prec = fh.FH_FP64 if precision == "fp64" else fh.FH_FP32_REFINED
    rc, H, sts, rep = ctx.solve_batch(devs, np.eye(6), eta=1e-10, precision=prec, eta_inner=1e-4)
    assert rc == 0, sts
    assert len(rep) == 3 and sorted(r["nsys"] for r in rep) == [1, 2, 3]
    # the groups ran concurrently; one after another they give the same result
    rc2, H2, sts2, rep2 = ctx.solve_batch(devs, np.eye(6), eta=1e-10, precision=prec,
                                          eta_inner=1e-4, serial=True)
    assert rc2 == 0
    _same_batch(H, sts, rep, H2, sts2, rep2)
    for i, (ph, n, m) in enumerate(sysl):
        wl = dict(dim=3, n=n, problem="elastic", element="hex8", phase=ph, mat=m, loads=np.eye(6))
        c1 = setup_context(wl)
        c1.solve(eta=1e-10)
        assert _rel(H[i], c1.get_homogenized()) < 1e-10, i
    ph, n, m = sysl[1]
    Ho, _, _ = oracle.homogenize(Problem(n, "elastic", "hex8", phase=ph, mat=m), np.eye(6), 1e-10)
    assert _rel(H[1], Ho) < 1e-10
