"""GPU parity of the two-node stencil (Fig. tiling c.2, N_n = 2, scalar)
through the C-ABI against oracle/two_node.py (pinned in
tests/test_oracle_two_node.py): operator, right-hand side, Hermitian symbol
with the rank-one zero-frequency pseudo-inverse, preconditioner, full solves
(C_hom, iterations, fluctuations) and the laminate closed form.

Tolerances as for the one-node stencils: step-level results to 1e-12 of the
largest entry, C_hom to 1e-10 relative, iterations +-max(1, 1 %),
fluctuations to 1e-8 relative in l2 at eta = 1e-10.
"""
import sys

import numpy as np
import pytest

from oracle import two_node as tn
from synth import circles2d, laminate
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


def _case(kind, n, seed=0, l=(1.0, 1.0)):
    """(workload dict for the library, oracle problem)."""
    rng = np.random.default_rng(seed)
    wl = dict(dim=2, n=tuple(n) + (1,), problem="scalar", element="tri4", loads=np.eye(2), l=l)
    if kind == "field":
        k = np.exp(rng.uniform(-2, 2, size=n[::-1]))
        wl["kfield"] = k
        # the oracle takes a conductivity field as one phase per pixel
        tp = tn.TwoNodeProblem(n, "scalar", np.arange(k.size).reshape(k.shape),
                               k.ravel()[:, None, None] * np.eye(2)[None], l=l)
    else:
        phase = rng.integers(0, 3, size=n[::-1]).astype(np.uint8)
        if kind == "aniso":
            mats = np.stack([random_spd(2, rng, 4.0) * (1 + 10 * p) for p in range(3)])
        else:
            mats = np.stack([(1.0 + 20 * p) * np.eye(2) for p in range(3)])
        wl["phase"], wl["mat"] = phase, mats
        tp = tn.TwoNodeProblem(n, "scalar", phase, mats, l=l)
    return wl, tp


def _ctx(wl):
    from paper_2203_02962_amd.runner import setup_context
    return setup_context(wl)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = [("iso", (12, 8), (1.0, 1.0)), ("aniso", (16, 18), (1.0, 0.7)),
         ("field", (12, 18), (1.0, 1.0)), ("iso", (6, 4), (1.0, 1.0))]


@pytest.mark.parametrize("kind,n,l", CASES)
def test_steps_match_oracle(fh, kind, n, l):
    say("two-node steps", kind, n)
    wl, tp = _case(kind, n, seed=1, l=l)
    ctx = _ctx(wl)
    F = 2 * tp.N
    rng = np.random.default_rng(2)
    u = rng.standard_normal(F)
    ud = torch.from_numpy(u).cuda()
    qd = torch.empty_like(ud)
    ctx.apply_operator(ud, qd)
    assert _rel(qd.cpu().numpy(), tn.assemble(tp) @ u) < 1e-12
    E = rng.standard_normal(2)
    bd = torch.empty(F, dtype=torch.float64, device="cuda")
    ctx.compute_rhs(E, bd)
    assert _rel(bd.cpu().numpy(), tn.rhs(tp, E)) < 1e-12
    # symbol: {k00, k11, Re k01, Im k01} of K^+ / N on the half spectrum
    Cref = tn.mean_material(tp)
    M = tn.TwoNodePreconditioner(tp, Cref)
    kd = torch.empty(ctx.symbol_size(), dtype=torch.float64, device="cuda")
    ctx.get_symbol(kd)
    nx, ny = n
    nxh = nx // 2 + 1
    K = M.Kplus.reshape(ny, nx, 2, 2)[:, :nxh] / tp.N       # [ky][kx]
    K = np.transpose(K, (1, 0, 2, 3))                         # [kx][ky]
    want = np.stack([K[..., 0, 0].real, K[..., 1, 1].real, K[..., 0, 1].real, K[..., 0, 1].imag])
    got = kd.cpu().numpy().reshape(4, nxh, ny)
    assert _rel(got, want) < 1e-12
    # the zero-frequency block is the rank-one pseudo-inverse, not zero
    assert np.abs(got[:, 0, 0]).max() > 0
    r = rng.standard_normal(F)
    rd = torch.from_numpy(r).cuda()
    zd = torch.empty_like(rd)
    ctx.apply_preconditioner(rd, zd)
    assert _rel(zd.cpu().numpy(), M.apply(r)) < 1e-12
    ctx.close()


@pytest.mark.parametrize("kind,n,l", CASES[:3])
def test_solve_matches_oracle(fh, kind, n, l):
    say("two-node solve", kind, n)
    wl, tp = _case(kind, n, seed=3, l=l)
    ctx = _ctx(wl)
    rc, st = ctx.solve(eta=1e-10)
    assert rc == 0, st
    H = ctx.get_homogenized()
    Ho, uo, res = tn.homogenize(tp, np.eye(2), 1e-10)
    assert _rel(H, Ho) < 1e-10
    for j in range(2):
        assert abs(st["iterations"][j] - res[j].iterations) <= max(1, 0.01 * res[j].iterations)
        u = torch.empty(2 * tp.N, dtype=torch.float64, device="cuda")
        ctx.get_fluctuation(j, u)
        u = u.cpu().numpy()
        assert np.linalg.norm(u - uo[j]) <= 1e-8 * np.linalg.norm(uo[j])
    ctx.close()


@pytest.mark.parametrize("axis", [0, 1])
def test_laminate_closed_form(fh, axis):
    n = (12, 18)
    rng = np.random.default_rng(9 + axis)
    layers = rng.integers(0, 2, size=n[axis])
    layers[0], layers[-1] = 0, 1
    phase = laminate(n, axis, layers).astype(np.uint8)
    mats = np.stack([np.eye(2), 37.0 * np.eye(2)])
    wl = dict(dim=2, n=n + (1,), problem="scalar", element="tri4", loads=np.eye(2),
              phase=phase, mat=mats)
    ctx = _ctx(wl)
    rc, st = ctx.solve(eta=1e-12)
    assert rc == 0
    H = ctx.get_homogenized()
    kl = np.array([[1.0, 37.0][v] for v in layers])
    ref = np.mean(kl) * np.eye(2)
    ref[axis, axis] = 1.0 / np.mean(1.0 / kl)
    assert np.abs(H - ref).max() <= 1e-10 * np.abs(ref).max()
    ctx.close()


def test_circles_workload_iterations(fh):
    """The paper's thermal setting (Sec. 6.1, where it compares the
    stencils) on the 32^2 circles workload with the two-node stencil:
    C_hom and the iteration counts match the oracle."""
    phase = circles2d(32, 8, (3.0, 6.0), seed=0)
    mats = np.stack([np.eye(2), 10.0 * np.eye(2)])
    wl = dict(dim=2, n=(32, 32, 1), problem="scalar", element="tri4", loads=np.eye(2),
              phase=phase.astype(np.uint8), mat=mats)
    ctx = _ctx(wl)
    rc, st = ctx.solve(eta=1e-10)
    assert rc == 0
    H = ctx.get_homogenized()
    tp = tn.TwoNodeProblem((32, 32), "scalar", phase, mats)
    Ho, _, res = tn.homogenize(tp, np.eye(2), 1e-10)
    say("32^2 circles iterations", st["iterations"], [r.iterations for r in res])
    assert _rel(H, Ho) < 1e-10
    for j in range(2):
        assert abs(st["iterations"][j] - res[j].iterations) <= max(1, 0.01 * res[j].iterations)
    ctx.close()


def test_two_node_rejections(fh):
    ctx = fh.Context(0)
    with pytest.raises(fh.FHError):
        ctx.set_grid((8, 8), "elastic", "tri4")
    ctx.close()
    wl, tp = _case("iso", (6, 4), seed=4)
    ctx = _ctx(wl)
    with pytest.raises(fh.FHError):
        ctx.eigen_bounds()
    ctx.close()
