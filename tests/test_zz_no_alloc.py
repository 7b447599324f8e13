"""GPU test of the no-allocation variant of the right-hand-side entry point:
fh_compute_rhs_noalloc stages the element-force tables in a static device
array instead of a hipMalloc'ed buffer.  Called through the C-ABI, it must
give exactly what fh_compute_rhs gives (same kernel, same tables), on two
calls in a row where the second input is smaller (fewer material tables,
smaller grid), so stale entries of the first call would show."""
import sys

import numpy as np
import pytest

from oracle.assembly import Problem, rhs
from synth import isotropic_mandel
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


def _case(n, problem, mats, seed):
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, len(mats), size=n[::-1]).astype(np.uint8)
    return phase, np.stack(mats)


def test_noalloc_rhs_matches_allocating_rhs_twice(fh):
    big = _case((16, 12, 8), "elastic",
                [isotropic_mandel(1.0, 0.3), isotropic_mandel(20.0, 0.25),
                 random_spd(6, np.random.default_rng(3))], 1)
    small = _case((6, 4, 4), "scalar", [np.eye(3), 7.0 * np.eye(3)], 2)
    E_big = np.array([0.3, -0.2, 0.1, 0.5, -0.4, 0.25])
    E_small = np.array([1.0, -0.5, 0.2])
    ctx = fh.Context(0)
    for (phase, mats), problem, E in ((big, "elastic", E_big), (small, "scalar", E_small)):
        n = phase.shape[::-1]
        say("no-alloc rhs", problem, n, "tables", len(mats))
        ctx.set_grid(n, problem, "hex8")
        ph = torch.from_numpy(phase).cuda()
        ctx.set_phases(ph, mats)
        F = ctx.nd * ctx.N
        b_ref = torch.full((F,), np.nan, dtype=torch.float64, device="cuda")
        b_new = torch.full((F,), np.nan, dtype=torch.float64, device="cuda")
        ctx.compute_rhs(E, b_ref)
        ctx.compute_rhs_noalloc(E, b_new)
        a, b = b_ref.cpu().numpy(), b_new.cpu().numpy()
        assert np.array_equal(a, b), np.abs(a - b).max()
        prob = Problem(tuple(n), problem, "hex8", phase=phase, mat=mats)
        bo = rhs(prob, E)
        assert np.abs(b - bo).max() <= 1e-12 * np.abs(bo).max()
    ctx.close()
