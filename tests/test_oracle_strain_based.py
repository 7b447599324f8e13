"""Pins of the strain-based scheme oracle (oracle/strain_based.py, Sec. 7.1)
against what the algebra and the paper's equivalence statement fix:

* Gamma0 Cref leaves compatible fields D u unchanged and is a projection;
* with Cref = I, Gamma0 tau is the weighted least-squares compatible part of
  tau (dense lstsq on a 3x3x3 grid);
* Gamma0 C is self-adjoint on compatible fields in the Cref-weighted inner
  product;
* CG on the strain unknown produces eps_k = D u_k for the displacement-based
  PCG iterates u_k, with the same residual history and iteration count
  (the equivalence of Sec. 7.1), and the same homogenized tensor;
* a homogeneous medium returns the macroscopic strain (zero fluctuation).
"""
import numpy as np
import pytest

import oracle
from oracle import strain_based as osb
from oracle.assembly import Problem, assemble_stiffness, gradient_at_quadrature, rhs
from oracle.pcg import pcg
from oracle.precond import Preconditioner
from synth import isotropic_mandel
from tests.helpers_tensor import random_spd


def _prob(n=(4, 3, 3), seed=0, aniso=False):
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    if aniso:
        mat = np.stack([random_spd(6, rng, 10.0), 20.0 * random_spd(6, rng, 10.0)])
    else:
        mat = np.stack([isotropic_mandel(1.0, 0.3), isotropic_mandel(30.0, 0.2)])
    return Problem(n, "elastic", "hex8", phase=phase, mat=mat)


def _field(prob, rng):
    return rng.normal(size=(prob.N, 8, 6))


@pytest.mark.parametrize("aniso", [False, True])
def test_green_operator_projects_onto_compatible_fields(aniso):
    prob = _prob(aniso=aniso, seed=1)
    rng = np.random.default_rng(2)
    Cref = oracle.mean_material(prob)
    G = osb.GreenOperator(prob, Cref)
    u = rng.normal(size=3 * prob.N)
    Du = gradient_at_quadrature(prob, u)
    GCref = lambda t: G.apply(np.einsum("mn,eqn->eqm", Cref, t))
    assert np.abs(GCref(Du) - Du).max() <= 1e-12 * np.abs(Du).max()
    tau = _field(prob, rng)
    once = GCref(tau)
    assert np.abs(GCref(once) - once).max() <= 1e-12 * np.abs(once).max()


def test_identity_reference_gives_least_squares_compatible_part():
    prob = _prob((3, 3, 3), seed=3)
    rng = np.random.default_rng(4)
    tau = _field(prob, rng)
    G = osb.GreenOperator(prob, np.eye(6))
    got = G.apply(tau)
    # dense D (rows (e, q, m)) and weights, least squares in the W-norm
    D = np.zeros((prob.N * 8 * 6, 3 * prob.N))
    for j in range(3 * prob.N):
        v = np.zeros(3 * prob.N)
        v[j] = 1.0
        D[:, j] = gradient_at_quadrature(prob, v).ravel()
    w = np.repeat(np.tile(prob.el.wfrac * prob.voxel_volume, prob.N), 6)
    sw = np.sqrt(w)
    u = np.linalg.lstsq(D * sw[:, None], tau.ravel() * sw, rcond=1e-12)[0]
    want = (D @ u).reshape(tau.shape)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_gamma_C_is_self_adjoint_on_compatible_fields():
    prob = _prob(seed=5, aniso=True)
    rng = np.random.default_rng(6)
    Cref = oracle.mean_material(prob)
    G = osb.GreenOperator(prob, Cref)
    Cv = prob.voxel_materials()
    C = lambda t: np.einsum("emn,eqn->eqm", Cv, t)
    a = gradient_at_quadrature(prob, rng.normal(size=3 * prob.N))
    b = gradient_at_quadrature(prob, rng.normal(size=3 * prob.N))
    lhs = osb.inner(prob, Cref, G.apply(C(a)), b)
    rhs_ = osb.inner(prob, Cref, a, G.apply(C(b)))
    assert abs(lhs - rhs_) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("aniso", [False, True])
def test_strain_iterates_equal_gradients_of_displacement_iterates(aniso):
    """Sec. 7.1: eps_k = D u_k for every k, same history and count."""
    prob = _prob((6, 4, 4), seed=7, aniso=aniso)
    Cref = oracle.mean_material(prob)
    E = np.array([0.3, -0.2, 0.1, 0.4, -0.1, 0.25])
    K = assemble_stiffness(prob)
    M = Preconditioner(prob, Cref)
    db_iters = []
    res = pcg(lambda v: K @ v, M.apply, rhs(prob, E), 1e-10, nd=3,
              callback=db_iters.append)
    sb = osb.cg_strain(prob, Cref, E, 1e-10, keep_iterates=True)
    assert sb.iterations == res.iterations
    assert np.abs(np.array(sb.history) - np.array(res.history)).max() <= 1e-9
    for uk, ek in zip(db_iters, sb.iterates):
        Du = gradient_at_quadrature(prob, uk)
        assert np.abs(ek - Du).max() <= 1e-9 * np.abs(Du).max()


def test_strain_based_homogenized_tensor_matches_displacement_based():
    prob = _prob((6, 4, 4), seed=8)
    Cref = oracle.mean_material(prob)
    loads = np.eye(6)
    H_db, _, _ = oracle.homogenize(prob, loads, 1e-12)
    eps = [osb.cg_strain(prob, Cref, E, 1e-12).eps for E in loads]
    H_sb = osb.homogenized_from_strain(prob, loads, eps)
    assert np.abs(H_sb - H_db).max() <= 1e-12 * np.abs(H_db).max()


def test_homogeneous_medium_returns_the_macroscopic_strain():
    """The right-hand side -Gamma0 C e vanishes up to the rounding of the
    nodal sums of equal element forces: the fluctuation is zero to rounding
    and C_hom = C0."""
    n = (4, 4, 4)
    C0 = isotropic_mandel(5.0, 0.25)
    prob = Problem(n, "elastic", "hex8", phase=np.zeros(n[::-1], dtype=np.uint8), mat=C0[None])
    loads = np.eye(6)
    eps = []
    for E in loads:
        r = osb.cg_strain(prob, C0, E, 1e-10)
        assert r.iterations <= 1 and np.abs(r.eps).max() <= 1e-25
        eps.append(r.eps)
    H = osb.homogenized_from_strain(prob, loads, eps)
    assert np.abs(H - C0).max() <= 1e-14 * np.abs(C0).max()
