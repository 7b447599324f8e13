"""Pins of the two-node stencil oracle (oracle/two_node.py, Fig. tiling c.2,
N_n = 2) against what the discretisation and the mathematics fix:

* the closed-form symbol of the unit-conductivity stencil: corner-corner 4,
  centre-centre 4, corner-centre -(1 + e^-i t1)(1 + e^-i t2), Hermitian and
  of rank 1 at xi = 0;
* the Fourier pseudo-inverse equals the dense Moore-Penrose pseudo-inverse of
  the assembled Kref (a genuine rank-deficient block at xi = 0), scalar and
  elastic;
* C = Cref converges in one PCG iteration;
* laminates (interfaces on pixel edges) reach the closed forms, scalar and
  elastic;
* PCG reaches the dense least-squares solution; Voigt/Reuss bounds;
* a homogeneous medium returns the macroscopic field.
"""
import numpy as np
import pytest

from oracle import two_node as tn
from oracle.pcg import pcg
from synth import isotropic_mandel, laminate
from tests.helpers_tensor import random_spd


def _tp(n, problem, seed=0, contrast=10.0, aniso=False):
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, 2, size=n[::-1])
    if problem == "scalar":
        if aniso:
            mats = np.stack([random_spd(2, rng, 3.0), contrast * random_spd(2, rng, 3.0)])
        else:
            mats = np.stack([np.eye(2), contrast * np.eye(2)])
    else:
        if aniso:
            mats = np.stack([random_spd(3, rng, 3.0), contrast * random_spd(3, rng, 3.0)])
        else:
            mats = np.stack([isotropic_mandel(1.0, 0.3, 2), isotropic_mandel(contrast, 0.2, 2)])
    return tn.TwoNodeProblem(n, problem, phase, mats)


def test_scalar_symbol_closed_form():
    n = (6, 4)
    # square pixels (h = 1/4): the closed form below assumes h_x = h_y
    tp = tn.TwoNodeProblem(n, "scalar", np.zeros(n[::-1], dtype=int), np.eye(2)[None],
                           l=(1.5, 1.0))
    K = tn.reference_symbol(tp, np.eye(2))
    t1 = 2 * np.pi * np.arange(n[0]) / n[0]
    t2 = 2 * np.pi * np.arange(n[1]) / n[1]
    T1, T2 = np.meshgrid(t1, t2)             # (ny, nx), x fastest after ravel
    k01 = -(1 + np.exp(-1j * T1)) * (1 + np.exp(-1j * T2))
    assert np.abs(K[:, 0, 0] - 4).max() <= 1e-14
    assert np.abs(K[:, 1, 1] - 4).max() <= 1e-14
    assert np.abs(K[:, 0, 1] - k01.ravel()).max() <= 1e-14
    assert np.abs(K[:, 1, 0] - np.conj(k01.ravel())).max() <= 1e-14
    lam = np.linalg.eigvalsh(K[0])
    assert abs(lam[0]) <= 1e-14 and abs(lam[1] - 8) <= 1e-14


@pytest.mark.parametrize("problem,aniso", [("scalar", False), ("scalar", True),
                                           ("elastic", False), ("elastic", True)])
def test_fourier_pseudo_inverse_is_dense_pseudo_inverse(problem, aniso):
    n = (4, 4) if problem == "scalar" else (4, 2)
    tp = _tp(n, problem, seed=3, aniso=aniso)
    Cref = tn.mean_material(tp)
    M = tn.TwoNodePreconditioner(tp, Cref)
    Kref = tn.assemble(tp, Cref).toarray()
    P = np.linalg.pinv(Kref, rcond=1e-10, hermitian=True)
    # the null space has dimension nd (constants of each component)
    s = np.linalg.svd(Kref, compute_uv=False)
    assert (s <= 1e-10 * s.max()).sum() == tp.nd
    rng = np.random.default_rng(4)
    for _ in range(3):
        r = rng.normal(size=Kref.shape[0])
        assert np.abs(M.apply(r) - P @ r).max() <= 1e-12 * np.abs(P @ r).max()


@pytest.mark.parametrize("problem", ["scalar", "elastic"])
def test_reference_equals_material_converges_in_one_iteration(problem):
    n = (6, 4)
    tp = _tp(n, problem, seed=5, aniso=True)
    tp.phase = np.zeros_like(tp.phase)
    C = tp.mat[0]
    K = tn.assemble(tp)
    M = tn.TwoNodePreconditioner(tp, C)
    rng = np.random.default_rng(6)
    b = K @ rng.normal(size=K.shape[0])
    r = pcg(lambda v: K @ v, M.apply, b, 1e-12)
    assert r.iterations == 1


def _laminate_2d_elastic(Cs, normal):
    """Laminate formula in 2D Mandel (11, 22, 12): traction components
    (n-set) continuous, tangential strains (p-set) continuous."""
    nset = [0, 2] if normal == 0 else [1, 2]
    pset = [1] if normal == 0 else [0]
    inv_nn = [np.linalg.inv(C[np.ix_(nset, nset)]) for C in Cs]
    Hnn = np.linalg.inv(np.mean(inv_nn, axis=0))
    A = np.mean([iv @ C[np.ix_(nset, pset)] for iv, C in zip(inv_nn, Cs)], axis=0)
    Bm = np.mean([C[np.ix_(pset, nset)] @ iv for iv, C in zip(inv_nn, Cs)], axis=0)
    Hpp = (np.mean([C[np.ix_(pset, pset)] - C[np.ix_(pset, nset)] @ iv @ C[np.ix_(nset, pset)]
                    for iv, C in zip(inv_nn, Cs)], axis=0) + Bm @ Hnn @ A)
    H = np.zeros((3, 3))
    H[np.ix_(nset, nset)] = Hnn
    H[np.ix_(nset, pset)] = Hnn @ A
    H[np.ix_(pset, nset)] = (Hnn @ A).T
    H[np.ix_(pset, pset)] = Hpp
    return H


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("problem", ["scalar", "elastic"])
def test_laminate_closed_form(problem, axis):
    n = (6, 4)
    rng = np.random.default_rng(7 + axis)
    layers = rng.integers(0, 2, size=n[axis])
    layers[0], layers[-1] = 0, 1
    phase = laminate(n, axis, layers)
    if problem == "scalar":
        mats = np.stack([np.eye(2), 23.0 * np.eye(2)])
    else:
        mats = np.stack([random_spd(3, rng, 4.0), 30.0 * random_spd(3, rng, 4.0)])
    tp = tn.TwoNodeProblem(n, problem, phase, mats)
    H, _, _ = tn.homogenize(tp, np.eye(tp.m), 1e-13)
    if problem == "scalar":
        kl = np.array([[1.0, 23.0][v] for v in layers])
        ref = np.mean(kl) * np.eye(2)
        ref[axis, axis] = 1.0 / np.mean(1.0 / kl)
    else:
        ref = _laminate_2d_elastic([mats[v] for v in layers], axis)
    assert np.abs(H - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("problem", ["scalar", "elastic"])
def test_pcg_matches_dense_least_squares_and_bounds(problem):
    n = (4, 4)
    tp = _tp(n, problem, seed=9, contrast=15.0)
    H, sols, res = tn.homogenize(tp, np.eye(tp.m), 1e-13)
    K = tn.assemble(tp).toarray()
    for E, u in zip(np.eye(tp.m), sols):
        ud = np.linalg.lstsq(K, tn.rhs(tp, E), rcond=1e-12)[0]
        # both are the minimum-norm representative (zero mean per component)
        assert np.abs(u - ud).max() <= 1e-10 * np.abs(ud).max()
    assert np.abs(H - H.T).max() <= 1e-13 * np.abs(H).max()
    C = tp.mat[np.asarray(tp.phase).ravel()]
    voigt = C.mean(axis=0)
    reuss = np.linalg.inv(np.linalg.inv(C).mean(axis=0))
    assert np.linalg.eigvalsh(voigt - H).min() >= -1e-12 * np.abs(H).max()
    assert np.linalg.eigvalsh(H - reuss).min() >= -1e-12 * np.abs(H).max()


def test_homogeneous_medium_returns_macroscopic_field():
    n = (6, 4)
    C0 = isotropic_mandel(3.0, 0.25, 2)
    tp = tn.TwoNodeProblem(n, "elastic", np.zeros(n[::-1], dtype=int), C0[None])
    scale = np.abs(C0).max() * tp.h.max()
    for E in np.eye(3):
        # equal element forces cancel at every node up to rounding
        assert np.abs(tn.rhs(tp, E)).max() <= 1e-15 * scale
    H, sols, res = tn.homogenize(tp, np.eye(3), 1e-10)
    assert all(np.abs(u).max() <= 1e-13 for u in sols)
    assert np.abs(H - C0).max() <= 1e-14 * np.abs(C0).max()
