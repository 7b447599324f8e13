"""Homogenized tensor (TEST INFRASTRUCTURE ONLY).

The paper imposes the macroscopic strain/gradient e through the split
eps = e + D u (Sec. 2, App. A) and takes the reference material as the
quadrature-weighted mean (Sec. 6.2).  It does not print a formula for the
homogenized tensor; reading (stated): the energy (bilinear) form

    C_hom[i, j] = (1/|Y|) sum_Q w_Q (e_i + D u_i)_Q^T C_Q (e_j + D u_j)_Q,

where u_j solves K u_j = b_j = -D^T W C e_j for the unit load e_j.  Its
error is quadratic in the solver error.  The stress average
<C (e_j + D u_j)> is provided as a diagnostic.
"""
from __future__ import annotations

import numpy as np

from .assembly import Problem, assemble_stiffness, gradient_at_quadrature, quadrature_weights, rhs
from .pcg import pcg
from .precond import Preconditioner


def mean_material(prob: Problem) -> np.ndarray:
    """Cref_mean = (1/|Y|) sum_Q C(x_Q) w_Q (Sec. 6.2).

    The voxel sum runs along a contiguous axis, where numpy sums pairwise
    (error ~ eps log N); a sum down the first axis of the (N, m, m) stack
    would add one voxel at a time, and for grids of two materials that
    rounding is systematic (about N eps, 1.5e-11 relative at 128^3)."""
    w = quadrature_weights(prob)
    C = prob.voxel_materials()
    m = C.shape[1]
    total = np.ascontiguousarray(C.reshape(prob.N, m * m).T).sum(axis=1).reshape(m, m)
    return total * w.sum() / prob.volume


def homogenized_energy(prob: Problem, loads: np.ndarray, sols) -> np.ndarray:
    w = quadrature_weights(prob)
    C = prob.voxel_materials()           # (N, m, m)
    eps = [gradient_at_quadrature(prob, u) + np.asarray(E)[None, None, :]
           for u, E in zip(sols, loads)]  # each (N, nq, m)
    nl = len(loads)
    H = np.zeros((nl, nl))
    for j in range(nl):
        sig = np.einsum("emn,eqn->eqm", C, eps[j])
        for i in range(nl):
            H[i, j] = np.einsum("q,eqm,eqm->", w, eps[i], sig) / prob.volume
    return H


def stress_average(prob: Problem, E: np.ndarray, u: np.ndarray) -> np.ndarray:
    w = quadrature_weights(prob)
    C = prob.voxel_materials()
    eps = gradient_at_quadrature(prob, u) + np.asarray(E)[None, None, :]
    sig = np.einsum("emn,eqn->eqm", C, eps)
    return np.einsum("q,eqm->m", w, sig) / prob.volume


def homogenize(prob: Problem, loads: np.ndarray, eta: float = 1e-10,
               Cref: np.ndarray | None = None, itmax: int = 10000,
               K=None, M: Preconditioner | None = None):
    """Solve every load case with PCG and return (C_hom, solutions, results)."""
    loads = np.atleast_2d(np.asarray(loads, dtype=float))
    if Cref is None:
        Cref = mean_material(prob)
    if K is None:
        K = assemble_stiffness(prob)
    if M is None:
        M = Preconditioner(prob, Cref)
    sols, results = [], []
    for E in loads:
        b = rhs(prob, E)
        res = pcg(lambda v: K @ v, M.apply, b, eta, itmax, nd=prob.ndof_node)
        sols.append(res.x)
        results.append(res)
    return homogenized_energy(prob, loads, sols), sols, results
