"""Strain-based scheme with the finite-element projection (TEST
INFRASTRUCTURE ONLY).

Paper Sec. 7.1 (eq. projection_chceme): multiplying the preconditioned
displacement-based system Kref^-1 K du = Kref^-1 b (eq. precondit_chceme) by
D from the left and taking the gradient field eps = D u as the unknown gives

    Gamma0 C d_eps = -Gamma0 sigma,   Gamma0 = D (D^T W Cref D)^+ D^T W,

with Gamma0 the discrete periodic Green operator of the FE discretisation
(for one-point triangles all weights are equal and W drops out, as the
paper notes; with W kept the same algebra holds for any quadrature rule).
Gamma0 maps a quadrature-point field onto the compatible fields D u; with
Cref = I_s it is the W-orthogonal projection (the least-squares compatible
part of a field).

The paper states that the two schemes generate the same iterates in exact
arithmetic: CG on the strain unknown, applied to Gamma0 C, produces
eps_k = D u_k for the PCG iterates u_k of the displacement scheme, when the
stopping criteria correspond.  Reading (stated): CG runs in the inner
product <a, b> = sum_Q w_Q a_Q^T Cref b_Q, in which Gamma0 C is self-
adjoint on compatible fields; the residual r^SB = D z^DB then has
<r^SB, r^SB> = r^DB . z^DB, so the strain-based stopping test on
sqrt(<r, r> / <r0, r0>) is the displacement-based test of Sec. 6.

Linear material only (C constant per voxel): sigma = C (e + eps).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .assembly import Problem, gradient_at_quadrature, quadrature_weights
from .plasticity import element_forces_to_nodes
from .assembly import B_matrices
from .precond import Preconditioner


def divergence(prob: Problem, tau: np.ndarray) -> np.ndarray:
    """D^T W tau for a quadrature-point field tau (N, nq, m)."""
    B = B_matrices(prob)
    w = quadrature_weights(prob)
    fe = np.einsum("q,qmi,eqm->ei", w, B, tau)
    return element_forces_to_nodes(prob, fe)


class GreenOperator:
    """Gamma0 tau = D Kref^+ D^T W tau (eq. projection_chceme), Kref^+ through
    the oracle's DFT pseudo-inverse (zero-frequency block pseudo-inverted)."""

    def __init__(self, prob: Problem, Cref: np.ndarray):
        self.prob = prob
        self.Cref = np.asarray(Cref, dtype=float)
        self.M = Preconditioner(prob, self.Cref)

    def apply(self, tau: np.ndarray) -> np.ndarray:
        return gradient_at_quadrature(self.prob, self.M.apply(divergence(self.prob, tau)))


def inner(prob: Problem, Cref: np.ndarray, a: np.ndarray, b: np.ndarray) -> float:
    """<a, b> = sum_Q w_Q a_Q^T Cref b_Q."""
    w = quadrature_weights(prob)
    return float(np.einsum("q,eqm,mn,eqn->", w, a, Cref, b))


@dataclass
class SBResult:
    eps: np.ndarray            # (N, nq, m) strain fluctuation D u
    iterations: int
    history: list = field(default_factory=list)   # sqrt(rho_k / rho_0)
    iterates: list = field(default_factory=list)  # eps_k (only if kept)


def cg_strain(prob: Problem, Cref: np.ndarray, E: np.ndarray, eta: float,
              itmax: int = 10000, keep_iterates: bool = False) -> SBResult:
    """CG on Gamma0 C eps = -Gamma0 C e from eps_0 = 0 in the inner product
    <., .> (linear material)."""
    G = GreenOperator(prob, Cref)
    Cv = prob.voxel_materials()                            # (N, m, m)
    E = np.asarray(E, dtype=float)

    def C_apply(t):
        return np.einsum("emn,eqn->eqm", Cv, t)

    nq = len(prob.el.wfrac)
    x = np.zeros((prob.N, nq, prob.nstrain))
    r = -G.apply(C_apply(np.broadcast_to(E, x.shape)))
    p = r.copy()
    rho = inner(prob, Cref, r, r)
    res = SBResult(x, 0)
    if rho == 0.0:
        return res
    rho0 = rho
    for k in range(1, itmax + 1):
        q = G.apply(C_apply(p))
        alpha = rho / inner(prob, Cref, p, q)
        x = x + alpha * p
        r = r - alpha * q
        rho_new = inner(prob, Cref, r, r)
        res.history.append(np.sqrt(max(rho_new, 0.0) / rho0))
        res.iterations = k
        if keep_iterates:
            res.iterates.append(x.copy())
        if rho_new <= eta * eta * rho0:
            break
        p = r + (rho_new / rho) * p
        rho = rho_new
    res.eps = x
    return res


def homogenized_from_strain(prob: Problem, loads: np.ndarray, eps_list) -> np.ndarray:
    """C_hom[i, j] = (1/|Y|) sum_Q w_Q (e_i + eps_i)^T C (e_j + eps_j)."""
    w = quadrature_weights(prob)
    Cv = prob.voxel_materials()
    tot = [e + np.asarray(E)[None, None, :] for e, E in zip(eps_list, loads)]
    nl = len(loads)
    H = np.zeros((nl, nl))
    for j in range(nl):
        s = np.einsum("emn,eqn->eqm", Cv, tot[j])
        for i in range(nl):
            H[i, j] = np.einsum("q,eqm,eqm->", w, tot[i], s) / prob.volume
    return H
