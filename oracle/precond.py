"""Reference-material preconditioner (TEST INFRASTRUCTURE ONLY).

Paper Sec. 4.1-4.2 (eqs. Kref, M, M_inverse), Sec. 5.2 (Alg. 2) and Sec. 5.3
(eq. block_inversion):

  * Kref = D^T W Cref D is assembled (assembly.assemble_stiffness);
  * applying Kref to the unit impulse of component beta at node 0 gives one
    column of every block K_ab; the DFT of block alpha of that column is the
    diagonal of K^_ab (Alg. 2);
  * per frequency the d_n x d_n block K^(xi) is pseudo-inverted; the
    zero-frequency block is singular (rigid-body modes) and gets the
    Moore-Penrose pseudo-inverse, the others the inverse (Sec. 5.3);
  * M^+ r = F^H K^+ F r (eq. M_inverse), with the DFT of naive_dft.py.

Reading (stated): the pseudo-inverse is computed from the Hermitian
eigen-decomposition of each block, eigenvalues at or below 1e-10 times the
largest eigenvalue over all frequencies being treated as zero.  For the
one-node stencils used here the whole zero-frequency block vanishes, so its
pseudo-inverse is the zero matrix.
"""
from __future__ import annotations

import numpy as np

from .assembly import Problem, assemble_stiffness
from .naive_dft import dft, idft


def reference_symbol(prob: Problem, Cref: np.ndarray) -> np.ndarray:
    """(N, nd, nd) complex K^(xi) by Alg. 2 (frequencies in numpy grid
    order, flattened x fastest)."""
    Kref = assemble_stiffness(prob, uniform=Cref)
    nd, N = prob.ndof_node, prob.N
    Khat = np.zeros((N, nd, nd), dtype=complex)
    for beta in range(nd):
        impulse = np.zeros(nd * N)
        impulse[beta * N] = 1.0
        col = Kref @ impulse
        for alpha in range(nd):
            blk = col[alpha * N:(alpha + 1) * N].reshape(prob.grid_shape)
            Khat[:, alpha, beta] = dft(blk).ravel()
    return Khat


def pseudo_inverse_blocks(Khat: np.ndarray, rtol: float = 1e-10) -> np.ndarray:
    """Moore-Penrose pseudo-inverse of every Hermitian block (eq.
    block_inversion; Alg. 2 pseudo-inverse of the singular block)."""
    lam, V = np.linalg.eigh(Khat)
    tol = rtol * np.max(np.abs(lam))
    inv = np.where(np.abs(lam) > tol, 1.0 / np.where(lam == 0, 1.0, lam), 0.0)
    return np.einsum("fik,fk,fjk->fij", V, inv, V.conj())


class Preconditioner:
    """z = M^+ r = F_d^H K^+ F_d r (eq. M_inverse)."""

    def __init__(self, prob: Problem, Cref: np.ndarray, Khat: np.ndarray | None = None):
        self.prob = prob
        self.Khat = reference_symbol(prob, Cref) if Khat is None else Khat
        self.Kplus = pseudo_inverse_blocks(self.Khat)

    def apply(self, r: np.ndarray) -> np.ndarray:
        prob = self.prob
        nd, N = prob.ndof_node, prob.N
        R = np.stack([dft(r[a * N:(a + 1) * N].reshape(prob.grid_shape)).ravel()
                      for a in range(nd)], axis=1)          # (N, nd)
        Z = np.einsum("fab,fb->fa", self.Kplus, R)
        z = np.concatenate([np.real(idft(Z[:, a].reshape(prob.grid_shape))).ravel()
                            for a in range(nd)])
        return z
