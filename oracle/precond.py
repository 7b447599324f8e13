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

from .assembly import Problem, assemble_stiffness, operator_rows
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


def _uniform_problem(prob: Problem, Cref: np.ndarray) -> Problem:
    """The same grid and stencil with the uniform reference material."""
    return Problem(prob.n, prob.problem, prob.elem,
                   phase=np.zeros(prob.grid_shape, dtype=np.int64),
                   mat=np.asarray(Cref, dtype=float)[None], l=prob.l)


def stencil_symbol(prob: Problem, Cref: np.ndarray) -> np.ndarray:
    """(N, nd, nd) complex K^(xi) by Alg. 2 for grids too large to assemble.

    The response of Kref to the unit impulse of component beta at node 0 is
    nonzero only at the nodes that share a pixel with node 0 (offsets in
    {-1, 0, 1}^d); those rows come from assembly.operator_rows with the
    uniform Cref.  The DFT of that column (naive_dft's convention) is then
    the sum over those nodes J of col[J] exp(-2 pi i sum_k xi_k J_k / n_k),
    evaluated at every frequency.  Same ordering as reference_symbol."""
    ref = _uniform_problem(prob, Cref)
    nd, N, dim = prob.ndof_node, prob.N, prob.dim
    n = np.array(prob.n)
    offs = np.array(list(np.ndindex(*(3,) * dim))) - 1          # (3^d, dim), x first
    coords = np.unique(offs % n[None, :], axis=0)                # distinct nodes
    flat = np.zeros(len(coords), dtype=np.int64)
    stride = 1
    for ax in range(dim):
        flat += coords[:, ax] * stride
        stride *= prob.n[ax]
    # per-axis phase factors exp(-2 pi i xi_k J_k / n_k), exponent reduced mod n_k
    xi = [np.arange(prob.n[ax]) for ax in range(dim)]
    Khat = np.zeros(prob.grid_shape + (nd, nd), dtype=complex)
    for beta in range(nd):
        impulse = np.zeros(nd * N)
        impulse[beta * N] = 1.0
        col = operator_rows(ref, impulse, flat)                  # (nd, nodes)
        for j, c in enumerate(coords):
            ph = np.ones((1,) * dim, dtype=complex)
            for ax in range(dim):
                e = np.exp(-2j * np.pi * ((xi[ax] * c[ax]) % prob.n[ax]) / prob.n[ax])
                shape = [1] * dim
                shape[dim - 1 - ax] = prob.n[ax]                 # numpy axes are z, y, x
                ph = ph * e.reshape(shape)
            for alpha in range(nd):
                Khat[..., alpha, beta] += col[alpha, j] * ph
    return Khat.reshape(N, nd, nd)


class FFTPreconditioner:
    """The M^+ r of Preconditioner for grids too large for the dense DFT:
    symbol from stencil_symbol, transforms by numpy.fft (a library FFT with
    the same unnormalised forward / 1/N inverse convention as naive_dft)."""

    def __init__(self, prob: Problem, Cref: np.ndarray):
        self.prob = prob
        self.Kplus = pseudo_inverse_blocks(stencil_symbol(prob, Cref))

    def apply(self, r: np.ndarray) -> np.ndarray:
        prob = self.prob
        nd, N = prob.ndof_node, prob.N
        R = np.stack([np.fft.fftn(r[a * N:(a + 1) * N].reshape(prob.grid_shape)).ravel()
                      for a in range(nd)], axis=1)
        Z = np.einsum("fab,fb->fa", self.Kplus, R)
        return np.concatenate([np.real(np.fft.ifftn(Z[:, a].reshape(prob.grid_shape))).ravel()
                               for a in range(nd)])
