"""Two-node stencil: four linear triangles per pixel (TEST INFRASTRUCTURE
ONLY).

Paper Sec. 3, Fig. tiling (c.2): a stencil with N_n = 2 nodes per pixel, the
pixel's lowest corner and its centre; the pixel is cut into four triangles,
each formed by the centre and one pixel edge, with one quadrature point
(the centroid) and weight V_p/4.  Degrees of freedom: d N_n N_p; here they
are numbered field-major, field f = s nd + alpha for node set s (0 =
corners, 1 = centres) and component alpha, then the pixel-grid index of the
node (x fastest).

The preconditioner follows Sec. 4-5 for N_n > 1: the blocks K_ab of Kref
between the 2 nd fields are block-circulant, so the DFT of the impulse
response of field b at node 0 gives column b of the (2 nd) x (2 nd) block
K^(xi) at every frequency (Alg. 2); K^(xi) is Hermitian (not real: the
centre sits half a pixel away from the corner) and at xi = 0 it has rank
d (N_n - 1) = nd, the constant fields of each component being its null
space; the Moore-Penrose pseudo-inverse of each block (eq. block_inversion)
is taken by eigen-decomposition with the same tolerance as the one-node
oracle.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .elements import scalar_gradient_rows, symmetric_gradient_rows
from .naive_dft import dft, idft
from .precond import pseudo_inverse_blocks

# node (set, dx, dy) of the pixel: corners (0, dx, dy), centre (1, 0, 0)
# triangles: (corner, corner, centre) for the bottom, right, top and left edge
TRIANGLES = [((0, 0, 0), (0, 1, 0), (1, 0, 0)),
             ((0, 1, 0), (0, 1, 1), (1, 0, 0)),
             ((0, 1, 1), (0, 0, 1), (1, 0, 0)),
             ((0, 0, 1), (0, 0, 0), (1, 0, 0))]


def _position(node):
    s, dx, dy = node
    return np.array([0.5, 0.5]) if s == 1 else np.array([float(dx), float(dy)])


def triangle_gradients(h):
    """Per triangle, the (3, 2) physical gradients of its three P1 basis
    functions: solve [1 x y] coefficients from the vertex positions."""
    out = []
    for tri in TRIANGLES:
        P = np.array([_position(v) for v in tri]) * np.asarray(h)[None, :]
        A = np.hstack([np.ones((3, 1)), P])
        coef = np.linalg.solve(A, np.eye(3))      # column i: basis i
        out.append(coef[1:, :].T)                  # (3 vertices, 2)
    return out


@dataclass
class TwoNodeProblem:
    n: tuple            # (nx, ny)
    problem: str        # 'scalar' or 'elastic'
    phase: np.ndarray   # (ny, nx) ints
    mat: np.ndarray     # (nphase, m, m)
    l: tuple = (1.0, 1.0)

    @property
    def N(self):
        return int(self.n[0] * self.n[1])

    @property
    def nd(self):
        return 2 if self.problem == "elastic" else 1

    @property
    def nfield(self):
        return 2 * self.nd

    @property
    def m(self):
        return 3 if self.problem == "elastic" else 2

    @property
    def h(self):
        return np.array(self.l) / np.array(self.n)

    @property
    def volume(self):
        return float(np.prod(self.l))

    def rows(self):
        return symmetric_gradient_rows(2) if self.problem == "elastic" else scalar_gradient_rows(2)

    def B_matrices(self):
        """(4 triangles, m, 3 nd) constant strain matrices."""
        grads = triangle_gradients(self.h)
        B = np.zeros((4, self.m, 3 * self.nd))
        for t in range(4):
            for (mm, alpha, beta, coef) in self.rows():
                for v in range(3):
                    B[t, mm, v * self.nd + alpha] += coef * grads[t][v, beta]
        return B

    def weight(self):
        return 0.25 * float(np.prod(self.h))

    def dof(self, node, alpha, x, y):
        """Global dof of vertex `node` of pixel (x, y), component alpha."""
        s, dx, dy = node
        nx, ny = self.n
        if s == 1:
            I = x + nx * y
        else:
            I = (x + dx) % nx + nx * ((y + dy) % ny)
        return (s * self.nd + alpha) * self.N + I


def assemble(tp: TwoNodeProblem, C_of_pixel=None) -> sp.csr_matrix:
    """K = sum over triangles of w B^T C B (eq. lin_system)."""
    B = tp.B_matrices()
    w = tp.weight()
    nx, ny = tp.n
    rows, cols, vals = [], [], []
    ph = np.asarray(tp.phase)
    for y in range(ny):
        for x in range(nx):
            C = tp.mat[ph[y, x]] if C_of_pixel is None else C_of_pixel
            for t, tri in enumerate(TRIANGLES):
                Ke = w * B[t].T @ C @ B[t]
                idx = [tp.dof(v, a, x, y) for v in tri for a in range(tp.nd)]
                for i, gi in enumerate(idx):
                    for j, gj in enumerate(idx):
                        rows.append(gi)
                        cols.append(gj)
                        vals.append(Ke[i, j])
    n = tp.nfield * tp.N
    K = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    return K


def rhs(tp: TwoNodeProblem, E) -> np.ndarray:
    """b = -D^T W C e."""
    B = tp.B_matrices()
    w = tp.weight()
    nx, ny = tp.n
    b = np.zeros(tp.nfield * tp.N)
    ph = np.asarray(tp.phase)
    E = np.asarray(E, dtype=float)
    for y in range(ny):
        for x in range(nx):
            C = tp.mat[ph[y, x]]
            for t, tri in enumerate(TRIANGLES):
                fe = w * B[t].T @ (C @ E)
                idx = [tp.dof(v, a, x, y) for v in tri for a in range(tp.nd)]
                b[idx] -= fe
    return b


def gradients(tp: TwoNodeProblem, u) -> np.ndarray:
    """(N_p, 4, m) strain / gradient D u at the four centroids of each pixel."""
    B = tp.B_matrices()
    nx, ny = tp.n
    out = np.zeros((tp.N, 4, tp.m))
    for y in range(ny):
        for x in range(nx):
            for t, tri in enumerate(TRIANGLES):
                idx = [tp.dof(v, a, x, y) for v in tri for a in range(tp.nd)]
                out[x + nx * y, t] = B[t] @ np.asarray(u)[idx]
    return out


def mean_material(tp: TwoNodeProblem) -> np.ndarray:
    """Quadrature-weighted mean (Sec. 6.2): all four triangles of a pixel carry
    its material."""
    ph = np.asarray(tp.phase).ravel()
    counts = np.bincount(ph, minlength=len(tp.mat)).astype(float)
    return np.einsum("p,pij->ij", counts, tp.mat) / tp.N


def reference_symbol(tp: TwoNodeProblem, Cref) -> np.ndarray:
    """(N_p, 2nd, 2nd) Hermitian K^(xi) by Alg. 2: the DFT over the pixel grid
    of each field block of the impulse responses of Kref."""
    Kref = assemble(tp, np.asarray(Cref, dtype=float))
    nf, N = tp.nfield, tp.N
    shape = (tp.n[1], tp.n[0])
    Khat = np.zeros((N, nf, nf), dtype=complex)
    for b in range(nf):
        imp = np.zeros(nf * N)
        imp[b * N] = 1.0
        col = Kref @ imp
        for a in range(nf):
            Khat[:, a, b] = dft(col[a * N:(a + 1) * N].reshape(shape)).ravel()
    return Khat


class TwoNodePreconditioner:
    """z = M^+ r: per-field DFT, Hermitian block pseudo-inverse, inverse DFT."""

    def __init__(self, tp: TwoNodeProblem, Cref):
        self.tp = tp
        self.Khat = reference_symbol(tp, Cref)
        self.Kplus = pseudo_inverse_blocks(self.Khat)

    def apply(self, r):
        tp = self.tp
        nf, N = tp.nfield, tp.N
        shape = (tp.n[1], tp.n[0])
        R = np.stack([dft(r[f * N:(f + 1) * N].reshape(shape)).ravel() for f in range(nf)], axis=1)
        Z = np.einsum("fab,fb->fa", self.Kplus, R)
        return np.concatenate([np.real(idft(Z[:, f].reshape(shape))).ravel() for f in range(nf)])


def homogenize(tp: TwoNodeProblem, loads, eta=1e-10, itmax=10000):
    """PCG (oracle.pcg) per load with Cref = mean; C_hom in energy form over
    the four centroids of every pixel."""
    from .pcg import pcg
    loads = np.atleast_2d(np.asarray(loads, dtype=float))
    Cref = mean_material(tp)
    K = assemble(tp)
    M = TwoNodePreconditioner(tp, Cref)
    sols, res = [], []
    for E in loads:
        r = pcg(lambda v: K @ v, M.apply, rhs(tp, E), eta, itmax)
        sols.append(r.x)
        res.append(r)
    w = tp.weight()
    C = tp.mat[np.asarray(tp.phase).ravel()]                 # (N, m, m)
    eps = [gradients(tp, u) + E[None, None, :] for u, E in zip(sols, loads)]
    nl = len(loads)
    H = np.zeros((nl, nl))
    for i in range(nl):
        for j in range(nl):
            H[i, j] = w * np.einsum("etm,emn,etn->", eps[i], C, eps[j]) / tp.volume
    return H, sols, res
