"""Assembled sparse stiffness and right-hand side (TEST INFRASTRUCTURE ONLY).

Paper Sec. 3: the gradient matrix D (eqs. Du_mat, grad_componets), the
quadrature weights W (eq. W_mat) and the material tangent C at the quadrature
points give K = D^T W C D (eq. lin_system) and, for a linear material and
u0 = 0, the right-hand side b = -D^T W C e.

Grouping the quadrature sum by pixel/voxel, K is the sum of element matrices
K_e = sum_q w_q B_q^T C_e B_q, where B_q holds the rows of D that belong to the
element's quadrature points restricted to its corner nodes.  This module
writes that sum out entry by entry into a CSR matrix with one row per degree
of freedom (component-major numbering alpha*N + I, I = flat node index, x
fastest) and 3^d neighbour offsets x d columns per row.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .elements import Element, element, scalar_gradient_rows, symmetric_gradient_rows


@dataclass
class Problem:
    """Periodic cell discretised on a regular grid (paper Sec. 2-3).

    n        grid size per axis, (nx, ny) or (nx, ny, nz)
    l        cell edge lengths (default 1), h = l / n
    problem  'scalar' (App. A) or 'elastic' (Sec. 2)
    elem     stencil name ('hex8', 'quad4', 'tri2')
    phase    integer grid (numpy order [z][y][x]) indexing `mat`, or None
    mat      (nphase, m, m) material tables: Mandel stiffness (m = d_m) or
             conductivity (m = d)
    kfield   per-voxel scalar conductivity grid (A = k I), used when phase is
             None (scalar problems only)
    """
    n: tuple
    problem: str
    elem: str
    phase: np.ndarray | None = None
    mat: np.ndarray | None = None
    kfield: np.ndarray | None = None
    l: tuple | None = None
    _el: Element = field(init=False, repr=False)

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        self._el = element(self.elem)
        assert self._el.dim == len(self.n)
        if self.l is None:
            self.l = (1.0,) * len(self.n)
        self.l = tuple(float(v) for v in self.l)

    @property
    def dim(self):
        return len(self.n)

    @property
    def el(self) -> Element:
        return self._el

    @property
    def h(self):
        return np.array(self.l) / np.array(self.n)

    @property
    def N(self):
        return int(np.prod(self.n))

    @property
    def ndof_node(self):
        return self.dim if self.problem == "elastic" else 1

    @property
    def nstrain(self):
        d = self.dim
        return d * (d + 1) // 2 if self.problem == "elastic" else d

    @property
    def grid_shape(self):
        """numpy shape of a nodal/voxel grid: (nz, ny, nx) or (ny, nx)."""
        return tuple(self.n[::-1])

    @property
    def volume(self):
        return float(np.prod(self.l))

    @property
    def voxel_volume(self):
        return float(np.prod(self.h))

    def gradient_rows(self):
        if self.problem == "elastic":
            return symmetric_gradient_rows(self.dim)
        return scalar_gradient_rows(self.dim)

    def voxel_materials(self) -> np.ndarray:
        """(N, m, m) material tangent of every pixel/voxel (element-wise
        constant, Sec. 4.3)."""
        if self.phase is not None:
            return self.mat[np.asarray(self.phase).ravel()]
        k = np.asarray(self.kfield, dtype=float).ravel()
        return k[:, None, None] * np.eye(self.dim)[None]


def B_matrices(prob: Problem) -> np.ndarray:
    """(nq, m, nc*nd) element gradient matrices, eq. Du_mat restricted to one
    pixel: B_q[m, a*nd + alpha] = sum of coef * dphi_a/dx_beta(x_q)."""
    el = prob.el
    nd = prob.ndof_node
    grad_phys = el.grad_ref / prob.h[None, None, :]
    nq, nc = grad_phys.shape[:2]
    B = np.zeros((nq, prob.nstrain, nc * nd))
    for (m, alpha, beta, coef) in prob.gradient_rows():
        for a in range(nc):
            B[:, m, a * nd + alpha] += coef * grad_phys[:, a, beta]
    return B


def quadrature_weights(prob: Problem) -> np.ndarray:
    """w_q = wfrac_q * V_p (Fig. tiling)."""
    return prob.el.wfrac * prob.voxel_volume


def element_matrix(prob: Problem, C: np.ndarray) -> np.ndarray:
    """K_e = sum_q w_q B_q^T C B_q for a constant material C (eq. lin_system
    restricted to one pixel)."""
    B = B_matrices(prob)
    w = quadrature_weights(prob)
    return np.einsum("q,qmi,mn,qnj->ij", w, B, C, B)


def _offsets(dim):
    return [np.array(o[::-1]) for o in itertools.product((-1, 0, 1), repeat=dim)]


def _shift_to_nodes(field_grid: np.ndarray, corner) -> np.ndarray:
    """Value at node I of the pixel e = I - corner (periodic): roll by +corner
    along each axis (numpy axes are reversed w.r.t. x, y, z)."""
    shift = tuple(int(c) for c in corner[::-1])
    return np.roll(field_grid, shift, axis=tuple(range(field_grid.ndim)))


def assemble_stiffness(prob: Problem, uniform: np.ndarray | None = None) -> sp.csr_matrix:
    """CSR K = D^T W C D (eq. lin_system) or, with `uniform` = Cref, the
    reference matrix Kref = D^T W Cref D (eq. Kref).

    Entry ((alpha, I), (beta, J)) = sum over pixels e containing both nodes,
    of K_e[(a, alpha), (b, beta)] with I = e + corner_a and J = e + corner_b.
    """
    el = prob.el
    nd = prob.ndof_node
    N = prob.N
    offs = _offsets(prob.dim)
    off_index = {tuple(o): i for i, o in enumerate(offs)}
    noff = len(offs)
    data = np.zeros((nd, N, noff, nd))
    nc = len(el.corners)
    if uniform is not None:
        Ke = element_matrix(prob, np.asarray(uniform, dtype=float))
        tables = Ke[None]
        key = np.zeros(prob.grid_shape, dtype=np.int64)
        scale = None
    elif prob.phase is not None:
        tables = np.stack([element_matrix(prob, C) for C in prob.mat])
        key = np.asarray(prob.phase).astype(np.int64)
        scale = None
    else:
        Ke = element_matrix(prob, np.eye(prob.dim))
        tables = Ke[None]
        key = np.zeros(prob.grid_shape, dtype=np.int64)
        scale = np.asarray(prob.kfield, dtype=float)
    for a in range(nc):
        key_at_I = _shift_to_nodes(key, el.corners[a]).ravel()
        sc_at_I = None if scale is None else _shift_to_nodes(scale, el.corners[a]).ravel()
        for b in range(nc):
            oi = off_index[tuple(el.corners[b] - el.corners[a])]
            blk = tables[:, a * nd:(a + 1) * nd, b * nd:(b + 1) * nd][key_at_I]  # (N, nd, nd)
            if sc_at_I is not None:
                blk = blk * sc_at_I[:, None, None]
            data[:, :, oi, :] += blk.transpose(1, 0, 2)
    # column indices: (beta, I + o) with periodic wrap
    coords = np.indices(prob.grid_shape).reshape(prob.dim, -1)[::-1]  # x, y(, z)
    n = np.array(prob.n)[:, None]
    cols = np.empty((noff, N), dtype=np.int64)
    for oi, o in enumerate(offs):
        c = (coords + o[:, None]) % n
        flat = c[0].copy()
        stride = 1
        for ax in range(1, prob.dim):
            stride *= prob.n[ax - 1]
            flat += c[ax] * stride
        cols[oi] = flat
    indices = np.empty((nd, N, noff, nd), dtype=np.int64)
    for beta in range(nd):
        indices[:, :, :, beta] = (beta * N + cols.T)[None]
    nnz = data.size
    idx_dtype = np.int32 if nd * N < 2 ** 31 and nnz < 2 ** 31 else np.int64
    indptr = np.arange(0, nnz + 1, noff * nd, dtype=idx_dtype)
    K = sp.csr_matrix((data.ravel(), indices.ravel().astype(idx_dtype), indptr),
                      shape=(nd * N, nd * N))
    if min(prob.n) < 3:
        K.sum_duplicates()
    return K


def rhs(prob: Problem, E: np.ndarray) -> np.ndarray:
    """b = -D^T W C e for a uniform macroscopic strain/gradient e
    (eq. lin_system with u_(0) = 0, sigma = C eps).  Returns a flat vector of
    length nd*N (component-major)."""
    el = prob.el
    nd = prob.ndof_node
    B = B_matrices(prob)
    w = quadrature_weights(prob)
    E = np.asarray(E, dtype=float)
    # per-material element force f = sum_q w_q B_q^T C E
    if prob.phase is not None:
        F = np.einsum("q,qmi,pmn,n->pi", w, B, prob.mat, E)
        key = np.asarray(prob.phase).astype(np.int64)
        scale = None
    else:
        F = np.einsum("q,qmi,mn,n->i", w, B, np.eye(prob.dim), E)[None]
        key = np.zeros(prob.grid_shape, dtype=np.int64)
        scale = np.asarray(prob.kfield, dtype=float)
    b = np.zeros((nd, prob.N))
    for a in range(len(el.corners)):
        key_at_I = _shift_to_nodes(key, el.corners[a]).ravel()
        f = F[key_at_I][:, a * nd:(a + 1) * nd]  # (N, nd)
        if scale is not None:
            f = f * _shift_to_nodes(scale, el.corners[a]).ravel()[:, None]
        b -= f.T
    return b.ravel()


def gradient_at_quadrature(prob: Problem, u: np.ndarray) -> np.ndarray:
    """(N, nq, m) strain/gradient D u at every quadrature point of every
    pixel (eq. Du_mat), u flat component-major."""
    el = prob.el
    nd = prob.ndof_node
    B = B_matrices(prob)
    ug = np.asarray(u, dtype=float).reshape((nd,) + prob.grid_shape)
    ue = np.empty((prob.N, len(el.corners) * nd))
    for a, c in enumerate(el.corners):
        # value at pixel e of node e + corner: roll by -corner
        shift = tuple(-int(v) for v in c[::-1])
        for alpha in range(nd):
            ue[:, a * nd + alpha] = np.roll(ug[alpha], shift,
                                            axis=tuple(range(prob.dim))).ravel()
    return np.einsum("qmi,ei->eqm", B, ue)


def operator_rows(prob: Problem, u: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """(K u) at selected nodes only, for grids too large to assemble:
    (K u)[(alpha, I)] = sum_a sum_b K_e[(a, alpha), (b, beta)] u[(beta, e + c_b)]
    over the pixels e = I - c_a that contain node I (eq. lin_system grouped by
    element).  `nodes` holds flat node indices; returns (nd, len(nodes))."""
    el = prob.el
    nd = prob.ndof_node
    nodes = np.asarray(nodes, dtype=np.int64)
    n = np.array(prob.n)
    coords = np.stack(np.unravel_index(nodes, prob.grid_shape)[::-1])  # x, y(, z)
    ug = np.asarray(u, dtype=float).reshape(nd, prob.N)
    if prob.phase is not None:
        tables = np.stack([element_matrix(prob, C) for C in prob.mat])
    else:
        tables = element_matrix(prob, np.eye(prob.dim))[None]

    def flat(c):
        c = c % n[:, None]
        out = c[0].copy()
        stride = 1
        for ax in range(1, prob.dim):
            stride *= prob.n[ax - 1]
            out += c[ax] * stride
        return out

    out = np.zeros((nd, nodes.size))
    for a, ca in enumerate(el.corners):
        e = flat(coords - ca[:, None])
        if prob.phase is not None:
            Ke = tables[np.asarray(prob.phase).ravel()[e]]
        else:
            Ke = tables[0][None] * np.asarray(prob.kfield).ravel()[e][:, None, None]
        for b, cb in enumerate(el.corners):
            J = flat(coords - ca[:, None] + cb[:, None])
            blk = Ke[:, a * nd:(a + 1) * nd, b * nd:(b + 1) * nd]  # (S, nd, nd)
            out += np.einsum("sab,bs->as", blk, ug[:, J])
    return out
