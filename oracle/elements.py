"""Reference discretisation stencils (TEST INFRASTRUCTURE ONLY).

Paper Sec. 3, Fig. tiling: a one-node stencil (N_n = 1) repeated on every
pixel/voxel.  Each stencil is described by

  corners   (nc, d) integer offsets of the pixel/voxel corner nodes, relative
            to the lowest corner (the node the pixel is attached to);
  grad_ref  (nq, nc, d) gradients of the corner shape functions with respect
            to the reference coordinates xi in [0, 1]^d, evaluated at the
            quadrature points (eq. grad_componets before the 1/h scaling);
  wfrac     (nq,) quadrature weights as fractions of the pixel volume V_p.

Stencils:
  'hex8'  3D trilinear hexahedron, 2x2x2 Gauss-Legendre points
          xi = 1/2 -+ 1/(2 sqrt 3), w = V_p/8 (3D analogue of Fig. tiling a.2);
  'quad4' 2D bilinear quadrilateral, 2x2 Gauss points, w = V_p/4 (a.2);
  'tri2'  2D pair of linear triangles per pixel split along the diagonal
          (0,0)-(1,1), one centroid point each, w = V_p/2 (b.2).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Element:
    name: str
    dim: int
    corners: np.ndarray   # (nc, d) int
    grad_ref: np.ndarray  # (nq, nc, d)
    wfrac: np.ndarray     # (nq,)
    qp_ref: np.ndarray    # (nq, d) reference coordinates of quadrature points


def _tensor_element(dim: int, name: str) -> Element:
    # corners with x varying fastest: node k = a0 + 2 a1 (+ 4 a2)
    corners = np.array([c[::-1] for c in itertools.product((0, 1), repeat=dim)])
    g = 0.5 / math.sqrt(3.0)
    pts1 = (0.5 - g, 0.5 + g)
    qps = np.array([p[::-1] for p in itertools.product(pts1, repeat=dim)])
    nq, nc = len(qps), len(corners)
    grad = np.zeros((nq, nc, dim))
    for q in range(nq):
        xi = qps[q]
        for a in range(nc):
            L = [xi[k] if corners[a, k] else 1.0 - xi[k] for k in range(dim)]
            dL = [1.0 if corners[a, k] else -1.0 for k in range(dim)]
            for k in range(dim):
                v = dL[k]
                for j in range(dim):
                    if j != k:
                        v *= L[j]
                grad[q, a, k] = v
    return Element(name, dim, corners, grad, np.full(nq, 1.0 / nq), qps)


def _tri2() -> Element:
    corners = np.array([(0, 0), (1, 0), (0, 1), (1, 1)])
    # T1 = {(0,0), (1,0), (1,1)}: barycentric 1-xi1, xi1-xi2, xi2
    # T2 = {(0,0), (1,1), (0,1)}: barycentric 1-xi2, xi1, xi2-xi1
    grad = np.zeros((2, 4, 2))
    grad[0, 0] = (-1.0, 0.0)
    grad[0, 1] = (1.0, -1.0)
    grad[0, 3] = (0.0, 1.0)
    grad[1, 0] = (0.0, -1.0)
    grad[1, 3] = (1.0, 0.0)
    grad[1, 2] = (-1.0, 1.0)
    qps = np.array([(2.0 / 3.0, 1.0 / 3.0), (1.0 / 3.0, 2.0 / 3.0)])
    return Element("tri2", 2, corners, grad, np.array([0.5, 0.5]), qps)


def element(name: str) -> Element:
    if name == "hex8":
        return _tensor_element(3, "hex8")
    if name == "quad4":
        return _tensor_element(2, "quad4")
    if name == "tri2":
        return _tri2()
    raise KeyError(name)


def symmetric_gradient_rows(dim: int):
    """Mandel symmetrized gradient (eq. mandel_grad, 3D extension).

    Returns a list of (m, alpha, beta, coef): strain component m receives
    coef * d u_alpha / d x_beta.  Order 3D: 11, 22, 33, 23, 13, 12; 2D: 11,
    22, 12.  Shear rows carry sqrt(2)/2 on each of the two partials.
    """
    s = math.sqrt(2.0) / 2.0
    if dim == 2:
        return [(0, 0, 0, 1.0), (1, 1, 1, 1.0), (2, 0, 1, s), (2, 1, 0, s)]
    return [(0, 0, 0, 1.0), (1, 1, 1, 1.0), (2, 2, 2, 1.0),
            (3, 1, 2, s), (3, 2, 1, s),
            (4, 0, 2, s), (4, 2, 0, s),
            (5, 0, 1, s), (5, 1, 0, s)]


def scalar_gradient_rows(dim: int):
    """Scalar gradient (eq. Dt_mat): row beta receives d w / d x_beta."""
    return [(b, 0, b, 1.0) for b in range(dim)]
