"""Guaranteed eigenvalue bounds of the preconditioned operator (TEST
INFRASTRUCTURE ONLY).

Paper Sec. 4.3: for every node I the bounds

    lambda_I^L = min over the quadrature points in supp(phi^I) of
                 lambda_min(Cref^-1 C(x_Q)),
    lambda_I^U = max over the same points of lambda_max(Cref^-1 C(x_Q)),

with generalized eigenvalues of the pair (C, Cref).  For element-wise
constant materials one pair (lambda_min, lambda_max) per pixel/voxel is
enough.  Each nodal bound is counted d times (once per displacement
component; once for scalar problems) and the two lists are sorted into
nondecreasing sequences.

Reading (stated, the paper does not say how the zero eigenvalues of the
periodic problem are counted): Kref^+ K has nd zero eigenvalues (constant
fields); its remaining eigenvalues mu_1 <= ... <= mu_M, M = nd N - nd,
satisfy L_(k+nd) <= mu_k <= U_(k) for the sorted lower and upper sequences
L and U (1-based).  The pins check this against dense generalized
eigenvalues on small grids.

The bound on the condition number is kappa = max_I lambda_I^U / min_I
lambda_I^L; the classical CG estimate then predicts at most
ceil(sqrt(kappa)/2 ln(2/eta)) iterations to reduce the energy-norm error by
eta.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.linalg as sla

from .assembly import Problem


def element_pairs(prob: Problem, Cref: np.ndarray):
    """(lo_e, hi_e), each (N,), extreme generalized eigenvalues of
    (C_e, Cref) for every pixel/voxel e (Sec. 4.3)."""
    Cref = np.asarray(Cref, dtype=float)
    if prob.phase is not None:
        lam = [sla.eigh(C, Cref, eigvals_only=True) for C in prob.mat]
        lo_p = np.array([v.min() for v in lam])
        hi_p = np.array([v.max() for v in lam])
        key = np.asarray(prob.phase).ravel().astype(np.int64)
        return lo_p[key], hi_p[key]
    k = np.asarray(prob.kfield, dtype=float).ravel()
    lam = sla.eigh(np.eye(prob.dim), Cref, eigvals_only=True)  # eigenvalues of Cref^-1
    return k * lam.min(), k * lam.max()


def node_bounds(prob: Problem, Cref: np.ndarray):
    """(lo, hi), each (N,): lambda_I^L and lambda_I^U of Sec. 4.3.  The
    support of the one-node stencil's basis function phi^I is the set of
    pixels that have I as a corner, e = I - c for every corner offset c."""
    lo_e, hi_e = element_pairs(prob, Cref)
    shape = prob.grid_shape
    lo = np.full(prob.N, np.inf)
    hi = np.full(prob.N, -np.inf)
    axes = tuple(range(prob.dim))
    for c in itertools.product((0, 1), repeat=prob.dim):
        shift = tuple(c)          # numpy axes are (z, y, x); any order covers all corners
        lo = np.minimum(lo, np.roll(lo_e.reshape(shape), shift, axis=axes).ravel())
        hi = np.maximum(hi, np.roll(hi_e.reshape(shape), shift, axis=axes).ravel())
    return lo, hi


def sorted_bounds(lo: np.ndarray, hi: np.ndarray, nd: int):
    """The nondecreasing sequences of Sec. 4.3: every nodal bound counted nd
    times."""
    return np.sort(np.repeat(lo, nd)), np.sort(np.repeat(hi, nd))


def kappa_bound(lo: np.ndarray, hi: np.ndarray) -> float:
    return float(np.max(hi) / np.min(lo))


def predicted_iterations(kappa: float, eta: float) -> int:
    """Classical CG estimate: the energy-norm error falls by eta within
    ceil(sqrt(kappa)/2 ln(2/eta)) iterations."""
    return int(math.ceil(0.5 * math.sqrt(kappa) * math.log(2.0 / eta)))
