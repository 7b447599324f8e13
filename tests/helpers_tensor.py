"""Tensor-notation helpers written for the tests only.

They restate textbook continuum mechanics (full fourth-order tensors, the
Mandel basis change) independently of the oracle's Mandel-matrix code, so that
a convention slip in either one shows up as a mismatch.
"""
import math

import numpy as np

_PAIR = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (1, 2): 3, (2, 1): 3,
         (0, 2): 4, (2, 0): 4, (0, 1): 5, (1, 0): 5}
_PAIR2 = {(0, 0): 0, (1, 1): 1, (0, 1): 2, (1, 0): 2}


def mandel_to_tensor(M: np.ndarray, dim: int) -> np.ndarray:
    pair = _PAIR if dim == 3 else _PAIR2
    C = np.zeros((dim,) * 4)
    for i in range(dim):
        for j in range(dim):
            for k in range(dim):
                for l in range(dim):
                    wij = 1.0 if i == j else math.sqrt(2.0)
                    wkl = 1.0 if k == l else math.sqrt(2.0)
                    C[i, j, k, l] = M[pair[i, j], pair[k, l]] / (wij * wkl)
    return C


def isotropic_tensor(lam: float, mu: float, dim: int = 3) -> np.ndarray:
    d = np.eye(dim)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def lame(E: float, nu: float):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def random_spd(m: int, rng, cond: float = 10.0) -> np.ndarray:
    A = rng.standard_normal((m, m))
    Q, _ = np.linalg.qr(A)
    lam = np.exp(rng.uniform(0.0, math.log(cond), m))
    return (Q * lam) @ Q.T
