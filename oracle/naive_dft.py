"""Naive discrete Fourier transform (TEST INFRASTRUCTURE ONLY).

Paper Sec. 4.2 and Alg. 2: diag(K^_ab) is obtained as the Fourier transform
of one column of the circulant block K_ab.  Reading (stated): the transform
in Alg. 2 is the *unnormalised* DFT

    X(xi) = sum_J x(J) exp(-2 pi i sum_k xi_k J_k / n_k),

and its inverse carries the factor 1/N, so that F^H K^ F of eq. M_inverse is
reproduced with the unitary F of Sec. 4.2.

This is the definition evaluated with dense DFT matrices applied along each
axis in turn (separable direct sum, O(N sum_k n_k) work, no butterflies).
Arrays are in numpy order [z][y][x] (or [y][x]); the transform covers every
axis.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(n: int, sign: int) -> np.ndarray:
    j = np.arange(n)
    # reduce j*k mod n before scaling so the angle is exact in integers
    return np.exp(sign * 2j * np.pi * (np.outer(j, j) % n) / n)


def _apply(x: np.ndarray, sign: int, axes) -> np.ndarray:
    y = np.asarray(x, dtype=complex)
    for ax in axes:
        F = dft_matrix(y.shape[ax], sign)
        y = np.moveaxis(np.tensordot(F, y, axes=([1], [ax])), 0, ax)
    return y


def dft(x: np.ndarray, axes=None) -> np.ndarray:
    """Unnormalised forward DFT over `axes` (default: all)."""
    axes = range(np.ndim(x)) if axes is None else axes
    return _apply(x, -1, axes)


def idft(X: np.ndarray, axes=None) -> np.ndarray:
    """Inverse DFT with the 1/N factor over `axes` (default: all)."""
    axes = list(range(np.ndim(X)) if axes is None else axes)
    N = int(np.prod([np.shape(X)[a] for a in axes]))
    return _apply(X, +1, axes) / N
