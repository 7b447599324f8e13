"""Preconditioned conjugate gradients (TEST INFRASTRUCTURE ONLY).

Paper Sec. 4.1 (PCG solves the symmetric form M^-1/2 K M^-1/2, written in
left-preconditioned notation, eq. prec_lin_system_general), Alg. 1 (the PCG
solve inside a Newton step; for a linear material and u_(0) = 0 the whole
algorithm is one PCG solve of K u = b) and Sec. 6 (termination: the
displacement-based scheme stops when the Kref^-1-norm of the residual falls
below eta^CG times its initial value).

Textbook PCG (Saad, Alg. 9.1), in plain numpy:

    x0 (zero, or a guess shifted to zero mean per component)
    r = b - K x, z = M r, p = z, rho = r.z, rho0 = rho
    repeat: q = K p; alpha = rho/(p.q); x += alpha p; r -= alpha q;
            z = M r; rho' = r.z; stop if rho' <= eta^2 rho0;
            beta = rho'/rho; p = z + beta p.

||r||_{M} = sqrt(r.z), so the stopping test is the relative M-norm test.
Status: 0 converged, 1 iteration limit reached, -4 breakdown (p.q <= 0).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class PCGResult:
    x: np.ndarray
    iterations: int
    status: int
    rho0: float
    rho: float
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)
    history: list = field(default_factory=list)   # sqrt(rho_k / rho0)


def zero_mean(x: np.ndarray, nd: int) -> np.ndarray:
    x = np.array(x, dtype=float).reshape(nd, -1)
    return (x - x.mean(axis=1, keepdims=True)).ravel()


def pcg(apply_K, apply_M, b: np.ndarray, eta: float, itmax: int = 10000,
        x0: np.ndarray | None = None, nd: int = 1,
        rho_ref: float | None = None, callback=None) -> PCGResult:
    """rho_ref: the squared norm the stopping test is relative to (default
    r0.z0; a warm start passes b.M b so that the test keeps measuring the
    residual against the zero-start one).  callback(x), if given, sees every
    iterate x_k, k >= 1 (a copy)."""
    b = np.asarray(b, dtype=float)
    x = np.zeros_like(b) if x0 is None else zero_mean(x0, nd)
    r = b - apply_K(x) if x0 is not None else b.copy()
    z = apply_M(r)
    p = z.copy()
    rho = float(np.dot(r, z))
    rho0 = rho if rho_ref is None else float(rho_ref)
    res = PCGResult(x, 0, 0, rho0, rho)
    if rho == 0.0 or (rho_ref is not None and rho <= eta * eta * rho0):
        return res
    for k in range(1, itmax + 1):
        q = apply_K(p)
        pq = float(np.dot(p, q))
        if not pq > 0.0:
            res.status = -4
            res.iterations = k - 1
            return res
        alpha = rho / pq
        x += alpha * p
        r -= alpha * q
        if callback is not None:
            callback(x.copy())
        z = apply_M(r)
        rho_new = float(np.dot(r, z))
        res.alphas.append(alpha)
        res.history.append(np.sqrt(max(rho_new, 0.0) / rho0))
        res.iterations = k
        res.rho = rho_new
        if rho_new <= eta * eta * rho0:
            return res
        beta = rho_new / rho
        res.betas.append(beta)
        rho = rho_new
        p = z + beta * p
    res.status = 1
    return res


def screened_guess(apply_K, apply_M, b: np.ndarray, x0: np.ndarray, nd: int):
    """Warm-start screen: keep the zero-mean guess only if its residual has a
    smaller M-norm than the zero start's (r.M r < b.M b).  Returns
    (accepted, guess or zeros, b.M b, r0.M r0)."""
    b = np.asarray(b, dtype=float)
    x = zero_mean(x0, nd)
    rb = float(np.dot(b, apply_M(b)))
    r = b - apply_K(x)
    rx = float(np.dot(r, apply_M(r)))
    if rx < rb:
        return True, x, rb, rx
    return False, np.zeros_like(b), rb, rx


def lanczos_ritz_values(alphas, betas) -> np.ndarray:
    """Eigenvalues of the Lanczos tridiagonal built from the PCG
    coefficients (Saad, Sec. 6.7.3): T_kk = 1/a_k + b_{k-1}/a_{k-1},
    T_k,k+1 = sqrt(b_k)/a_k.  They approximate eigenvalues of M^+ K."""
    m = len(alphas)
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k + 1 < m:
            T[k, k + 1] = T[k + 1, k] = np.sqrt(betas[k]) / alphas[k]
    return np.linalg.eigvalsh(T)
