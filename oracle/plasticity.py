"""Newton-PCG for a nonlinear (elasto-plastic) material (TEST INFRASTRUCTURE
ONLY).

Paper Sec. 3 (eq. non_lin_system: the nodal equilibrium D^T W sigma(e + D u)
= 0), Sec. 3.1 (Newton linearisation, eq. lin_system: K_(i) du = b_(i) with
K_(i) = D^T W C_(i) D, b_(i) = -D^T W sigma(e + D u_(i)), C_(i) the
consistent tangent at the quadrature points), Alg. 1 (the Newton loop: for
every step update the internal variables, form the right-hand side and the
tangent, assemble the preconditioner, solve with PCG to eta^CG, update
u_(i+1) = u_(i) + du, stop when ||du|| <= eta^NW ||u_(i+1)||), Sec. 5.2
(re-assembly of the preconditioner when the tangent changes) and Sec. 6.3
(two phases that share the elastic constants and differ in the initial yield
stress and the linear hardening modulus, macroscopic strain applied in load
increments).

Material (stated reading: the paper's Sec. 6.3 model is finite-strain; the
build uses its small-strain counterpart): von Mises plasticity with linear
isotropic hardening, per phase the bulk modulus K, shear modulus G, initial
yield stress sy0 and hardening modulus H (yield stress sy0 + H alpha, alpha
the equivalent plastic strain).  Internal variables per quadrature point:
the plastic strain eps_p (Mandel, deviatoric) and alpha.  Stress update from
the committed state of the previous increment by the radial return of
Simo & Hughes (Computational Inelasticity, Sec. 3.3):

    s_tr = 2G (dev eps - eps_p_n),  f = |s_tr| - sqrt(2/3) (sy0 + H alpha_n)
    elastic (f <= 0): sigma = K tr(eps) 1 + s_tr, C = K 1(x)1 + 2G P_dev
    plastic: dg = f / (2G + 2H/3), n = s_tr / |s_tr|,
             sigma = K tr(eps) 1 + s_tr - 2G dg n,
             eps_p = eps_p_n + dg n, alpha = alpha_n + sqrt(2/3) dg,
             C = K 1(x)1 + 2G th P_dev - 2G thb n(x)n,
             th = 1 - 2G dg / |s_tr|, thb = 1 / (1 + H/(3G)) - (1 - th).

Mandel vectors make |.| the Frobenius norm of the tensor and P_dev =
I - (1/3) 1(x)1 with 1 = (1, 1, 1, 0, 0, 0).

Reference material (stated reading of Alg. 1 "preconditioner assembly"):
mode 'tangent' re-assembles K^ref every Newton step from the quadrature-
weighted mean of the current tangent (Sec. 6.2's mean, applied to C_(i));
mode 'elastic' keeps the mean elastic stiffness throughout.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .assembly import B_matrices, Problem, _shift_to_nodes, quadrature_weights
from .pcg import pcg
from .precond import FFTPreconditioner, Preconditioner

ONE = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
# Reading (stated; the paper's Alg. 1 assumes exact arithmetic): a nodal
# residual whose 2-norm is at most this fraction of the 2-norm of the element
# forces it sums is rounding noise (e.g. a uniform stress) and counts as
# equilibrium, with no PCG solve: the relative PCG stopping test is
# meaningless for such a right-hand side.
RESIDUAL_FLOOR = 1e-12
P_DEV = np.eye(6) - np.outer(ONE, ONE) / 3.0
SQ23 = math.sqrt(2.0 / 3.0)


def return_mapping(eps, eps_p_n, alpha_n, K, G, sy0, H):
    """Radial return for arrays of quadrature points.

    eps, eps_p_n: (..., 6) Mandel; alpha_n, K, G, sy0, H: (...,).
    Returns sigma (..., 6), tangent C (..., 6, 6), eps_p (..., 6),
    alpha (...,), plastic mask (...,)."""
    eps = np.asarray(eps, dtype=float)
    tr = eps[..., 0] + eps[..., 1] + eps[..., 2]
    dev = eps - (tr / 3.0)[..., None] * ONE
    s_tr = 2.0 * G[..., None] * (dev - eps_p_n)
    ns = np.sqrt(np.sum(s_tr * s_tr, axis=-1))
    f = ns - SQ23 * (sy0 + H * alpha_n)
    plastic = f > 0.0
    dg = np.where(plastic, f / (2.0 * G + 2.0 * H / 3.0), 0.0)
    n = np.where(plastic[..., None], s_tr / np.where(ns > 0, ns, 1.0)[..., None], 0.0)
    sigma = (K * tr)[..., None] * ONE + s_tr - (2.0 * G * dg)[..., None] * n
    eps_p = eps_p_n + dg[..., None] * n
    alpha = alpha_n + SQ23 * dg
    th = np.where(plastic, 1.0 - 2.0 * G * dg / np.where(ns > 0, ns, 1.0), 1.0)
    thb = np.where(plastic, 1.0 / (1.0 + H / (3.0 * G)) - (1.0 - th), 0.0)
    C = (K[..., None, None] * np.outer(ONE, ONE) + (2.0 * G * th)[..., None, None] * P_DEV
         - (2.0 * G * thb)[..., None, None] * n[..., :, None] * n[..., None, :])
    return sigma, C, eps_p, alpha, plastic


@dataclass
class PlasticProblem:
    """3D hex8 grid with a phase field; params (nphase, 4) = K, G, sy0, H."""
    n: tuple
    phase: np.ndarray
    params: np.ndarray
    prob: Problem = field(init=False)

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        self.params = np.asarray(self.params, dtype=float)
        # elastic stiffness per phase (the material of the underlying linear problem)
        mats = []
        for K, G, _, _ in self.params:
            mats.append(K * np.outer(ONE, ONE) + 2.0 * G * P_DEV)
        self.prob = Problem(self.n, "elastic", "hex8", phase=self.phase, mat=np.stack(mats))

    def qp_params(self):
        """(N, nq) arrays K, G, sy0, H at every quadrature point."""
        ph = np.asarray(self.phase).ravel()
        nq = len(self.prob.el.wfrac)
        return [np.repeat(self.params[ph, k][:, None], nq, axis=1) for k in range(4)]


def strain_at_qp(pp: PlasticProblem, u, E):
    """(N, nq, 6) total strain e + D u at every quadrature point (eq. Du_mat)."""
    from .assembly import gradient_at_quadrature
    return gradient_at_quadrature(pp.prob, u) + np.asarray(E, dtype=float)[None, None, :]


def element_forces_to_nodes(prob: Problem, fe: np.ndarray) -> np.ndarray:
    """Scatter per-element corner forces fe (N, nc*nd) to the nodes: node
    I = e + corner_a receives fe[e, a]; flat component-major output."""
    el = prob.el
    nd = prob.ndof_node
    out = np.zeros((nd, prob.N))
    for a, c in enumerate(el.corners):
        for alpha in range(nd):
            g = fe[:, a * nd + alpha].reshape(prob.grid_shape)
            out[alpha] += _shift_to_nodes(g, c).ravel()
    return out.ravel()


def internal_force(pp: PlasticProblem, sigma: np.ndarray, with_scale: bool = False):
    """D^T W sigma for a stress (N, nq, 6) at the quadrature points.  With
    with_scale, also the 2-norm of the element forces before they are summed
    at the nodes: the size of the terms whose cancellation leaves rounding
    noise in the nodal sums."""
    B = B_matrices(pp.prob)
    w = quadrature_weights(pp.prob)
    fe = np.einsum("q,qmi,eqm->ei", w, B, sigma)
    f = element_forces_to_nodes(pp.prob, fe)
    if with_scale:
        return f, float(np.sqrt(np.sum(fe * fe)))
    return f


def tangent_stiffness(pp: PlasticProblem, C: np.ndarray) -> sp.csr_matrix:
    """Assembled K_(i) = D^T W C_(i) D with a tangent C (N, nq, 6, 6) per
    quadrature point (eq. lin_system)."""
    prob = pp.prob
    el = prob.el
    nd = prob.ndof_node
    B = B_matrices(prob)
    w = quadrature_weights(prob)
    Ke = np.einsum("q,qmi,eqmn,qnj->eij", w, B, C, B)  # (N, 24, 24)
    N = prob.N
    n = np.array(prob.n)
    coords = np.indices(prob.grid_shape).reshape(3, -1)[::-1]
    rows, cols, vals = [], [], []
    for a, ca in enumerate(el.corners):
        Ia = (coords + ca[:, None]) % n[:, None]
        Ia = Ia[0] + n[0] * (Ia[1] + n[1] * Ia[2])
        for b, cb in enumerate(el.corners):
            Ib = (coords + cb[:, None]) % n[:, None]
            Ib = Ib[0] + n[0] * (Ib[1] + n[1] * Ib[2])
            for al in range(nd):
                for be in range(nd):
                    rows.append(al * N + Ia)
                    cols.append(be * N + Ib)
                    vals.append(Ke[:, a * nd + al, b * nd + be])
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nd * N, nd * N)).tocsr()
    K.sum_duplicates()
    return K


def mean_tangent(pp: PlasticProblem, C: np.ndarray) -> np.ndarray:
    """Quadrature-weighted mean of a per-point tangent (Sec. 6.2)."""
    w = quadrature_weights(pp.prob)
    flat = np.ascontiguousarray(np.einsum("q,eqmn->mneq", w, C).reshape(36, -1))
    return (flat.sum(axis=1) / pp.prob.volume).reshape(6, 6)


@dataclass
class IncrementResult:
    newton_steps: int
    pcg_iterations: list
    du_ratios: list           # ||du|| / ||u_(i+1)|| per Newton step
    macro_stress: np.ndarray  # (1/|Y|) sum_Q w_Q sigma_Q at the converged u
    plastic_fraction: float   # share of quadrature points that yielded
    converged: bool


def newton_solve(pp: PlasticProblem, E_final, nincr: int, eta_nw: float = 1e-8,
                 eta_cg: float = 1e-10, itmax_nw: int = 50, itmax_cg: int = 10000,
                 ref: str = "tangent", fft: bool = False):
    """Alg. 1 over `nincr` equal increments of the macroscopic strain,
    e_k = (k / nincr) E_final, each Newton loop starting from the previous
    increment's converged u.  Returns (u, eps_p, alpha, [IncrementResult]).
    fft=True uses the FFT form of the preconditioner (larger grids)."""
    prob = pp.prob
    N, nq = prob.N, len(prob.el.wfrac)
    Kq, Gq, syq, Hq = pp.qp_params()
    eps_p = np.zeros((N, nq, 6))
    alpha = np.zeros((N, nq))
    u = np.zeros(3 * N)
    w = quadrature_weights(prob)
    results = []
    E_final = np.asarray(E_final, dtype=float)
    M_elastic = None
    for k in range(1, nincr + 1):
        E = E_final * (k / nincr)
        its, ratios = [], []
        converged = False
        for i in range(itmax_nw):
            eps = strain_at_qp(pp, u, E)
            sig, C, _, _, _ = return_mapping(eps, eps_p, alpha, Kq, Gq, syq, Hq)
            f, fscale = internal_force(pp, sig, with_scale=True)
            b = -f
            if np.linalg.norm(b) <= RESIDUAL_FLOOR * fscale:
                # equilibrium to rounding: no step is taken (du = 0)
                its.append(0)
                ratios.append(0.0)
                converged = True
                break
            Kt = tangent_stiffness(pp, C)
            if ref == "tangent":
                Cref = mean_tangent(pp, C)
                M = (FFTPreconditioner if fft else Preconditioner)(prob, Cref)
            else:
                if M_elastic is None:
                    from .homog import mean_material
                    M_elastic = (FFTPreconditioner if fft else Preconditioner)(
                        prob, mean_material(prob))
                M = M_elastic
            res = pcg(lambda v: Kt @ v, M.apply, b, eta_cg, itmax_cg, nd=3)
            its.append(res.iterations)
            u = u + res.x
            nu_ = float(np.linalg.norm(u))
            ndu = float(np.linalg.norm(res.x))
            ratios.append(ndu / nu_ if nu_ > 0 else 0.0)
            if ndu <= eta_nw * nu_:
                converged = True
                break
        # commit the internal variables at the converged displacement
        eps = strain_at_qp(pp, u, E)
        sig, _, eps_p, alpha, plastic = return_mapping(eps, eps_p, alpha, Kq, Gq, syq, Hq)
        macro = np.einsum("q,eqm->m", w, sig) / prob.volume
        results.append(IncrementResult(len(its), its, ratios, macro,
                                       float(np.mean(plastic)), converged))
    return u, eps_p, alpha, results
