"""Pins of the Newton-PCG oracle for the elasto-plastic material
(oracle/plasticity.py) against what the mathematics fixes, independent of the
oracle's own Mandel formulation:

* the textbook pure-shear response of linear-hardening von Mises plasticity
  (closed form);
* the consistent tangent against central differences of the stress update;
* a material that never yields reduces Alg. 1 to the linear solve;
* a homogeneous cell keeps u = 0 and returns the single-point response;
* an independent brute-force equilibrium residual written with 3x3 tensors,
  equivalent-stress radial return and trilinear shape functions built from
  their definition, and a dense Newton on it with a finite-difference
  Jacobian, on a 3x3x2 grid over two increments;
* quadratic convergence of the Newton steps.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import plasticity as op
from oracle.assembly import Problem


def _params(E=1.0, nu=0.3, sy0=0.0015, H=0.005):
    K = E / (3.0 * (1.0 - 2.0 * nu))
    G = E / (2.0 * (1.0 + nu))
    return np.array([K, G, sy0, H])


def test_pure_shear_closed_form():
    """Tensor shear strain eps12 = gamma/2 from the virgin state: elastic
    tau = G gamma up to tau = sy0/sqrt(3); beyond, with equivalent plastic
    strain gamma_p/sqrt(3), tau = G (gamma - gamma_p) and
    sqrt(3) tau = sy0 + H gamma_p / sqrt(3)."""
    K, G, sy0, H = _params()
    gammas = np.linspace(0.0, 0.03, 61)
    eps = np.zeros((gammas.size, 6))
    eps[:, 5] = math.sqrt(2.0) * gammas / 2.0          # Mandel: sqrt(2) eps12
    one = np.ones(gammas.size)
    sig, C, eps_p, alpha, plastic = op.return_mapping(eps, np.zeros_like(eps), 0 * one,
                                                      K * one, G * one, sy0 * one, H * one)
    tau = sig[:, 5] / math.sqrt(2.0)
    gp = np.maximum(0.0, (G * gammas - sy0 / math.sqrt(3.0)) / (G + H / 3.0))
    tau_exact = G * (gammas - gp)
    assert np.abs(tau - tau_exact).max() <= 1e-14
    assert np.abs(sig[:, :5]).max() <= 1e-15
    assert np.array_equal(plastic, gp > 0)
    assert np.abs(alpha - gp / math.sqrt(3.0)).max() <= 1e-15
    assert np.abs(eps_p[:, 5] - math.sqrt(2.0) * gp / 2.0).max() <= 1e-15


def _fd_tangent(eps, eps_p, alpha, K, G, sy0, H, h=1e-7):
    C = np.zeros((6, 6))
    for j in range(6):
        d = np.zeros(6)
        d[j] = h
        sp_ = op.return_mapping(eps + d, eps_p, alpha, K, G, sy0, H)[0]
        sm_ = op.return_mapping(eps - d, eps_p, alpha, K, G, sy0, H)[0]
        C[:, j] = (sp_ - sm_) / (2 * h)
    return C


def test_consistent_tangent_is_the_derivative_of_the_stress_update():
    rng = np.random.default_rng(3)
    K, G, sy0, H = (np.array(v) for v in _params())
    seen = set()
    for trial in range(40):
        eps = rng.normal(scale=0.004 if trial % 2 else 0.0004, size=6)
        dev_p = rng.normal(scale=0.001, size=6)
        dev_p[:3] -= dev_p[:3].mean()
        alpha = np.array(abs(rng.normal(scale=0.001)))
        sig, C, _, _, plastic = op.return_mapping(eps, dev_p, alpha, K, G, sy0, H)
        Cfd = _fd_tangent(eps, dev_p, alpha, K, G, sy0, H)
        assert np.abs(C - Cfd).max() <= 2e-7 * np.abs(C).max()
        assert np.allclose(C, C.T, atol=1e-15)
        assert np.linalg.eigvalsh(C).min() > 0.0
        seen.add(bool(plastic))
    assert seen == {True, False}


def _spheres_case(n, seed, contrast=1.0):
    from synth import spheres
    phase, _, _ = spheres(n[0], (0.8, 1.4), 0.3, seed=seed)
    phase = np.ascontiguousarray(phase[:n[2], :n[1], :n[0]])
    soft = _params(1.0, 0.3, 0.0015, 0.005)
    hard = _params(contrast, 0.3, 0.003, 0.01)
    return op.PlasticProblem(n, phase.astype(np.uint8), np.stack([soft, hard]))


def test_material_that_never_yields_is_the_linear_solve():
    pp = _spheres_case((6, 6, 6), 1, contrast=5.0)
    pp.params[:, 2] = 1e30
    E = np.array([0.3, -0.1, 0.2, 0.05, -0.02, 0.1])
    u, eps_p, alpha, res = op.newton_solve(pp, E, 1, eta_nw=1e-9, eta_cg=1e-12)
    assert res[0].converged and res[0].newton_steps <= 2
    H, sols, _ = oracle.homogenize(pp.prob, E[None], 1e-12)
    assert np.linalg.norm(u - sols[0]) <= 1e-10 * np.linalg.norm(sols[0])
    assert not eps_p.any() and not alpha.any()
    # macroscopic stress of a linear material: C_hom E (energy form)
    assert np.abs(res[0].macro_stress @ E - H[0, 0]).max() <= 1e-10 * abs(H[0, 0])


def test_homogeneous_cell_returns_the_point_response():
    n = (4, 4, 4)
    pp = op.PlasticProblem(n, np.zeros(n, dtype=np.uint8), _params()[None])
    E = np.array([0.004, -0.004, 0.0, 0.0, 0.0, 0.0])
    u, eps_p, alpha, res = op.newton_solve(pp, E, 3)
    assert np.abs(u).max() == 0.0
    K, G, sy0, H = _params()
    # one-step return from the virgin state along this proportional path
    s3 = op.return_mapping(E, np.zeros(6), np.array(0.0), np.array(K), np.array(G),
                           np.array(sy0), np.array(H))[0]
    assert np.abs(res[-1].macro_stress - s3).max() <= 1e-15
    assert res[-1].plastic_fraction == 1.0


# ---------------------------------------------------------------- brute force
def _brute_residual(n, phase, params, u, E, state):
    """D^T W sigma written with 3x3 tensors: trilinear shape functions and
    their gradients from the definition, 2-point Gauss rule per axis, von
    Mises radial return in equivalent-stress form.  Returns (r, new_state)
    with state = (eps_p tensors (N,8,3,3), alpha (N,8))."""
    nx, ny, nz = n
    N = nx * ny * nz
    h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
    g = 0.5 / math.sqrt(3.0)
    pts = [0.5 - g, 0.5 + g]
    U = u.reshape(3, N)
    Et = np.array([[E[0], E[5] / math.sqrt(2), E[4] / math.sqrt(2)],
                   [E[5] / math.sqrt(2), E[1], E[3] / math.sqrt(2)],
                   [E[4] / math.sqrt(2), E[3] / math.sqrt(2), E[2]]])
    f = np.zeros((3, N))
    eps_p_all, alpha_all = state
    new_ep, new_al = eps_p_all.copy(), alpha_all.copy()
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        e = x + nx * (y + ny * z)
        K, G, sy0, H = params[phase[z, y, x]]
        nodes = []
        for cz, cy, cx in itertools.product((0, 1), repeat=3):
            nodes.append(((x + cx) % nx + nx * (((y + cy) % ny) + ny * ((z + cz) % nz)),
                          (cx, cy, cz)))
        for q, (pz, py, px) in enumerate(itertools.product(pts, repeat=3)):
            xi = (px, py, pz)
            grads = []
            for I, c in nodes:
                val = [xi[k] if c[k] else 1 - xi[k] for k in range(3)]
                dv = [1.0 if c[k] else -1.0 for k in range(3)]
                gr = np.array([dv[0] * val[1] * val[2], val[0] * dv[1] * val[2],
                               val[0] * val[1] * dv[2]]) / h
                grads.append((I, gr))
            Gu = np.zeros((3, 3))
            for I, gr in grads:
                Gu += np.outer(U[:, I], gr)
            eps = 0.5 * (Gu + Gu.T) + Et
            ep = eps_p_all[e, q]
            s_tr = 2 * G * (eps - np.trace(eps) / 3 * np.eye(3) - ep)
            q_tr = math.sqrt(1.5 * np.sum(s_tr * s_tr))
            fy = q_tr - (sy0 + H * alpha_all[e, q])
            s = s_tr
            if fy > 0:
                da = fy / (3 * G + H)
                s = s_tr * (1 - 3 * G * da / q_tr)
                new_ep[e, q] = ep + 1.5 * da * s_tr / q_tr
                new_al[e, q] = alpha_all[e, q] + da
            sig = K * np.trace(eps) * np.eye(3) + s
            w = h.prod() / 8
            for I, gr in grads:
                f[:, I] += w * sig @ gr
    return f.ravel(), (new_ep, new_al)


def test_oracle_internal_force_matches_brute_force():
    n = (3, 3, 2)
    rng = np.random.default_rng(7)
    phase = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    params = np.stack([_params(1.0, 0.3, 0.0015, 0.005), _params(3.0, 0.25, 0.003, 0.01)])
    pp = op.PlasticProblem(n, phase, params)
    u = rng.normal(scale=0.0003, size=3 * pp.prob.N)
    E = np.array([0.0012, -0.0008, 0.0004, 0.0006, -0.0004, 0.0008])
    eps = op.strain_at_qp(pp, u, E)
    Kq, Gq, syq, Hq = pp.qp_params()
    sig, _, _, _, plastic = op.return_mapping(eps, np.zeros(eps.shape), np.zeros(eps.shape[:2]),
                                              Kq, Gq, syq, Hq)
    assert 0 < plastic.mean() < 1
    fo = op.internal_force(pp, sig)
    N = pp.prob.N
    fb, _ = _brute_residual(n, phase, params, u, E,
                            (np.zeros((N, 8, 3, 3)), np.zeros((N, 8))))
    assert np.abs(fo - fb).max() <= 1e-13 * np.abs(fb).max()


def test_newton_matches_dense_newton_on_brute_residual():
    """Two increments on a 3x3x2 grid: the oracle's Newton-PCG (assembled
    tangent, FFT-free naive-DFT preconditioner) against a dense Newton on
    the brute-force residual with a central-difference Jacobian and
    least-squares steps, each committing its own internal variables."""
    n = (3, 3, 2)
    rng = np.random.default_rng(11)
    phase = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    params = np.stack([_params(1.0, 0.3, 0.0015, 0.005), _params(3.0, 0.25, 0.003, 0.01)])
    pp = op.PlasticProblem(n, phase, params)
    Ef = np.array([0.006, -0.004, 0.0, 0.002, 0.0, 0.001])
    u_o, ep_o, al_o, res = op.newton_solve(pp, Ef, 2, eta_nw=1e-12, eta_cg=1e-13)
    assert all(r.converged for r in res)
    N = pp.prob.N
    state = (np.zeros((N, 8, 3, 3)), np.zeros((N, 8)))
    u = np.zeros(3 * N)
    for k in (1, 2):
        E = Ef * k / 2
        for it in range(30):
            r, _ = _brute_residual(n, phase, params, u, E, state)
            if np.abs(r).max() <= 1e-15:
                break
            J = np.zeros((3 * N, 3 * N))
            hstep = 1e-7
            for j in range(3 * N):
                d = np.zeros(3 * N)
                d[j] = hstep
                J[:, j] = (_brute_residual(n, phase, params, u + d, E, state)[0]
                           - _brute_residual(n, phase, params, u - d, E, state)[0]) / (2 * hstep)
            du = np.linalg.lstsq(J, -r, rcond=1e-10)[0]
            u = u + du
            u = (u.reshape(3, N) - u.reshape(3, N).mean(axis=1, keepdims=True)).ravel()
            if np.linalg.norm(du) <= 1e-12 * np.linalg.norm(u):
                break
        _, state = _brute_residual(n, phase, params, u, E, state)
    assert np.linalg.norm(u_o - u) <= 1e-7 * np.linalg.norm(u)
    assert np.abs(al_o - state[1]).max() <= 1e-7 * np.abs(state[1]).max()
    assert (al_o > 0).sum() == (state[1] > 0).sum() > 0


def test_newton_converges_quadratically():
    pp = _spheres_case((8, 8, 8), 2, contrast=3.0)
    E = np.array([0.006, -0.006, 0.0, 0.0, 0.0, 0.0])
    _, _, _, res = op.newton_solve(pp, E, 1, eta_nw=1e-11, eta_cg=1e-13)
    r = res[0].du_ratios
    assert res[0].converged and 3 <= len(r) <= 8
    assert res[0].plastic_fraction > 0.2
    # each step at least squares the previous (with a constant) once in the
    # asymptotic range
    for a, b in zip(r[1:-1], r[2:]):
        if a < 1e-3:
            assert b <= 10 * a * a + 1e-13


def test_mean_tangent_of_elastic_points_is_the_mean_stiffness():
    pp = _spheres_case((6, 6, 6), 3, contrast=4.0)
    Kq, Gq, syq, Hq = pp.qp_params()
    eps = np.zeros((pp.prob.N, 8, 6))
    _, C, _, _, _ = op.return_mapping(eps, eps, np.zeros((pp.prob.N, 8)), Kq, Gq, syq, Hq)
    assert np.abs(op.mean_tangent(pp, C) - oracle.mean_material(pp.prob)).max() <= 1e-14 * 4
