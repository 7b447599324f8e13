"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks it against an
independent route (closed forms, a library routine, dense linear algebra,
brute-force quadrature of the FE interpolant in tensor notation, invariants
the paper states).
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle.assembly import Problem, assemble_stiffness, rhs
from oracle.naive_dft import dft, idft
from oracle.pcg import lanczos_ritz_values, pcg
from oracle.precond import Preconditioner, reference_symbol
from synth import isotropic_conductivity, isotropic_mandel, laminate, spheres
from tests.helpers_tensor import isotropic_tensor, lame, mandel_to_tensor, random_spd

RNG = np.random.default_rng(12345)


def two_phase(n, problem, elem, phase, C0, C1):
    return Problem(n, problem, elem, phase=phase.astype(np.uint8), mat=np.stack([C0, C1]))


# ---------------------------------------------------------------- elements

@pytest.mark.parametrize("name", ["hex8", "quad4", "tri2"])
def test_partition_of_unity_and_weights(name):
    el = oracle.element(name)
    # gradients of shape functions sum to zero at every point (constants are
    # reproduced exactly); weights sum to the pixel volume (Fig. tiling).
    assert np.abs(el.grad_ref.sum(axis=1)).max() < 1e-15
    assert abs(el.wfrac.sum() - 1.0) < 1e-15


def test_two_point_gauss_exact_for_quadratics():
    el = oracle.element("quad4")
    xs = np.unique(el.qp_ref[:, 0])
    # int_0^1 xi^2 = 1/3 and int_0^1 xi^3 = 1/4 with weights 1/2 each
    assert abs(0.5 * (xs ** 2).sum() - 1.0 / 3.0) < 1e-15
    assert abs(0.5 * (xs ** 3).sum() - 0.25) < 1e-15


# ---------------------------------------------- energy by an independent route

def _interp_multilinear(vals, xi):
    """vals[a0, a1(, a2)] corner values; multilinear interpolation."""
    dim = vals.ndim
    out = 0.0
    for a in itertools.product((0, 1), repeat=dim):
        w = 1.0
        for k in range(dim):
            w *= xi[k] if a[k] else 1.0 - xi[k]
        out += vals[a] * w
    return out


def _interp_tri2(vals, xi):
    u00, u10, u01, u11 = vals[0, 0], vals[1, 0], vals[0, 1], vals[1, 1]
    if xi[1] <= xi[0]:   # lower triangle (0,0)-(1,0)-(1,1)
        return u00 + (u10 - u00) * xi[0] + (u11 - u10) * xi[1]
    return u00 + (u11 - u01) * xi[0] + (u01 - u00) * xi[1]


def _energy_brute_force(prob, u, Ctensor_of_voxel):
    """sum_e int_e grad(u):C:grad(u) with the FE interpolant evaluated
    directly, its gradient by central differences (exact for functions that
    are linear along the difference direction) and a 3-point Gauss-Legendre
    rule per axis (tensor elements) or the triangle area (tri2)."""
    dim, h = prob.dim, prob.h
    nd = prob.ndof_node
    ug = u.reshape((nd,) + prob.grid_shape)
    g3, w3 = np.polynomial.legendre.leggauss(3)
    g3, w3 = 0.5 * (g3 + 1.0), 0.5 * w3
    if prob.elem == "tri2":
        pts = [((2 / 3, 1 / 3), 0.5), ((1 / 3, 2 / 3), 0.5)]
        interp = _interp_tri2
    else:
        pts = [(p, np.prod(w)) for p, w in zip(itertools.product(g3, repeat=dim),
                                               itertools.product(w3, repeat=dim))]
        interp = _interp_multilinear
    delta = 0.05
    total = 0.0
    Vp = float(np.prod(h))
    for e in itertools.product(*[range(n) for n in prob.n]):
        corner_vals = np.zeros((nd,) + (2,) * dim)
        for a in itertools.product((0, 1), repeat=dim):
            node = tuple((e[k] + a[k]) % prob.n[k] for k in range(dim))
            for c in range(nd):
                corner_vals[(c,) + a] = ug[(c,) + node[::-1]]
        Ct = Ctensor_of_voxel(e)
        for xi, w in pts:
            G = np.zeros((nd, dim))
            for beta in range(dim):
                xp = list(xi); xm = list(xi)
                xp[beta] += delta; xm[beta] -= delta
                for c in range(nd):
                    G[c, beta] = (interp(corner_vals[c], xp) - interp(corner_vals[c], xm)) / (2 * delta * h[beta])
            if nd == 1:
                dens = G[0] @ Ct @ G[0]
            else:
                eps = 0.5 * (G + G.T)
                dens = np.einsum("ij,ijkl,kl->", eps, Ct, eps)
            total += w * Vp * dens
    return total


@pytest.mark.parametrize("elem,problem,n", [
    ("hex8", "elastic", (4, 3, 5)), ("hex8", "scalar", (4, 5, 3)),
    ("quad4", "elastic", (5, 4)), ("quad4", "scalar", (4, 6)),
    ("tri2", "elastic", (5, 4)), ("tri2", "scalar", (4, 6))])
def test_energy_matches_brute_force_quadrature(elem, problem, n):
    rng = np.random.default_rng(7)
    dim = len(n)
    phase = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    if problem == "elastic":
        M0 = random_spd(3 * dim - 3, rng)
        M1 = random_spd(3 * dim - 3, rng)
        tens = [mandel_to_tensor(M0, dim), mandel_to_tensor(M1, dim)]
    else:
        M0 = random_spd(dim, rng)
        M1 = random_spd(dim, rng)
        tens = [M0, M1]
    prob = Problem(n, problem, elem, phase=phase, mat=np.stack([M0, M1]),
                   l=tuple(0.7 + 0.3 * k for k in range(dim)))
    K = assemble_stiffness(prob)
    u = rng.standard_normal(prob.ndof_node * prob.N)
    e_oracle = u @ (K @ u)
    e_brute = _energy_brute_force(prob, u, lambda e: tens[phase[e[::-1]]])
    assert abs(e_oracle - e_brute) <= 1e-12 * abs(e_brute)
    assert abs(K - K.T).max() <= 1e-14 * abs(K).max()


def test_isotropic_mandel_table_matches_lame_tensor():
    lam, mu = lame(3.0, 0.27)
    T = mandel_to_tensor(isotropic_mandel(3.0, 0.27), 3)
    assert np.abs(T - isotropic_tensor(lam, mu)).max() < 1e-14


# ----------------------------------------------------------- naive DFT

def test_naive_dft_matches_library_fft():
    x = RNG.standard_normal((6, 4, 9)) + 1j * RNG.standard_normal((6, 4, 9))
    assert np.abs(dft(x) - np.fft.fftn(x)).max() < 1e-12
    assert np.abs(idft(x) - np.fft.ifftn(x)).max() < 1e-14


# ------------------------------------------------------ Fourier symbol (P6)

def _m(theta, h):
    return h * (2.0 + np.cos(theta)) / 3.0


def _s(theta, h):
    return (2.0 - 2.0 * np.cos(theta)) / h


def _symbol_tensor_element(n, l, Ct):
    """Closed form of K^ for Q1 elements, exact integration: K^_ag =
    sum_bd C_abgd G_bd with G_bb = s(theta_b) prod m(theta_other) and
    G_bd = sin(theta_b) sin(theta_d) prod_{other} m(theta) (b != d)."""
    dim = len(n)
    h = np.array(l) / np.array(n)
    th = np.meshgrid(*[2 * np.pi * np.arange(k) / k for k in n[::-1]], indexing="ij")[::-1]
    G = np.zeros((dim, dim) + tuple(n[::-1]))
    for b in range(dim):
        for d in range(dim):
            val = np.ones(tuple(n[::-1]))
            for k in range(dim):
                if b == d == k:
                    val = val * _s(th[k], h[k])
                elif k == b or k == d:
                    val = val * np.sin(th[k])
                else:
                    val = val * _m(th[k], h[k])
            G[b, d] = val
    if Ct.ndim == 2:    # scalar conductivity
        return np.einsum("bd,bd...->...", Ct, G)[..., None, None]
    return np.moveaxis(np.einsum("abgd,bd...->...ag", Ct, G), (-2, -1), (-2, -1))


@pytest.mark.parametrize("problem", ["scalar", "elastic"])
def test_symbol_hex8_closed_form(problem):
    rng = np.random.default_rng(3)
    n, l = (5, 4, 6), (1.0, 0.8, 1.3)
    if problem == "elastic":
        M = random_spd(6, rng)
        Ct = mandel_to_tensor(M, 3)
    else:
        M = random_spd(3, rng)
        Ct = M
    prob = Problem(n, problem, "hex8", phase=np.zeros(n[::-1], np.uint8), mat=M[None], l=l)
    Khat = reference_symbol(prob, M).reshape(tuple(n[::-1]) + (prob.ndof_node,) * 2)
    ref = _symbol_tensor_element(n, l, Ct)
    assert np.abs(Khat - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(Khat.imag).max() < 1e-14 * np.abs(ref).max()
    assert np.abs(Khat[0, 0, 0]).max() < 1e-14 * np.abs(ref).max()


def test_symbol_quad4_closed_form():
    rng = np.random.default_rng(4)
    n, l = (6, 5), (1.0, 0.6)
    M = random_spd(3, rng)
    prob = Problem(n, "elastic", "quad4", phase=np.zeros(n[::-1], np.uint8), mat=M[None], l=l)
    Khat = reference_symbol(prob, M).reshape(tuple(n[::-1]) + (2, 2))
    ref = _symbol_tensor_element(n, l, mandel_to_tensor(M, 2))
    assert np.abs(Khat - ref).max() < 1e-12 * np.abs(ref).max()


def test_symbol_tri2_is_five_point_laplacian():
    n = (8, 6)
    k = 2.5
    prob = Problem(n, "scalar", "tri2", phase=np.zeros(n[::-1], np.uint8),
                   mat=isotropic_conductivity(k, 2)[None])
    Khat = reference_symbol(prob, k * np.eye(2)).reshape(n[::-1])
    t2, t1 = np.meshgrid(2 * np.pi * np.arange(n[1]) / n[1], 2 * np.pi * np.arange(n[0]) / n[0],
                         indexing="ij")
    # right triangles: the hypotenuse couples nothing (cot 90 deg = 0), so
    # the stencil is the anisotropic 5-point Laplacian
    h1, h2 = 1.0 / n[0], 1.0 / n[1]
    ref = k * ((h2 / h1) * (2.0 - 2.0 * np.cos(t1)) + (h1 / h2) * (2.0 - 2.0 * np.cos(t2)))
    assert np.abs(Khat - ref).max() < 1e-13 * k


# -------------------------------------------- preconditioner = pinv(Kref)

@pytest.mark.parametrize("elem,problem,n", [("hex8", "elastic", (4, 4, 3)),
                                            ("tri2", "scalar", (6, 4)),
                                            ("hex8", "scalar", (3, 4, 5))])
def test_preconditioner_is_dense_pseudo_inverse(elem, problem, n):
    rng = np.random.default_rng(5)
    m = 3 * len(n) - 3 if problem == "elastic" else len(n)
    Cref = random_spd(m, rng)
    prob = Problem(n, problem, elem, phase=np.zeros(n[::-1], np.uint8), mat=Cref[None])
    Kref = assemble_stiffness(prob, uniform=Cref).toarray()
    P = np.linalg.pinv(Kref, rcond=1e-10)
    M = Preconditioner(prob, Cref)
    for _ in range(3):
        r = rng.standard_normal(Kref.shape[0])
        z = M.apply(r)
        zd = P @ r
        assert np.abs(z - zd).max() < 1e-11 * np.abs(zd).max()


# ----------------------------------------------------- P1 homogeneous medium

def test_homogeneous_medium_returns_macroscopic_field():
    n = (4, 5, 6)
    C0 = isotropic_mandel(2.0, 0.25)
    prob = Problem(n, "elastic", "hex8", phase=np.zeros(n[::-1], np.uint8), mat=C0[None])
    loads = np.eye(6)
    # D^T W annihilates uniform fields: b = 0 up to cancellation roundoff
    # (relative to the force one voxel puts on one node, ~ |C| h^2)
    scale = np.abs(C0).max() * prob.h.prod() / prob.h.min()
    for E in loads:
        assert np.abs(rhs(prob, E)).max() < 1e-15 * scale
    # u = 0 then returns the macroscopic field: C_hom = C0 exactly
    zero = [np.zeros(3 * prob.N)] * 6
    assert np.abs(oracle.homogenized_energy(prob, loads, zero) - C0).max() < 1e-13 * np.abs(C0).max()
    H, sols, res = oracle.homogenize(prob, loads, 1e-10, itmax=20)
    assert np.abs(H - C0).max() < 1e-13 * np.abs(C0).max()


# --------------------------------------- P2 C = Cref: one PCG iteration

@pytest.mark.parametrize("elem,problem,n", [("hex8", "elastic", (5, 4, 4)),
                                            ("tri2", "scalar", (8, 8))])
def test_reference_equals_material_converges_in_one_iteration(elem, problem, n):
    rng = np.random.default_rng(9)
    m = 3 * len(n) - 3 if problem == "elastic" else len(n)
    C = random_spd(m, rng)
    prob = Problem(n, problem, elem, phase=np.zeros(n[::-1], np.uint8), mat=C[None])
    K = assemble_stiffness(prob)
    M = Preconditioner(prob, C)
    nd = prob.ndof_node
    b = rng.standard_normal(nd * prob.N).reshape(nd, -1)
    b = (b - b.mean(axis=1, keepdims=True)).ravel()
    res = pcg(lambda v: K @ v, M.apply, b, 1e-12, nd=nd)
    assert res.iterations == 1 and res.status == 0
    # M^+ K is the identity on zero-mean vectors
    x = rng.standard_normal(nd * prob.N).reshape(nd, -1)
    x = (x - x.mean(axis=1, keepdims=True)).ravel()
    assert np.abs(M.apply(K @ x) - x).max() < 1e-11


# -------------------------------------------------------- P3 laminates

def _laminate_scalar(kvals, frac_axis):
    k = np.asarray(kvals, float)
    return 1.0 / np.mean(1.0 / k), np.mean(k)


@pytest.mark.parametrize("elem,n", [("hex8", (6, 5, 4)), ("tri2", (6, 4)), ("quad4", (5, 6))])
@pytest.mark.parametrize("axis", [0, 1])
def test_laminate_scalar_closed_form(elem, n, axis):
    dim = len(n)
    rng = np.random.default_rng(11 + axis)
    layers = rng.integers(0, 2, size=n[axis])
    layers[0], layers[1] = 0, 1
    kv = (1.0, 37.0)
    phase = laminate(n, axis, layers)
    prob = two_phase(n, "scalar", elem, phase, kv[0] * np.eye(dim), kv[1] * np.eye(dim))
    H, _, _ = oracle.homogenize(prob, np.eye(dim), 1e-13)
    kl = np.array([kv[v] for v in layers])
    harm, arith = 1.0 / np.mean(1.0 / kl), np.mean(kl)
    ref = arith * np.eye(dim)
    ref[axis, axis] = harm
    assert np.abs(H - ref).max() < 1e-11 * arith


_NSET = {0: [0, 4, 5], 1: [1, 3, 5], 2: [2, 3, 4]}


def _laminate_elastic(Cs, normal):
    """Classical laminate formula in an orthonormal (Mandel) basis: strain
    components tangential to the layers (p-set) are continuous, tractions
    (n-set stress components) are continuous."""
    nset = _NSET[normal]
    pset = [i for i in range(6) if i not in nset]
    inv_nn = [np.linalg.inv(C[np.ix_(nset, nset)]) for C in Cs]
    Hnn = np.linalg.inv(np.mean(inv_nn, axis=0))
    A = np.mean([iv @ C[np.ix_(nset, pset)] for iv, C in zip(inv_nn, Cs)], axis=0)
    Bm = np.mean([C[np.ix_(pset, nset)] @ iv for iv, C in zip(inv_nn, Cs)], axis=0)
    Hpp = (np.mean([C[np.ix_(pset, pset)] - C[np.ix_(pset, nset)] @ iv @ C[np.ix_(nset, pset)]
                    for iv, C in zip(inv_nn, Cs)], axis=0) + Bm @ Hnn @ A)
    H = np.zeros((6, 6))
    H[np.ix_(nset, nset)] = Hnn
    H[np.ix_(nset, pset)] = Hnn @ A
    H[np.ix_(pset, nset)] = (Hnn @ A).T
    H[np.ix_(pset, pset)] = Hpp
    return H


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_elastic_closed_form_anisotropic(axis):
    rng = np.random.default_rng(20 + axis)
    n = (5, 4, 6)
    layers = rng.integers(0, 2, size=n[axis])
    layers[0], layers[-1] = 0, 1
    C0 = random_spd(6, rng, 5.0)
    C1 = 40.0 * random_spd(6, rng, 5.0)
    phase = laminate(n, axis, layers)
    prob = two_phase(n, "elastic", "hex8", phase, C0, C1)
    H, _, _ = oracle.homogenize(prob, np.eye(6), 1e-13)
    ref = _laminate_elastic([C0 if v == 0 else C1 for v in layers], axis)
    assert np.abs(H - ref).max() < 1e-11 * np.abs(ref).max()


# ------------------------------------------------ P4 dense direct solve

@pytest.mark.parametrize("elem,problem,n", [("hex8", "elastic", (4, 4, 4)),
                                            ("tri2", "scalar", (4, 4)),
                                            ("quad4", "elastic", (4, 4))])
def test_pcg_matches_dense_least_squares(elem, problem, n):
    rng = np.random.default_rng(31)
    dim = len(n)
    phase = rng.integers(0, 2, size=n[::-1])
    m = 3 * dim - 3 if problem == "elastic" else dim
    C0 = random_spd(m, rng)
    C1 = 30.0 * random_spd(m, rng)
    prob = two_phase(n, problem, elem, phase, C0, C1)
    K = assemble_stiffness(prob)
    Kd = K.toarray()
    Cref = oracle.mean_material(prob)
    M = Preconditioner(prob, Cref)
    for E in np.eye(m)[:2]:
        b = rhs(prob, E)
        res = pcg(lambda v: K @ v, M.apply, b, 1e-14, nd=prob.ndof_node)
        x_ls = np.linalg.lstsq(Kd, b, rcond=1e-12)[0]   # minimum-norm = zero mean
        assert np.abs(res.x - x_ls).max() < 1e-10 * np.abs(x_ls).max()


# ------------------------------------ reference material = mean (Sec. 6.2)

@pytest.mark.parametrize("elem,problem,n,l", [("hex8", "elastic", (5, 4, 3), (1.0, 2.0, 0.5)),
                                              ("tri2", "scalar", (6, 4), None),
                                              ("quad4", "elastic", (3, 5), (3.0, 1.0))])
def test_mean_material_two_phase_closed_form(elem, problem, n, l):
    """The quadrature-weighted mean of an element-wise constant material is
    (1 - f) C0 + f C1 with f the inclusion's share of the pixels: every
    pixel carries the same total weight V_p (the weights of a stencil sum
    to the pixel volume), so the mean depends only on the counts.  f comes
    from integer counts here, not from the oracle's weights."""
    rng = np.random.default_rng(41)
    dim = len(n)
    m = 3 * dim - 3 if problem == "elastic" else dim
    phase = rng.integers(0, 2, size=n[::-1])
    C0, C1 = random_spd(m, rng), 17.0 * random_spd(m, rng)
    prob = Problem(n, problem, elem, phase=phase.astype(np.uint8), mat=np.stack([C0, C1]), l=l)
    n1 = int(np.count_nonzero(phase))
    N = int(np.prod(n))
    want = (N - n1) / N * C0 + n1 / N * C1
    assert np.abs(oracle.mean_material(prob) - want).max() < 1e-14 * np.abs(want).max()


def test_mean_material_of_a_field_is_the_exact_sum():
    """Per-voxel conductivity: the mean is sum(k)/N, checked against
    math.fsum (exactly rounded) on a field whose entries span six decades."""
    rng = np.random.default_rng(43)
    n = (6, 5, 4)
    k = np.exp(rng.uniform(-7.0, 7.0, size=n[::-1]))
    prob = Problem(n, "scalar", "hex8", kfield=k, l=(0.5, 1.0, 3.0))
    want = math.fsum(k.ravel().tolist()) / k.size
    got = oracle.mean_material(prob)
    assert np.abs(got - want * np.eye(3)).max() <= 4e-16 * want


# ------------------------ stress average vs energy form at the exact solution

@pytest.mark.parametrize("elem,problem,n", [("hex8", "elastic", (4, 3, 4)),
                                            ("quad4", "scalar", (5, 4)),
                                            ("tri2", "elastic", (4, 5))])
def test_stress_average_equals_energy_columns_at_exact_solution(elem, problem, n):
    """At the exact discrete solution the test function u_i in the
    equilibrium of u_j makes <D u_i . sigma_j> vanish, so e_i . <sigma_j>
    equals the energy form C_hom[i, j].  The solutions here come from a dense
    least-squares solve of the assembled system, not from PCG."""
    rng = np.random.default_rng(47)
    dim = len(n)
    m = 3 * dim - 3 if problem == "elastic" else dim
    phase = rng.integers(0, 2, size=n[::-1])
    prob = Problem(n, problem, elem, phase=phase.astype(np.uint8),
                   mat=np.stack([random_spd(m, rng), 40.0 * random_spd(m, rng)]))
    Kd = assemble_stiffness(prob).toarray()
    loads = np.eye(m)
    sols = [np.linalg.lstsq(Kd, rhs(prob, E), rcond=1e-12)[0] for E in loads]
    H = oracle.homogenized_energy(prob, loads, sols)
    S = np.stack([oracle.stress_average(prob, E, u) for E, u in zip(loads, sols)], axis=1)
    assert np.abs(S - H).max() < 1e-11 * np.abs(H).max()


def test_stress_average_of_a_laminate_is_the_closed_form():
    """Scalar laminate normal to x: the flux average under a unit gradient
    along the normal is the harmonic mean, across it the arithmetic mean
    (the FE space holds the exact piecewise-linear solution)."""
    kvals = np.array([1.0, 1.0, 7.0, 30.0, 7.0, 2.0])
    n = (6, 4, 3)
    kf = np.broadcast_to(kvals[None, None, :], n[::-1]).copy()
    prob = Problem(n, "scalar", "hex8", kfield=kf)
    Kd = assemble_stiffness(prob).toarray()
    harm, arit = 1.0 / np.mean(1.0 / kvals), np.mean(kvals)
    for j, want in ((0, [harm, 0, 0]), (1, [0, arit, 0])):
        E = np.eye(3)[j]
        u = np.linalg.lstsq(Kd, rhs(prob, E), rcond=1e-12)[0]
        got = oracle.stress_average(prob, E, u)
        assert np.abs(got - np.array(want)).max() < 1e-12 * arit


# ------------------------------------------- P5 Voigt / Reuss and symmetry

def test_discrete_bounds_and_symmetry():
    n = 12
    phase, _, _ = spheres(n, (2.0, 3.5), 0.3, seed=4)
    C0, C1 = isotropic_mandel(1.0, 0.3), isotropic_mandel(50.0, 0.2)
    prob = two_phase((n,) * 3, "elastic", "hex8", phase, C0, C1)
    H, _, _ = oracle.homogenize(prob, np.eye(6), 1e-11)
    f = phase.mean()
    voigt = (1 - f) * C0 + f * C1
    reuss = np.linalg.inv((1 - f) * np.linalg.inv(C0) + f * np.linalg.inv(C1))
    assert np.abs(H - H.T).max() < 1e-12 * np.abs(H).max()
    assert np.linalg.eigvalsh(voigt - H).min() > -1e-10
    assert np.linalg.eigvalsh(H - reuss).min() > -1e-10
    assert np.linalg.eigvalsh(H).min() > 0


# ---------------------------------------- P7 eigenvalue bounds (Sec. 4.3)

def test_ritz_values_inside_guaranteed_bounds_and_iteration_bound():
    n = 14
    phase, _, _ = spheres(n, (2.0, 4.0), 0.3, seed=8)
    C0, C1 = isotropic_mandel(1.0, 0.3), isotropic_mandel(100.0, 0.3)
    prob = two_phase((n,) * 3, "elastic", "hex8", phase, C0, C1)
    K = assemble_stiffness(prob)
    Cref = oracle.mean_material(prob)
    M = Preconditioner(prob, Cref)
    eta = 1e-10
    res = pcg(lambda v: K @ v, M.apply, rhs(prob, np.eye(6)[0]), eta, nd=3)
    lo = min(np.linalg.eigvals(np.linalg.solve(Cref, C)).real.min() for C in (C0, C1))
    hi = max(np.linalg.eigvals(np.linalg.solve(Cref, C)).real.max() for C in (C0, C1))
    ritz = lanczos_ritz_values(res.alphas[:-1], res.betas)
    assert ritz.min() >= lo * (1 - 1e-8) and ritz.max() <= hi * (1 + 1e-8)
    kappa = hi / lo
    assert res.iterations <= math.ceil(0.5 * math.sqrt(kappa) * math.log(2 / eta))


def _nonzero_spectrum(prob, Cref):
    """Nonzero generalized eigenvalues of (K, Kref), i.e. of Kref^+ K, from
    dense matrices restricted to zero-mean fields."""
    import scipy.linalg as sla
    K = assemble_stiffness(prob).toarray()
    Kr = assemble_stiffness(prob, uniform=Cref).toarray()
    nd, N = prob.ndof_node, prob.N
    Z = np.zeros((nd * N, nd))
    for a in range(nd):
        Z[a * N:(a + 1) * N, a] = 1.0
    Q, _ = np.linalg.qr(np.hstack([Z, np.random.default_rng(5).standard_normal((nd * N, nd * N - nd))]))
    B = Q[:, nd:]
    return np.sort(sla.eigh(B.T @ K @ B, B.T @ Kr @ B, eigvals_only=True))


@pytest.mark.parametrize("elem,problem,n,ref", [("hex8", "elastic", (3, 3, 4), "mean"),
                                                ("hex8", "scalar", (4, 3, 3), "random"),
                                                ("quad4", "elastic", (4, 5), "random"),
                                                ("tri2", "scalar", (5, 4), "mean")])
def test_eigen_bounds_enclose_the_dense_spectrum(elem, problem, n, ref):
    """Sec. 4.3: with every nodal bound counted nd times and both lists
    sorted, the k-th nonzero eigenvalue of Kref^+ K lies between the
    (k + nd)-th lower bound and the k-th upper bound (dense eigenvalues)."""
    from oracle import bounds
    rng = np.random.default_rng(53)
    dim = len(n)
    m = 3 * dim - 3 if problem == "elastic" else dim
    mats = np.stack([random_spd(m, rng) * 10.0 ** rng.uniform(-2, 2) for _ in range(3)])
    phase = rng.integers(0, 3, size=n[::-1]).astype(np.uint8)
    prob = Problem(n, problem, elem, phase=phase, mat=mats)
    Cref = oracle.mean_material(prob) if ref == "mean" else random_spd(m, rng)
    mu = _nonzero_spectrum(prob, Cref)
    lo, hi = bounds.node_bounds(prob, Cref)
    L, U = bounds.sorted_bounds(lo, hi, prob.ndof_node)
    nd = prob.ndof_node
    assert np.all(L[nd:] <= mu * (1 + 1e-10))
    assert np.all(mu <= U[:mu.size] * (1 + 1e-10))
    assert mu.max() / mu.min() <= bounds.kappa_bound(lo, hi) * (1 + 1e-10)


def test_eigen_bounds_isotropic_closed_form():
    """Isotropic phases against an isotropic reference: the generalized
    eigenvalues are the bulk ratio (3 lambda + 2 mu)/(3 lambda_r + 2 mu_r)
    once and the shear ratio mu/mu_r five times, so each voxel's pair is
    (min, max) of the two ratios; a node takes the extremes over the eight
    voxels around it."""
    from oracle import bounds
    n = (4, 3, 5)
    rng = np.random.default_rng(57)
    phase = rng.integers(0, 2, size=n[::-1]).astype(np.uint8)
    E, nu = (1.0, 80.0), (0.3, 0.2)
    prob = Problem(n, "elastic", "hex8", phase=phase,
                   mat=np.stack([isotropic_mandel(e, v) for e, v in zip(E, nu)]))
    Er, nur = 10.0, 0.35
    Cref = isotropic_mandel(Er, nur)
    lam = lambda e, v: e * v / ((1 + v) * (1 - 2 * v))
    mu = lambda e, v: e / (2 * (1 + v))
    bulk = [(3 * lam(e, v) + 2 * mu(e, v)) / (3 * lam(Er, nur) + 2 * mu(Er, nur)) for e, v in zip(E, nu)]
    shear = [mu(e, v) / mu(Er, nur) for e, v in zip(E, nu)]
    lo_p = np.array([min(b, s) for b, s in zip(bulk, shear)])
    hi_p = np.array([max(b, s) for b, s in zip(bulk, shear)])
    lo, hi = bounds.node_bounds(prob, Cref)
    # brute force over the voxel neighbourhood of every node
    for I in range(prob.N):
        x, y, z = I % n[0], (I // n[0]) % n[1], I // (n[0] * n[1])
        ph = [phase[(z - cz) % n[2], (y - cy) % n[1], (x - cx) % n[0]]
              for cx, cy, cz in itertools.product((0, 1), repeat=3)]
        assert abs(lo[I] - lo_p[ph].min()) < 1e-13 * lo_p.max()
        assert abs(hi[I] - hi_p[ph].max()) < 1e-13 * hi_p.max()


def test_eigen_bounds_reference_equal_to_material():
    """C = Cref in every voxel: every bound is 1 and the bound on the
    condition number is 1 (the "geometrically optimal" case of Sec. 4.3)."""
    from oracle import bounds
    C = random_spd(6, np.random.default_rng(59))
    prob = Problem((3, 4, 3), "elastic", "hex8", phase=np.zeros((3, 4, 3), np.uint8), mat=C[None])
    lo, hi = bounds.node_bounds(prob, C)
    assert np.abs(lo - 1).max() < 1e-13 and np.abs(hi - 1).max() < 1e-13
    assert abs(bounds.kappa_bound(lo, hi) - 1) < 1e-13
    kf = np.exp(np.random.default_rng(61).uniform(-3, 3, size=(4, 5, 6)))
    prob = Problem((6, 5, 4), "scalar", "hex8", kfield=kf)
    lo, hi = bounds.node_bounds(prob, 2.0 * np.eye(3))
    assert abs(bounds.kappa_bound(lo, hi) - kf.max() / kf.min()) < 1e-12 * kf.max() / kf.min()


# ----------------------------------- P9 translation, permutation, linearity

def test_translation_and_axis_permutation_invariance():
    n = (6, 6, 6)
    phase, _, _ = spheres(6, (1.5, 2.2), 0.25, seed=2)
    C0, C1 = isotropic_mandel(1.0, 0.3), isotropic_mandel(20.0, 0.3)
    base, _, _ = oracle.homogenize(two_phase(n, "elastic", "hex8", phase, C0, C1), np.eye(6), 1e-12)
    shifted, _, _ = oracle.homogenize(
        two_phase(n, "elastic", "hex8", np.roll(phase, (1, 3, 2), axis=(0, 1, 2)), C0, C1),
        np.eye(6), 1e-12)
    assert np.abs(base - shifted).max() < 1e-10 * np.abs(base).max()
    # swap x and y: numpy axes (z, y, x) -> (z, x, y)
    swapped, _, _ = oracle.homogenize(
        two_phase(n, "elastic", "hex8", np.swapaxes(phase, 1, 2), C0, C1), np.eye(6), 1e-12)
    perm = [1, 0, 2, 4, 3, 5]   # 11<->22, 23<->13
    assert np.abs(swapped - base[np.ix_(perm, perm)]).max() < 1e-10 * np.abs(base).max()


def test_linearity_in_the_load():
    n = (5, 6, 4)
    rng = np.random.default_rng(41)
    phase = rng.integers(0, 2, size=n[::-1])
    prob = two_phase(n, "elastic", "hex8", phase, isotropic_mandel(1, 0.3), isotropic_mandel(10, 0.3))
    K = assemble_stiffness(prob)
    M = Preconditioner(prob, oracle.mean_material(prob))
    a = rng.standard_normal(6)
    sols = [pcg(lambda v: K @ v, M.apply, rhs(prob, E), 1e-14, nd=3).x for E in np.eye(6)]
    comb = pcg(lambda v: K @ v, M.apply, rhs(prob, a), 1e-14, nd=3).x
    ref = sum(ai * s for ai, s in zip(a, sols))
    assert np.abs(comb - ref).max() < 1e-10 * np.abs(ref).max()


def test_operator_rows_match_assembled_rows():
    rng = np.random.default_rng(50)
    for elem, problem, n in [("hex8", "elastic", (5, 4, 6)), ("tri2", "scalar", (6, 5))]:
        phase = rng.integers(0, 3, size=n[::-1])
        m = 3 * len(n) - 3 if problem == "elastic" else len(n)
        prob = Problem(n, problem, elem, phase=phase.astype(np.uint8),
                       mat=np.stack([random_spd(m, rng) for _ in range(3)]))
        K = assemble_stiffness(prob)
        u = rng.standard_normal(K.shape[0])
        nodes = rng.choice(prob.N, 17, replace=False)
        full = (K @ u).reshape(prob.ndof_node, prob.N)[:, nodes]
        from oracle.assembly import operator_rows
        assert np.abs(operator_rows(prob, u, nodes) - full).max() < 1e-13 * np.abs(full).max()


def test_stencil_symbol_and_fft_preconditioner_match_dense_forms():
    """The large-grid preconditioner (Alg. 2 symbol as a sum over the nonzero
    impulse-response nodes, numpy FFT) against the assembled Kref with the
    dense DFT matrices, on grids that include a 2-node axis (stencil
    neighbours wrap onto the same node)."""
    from oracle.precond import FFTPreconditioner, stencil_symbol
    rng = np.random.default_rng(51)
    for elem, problem, n in [("hex8", "elastic", (6, 4, 5)), ("hex8", "scalar", (5, 6, 4)),
                             ("hex8", "elastic", (2, 3, 4)), ("quad4", "elastic", (7, 5)),
                             ("tri2", "scalar", (4, 6))]:
        dim = len(n)
        m = dim * (dim + 1) // 2 if problem == "elastic" else dim
        prob = Problem(n, problem, elem, phase=rng.integers(0, 2, size=n[::-1]),
                       mat=np.stack([random_spd(m, rng) for _ in range(2)]))
        Cref = random_spd(m, rng)
        K1 = reference_symbol(prob, Cref)
        K2 = stencil_symbol(prob, Cref)
        assert np.abs(K1 - K2).max() < 1e-13 * np.abs(K1).max()
        r = rng.standard_normal(prob.ndof_node * prob.N)
        z1 = Preconditioner(prob, Cref).apply(r)
        z2 = FFTPreconditioner(prob, Cref).apply(r)
        assert np.abs(z1 - z2).max() < 1e-12 * np.abs(z1).max()


# ------------------------------------------------ initial guess and screen

def test_warm_started_pcg_reaches_dense_solution_and_screen():
    """A guess u0 (the initial displacement of the Newton scheme of Alg. 1):
    PCG from it with the test relative to b.M b reaches the minimum-norm
    dense solution; the exact solution as guess needs no iteration; the
    screen accepts a good guess and rejects a bad one."""
    from oracle.pcg import screened_guess
    rng = np.random.default_rng(41)
    n = (4, 4, 4)
    phase = rng.integers(0, 2, size=n[::-1])
    C0 = random_spd(6, rng)
    prob = two_phase(n, "elastic", "hex8", phase, C0, 20.0 * random_spd(6, rng))
    K = assemble_stiffness(prob)
    M = Preconditioner(prob, oracle.mean_material(prob))
    b = rhs(prob, np.eye(6)[3])
    x_ls = np.linalg.lstsq(K.toarray(), b, rcond=1e-12)[0]
    AK = lambda v: K @ v  # noqa: E731
    nd = prob.ndof_node
    # exact solution shifted by a constant: accepted, zero iterations
    ok, x0, rb, rx = screened_guess(AK, M.apply, b, x_ls + 3.0, nd)
    assert ok and rx < 1e-20 * rb
    res = pcg(AK, M.apply, b, 1e-10, x0=x0, nd=nd, rho_ref=rb)
    assert res.iterations == 0 and np.abs(res.x - x_ls).max() < 1e-12 * np.abs(x_ls).max()
    # perturbed solution: accepted, converges to the same point in fewer steps
    ok, x0, rb, rx = screened_guess(AK, M.apply, b, x_ls + 0.01 * np.abs(x_ls).max() *
                                  rng.standard_normal(b.size), nd)
    assert ok and rx < rb
    warm = pcg(AK, M.apply, b, 1e-12, x0=x0, nd=nd, rho_ref=rb)
    cold = pcg(AK, M.apply, b, 1e-12, nd=nd)
    assert warm.status == 0 and np.abs(warm.x - x_ls).max() < 1e-9 * np.abs(x_ls).max()
    assert warm.iterations < cold.iterations
    assert warm.history[-1] ** 2 * warm.rho0 <= (1e-12) ** 2 * rb * (1 + 1e-12)
    # a guess far worse than zero is rejected
    ok, x0, rb, rx = screened_guess(AK, M.apply, b, 1e3 * rng.standard_normal(b.size), nd)
    assert not ok and rx >= rb and not x0.any()
