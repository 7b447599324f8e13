"""Plant plausible mistakes in the oracle (CPU only) and check that the pins
catch each one: a dropped sqrt(2)/2 on shear rows, Gauss points moved, a
periodic shift taken the wrong way, a dropped quadrature weight, a sign slip in
the right-hand side, an unnormalised inverse DFT, a zero-frequency block
inverted instead of pseudo-inverted, in the large-grid preconditioner a
symbol built from the wrong rows or an unnormalised inverse FFT, and in the
homogenization helpers an unweighted or scaled mean material and a stress
average without the macroscopic strain."""
import sys

import numpy as np
import pytest

import oracle.assembly as asm
import oracle.homog as ohom
import oracle.naive_dft as odft
import oracle.elements as oel
import oracle.precond as opre
from tests import test_oracle_pins as pins


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    except (np.linalg.LinAlgError, FloatingPointError, ValueError):
        return True
    return False


def _all_pin_checks():
    return [
        (pins.test_energy_matches_brute_force_quadrature, ("hex8", "elastic", (4, 3, 5))),
        (pins.test_energy_matches_brute_force_quadrature, ("tri2", "scalar", (4, 6))),
        (pins.test_laminate_elastic_closed_form_anisotropic, (1,)),
        (pins.test_laminate_scalar_closed_form, ("hex8", (6, 5, 4), 0)),
        (pins.test_symbol_hex8_closed_form, ("elastic",)),
        (pins.test_preconditioner_is_dense_pseudo_inverse, ("hex8", "elastic", (4, 4, 3))),
        (pins.test_reference_equals_material_converges_in_one_iteration, ("hex8", "elastic", (5, 4, 4))),
        (pins.test_stencil_symbol_and_fft_preconditioner_match_dense_forms, ()),
    ]


def _caught():
    return any(_fails(fn, *args) for fn, args in _all_pin_checks())


def test_unmutated_oracle_passes_every_check():
    assert not _caught()


def test_catches_wrong_shear_factor(monkeypatch):
    orig = oel.symmetric_gradient_rows

    def bad(dim):
        return [(m, a, b, 1.0 if a != b else c) for (m, a, b, c) in orig(dim)]
    monkeypatch.setattr(asm, "symmetric_gradient_rows", bad)
    assert _caught()


def test_catches_wrong_gauss_points(monkeypatch):
    orig = oel._tensor_element

    def bad(dim, name):
        el = orig(dim, name)
        g = 1.0 / 3.0
        qp = np.where(el.qp_ref < 0.5, g, 1.0 - g)
        grad = np.zeros_like(el.grad_ref)
        for q in range(len(qp)):
            for a in range(len(el.corners)):
                for k in range(dim):
                    v = 1.0 if el.corners[a, k] else -1.0
                    for j in range(dim):
                        if j != k:
                            v *= qp[q, j] if el.corners[a, j] else 1.0 - qp[q, j]
                    grad[q, a, k] = v
        return oel.Element(el.name, dim, el.corners, grad, el.wfrac, qp)
    monkeypatch.setattr(oel, "_tensor_element", bad)
    assert _caught()


def test_catches_shift_in_wrong_direction(monkeypatch):
    def bad(field_grid, corner):
        shift = tuple(-int(c) for c in corner[::-1])
        return np.roll(field_grid, shift, axis=tuple(range(field_grid.ndim)))
    monkeypatch.setattr(asm, "_shift_to_nodes", bad)
    assert _caught()


def test_catches_dropped_quadrature_weight(monkeypatch):
    monkeypatch.setattr(asm, "quadrature_weights", lambda prob: prob.el.wfrac)
    assert _caught()


def test_catches_rhs_sign_slip(monkeypatch):
    orig = asm.rhs
    monkeypatch.setattr(asm, "rhs", lambda prob, E: -orig(prob, E))
    import oracle.homog as hom
    monkeypatch.setattr(hom, "rhs", lambda prob, E: -orig(prob, E))
    assert _caught()


def test_catches_unnormalised_inverse_dft(monkeypatch):
    monkeypatch.setattr(opre, "idft", lambda X, axes=None: odft._apply(X, +1, range(np.ndim(X))))
    assert _caught()


def test_catches_large_grid_symbol_from_wrong_rows(monkeypatch):
    # the impulse response read at one node only, instead of at every
    # neighbour of the impulse
    orig = asm.operator_rows
    monkeypatch.setattr(opre, "operator_rows",
                        lambda prob, u, nodes: orig(prob, u, np.repeat(nodes[:1], len(nodes))))
    assert _caught()


def test_catches_large_grid_unnormalised_inverse_fft(monkeypatch):
    fftn = np.fft.fftn
    monkeypatch.setattr(np.fft, "ifftn", lambda a: np.conj(fftn(np.conj(a))))
    assert _caught()


def test_catches_zero_frequency_inverted(monkeypatch):
    def bad(Khat, rtol=1e-10):
        lam, V = np.linalg.eigh(Khat)
        return np.einsum("fik,fk,fjk->fij", V, 1.0 / lam, V.conj())
    monkeypatch.setattr(opre, "pseudo_inverse_blocks", bad)
    with np.errstate(all="ignore"):
        assert _caught()


# ------------------------------------------------------------ warm-start net
import torch  # noqa: E402

import oracle.convnet as ocn  # noqa: E402
from tests import test_oracle_convnet as npins  # noqa: E402


def _net_pins_fail():
    checks = [npins.test_conv_matches_library_circular_conv3d,
              npins.test_manual_backward_matches_autograd,
              npins.test_loss_closed_form_and_gradient,
              npins.test_gradient_finite_differences]
    return any(_fails(fn) for fn in checks)


def _input_grad_wrong_shift(dy, W):
    dx = None
    for t, (dz, dyy, ddx) in enumerate(ocn.TAPS):
        ds = torch.roll(dy, shifts=(-dz, -dyy, -ddx), dims=(2, 3, 4))
        term = torch.einsum("oc,bozyx->bczyx", W[t], ds)
        dx = term if dx is None else dx + term
    return dx


def _conv_taps_transposed(x, W, b):
    y = b.view(1, -1, 1, 1, 1).expand(x.shape[0], -1, *x.shape[2:]).clone()
    for t, (dz, dy, dx) in enumerate(ocn.TAPS):
        xs = torch.roll(x, shifts=(-dx, -dy, -dz), dims=(2, 3, 4))
        y += torch.einsum("oc,bczyx->bozyx", W[t], xs)
    return y


@pytest.mark.parametrize("name,mutant", [
    ("conv_input_grad", _input_grad_wrong_shift),
    ("conv", _conv_taps_transposed),
    ("loss_grad", lambda O, T: 0.5 * (lambda e: sum(
        2.0 * e - torch.roll(e, 1, d) - torch.roll(e, -1, d) for d in (2, 3, 4)))(O - T)
        * (2.0 / (3.0 * O.numel()))),
    ("up_adjoint", lambda y: ocn.pool(y)),
    ("leaky_grad_from_output", lambda y: torch.ones_like(y)),
])
def test_net_pins_catch_planted_mistake(monkeypatch, name, mutant):
    monkeypatch.setattr(ocn, name, mutant)
    assert _net_pins_fail()


# ------------------------------------------------ mean material and stress

def _mean_pins():
    return [
        (pins.test_mean_material_two_phase_closed_form, ("hex8", "elastic", (5, 4, 3),
                                                         (1.0, 2.0, 0.5))),
        (pins.test_mean_material_of_a_field_is_the_exact_sum, ()),
    ]


def test_unmutated_mean_and_stress_pins_pass():
    assert not any(_fails(fn, *a) for fn, a in _mean_pins())
    assert not _fails(pins.test_stress_average_equals_energy_columns_at_exact_solution,
                      "hex8", "elastic", (4, 3, 4))
    assert not _fails(pins.test_stress_average_of_a_laminate_is_the_closed_form)


def test_catches_unweighted_mean_material(monkeypatch):
    """Mean over the distinct phases instead of over the pixels."""
    def bad(prob):
        if prob.phase is not None:
            return np.mean(prob.mat, axis=0)
        return np.mean(np.asarray(prob.kfield)) * np.eye(prob.dim)
    monkeypatch.setattr(oracle_mod(), "mean_material", bad)
    assert any(_fails(fn, *a) for fn, a in _mean_pins())


def test_catches_mean_material_not_divided_by_the_volume(monkeypatch):
    orig = ohom.mean_material

    def bad(prob):
        return orig(prob) * prob.volume
    monkeypatch.setattr(oracle_mod(), "mean_material", bad)
    assert any(_fails(fn, *a) for fn, a in _mean_pins())


def test_catches_mean_material_with_one_voxel_dropped(monkeypatch):
    orig = ohom.mean_material

    def bad(prob):
        C = prob.voxel_materials()
        return orig(prob) - C[-1] / prob.N
    monkeypatch.setattr(oracle_mod(), "mean_material", bad)
    assert any(_fails(fn, *a) for fn, a in _mean_pins())


def test_catches_stress_average_without_macroscopic_strain(monkeypatch):
    def bad(prob, E, u):
        w = asm.quadrature_weights(prob)
        C = prob.voxel_materials()
        eps = asm.gradient_at_quadrature(prob, u)
        sig = np.einsum("emn,eqn->eqm", C, eps)
        return np.einsum("q,eqm->m", w, sig) / prob.volume
    monkeypatch.setattr(oracle_mod(), "stress_average", bad)
    assert _fails(pins.test_stress_average_equals_energy_columns_at_exact_solution,
                  "hex8", "elastic", (4, 3, 4))
    assert _fails(pins.test_stress_average_of_a_laminate_is_the_closed_form)


def oracle_mod():
    import oracle
    return oracle


# ------------------------------------------------- eigenvalue bounds (Sec. 4.3)

def _bounds_pins():
    return [
        (pins.test_eigen_bounds_enclose_the_dense_spectrum, ("hex8", "elastic", (3, 3, 4), "mean")),
        (pins.test_eigen_bounds_enclose_the_dense_spectrum, ("quad4", "elastic", (4, 5), "random")),
        (pins.test_eigen_bounds_isotropic_closed_form, ()),
        (pins.test_eigen_bounds_reference_equal_to_material, ()),
    ]


def test_unmutated_bounds_pins_pass():
    assert not any(_fails(fn, *a) for fn, a in _bounds_pins())


def test_catches_bounds_without_the_reference(monkeypatch):
    """Eigenvalues of C instead of Cref^-1 C."""
    import oracle.bounds as ob
    import scipy.linalg as sla

    def bad(prob, Cref):
        if prob.phase is not None:
            lam = [np.linalg.eigvalsh(C) for C in prob.mat]
            key = np.asarray(prob.phase).ravel().astype(np.int64)
            return np.array([v.min() for v in lam])[key], np.array([v.max() for v in lam])[key]
        k = np.asarray(prob.kfield, dtype=float).ravel()
        return k, k
    monkeypatch.setattr(ob, "element_pairs", bad)
    assert any(_fails(fn, *a) for fn, a in _bounds_pins())


def test_catches_bounds_from_one_voxel_only(monkeypatch):
    """Support of phi^I taken as the node's own voxel instead of all the
    voxels that share the node."""
    import oracle.bounds as ob

    def bad(prob, Cref):
        return ob.element_pairs(prob, Cref)
    monkeypatch.setattr(ob, "node_bounds", bad)
    assert any(_fails(fn, *a) for fn, a in _bounds_pins())


def test_catches_bounds_with_min_and_max_swapped(monkeypatch):
    import oracle.bounds as ob
    orig = ob.element_pairs

    def bad(prob, Cref):
        lo, hi = orig(prob, Cref)
        return hi, lo
    monkeypatch.setattr(ob, "element_pairs", bad)
    assert any(_fails(fn, *a) for fn, a in _bounds_pins())


# ------------------------------------------------ elasto-plastic Newton oracle
import oracle.plasticity as opl  # noqa: E402
from tests import test_oracle_plasticity as ppins  # noqa: E402


def _plastic_checks():
    return [
        (ppins.test_pure_shear_closed_form, ()),
        (ppins.test_consistent_tangent_is_the_derivative_of_the_stress_update, ()),
        (ppins.test_oracle_internal_force_matches_brute_force, ()),
        (ppins.test_homogeneous_cell_returns_the_point_response, ()),
        (ppins.test_newton_converges_quadratically, ()),
    ]


def _plastic_caught():
    return any(_fails(fn, *args) for fn, args in _plastic_checks())


def _radial_return(eps, eps_p_n, alpha_n, K, G, sy0, H, hard=2.0 / 3.0, sq=None,
                   thb_full=True):
    """The oracle's stress update with knobs for planted mistakes."""
    sq = opl.SQ23 if sq is None else sq
    ONE, P = opl.ONE, opl.P_DEV
    eps = np.asarray(eps, dtype=float)
    tr = eps[..., 0] + eps[..., 1] + eps[..., 2]
    s_tr = 2.0 * G[..., None] * (eps - (tr / 3.0)[..., None] * ONE - eps_p_n)
    ns = np.sqrt(np.sum(s_tr * s_tr, axis=-1))
    f = ns - sq * (sy0 + H * alpha_n)
    pl = f > 0.0
    dg = np.where(pl, f / (2.0 * G + hard * H), 0.0)
    n = np.where(pl[..., None], s_tr / np.where(ns > 0, ns, 1.0)[..., None], 0.0)
    sigma = (K * tr)[..., None] * ONE + s_tr - (2.0 * G * dg)[..., None] * n
    th = np.where(pl, 1.0 - 2.0 * G * dg / np.where(ns > 0, ns, 1.0), 1.0)
    thb = np.where(pl, 1.0 / (1.0 + H / (3.0 * G)) - ((1.0 - th) if thb_full else 0.0), 0.0)
    C = (K[..., None, None] * np.outer(ONE, ONE) + (2.0 * G * th)[..., None, None] * P
         - (2.0 * G * thb)[..., None, None] * n[..., :, None] * n[..., None, :])
    return sigma, C, eps_p_n + dg[..., None] * n, alpha_n + sq * dg, pl


def test_unmutated_plasticity_pins_pass(monkeypatch):
    monkeypatch.setattr(opl, "return_mapping", _radial_return)  # same arithmetic
    assert not _plastic_caught()


@pytest.mark.parametrize("name,kw", [
    ("yield radius without sqrt(2/3)", dict(sq=1.0)),
    ("hardening denominator 2G + H", dict(hard=1.0)),
    ("tangent without the (1 - theta) term", dict(thb_full=False)),
])
def test_plasticity_pins_catch_stress_update_mistakes(monkeypatch, name, kw):
    monkeypatch.setattr(opl, "return_mapping",
                        lambda *a: _radial_return(*a, **kw))
    assert _plastic_caught(), name


def test_plasticity_pins_catch_residual_sign_slip(monkeypatch):
    orig = opl.internal_force

    def bad(pp, sigma, with_scale=False):
        out = orig(pp, sigma, with_scale)
        return (-out[0], out[1]) if with_scale else -out
    monkeypatch.setattr(opl, "internal_force", bad)
    assert _plastic_caught()


def test_plasticity_pins_catch_uncommitted_state(monkeypatch):
    """Internal variables never carried to the next increment."""
    orig = opl.return_mapping

    def bad(eps, eps_p_n, alpha_n, *rest):
        s, C, _, _, pl = orig(eps, eps_p_n, alpha_n, *rest)
        return s, C, eps_p_n, alpha_n, pl
    monkeypatch.setattr(opl, "return_mapping", bad)
    assert _fails(ppins.test_newton_matches_dense_newton_on_brute_residual) or _plastic_caught()


# ------------------------------------------------- strain-based scheme oracle
import oracle.strain_based as osbm  # noqa: E402
from tests import test_oracle_strain_based as sbpins  # noqa: E402


def _sb_caught():
    checks = [
        (sbpins.test_green_operator_projects_onto_compatible_fields, (True,)),
        (sbpins.test_identity_reference_gives_least_squares_compatible_part, ()),
        (sbpins.test_strain_iterates_equal_gradients_of_displacement_iterates, (True,)),
    ]
    return any(_fails(fn, *args) for fn, args in checks)


def test_unmutated_strain_based_pins_pass():
    assert not _sb_caught()


def test_sb_pins_catch_divergence_without_weights(monkeypatch):
    orig = osbm.divergence
    monkeypatch.setattr(osbm, "divergence",
                        lambda prob, tau: orig(prob, tau) / prob.voxel_volume * 8.0)
    assert _sb_caught()


def test_sb_pins_catch_green_operator_without_the_reference(monkeypatch):
    orig = osbm.GreenOperator.__init__

    def bad(self, prob, Cref):
        orig(self, prob, np.eye(np.asarray(Cref).shape[0]) * np.trace(Cref) / len(Cref))
        self.Cref = np.asarray(Cref, dtype=float)
    monkeypatch.setattr(osbm.GreenOperator, "__init__", bad)
    assert _sb_caught()


def test_sb_pins_catch_inner_product_without_the_reference(monkeypatch):
    orig = osbm.inner
    monkeypatch.setattr(osbm, "inner", lambda prob, Cref, a, b: orig(prob, np.eye(6), a, b))
    assert _sb_caught()


# ------------------------------------------------- two-node stencil oracle
import oracle.two_node as otn  # noqa: E402
from tests import test_oracle_two_node as tnpins  # noqa: E402


def _tn_caught():
    checks = [
        (tnpins.test_scalar_symbol_closed_form, ()),
        (tnpins.test_fourier_pseudo_inverse_is_dense_pseudo_inverse, ("scalar", True)),
        (tnpins.test_fourier_pseudo_inverse_is_dense_pseudo_inverse, ("elastic", True)),
        (tnpins.test_laminate_closed_form, ("elastic", 0)),
    ]
    return any(_fails(fn, *args) for fn, args in checks)


def test_unmutated_two_node_pins_pass():
    assert not _tn_caught()


def test_two_node_pins_catch_zero_frequency_block_set_to_zero(monkeypatch):
    """The one-node rule K^+(0) = 0 applied to the rank-deficient (not zero)
    two-node block."""
    orig = otn.pseudo_inverse_blocks

    def bad(Khat, rtol=1e-10):
        P = orig(Khat, rtol)
        P[0] = 0.0
        return P
    monkeypatch.setattr(otn, "pseudo_inverse_blocks", bad)
    assert _tn_caught()


def test_two_node_pins_catch_centre_in_the_wrong_place(monkeypatch):
    monkeypatch.setattr(otn, "_position", lambda node: (np.array([0.5, 0.4]) if node[0] == 1
                                                        else np.array(node[1:], dtype=float)))
    assert _tn_caught()


def test_two_node_pins_catch_transposed_symbol(monkeypatch):
    orig = otn.reference_symbol
    monkeypatch.setattr(otn, "reference_symbol",
                        lambda tp, Cref: np.transpose(orig(tp, Cref), (0, 2, 1)))
    assert _tn_caught()


def test_two_node_pins_catch_half_pixel_weight(monkeypatch):
    monkeypatch.setattr(otn.TwoNodeProblem, "weight", lambda self: 0.5 * float(np.prod(self.h)))
    assert _tn_caught()
