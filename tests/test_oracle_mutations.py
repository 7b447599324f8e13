"""Plant plausible mistakes in the oracle (CPU only) and check that the pins
catch each one: a dropped sqrt(2)/2 on shear rows, Gauss points moved, a
periodic shift taken the wrong way, a dropped quadrature weight, a sign slip in
the right-hand side, an unnormalised inverse DFT, a zero-frequency block
inverted instead of pseudo-inverted."""
import sys

import numpy as np
import pytest

import oracle.assembly as asm
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


def test_catches_zero_frequency_inverted(monkeypatch):
    def bad(Khat, rtol=1e-10):
        lam, V = np.linalg.eigh(Khat)
        return np.einsum("fik,fk,fjk->fij", V, 1.0 / lam, V.conj())
    monkeypatch.setattr(opre, "pseudo_inverse_blocks", bad)
    with np.errstate(all="ignore"):
        assert _caught()
