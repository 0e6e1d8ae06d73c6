"""Planted mistakes in the oracle must fail at least one pin.

Each case patches a deliberately wrong variant into the oracle (on the CPU,
inside this test only) and runs a set of pins from test_oracle.py; the pins
must raise.  This shows the pins are strong enough to catch a dropped term,
a wrong sign, a wrong index or a transposed operand.
"""
import numpy as np
import pytest

from oracle import cg as ocg
from oracle import wilson
from oracle.gamma import GAMMA, IDENTITY4

import test_oracle as T


def _hop(mutation):
    """A copy of the stencil's hopping term with one planted mistake."""

    def hopping_4d(U4, psi4, fwd_sign, antiperiodic_t=True):
        out = np.zeros_like(psi4)
        nT = psi4.shape[0]
        for mu in range(4):
            if mutation == "drop_direction" and mu == 2:
                continue
            ax = {0: 3, 1: 2, 2: 1, 3: 0}[mu]
            Umu = U4[..., mu, :, :]
            fwd = np.roll(psi4, -1, axis=ax)
            if mu == 3 and antiperiodic_t and mutation != "no_antiperiodic":
                fwd[0 if mutation == "boundary_at_t0" else nT - 1] *= -1.0
            if mutation == "transposed_link":
                Uf = np.einsum("...ba,...sb->...sa", Umu, fwd)
            else:
                Uf = np.einsum("...ab,...sb->...sa", Umu, fwd)
            out += np.einsum("st,...tc->...sc", IDENTITY4 + fwd_sign * GAMMA[mu], Uf)
            Ub = np.roll(Umu, +1, axis=ax) if mutation == "shifted_back_link" else Umu
            w = np.einsum("...ba,...sb->...sa", Ub.conj(), psi4)
            bwd = np.roll(w, +1, axis=ax)
            if mu == 3 and antiperiodic_t and mutation not in ("no_antiperiodic",
                                                              "boundary_forward_only"):
                bwd[1 if mutation == "boundary_at_t0" else 0] *= -1.0
            sgn = fwd_sign if mutation == "same_projector" else -fwd_sign
            out += np.einsum("st,...tc->...sc", IDENTITY4 + sgn * GAMMA[mu], bwd)
        return out

    return hopping_4d


PINS = [
    lambda: T.test_stencil_equals_dense((2, 2, 2, 4), False),
    lambda: T.test_fft_propagator_vs_cg((4, 4, 4, 4)),
    lambda: T.test_gauge_covariance(False),
    lambda: T.test_plane_wave_eigen((4, 4, 4, 4), np.random.default_rng(1)),
    lambda: T.test_adjoint_dot_and_gamma5((4, 4, 4, 4)),
    lambda: T.test_translation_covariance((0, 0, 0, 3), True, False),
]


def _some_pin_fails():
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            return True
    return False


def test_pins_pass_unmutated():
    assert not _some_pin_fails()


@pytest.mark.parametrize("mutation", ["drop_direction", "no_antiperiodic", "transposed_link",
                                      "shifted_back_link", "same_projector", "boundary_at_t0",
                                      "boundary_forward_only"])
def test_stencil_mutation_caught(monkeypatch, mutation):
    monkeypatch.setattr(wilson, "hopping_4d", _hop(mutation))
    assert _some_pin_fails()


@pytest.mark.parametrize("mutation", ["boundary_at_t0", "boundary_forward_only"])
def test_translation_pin_alone_catches_boundary_mistakes(monkeypatch, mutation):
    monkeypatch.setattr(wilson, "hopping_4d", _hop(mutation))
    with pytest.raises(AssertionError):
        T.test_translation_covariance((0, 0, 0, 3), True, False)


def test_swapped_projectors_caught(monkeypatch):
    monkeypatch.setattr(wilson, "GAMMA", -GAMMA)
    assert _some_pin_fails()


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_cg_wrong_step_length_caught(monkeypatch):
    real_dot = ocg._dot_re
    calls = {"n": 0}

    def bad_dot(a, b):
        # every second call is ||D p||^2: plant ||D p||^2 * 1.01
        calls["n"] += 1
        v = real_dot(a, b)
        return v * 1.01 if calls["n"] % 2 == 0 else v

    monkeypatch.setattr(ocg, "_dot_re", bad_dot)
    with pytest.raises(AssertionError):
        T.test_cg_vs_lapack_tiny((2, 2, 2, 2), 1, 0.12)


def test_cgne_swapped_operators_caught(monkeypatch):
    # CG on D^dag D y = b with x = D y (operators exchanged) must fail the pin
    real = ocg.cgne
    monkeypatch.setattr(ocg, "cgne", lambda mv, mvd, b, **kw: real(mvd, mv, b, **kw))
    with pytest.raises(AssertionError):
        T.test_cgne_vs_lapack_tiny((2, 2, 2, 4), 3, 0.124)


def _lanczos(mutation):
    """A copy of the Lanczos condition estimate with one planted mistake."""

    def lanczos_condition(alphas, betas):
        n = len(alphas)
        T = np.zeros((n, n))
        for k in range(n):
            if mutation == "diag_same_index":
                T[k, k] = 1.0 / alphas[k] + (betas[k] / alphas[k] if k > 0 else 0.0)
            else:
                T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
            if k + 1 < n:
                off = betas[k] if mutation == "no_sqrt" else np.sqrt(betas[k])
                T[k, k + 1] = T[k + 1, k] = off / alphas[k]
        ev = np.linalg.eigvalsh(T)
        return float(ev[-1] / ev[0])

    return lanczos_condition


LANCZOS_PINS = [
    lambda: T.test_lanczos_condition_vs_dense_eigenvalues((2, 2, 2, 2), 1, 0.12, T.synth.HAAR),
    lambda: T.test_lanczos_condition_free_field_closed_form(),
]


@pytest.mark.parametrize("mutation", ["none", "no_sqrt", "diag_same_index"])
def test_lanczos_mutation_caught(monkeypatch, mutation):
    monkeypatch.setattr(ocg, "lanczos_condition", _lanczos(mutation))
    failed = False
    for pin in LANCZOS_PINS:
        try:
            pin()
        except AssertionError:
            failed = True
    assert failed == (mutation != "none")
