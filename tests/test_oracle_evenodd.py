"""Pins of the oracle's even-odd (Schur complement) solve against dense
linear algebra: the block structure of the dense matrix of Eq. (1), the
dense Schur complement, adjointness, LAPACK solutions, and planted mistakes
that some pin must catch."""
import numpy as np
import pytest

import synth
from oracle import cg, dense, evenodd, wilson


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _blocks(U, dims, k):
    """Dense D and the row/column index sets of even and odd sites."""
    Dm = dense.dense_D(U, dims, k)
    par = evenodd.parity(dims)
    ev = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in np.flatnonzero(par == 0)])
    od = np.concatenate([np.arange(12 * s, 12 * s + 12) for s in np.flatnonzero(par == 1)])
    return Dm, ev, od


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4), (2, 4, 2, 2)])
def test_same_parity_blocks_are_identity(dims):
    U = synth.gauge(dims, 71, synth.HAAR)
    Dm, ev, od = _blocks(U, dims, 0.13)
    assert np.abs(Dm[np.ix_(ev, ev)] - np.eye(len(ev))).max() == 0.0
    assert np.abs(Dm[np.ix_(od, od)] - np.eye(len(od))).max() == 0.0


@pytest.mark.parametrize("dims,dagger", [((2, 2, 2, 4), False), ((2, 2, 2, 4), True),
                                         ((2, 4, 2, 2), False)])
def test_apply_M_equals_dense_schur_complement(dims, dagger):
    U = synth.gauge(dims, 72, synth.EXP)
    k = 0.124
    Dm, ev, od = _blocks(U, dims, k)
    if dagger:
        Dm = Dm.conj().T
    Mdense = Dm[np.ix_(ev, ev)] - Dm[np.ix_(ev, od)] @ Dm[np.ix_(od, ev)]
    v = evenodd.project(synth.gaussian_spinor(dims, 73), evenodd.parity(dims), 0)
    got = dense.flat(evenodd.apply_M(U, v, dims, k, dagger=dagger))
    want = np.zeros_like(got)
    want[ev] = Mdense @ dense.flat(v)[ev]
    assert rel(got, want) < 1e-14


def test_M_adjoint():
    dims = (4, 2, 4, 4)
    U = synth.gauge(dims, 74, synth.EXP)
    par = evenodd.parity(dims)
    u = evenodd.project(synth.gaussian_spinor(dims, 75), par, 0)
    v = evenodd.project(synth.gaussian_spinor(dims, 76), par, 0)
    lhs = wilson.dot(u, evenodd.apply_M(U, v, dims, 0.13))
    rhs = wilson.dot(evenodd.apply_M(U, u, dims, 0.13, dagger=True), v)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


@pytest.mark.parametrize("dims,seed,kappa", [((2, 2, 2, 2), 1, 0.12), ((2, 2, 2, 4), 3, 0.124),
                                             ((4, 2, 2, 2), 5, 0.15)])
def test_evenodd_solve_vs_lapack(dims, seed, kappa):
    U = synth.gauge(dims, seed, synth.HAAR)
    b = synth.gaussian_spinor(dims, seed + 50)
    x, it, info = evenodd.solve(U, b, dims, kappa, tol=1e-13)
    want = dense.unflat(np.linalg.solve(dense.dense_D(U, dims, kappa), dense.flat(b)))
    assert info["converged"] and rel(x, want) < 1e-11


def test_evenodd_config1_and_fewer_iterations():
    """4^4 configuration: the Schur solve reaches the dense solution, with
    fewer CG iterations than CGNR on the full lattice."""
    dims = (4, 4, 4, 4)
    U = synth.gauge(dims, 1, synth.HAAR)
    b = synth.point_source(dims, 0, 0, 0)
    k = 0.12
    x, it, _ = evenodd.solve(U, b, dims, k, tol=1e-10)
    want = dense.unflat(np.linalg.solve(dense.dense_D(U, dims, k), dense.flat(b)))
    assert rel(x, want) < 1e-9
    _, it_full, _ = cg.cgnr(lambda v: wilson.apply_D(U, v, dims, k),
                            lambda v: wilson.apply_Ddag(U, v, dims, k), b, tol=1e-10)
    assert it < it_full


def test_evenodd_plus_kappa_sign():
    dims = (2, 2, 2, 4)
    U = synth.gauge(dims, 7, synth.HAAR)
    b = synth.gaussian_spinor(dims, 8)
    x, _, _ = evenodd.solve(U, b, dims, 0.12, tol=1e-13, hop_sign=+1)
    want = dense.unflat(np.linalg.solve(dense.dense_D(U, dims, 0.12, hop_sign=+1), dense.flat(b)))
    assert rel(x, want) < 1e-11


# planted mistakes -----------------------------------------------------------

def test_missing_source_correction_caught(monkeypatch):
    # b^_e = b_e (the - D_eo b_o term dropped) must fail the LAPACK pin
    real_project = evenodd.project
    calls = {"n": 0}

    def bad_project(v, par, p):
        calls["n"] += 1
        out = real_project(v, par, p)
        return out * 0.0 if calls["n"] == 3 else out  # P_e D b_o -> 0 in solve()

    monkeypatch.setattr(evenodd, "project", bad_project)
    with pytest.raises(AssertionError):
        test_evenodd_solve_vs_lapack((2, 2, 2, 4), 3, 0.124)


def test_wrong_adjoint_caught(monkeypatch):
    # M^dag built from D instead of D^dag must fail the adjoint pin
    real = evenodd.apply_M
    monkeypatch.setattr(evenodd, "apply_M",
                        lambda U, v, dims, k, dagger=False, *a, **kw: real(U, v, dims, k, False,
                                                                           *a, **kw))
    with pytest.raises(AssertionError):
        test_M_adjoint()
