"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
Clifford algebra of the Appendix A basis, an independently assembled dense
matrix, the closed-form free-field spectrum, an FFT propagator, the adjoint
relation and gamma_5-hermiticity of Sec. 2.2, gauge covariance, LAPACK
solves, and the published SplitMix64 test vector.  test_oracle_mutations.py
shows that planted mistakes in the oracle fail these pins.
"""
import os

import numpy as np
import pytest

import synth
from oracle import cg, dense, free, gauge, wilson
from oracle.gamma import GAMMA, GAMMA5, IDENTITY4

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cx(a):
    return wilson.to_complex(a)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


# --------------------------------------------------------------- generators

def test_splitmix64_published_vector():
    want = []
    for line in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            want.append(int(line, 16))
    got = [int(v) for v in synth.splitmix_stream(0, len(want))]
    assert got == want


@pytest.mark.parametrize("kind", [synth.HAAR, synth.EXP])
def test_su3_links(kind):
    U = cx(synth.gauge((4, 2, 2, 4), 7, kind, 0.3))
    I3 = np.eye(3)
    assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - I3).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    row3 = np.conj(np.cross(U[..., 0, :], U[..., 1, :]))
    assert np.abs(row3 - U[..., 2, :]).max() < 1e-15


def test_generator_chunking_and_determinism():
    dims = (4, 4, 4, 6)
    full = synth.gauge(dims, 11, synth.EXP, 0.3)
    part = synth.gauge(dims, 11, synth.EXP, 0.3, t0=2, t1=5)
    v3 = 64
    assert np.array_equal(full[2 * v3:5 * v3], part)
    s = synth.gaussian_spinor(dims, 5)
    assert np.array_equal(s[100:200], synth.gaussian_spinor(dims, 5, 100, 200))
    assert abs(s.mean()) < 0.05 and abs(s.std() - 1) < 0.05


def test_exp_links_are_near_identity():
    # eps = 0.3 links sit near 1: mean |U - 1| well below Haar's
    U = cx(synth.gauge((4, 4, 4, 4), 2, synth.EXP, 0.3))
    H = cx(synth.gauge((4, 4, 4, 4), 2, synth.HAAR))
    assert np.abs(U - np.eye(3)).mean() < 0.5 * np.abs(H - np.eye(3)).mean()


# --------------------------------------------------------------- gamma basis

def test_clifford_algebra_and_gamma5():
    for m in range(4):
        assert np.allclose(GAMMA[m], GAMMA[m].conj().T)
        for n in range(4):
            anti = GAMMA[m] @ GAMMA[n] + GAMMA[n] @ GAMMA[m]
            assert np.allclose(anti, 2 * (m == n) * IDENTITY4)
    assert np.allclose(GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3], GAMMA5)
    for m in range(4):
        assert np.allclose(GAMMA5 @ GAMMA[m], -GAMMA[m] @ GAMMA5)


def test_projectors_rank_two():
    for m in range(4):
        for s in (+1, -1):
            P = IDENTITY4 + s * GAMMA[m]
            assert np.linalg.matrix_rank(P) == 2
            assert np.allclose(P @ P, 2 * P)


# --------------------------------------------------------------- stencil vs dense

DENSE_DIMS = [(2, 2, 2, 2), (2, 2, 4, 2), (4, 2, 2, 2), (2, 4, 2, 2), (2, 2, 2, 4)]


@pytest.mark.parametrize("dims", DENSE_DIMS)
@pytest.mark.parametrize("dagger", [False, True])
def test_stencil_equals_dense(dims, dagger):
    U = synth.gauge(dims, 3, synth.HAAR)
    psi = synth.gaussian_spinor(dims, 4)
    k = 0.137
    M = dense.dense_D(U, dims, k)
    if dagger:
        M = M.conj().T
        got = wilson.apply_Ddag(U, psi, dims, k)
    else:
        got = wilson.apply_D(U, psi, dims, k)
    want = dense.unflat(M @ dense.flat(psi))
    assert np.abs(got - want).max() < 1e-14


def test_dense_gamma5_hermiticity():
    dims = (2, 2, 2, 2)
    U = synth.gauge(dims, 8, synth.HAAR)
    M = dense.dense_D(U, dims, 0.19)
    G5 = dense.gamma5_matrix(16)
    assert np.abs(G5 @ M @ G5 - M.conj().T).max() < 1e-15


def test_kappa_zero_is_identity():
    dims = (2, 2, 2, 2)
    U = synth.gauge(dims, 8, synth.HAAR)
    assert np.array_equal(dense.dense_D(U, dims, 0.0), np.eye(192))
    psi = synth.gaussian_spinor((4, 2, 2, 4), 1)
    U2 = synth.gauge((4, 2, 2, 4), 1, synth.EXP)
    assert np.array_equal(wilson.apply_D(U2, psi, (4, 2, 2, 4), 0.0), psi)


def test_apply_at_sites_matches_full():
    dims = (4, 6, 8, 10)
    U = synth.gauge(dims, 21, synth.EXP)
    psi = synth.gaussian_spinor(dims, 22)
    k = 0.124
    Uc = cx(U)
    pc = cx(psi)
    sites = [0, 1, 3, 4 * 6 * 8 * 10 - 1, 4 * 6 * 8 * 9, 4 * 6 * 8 - 1, 777, 1234]
    for dag in (False, True):
        full = cx(wilson.apply_Ddag(U, psi, dims, k) if dag else wilson.apply_D(U, psi, dims, k))
        got = wilson.apply_D_sites(lambda s: Uc[s], lambda s: pc[s], dims, k, sites, dagger=dag)
        assert np.abs(got - full[sites]).max() < 1e-14


# --------------------------------------------------------------- free field

@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4), (4, 2, 2, 2)])
@pytest.mark.parametrize("anti", [True, False])
def test_free_spectrum_dense(dims, anti):
    U = synth.gauge_unit(dims)
    k = 0.11
    M = dense.dense_D(U, dims, k, antiperiodic_t=anti)
    ev = np.linalg.eigvals(M)
    want = free.spectrum(dims, k, anti)
    key = lambda z: (round(z.real, 9), round(z.imag, 9))  # noqa: E731
    a = np.array(sorted(ev, key=key))
    b = np.array(sorted(want, key=key))
    assert np.abs(a - b).max() < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10)])
def test_plane_wave_eigen(dims, rng):
    U = synth.gauge_unit(dims)
    k = 0.124
    ps = free.momenta(dims)
    for idx in rng.choice(len(ps), 4, replace=False):
        p = ps[idx]
        chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        psi = free.plane_wave(dims, p, chi)
        a, b = free.a_b(p, k)
        Dp = a * IDENTITY4 + 1j * np.einsum("m,mst->st", b, GAMMA)
        want_D = free.plane_wave(dims, p, Dp @ chi)
        assert rel(wilson.apply_D(U, psi, dims, k), want_D) < 1e-13
        lam = free.DdagD_eigenvalue(p, k)
        assert rel(wilson.apply_DdagD(U, psi, dims, k), lam * psi) < 1e-13


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 4, 8)])
def test_fft_propagator_vs_cg(dims):
    U = synth.gauge_unit(dims)
    k = 0.12
    eta = synth.point_source(dims, 1, 2, site=5)
    D = lambda v: wilson.apply_D(U, v, dims, k)  # noqa: E731
    Dd = lambda v: wilson.apply_Ddag(U, v, dims, k)  # noqa: E731
    x, it, info = cg.cgnr(D, Dd, eta, tol=1e-12)
    assert info["converged"]
    want = free.solve_fft(dims, k, eta)
    assert rel(x, want) < 1e-10
    # and the FFT solution solves D psi = eta
    assert rel(D(want), eta) < 1e-12


# --------------------------------------------------------------- adjoint and covariance

@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 8, 10)])
def test_adjoint_dot_and_gamma5(dims):
    U = synth.gauge(dims, 31, synth.HAAR)
    phi = synth.gaussian_spinor(dims, 32)
    psi = synth.gaussian_spinor(dims, 33)
    k = 0.13
    lhs = wilson.dot(phi, wilson.apply_Ddag(U, psi, dims, k))
    rhs = wilson.dot(wilson.apply_D(U, phi, dims, k), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-14
    g5 = np.array([1, 1, -1, -1], dtype=np.float64)[None, :, None, None]
    got = g5 * wilson.apply_D(U, g5 * psi, dims, k)
    assert rel(got, wilson.apply_Ddag(U, psi, dims, k)) < 1e-15


@pytest.mark.parametrize("dagger", [False, True])
def test_gauge_covariance(dagger):
    dims = (4, 6, 8, 10)
    U = synth.gauge(dims, 41, synth.EXP)
    psi = synth.gaussian_spinor(dims, 42)
    G = synth.gauge_rotation(dims, 43)
    k = 0.125
    f = wilson.apply_Ddag if dagger else wilson.apply_D
    Up = gauge.transform_gauge(U, G, dims)
    lhs = f(Up, gauge.transform_spinor(psi, G), dims, k)
    rhs = gauge.transform_spinor(f(U, psi, dims, k), G)
    assert rel(lhs, rhs) < 1e-14


def _shift4(a, dims, s):
    """Canonical field moved by s = (sx, sy, sz, st): out(x + s) = a(x)."""
    Lx, Ly, Lz, Lt = dims
    f = a.reshape((Lt, Lz, Ly, Lx) + a.shape[1:])
    f = np.roll(f, (s[3], s[2], s[1], s[0]), axis=(0, 1, 2, 3))
    return np.ascontiguousarray(f.reshape(a.shape))


@pytest.mark.parametrize("s", [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1),
                               (3, 2, 5, 7)])
@pytest.mark.parametrize("anti", [False, True])
@pytest.mark.parametrize("dagger", [False, True])
def test_translation_covariance(s, anti, dagger):
    # The lattice is periodic in x, y, z, so shifting links and source shifts
    # D psi.  An antiperiodic t boundary is a sign on the links that cross
    # t = T-1 -> 0; after a t shift by s_t it sits on the links leaving
    # t = s_t - 1, and the +-1 gauge rotation g(t) = -1 for t < s_t moves it
    # back: D[U'] (g psi') = g (D[U] psi)'.  A misplaced or doubled boundary
    # sign breaks this.
    dims = (4, 6, 8, 10)
    U = synth.gauge(dims, 47, synth.EXP)
    psi = synth.gaussian_spinor(dims, 48)
    k = 0.125
    f = wilson.apply_Ddag if dagger else wilson.apply_D
    Us, ps = _shift4(U, dims, s), _shift4(psi, dims, s)
    t = np.array([wilson.coords(x, dims)[3] for x in range(psi.shape[0])])
    g = np.where(anti & (t < s[3]), -1.0, 1.0)[:, None, None, None]
    lhs = f(Us, g * ps, dims, k, antiperiodic_t=anti)
    rhs = g * _shift4(f(U, psi, dims, k, antiperiodic_t=anti), dims, s)
    assert rel(lhs, rhs) < 1e-15
    if anti and s[3]:
        # without the rotation the boundary is in the wrong place
        assert rel(f(Us, ps, dims, k, antiperiodic_t=True),
                   _shift4(f(U, psi, dims, k, antiperiodic_t=True), dims, s)) > 1e-3


def test_sign_convention_equivalence():
    # D_{+kappa} = eps D_{-kappa} eps, eps(x) = (-1)^(x+y+z+t), even extents
    dims = (4, 2, 6, 4)
    U = synth.gauge(dims, 51, synth.EXP)
    psi = synth.gaussian_spinor(dims, 52)
    V = 4 * 2 * 6 * 4
    eps = np.array([(-1) ** sum(wilson.coords(s, dims)) for s in range(V)],
                   dtype=np.float64)[:, None, None, None]
    a = wilson.apply_D(U, psi, dims, 0.12, hop_sign=+1)
    b = eps * wilson.apply_D(U, eps * psi, dims, 0.12, hop_sign=-1)
    assert np.abs(a - b).max() < 1e-15


def test_normal_operator_positive_and_linear(rng):
    dims = (4, 4, 2, 4)
    U = synth.gauge(dims, 61, synth.HAAR)
    a = synth.gaussian_spinor(dims, 62)
    b = synth.gaussian_spinor(dims, 63)
    k = 0.13
    AD = lambda v: wilson.apply_DdagD(U, v, dims, k)  # noqa: E731
    assert wilson.dot(a, AD(a)).real > 0
    assert abs(wilson.dot(a, AD(a)).imag) < 1e-10
    c = 0.7
    assert rel(AD(a + c * b), AD(a) + c * AD(b)) < 1e-15
    assert abs(wilson.dot(a, AD(a)).real - wilson.norm2(wilson.apply_D(U, a, dims, k))) < 1e-10


# --------------------------------------------------------------- CG vs LAPACK

def _solve_dense(U, dims, k, b):
    M = dense.dense_D(U, dims, k)
    return dense.unflat(np.linalg.solve(M, dense.flat(b)))


@pytest.mark.parametrize("dims,seed,kappa", [((2, 2, 2, 2), 1, 0.12), ((2, 2, 2, 4), 3, 0.124)])
def test_cg_vs_lapack_tiny(dims, seed, kappa):
    U = synth.gauge(dims, seed, synth.HAAR)
    b = synth.point_source(dims)
    D = lambda v: wilson.apply_D(U, v, dims, kappa)  # noqa: E731
    Dd = lambda v: wilson.apply_Ddag(U, v, dims, kappa)  # noqa: E731
    x, it, info = cg.cgnr(D, Dd, b, tol=1e-13)
    want = _solve_dense(U, dims, kappa, b)
    assert rel(x, want) < 1e-12
    # a dense-matrix CG reaches the same iterate count and solution
    M = dense.dense_D(U, dims, kappa)
    Dm = lambda v: dense.unflat(M @ dense.flat(v))  # noqa: E731
    Dmd = lambda v: dense.unflat(M.conj().T @ dense.flat(v))  # noqa: E731
    x2, it2, _ = cg.cgnr(Dm, Dmd, b, tol=1e-13)
    assert abs(it - it2) <= 1
    assert rel(x2, want) < 1e-12


def test_cg_config1_4x4_vs_lapack():
    """4^4, kappa 0.12, Haar-QR links seed 1, point source at the origin."""
    dims = (4, 4, 4, 4)
    U = synth.gauge(dims, 1, synth.HAAR)
    b = synth.point_source(dims, 0, 0, 0)
    k = 0.12
    D = lambda v: wilson.apply_D(U, v, dims, k)  # noqa: E731
    Dd = lambda v: wilson.apply_Ddag(U, v, dims, k)  # noqa: E731
    x, it, info = cg.cgnr(D, Dd, b, tol=1e-10)
    assert info["converged"]
    want = _solve_dense(U, dims, k, b)
    cond = cg.lanczos_condition(info["alphas"], info["betas"])
    assert cond > 1
    assert rel(x, want) < 1e-9
    assert rel(D(x), b) < 1e-8


@pytest.mark.parametrize("dims,seed,kappa", [((2, 2, 2, 2), 1, 0.12), ((2, 2, 2, 4), 3, 0.124)])
def test_cgne_vs_lapack_tiny(dims, seed, kappa):
    """The paper's form (CG on D D^dag y = b, x = D^dag y) reaches the dense
    solution, with the true residual of D x = b at the tolerance."""
    U = synth.gauge(dims, seed, synth.HAAR)
    b = synth.gaussian_spinor(dims, seed + 40)
    D = lambda v: wilson.apply_D(U, v, dims, kappa)  # noqa: E731
    Dd = lambda v: wilson.apply_Ddag(U, v, dims, kappa)  # noqa: E731
    x, it, info = cg.cgne(D, Dd, b, tol=1e-13)
    want = _solve_dense(U, dims, kappa, b)
    assert info["converged"] and rel(x, want) < 1e-12
    assert rel(D(x), b) <= 1e-12


def test_cgne_config1_and_paper_sign():
    """4^4 configuration: CGNE and CGNR agree; with the paper's +kappa sign
    the solution is eps x_- (D_+ = eps D_- eps, even extents)."""
    dims = (4, 4, 4, 4)
    U = synth.gauge(dims, 1, synth.HAAR)
    b = synth.point_source(dims, 0, 0, 0)
    k = 0.12
    D = lambda v: wilson.apply_D(U, v, dims, k)  # noqa: E731
    Dd = lambda v: wilson.apply_Ddag(U, v, dims, k)  # noqa: E731
    xe, ite, _ = cg.cgne(D, Dd, b, tol=1e-11)
    xr, itr, _ = cg.cgnr(D, Dd, b, tol=1e-11)
    assert rel(xe, xr) < 1e-9 and rel(xe, _solve_dense(U, dims, k, b)) < 1e-9
    Dp = lambda v: wilson.apply_D(U, v, dims, k, hop_sign=+1)  # noqa: E731
    Dpd = lambda v: wilson.apply_Ddag(U, v, dims, k, hop_sign=+1)  # noqa: E731
    xp, itp, _ = cg.cgne(Dp, Dpd, b, tol=1e-11)
    V = int(np.prod(dims))
    eps = np.array([(-1) ** sum(wilson.coords(s, dims)) for s in range(V)],
                   dtype=np.float64)[:, None, None, None]
    assert rel(xp, eps * cg.cgne(D, Dd, eps * b, tol=1e-11)[0]) < 1e-9
    assert abs(itp - ite) <= 1


def test_cg_warm_start_from_solution():
    dims = (2, 2, 2, 4)
    U = synth.gauge(dims, 5, synth.HAAR)
    b = synth.gaussian_spinor(dims, 6)
    k = 0.11
    D = lambda v: wilson.apply_D(U, v, dims, k)  # noqa: E731
    Dd = lambda v: wilson.apply_Ddag(U, v, dims, k)  # noqa: E731
    want = _solve_dense(U, dims, k, b)
    x, it, info = cg.cgnr(D, Dd, b, tol=1e-10, x0=want)
    assert it == 0 and rel(x, want) < 1e-14


def test_solution_gauge_covariance():
    dims = (4, 2, 2, 4)
    U = synth.gauge(dims, 71, synth.EXP)
    b = synth.gaussian_spinor(dims, 72)
    G = synth.gauge_rotation(dims, 73)
    k = 0.12
    Up = gauge.transform_gauge(U, G, dims)
    bp = gauge.transform_spinor(b, G)
    x, _, _ = cg.cgnr(lambda v: wilson.apply_D(U, v, dims, k),
                      lambda v: wilson.apply_Ddag(U, v, dims, k), b, tol=1e-12)
    xp, _, _ = cg.cgnr(lambda v: wilson.apply_D(Up, v, dims, k),
                       lambda v: wilson.apply_Ddag(Up, v, dims, k), bp, tol=1e-12)
    assert rel(xp, gauge.transform_spinor(x, G)) < 1e-10


# --------------------------------------------------------------- paper's printed numbers

def test_paper_table4_from_formula():
    rows = []
    for line in open(os.path.join(GOLDEN, "paper_table4.txt")):
        if line.strip() and not line.startswith("#"):
            name, delta, nu, tau, printed = line.split()
            rows.append((name, float(delta), float(nu) * 1e6, float(tau), float(printed)))
    V, f = 6 ** 3 * 8, 1464
    for name, delta, nu, tau, printed in rows:
        perf = V * f * nu / (V * delta + tau) / 1e9
        assert abs(perf - printed) / printed < 5e-3, name
    assert (9 * 24 + 8 * 18) * 8 == 2880


# ------------------------------------------------------------------ condition estimate
#
# cg.lanczos_condition turns CG's step lengths into the Lanczos tridiagonal of
# D^dag D (Sec. 2.2 iteration; the Ritz values of that matrix interlace the
# spectrum).  Its largest-to-smallest Ritz ratio can therefore never exceed
# the exact condition number, and once CG has converged it must be close to
# it.  Two independent pins: the eigenvalues of the dense D^dag D on 2^4-type
# lattices, and the free-field closed form a(p)^2 + |b(p)|^2 at 4^4.

@pytest.mark.parametrize("dims,seed,kappa,kind", [((2, 2, 2, 2), 1, 0.12, synth.HAAR),
                                                  ((2, 2, 2, 4), 3, 0.15, synth.HAAR),
                                                  ((2, 2, 2, 2), 5, 0.124, synth.EXP)])
def test_lanczos_condition_vs_dense_eigenvalues(dims, seed, kappa, kind):
    U = synth.gauge(dims, seed, kind, 0.3)
    M = dense.dense_D(U, dims, kappa)
    ev = np.linalg.eigvalsh(M.conj().T @ M)
    exact = ev[-1] / ev[0]
    b = synth.gaussian_spinor(dims, seed + 10)
    D = lambda v: wilson.apply_D(U, v, dims, kappa)  # noqa: E731
    Dd = lambda v: wilson.apply_Ddag(U, v, dims, kappa)  # noqa: E731
    _, _, info = cg.cgnr(D, Dd, b, tol=1e-10)
    est = cg.lanczos_condition(info["alphas"], info["betas"])
    assert est <= exact * (1 + 1e-9), (est, exact)
    assert est >= 0.99 * exact, (est, exact)


def test_lanczos_condition_free_field_closed_form():
    """U = 1 on 4^4 (antiperiodic t): D^dag D is a(p)^2 + |b(p)|^2 times the
    identity on each momentum, so cond = max / min over the allowed momenta."""
    dims = (4, 4, 4, 4)
    kappa = 0.12
    lam = np.array([free.DdagD_eigenvalue(p, kappa) for p in free.momenta(dims)])
    exact = lam.max() / lam.min()
    U = synth.gauge_unit(dims)
    b = synth.gaussian_spinor(dims, 77)
    D = lambda v: wilson.apply_D(U, v, dims, kappa)  # noqa: E731
    Dd = lambda v: wilson.apply_Ddag(U, v, dims, kappa)  # noqa: E731
    _, it, info = cg.cgnr(D, Dd, b, tol=1e-10)
    est = cg.lanczos_condition(info["alphas"], info["betas"])
    assert est <= exact * (1 + 1e-9), (est, exact)
    assert est >= 0.999 * exact, (est, exact)
    # CG on a scalar-per-momentum operator ends within the number of its
    # distinct eigenvalues (one more step in floating point)
    assert it <= len(np.unique(np.round(lam, 12))) + 1
