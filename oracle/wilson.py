"""The Wilson-Dirac operator of Eq. (1), Sec. 2.1, and its adjoint (oracle).

Definition implemented (the sign of the hopping term is a parameter):

  (D psi)(x) = psi(x) + s * kappa * sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                                          + (1 + gamma_mu) U_mu(x - mu)^dag psi(x - mu) ]

Eq. (1) prints s = +1; the operator this project solves uses s = -1
(D = 1 - kappa * hopping).  On lattices with even extents the two are
related by D_{+}(kappa) = eps D_{-}(kappa) eps with eps(x) = (-1)^(x+y+z+t),
so they share spectrum and CG iteration counts (pinned in the tests).

Readings of garbled or silent points in Eq. (1):
* The backward term's link is the conjugate transpose of U_mu on the edge
  from x - mu to x, i.e. U_mu(x - mu)^dag (its mu subscript is missing in
  the printed equation).
* The forward hop x -> x + mu carries P^{-mu} = 1 - gamma_mu and the
  backward hop carries P^{+mu} = 1 + gamma_mu, as printed.
* Boundary conditions: periodic in x, y, z; antiperiodic in t when
  ``antiperiodic_t`` (Sec. 2.3 allows periodic or antiperiodic conditions).
  A hop that crosses the t boundary (T-1 -> 0 forward, 0 -> T-1 backward)
  picks up a factor -1.  On an extent-2 direction the forward and backward
  neighbours coincide and both contributions add.

Layouts.  The public functions take canonical float64 arrays:
  gauge  (V, 4, 3, 3, 2): U_mu(s)[a][b] (re, im), mu = 0..3 = x, y, z, t
  spinor (V, 4, 3, 2):    psi(s)[spin][colour] (re, im)
  site s = x + Lx*(y + Ly*(z + Lz*t)).
Internally fields are complex128 arrays indexed [t, z, y, x, ...].
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA, IDENTITY4

# lattice direction mu -> axis of the [t, z, y, x] array
_AXIS = {0: 3, 1: 2, 2: 1, 3: 0}


def to_complex(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.view(np.complex128)[..., 0]


def to_real(c: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.complex128)
    return c.view(np.float64).reshape(c.shape + (2,))


def gauge_4d(U: np.ndarray, dims) -> np.ndarray:
    """canonical (V,4,3,3,2) -> complex (T, Z, Y, X, 4, 3, 3)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    return to_complex(U).reshape(lt, lz, ly, lx, 4, 3, 3)


def spinor_4d(psi: np.ndarray, dims) -> np.ndarray:
    """canonical (V,4,3,2) -> complex (T, Z, Y, X, 4, 3)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    return to_complex(psi).reshape(lt, lz, ly, lx, 4, 3)


def spinor_flat(psi4: np.ndarray) -> np.ndarray:
    """complex (T, Z, Y, X, 4, 3) -> canonical (V, 4, 3, 2)."""
    return to_real(psi4.reshape(-1, 4, 3))


def _spin(P: np.ndarray, v: np.ndarray) -> np.ndarray:
    # (P v)[..., s, c] = sum_t P[s, t] v[..., t, c]
    return np.einsum("st,...tc->...sc", P, v)


def _colour(U: np.ndarray, v: np.ndarray) -> np.ndarray:
    # (U v)[..., s, a] = sum_b U[..., a, b] v[..., s, b]
    return np.einsum("...ab,...sb->...sa", U, v)


def _colour_dag(U: np.ndarray, v: np.ndarray) -> np.ndarray:
    # (U^dag v)[..., s, a] = sum_b conj(U[..., b, a]) v[..., s, b]
    return np.einsum("...ba,...sb->...sa", U.conj(), v)


def hopping_4d(U4: np.ndarray, psi4: np.ndarray, fwd_sign: int, antiperiodic_t: bool = True):
    """H psi = sum_mu [ (1 + f gamma_mu) U_mu(x) psi(x+mu) + (1 - f gamma_mu) U_mu(x-mu)^dag psi(x-mu) ].

    fwd_sign f = -1 gives the hopping term of Eq. (1); f = +1 its adjoint.
    """
    out = np.zeros_like(psi4)
    T = psi4.shape[0]
    for mu in range(4):
        ax = _AXIS[mu]
        Umu = U4[..., mu, :, :]
        # forward neighbour: fwd[x] = psi[x + mu]
        fwd = np.roll(psi4, -1, axis=ax)
        if mu == 3 and antiperiodic_t:
            fwd[T - 1] *= -1.0
        out += _spin(IDENTITY4 + fwd_sign * GAMMA[mu], _colour(Umu, fwd))
        # backward neighbour: W(y) = U_mu(y)^dag psi(y), taken at y = x - mu
        w = _colour_dag(Umu, psi4)
        bwd = np.roll(w, +1, axis=ax)
        if mu == 3 and antiperiodic_t:
            bwd[0] *= -1.0
        out += _spin(IDENTITY4 - fwd_sign * GAMMA[mu], bwd)
    return out


def apply_D(U: np.ndarray, psi: np.ndarray, dims, kappa: float, antiperiodic_t: bool = True,
            hop_sign: int = -1) -> np.ndarray:
    """D psi on canonical arrays (Eq. (1) with the hopping sign ``hop_sign``)."""
    U4 = gauge_4d(U, dims)
    p4 = spinor_4d(psi, dims)
    out = p4 + hop_sign * kappa * hopping_4d(U4, p4, -1, antiperiodic_t)
    return spinor_flat(out)


def apply_Ddag(U: np.ndarray, psi: np.ndarray, dims, kappa: float, antiperiodic_t: bool = True,
               hop_sign: int = -1) -> np.ndarray:
    """D^dag psi.

    The adjoint of the hop x <- x + mu with weight (1 - gamma_mu) U_mu(x) is
    the hop x <- x - mu with weight (1 - gamma_mu)^dag U_mu(x - mu)^dag =
    (1 - gamma_mu) U_mu(x - mu)^dag (the gamma_mu are Hermitian); likewise
    for the backward hop.  The boundary signs are real, so D^dag is D with
    the two projectors exchanged (kappa real).
    """
    U4 = gauge_4d(U, dims)
    p4 = spinor_4d(psi, dims)
    out = p4 + hop_sign * kappa * hopping_4d(U4, p4, +1, antiperiodic_t)
    return spinor_flat(out)


def apply_DdagD(U, psi, dims, kappa, antiperiodic_t=True):
    return apply_Ddag(U, apply_D(U, psi, dims, kappa, antiperiodic_t), dims, kappa,
                      antiperiodic_t)


def apply_D_multi(U, psis, dims, kappa, dagger=False, antiperiodic_t=True):
    """Apply D (or D^dag) to each of a stack of spinors (nrhs, V, 4, 3, 2)."""
    f = apply_Ddag if dagger else apply_D
    return np.stack([f(U, p, dims, kappa, antiperiodic_t) for p in psis])


def coords(s: int, dims):
    lx, ly, lz, lt = (int(d) for d in dims)
    x = s % lx
    y = (s // lx) % ly
    z = (s // (lx * ly)) % lz
    t = s // (lx * ly * lz)
    return [x, y, z, t]


def site_index(c, dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return int(c[0] + lx * (c[1] + ly * (c[2] + lz * c[3])))


def apply_D_sites(U_at, psi_at, dims, kappa: float, sites, dagger: bool = False,
                  antiperiodic_t: bool = True) -> np.ndarray:
    """(D psi)(s) or (D^dag psi)(s) at chosen sites only, one site at a time.

    ``U_at(s)`` returns the complex (4, 3, 3) links of site s and ``psi_at(s)``
    the complex (4, 3) spinor of site s, so a caller can serve them from a
    huge lattice (or generate them on demand) without holding the field in
    this process.  Returns complex (len(sites), 4, 3).
    """
    f = +1 if dagger else -1  # forward projector 1 + f gamma
    res = []
    for s in sites:
        c = coords(int(s), dims)
        acc = np.zeros((4, 3), dtype=np.complex128)
        for mu in range(4):
            L = int(dims[mu])
            cf = list(c)
            cf[mu] = (c[mu] + 1) % L
            cb = list(c)
            cb[mu] = (c[mu] - 1) % L
            sf, sb = site_index(cf, dims), site_index(cb, dims)
            ph_f = -1.0 if (mu == 3 and antiperiodic_t and c[3] == L - 1) else 1.0
            ph_b = -1.0 if (mu == 3 and antiperiodic_t and c[3] == 0) else 1.0
            Uf = U_at(int(s))[mu]
            Ub = U_at(sb)[mu]
            acc += ph_f * (IDENTITY4 + f * GAMMA[mu]) @ (psi_at(sf) @ Uf.T)
            acc += ph_b * (IDENTITY4 - f * GAMMA[mu]) @ (psi_at(sb) @ Ub.conj())
        res.append(psi_at(int(s)) - kappa * acc)
    return np.array(res)


def norm2(v: np.ndarray) -> float:
    """Squared 2-norm of a canonical real-pair array (sum of squares)."""
    return float(np.sum(np.asarray(v, dtype=np.float64) ** 2))


def dot(a: np.ndarray, b: np.ndarray) -> complex:
    """<a, b> = sum conj(a) b for canonical arrays."""
    return complex(np.vdot(to_complex(a).ravel(), to_complex(b).ravel()))
