"""Dense matrix of the operator of Eq. (1), Sec. 2.1, assembled entry by entry.

An independent route to D for tiny lattices (2^4 gives 192 x 192): explicit
loops over sites, the eight hops, and the (spin, colour) x (spin, colour)
entries of each hop block.  Row/column index = 12*s + 3*spin + colour.  No
array rolls and no einsum, so a mistake in the stencil code of ``wilson``
does not repeat here.  The same readings apply as in ``wilson``: backward
link U_mu(x-mu)^dag, forward projector 1 - gamma_mu, backward 1 + gamma_mu,
antiperiodic t by a -1 on hops across the t boundary, and contributions of
coinciding neighbours (extent 2) added.
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA


def _coords(s, dims):
    lx, ly, lz, _ = dims
    return [s % lx, (s // lx) % ly, (s // (lx * ly)) % lz, s // (lx * ly * lz)]


def _index(c, dims):
    lx, ly, lz, _ = dims
    return c[0] + lx * (c[1] + ly * (c[2] + lz * c[3]))


def dense_D(U: np.ndarray, dims, kappa: float, antiperiodic_t: bool = True,
            hop_sign: int = -1) -> np.ndarray:
    """12V x 12V complex matrix of D.  U canonical (V, 4, 3, 3, 2)."""
    dims = [int(d) for d in dims]
    V = dims[0] * dims[1] * dims[2] * dims[3]
    Uc = np.asarray(U, dtype=np.float64)
    N = 12 * V
    M = np.zeros((N, N), dtype=np.complex128)
    for s in range(V):
        for k in range(12):
            M[12 * s + k, 12 * s + k] += 1.0
        c = _coords(s, dims)
        for mu in range(4):
            L = dims[mu]
            for direction in (+1, -1):
                cn = list(c)
                cn[mu] = (c[mu] + direction) % L
                n = _index(cn, dims)
                phase = 1.0
                if mu == 3 and antiperiodic_t:
                    if direction == +1 and c[3] == L - 1:
                        phase = -1.0
                    if direction == -1 and c[3] == 0:
                        phase = -1.0
                for a in range(3):
                    for b in range(3):
                        if direction == +1:
                            # U_mu(x)[a][b]
                            u = complex(Uc[s, mu, a, b, 0], Uc[s, mu, a, b, 1])
                        else:
                            # (U_mu(x - mu)^dag)[a][b] = conj(U_mu(x - mu)[b][a])
                            u = complex(Uc[n, mu, b, a, 0], -Uc[n, mu, b, a, 1])
                        for al in range(4):
                            for be in range(4):
                                # P^{-mu} = 1 - gamma_mu forward, P^{+mu} = 1 + gamma_mu backward
                                pab = (1.0 if al == be else 0.0) - direction * GAMMA[mu][al, be]
                                if pab == 0:
                                    continue
                                M[12 * s + 3 * al + a, 12 * n + 3 * be + b] += (
                                    hop_sign * kappa * phase * pab * u)
    return M


def flat(psi: np.ndarray) -> np.ndarray:
    """canonical spinor (V, 4, 3, 2) -> complex vector of length 12V."""
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    return psi.view(np.complex128).reshape(-1)


def unflat(v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.complex128)
    return v.view(np.float64).reshape(-1, 4, 3, 2)


def gamma5_matrix(V: int) -> np.ndarray:
    """gamma_5 acting on every site: diag over (site, spin, colour)."""
    g = np.tile(np.repeat(np.array([1.0, 1.0, -1.0, -1.0]), 3), V)
    return np.diag(g.astype(np.complex128))
