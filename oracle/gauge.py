"""Gauge transformations (a pin for link indexing and U versus U^dag).

With G(x) in SU(3) on every site, U'_mu(x) = G(x) U_mu(x) G(x + mu)^dag and
psi'(x) = G(x) psi(x).  The operator of Eq. (1) then satisfies
D[U'] psi' = G D[U] psi, since every hop carries U between the colour frames
of its two end points.  The antiperiodic sign is a real scalar and commutes
with G; G itself is periodic.
"""
from __future__ import annotations

import numpy as np


def _cx(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.complex128)[..., 0]


def _re(c):
    c = np.ascontiguousarray(c)
    return c.view(np.float64).reshape(c.shape + (2,))


def transform_gauge(U: np.ndarray, G: np.ndarray, dims) -> np.ndarray:
    """U (V,4,3,3,2), G (V,3,3,2) -> U' (V,4,3,3,2)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    Uc = _cx(U).reshape(lt, lz, ly, lx, 4, 3, 3)
    Gc = _cx(G).reshape(lt, lz, ly, lx, 3, 3)
    axis = {0: 3, 1: 2, 2: 1, 3: 0}
    out = np.empty_like(Uc)
    for mu in range(4):
        Gn = np.roll(Gc, -1, axis=axis[mu])  # G(x + mu)
        out[..., mu, :, :] = Gc @ Uc[..., mu, :, :] @ np.conj(np.swapaxes(Gn, -1, -2))
    return _re(out.reshape(-1, 4, 3, 3))


def transform_spinor(psi: np.ndarray, G: np.ndarray) -> np.ndarray:
    """psi (V,4,3,2) -> G(x) psi(x) on the colour index."""
    p = _cx(psi)
    g = _cx(G)
    out = np.einsum("sab,skb->ska", g, p)
    return _re(out)
