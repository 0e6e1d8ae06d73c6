"""Even-odd (Schur complement) form of D x = b (oracle; test infrastructure).

Not in the paper: a standard technique for the Wilson operator of Eq. (1),
written here from its definition.  Sites split by parity (x+y+z+t) mod 2.
The hopping term of Eq. (1) only couples nearest neighbours, which have
opposite parity, so in (even, odd) blocks

    D = [[1, D_eo], [D_oe, 1]],   D_eo = P_e D P_o,   D_oe = P_o D P_e,

with P_e / P_o the projections onto even / odd sites.  Eliminating the odd
sites gives the Schur complement on the even sites:

    M x_e = b^_e,   M = 1 - D_eo D_oe,   b^_e = b_e - D_eo b_o,
    x_o = b_o - D_oe x_e.

M^dag = 1 - (D^dag)_eo (D^dag)_oe, since (D_oe)^dag = (D^dag)_eo.  The solve
runs CGNR on M (M^dag M x_e = M^dag b^_e).  Everything acts on full-lattice
canonical arrays through parity masks, so each step reads off the block
definition above.
"""
from __future__ import annotations

import numpy as np

from . import cg, wilson


def parity(dims) -> np.ndarray:
    """(V,) array of site parities (x+y+z+t) mod 2, canonical site order."""
    lx, ly, lz, lt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    return ((x + y + z + t) % 2).reshape(-1)


def project(v: np.ndarray, par: np.ndarray, p: int) -> np.ndarray:
    """Keep the sites of parity p (v canonical (V, 4, 3, 2) or (..., V, 4, 3, 2))."""
    mask = (par == p).astype(np.float64)[:, None, None, None]
    return v * mask


def _op(U, dims, kappa, dagger, hop_sign, antiperiodic_t):
    f = wilson.apply_Ddag if dagger else wilson.apply_D
    return lambda v: f(U, v, dims, kappa, antiperiodic_t=antiperiodic_t, hop_sign=hop_sign)


def apply_M(U, ve, dims, kappa: float, dagger: bool = False, hop_sign: int = -1,
            antiperiodic_t: bool = True) -> np.ndarray:
    """M v_e = v_e - D_eo D_oe v_e (dagger: M^dag with D^dag's blocks) for a
    field supported on even sites; the result is supported on even sites."""
    par = parity(dims)
    Dx = _op(U, dims, kappa, dagger, hop_sign, antiperiodic_t)
    ve = project(ve, par, 0)
    w_o = project(Dx(ve), par, 1)         # D_oe v_e
    return ve - project(Dx(w_o), par, 0)  # v_e - D_eo w_o


def solve(U, b, dims, kappa: float, tol: float = 1e-10, hop_sign: int = -1,
          antiperiodic_t: bool = True, max_iter: int = 20000):
    """x = D^{-1} b through the Schur complement.  Returns (x, iterations,
    info) with info from CGNR on M (its 'rel_resid' is relative to
    ||M^dag b^_e||)."""
    par = parity(dims)
    D = _op(U, dims, kappa, False, hop_sign, antiperiodic_t)
    b = np.asarray(b, dtype=np.float64)
    b_o = project(b, par, 1)
    bhat = project(b, par, 0) - project(D(b_o), par, 0)  # b_e - D_eo b_o
    M = lambda v: apply_M(U, v, dims, kappa, False, hop_sign, antiperiodic_t)  # noqa: E731
    Md = lambda v: apply_M(U, v, dims, kappa, True, hop_sign, antiperiodic_t)  # noqa: E731
    x_e, it, info = cg.cgnr(M, Md, bhat, tol=tol, max_iter=max_iter)
    x_e = project(x_e, par, 0)
    x_o = b_o - project(D(x_e), par, 1)  # b_o - D_oe x_e
    return x_e + x_o, it, info
