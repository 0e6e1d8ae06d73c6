"""Free field (all links U = 1): the operator of Eq. (1) in momentum space.

A plane wave psi(x) = exp(i p.x) chi with constant spinor-colour chi gives,
for the operator D = 1 - kappa * hopping (Sec. 2.1 projectors 1 -+ gamma),

  D(p) = a(p) * 1 + i * sum_mu b_mu(p) gamma_mu,
  a(p) = 1 - 2 kappa sum_mu cos p_mu,   b_mu(p) = 2 kappa sin p_mu,

because (1 - gamma) e^{i p} + (1 + gamma) e^{-i p} = 2 cos p - 2 i gamma sin p.
The gamma_mu anticommute and square to 1 (Appendix A), so
(sum b gamma)^2 = |b|^2: the eigenvalues of D(p) are a +- i |b|, each
6-fold (2 spin x 3 colour), and D^dag D(p) = a^2 + |b|^2 times the identity.
D(p)^{-1} = (a - i b.gamma) / (a^2 + |b|^2).

Allowed momenta: p_mu = 2 pi n / L_mu in x, y, z; antiperiodic t gives
p_t = (2 n + 1) pi / T (the plane wave must change sign across the t
boundary, matching the -1 on boundary hops).
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA


def momenta(dims, antiperiodic_t: bool = True):
    """List of allowed 4-momenta (p_x, p_y, p_z, p_t)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    ps = []
    for nt in range(lt):
        pt = (2 * nt + (1 if antiperiodic_t else 0)) * np.pi / lt
        for nz in range(lz):
            for ny in range(ly):
                for nx in range(lx):
                    ps.append((2 * np.pi * nx / lx, 2 * np.pi * ny / ly, 2 * np.pi * nz / lz, pt))
    return np.array(ps)


def a_b(p, kappa):
    p = np.asarray(p, dtype=np.float64)
    a = 1.0 - 2.0 * kappa * np.sum(np.cos(p), axis=-1)
    b = 2.0 * kappa * np.sin(p)
    return a, b


def spectrum(dims, kappa: float, antiperiodic_t: bool = True) -> np.ndarray:
    """All 12V eigenvalues of the free D (closed form)."""
    ps = momenta(dims, antiperiodic_t)
    a, b = a_b(ps, kappa)
    bn = np.sqrt(np.sum(b * b, axis=-1))
    ev = np.concatenate([np.repeat(a + 1j * bn, 6), np.repeat(a - 1j * bn, 6)])
    return ev


def DdagD_eigenvalue(p, kappa: float) -> float:
    a, b = a_b(p, kappa)
    return float(a * a + np.sum(b * b))


def plane_wave(dims, p, chi: np.ndarray) -> np.ndarray:
    """exp(i p.x) chi on the lattice, canonical (V, 4, 3, 2).  chi complex (4, 3)."""
    lx, ly, lz, lt = (int(d) for d in dims)
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t)).reshape(-1)
    f = ph[:, None, None] * np.asarray(chi, dtype=np.complex128)[None]
    return np.ascontiguousarray(f).view(np.float64).reshape(-1, 4, 3, 2)


def solve_fft(dims, kappa: float, eta: np.ndarray, antiperiodic_t: bool = True) -> np.ndarray:
    """psi = D^{-1} eta for U = 1 by FFT.

    Antiperiodic t is handled by the twist phi(x) = exp(-i pi t / T) field(x),
    which is periodic, with momentum p_t = q_t + pi / T for FFT index q_t.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    e = np.ascontiguousarray(eta, dtype=np.float64).view(np.complex128)[..., 0]
    e = e.reshape(lt, lz, ly, lx, 4, 3)
    shift = np.pi / lt if antiperiodic_t else 0.0
    tw = np.exp(-1j * shift * np.arange(lt))[:, None, None, None, None, None]
    F = np.fft.fftn(e * tw, axes=(0, 1, 2, 3))
    qt = 2 * np.pi * np.fft.fftfreq(lt) * 1.0 + shift
    qz = 2 * np.pi * np.fft.fftfreq(lz)
    qy = 2 * np.pi * np.fft.fftfreq(ly)
    qx = 2 * np.pi * np.fft.fftfreq(lx)
    PT, PZ, PY, PX = np.meshgrid(qt, qz, qy, qx, indexing="ij")
    P = np.stack([PX, PY, PZ, PT], axis=-1)  # (T, Z, Y, X, 4) in mu order x,y,z,t
    a, b = a_b(P, kappa)
    den = a * a + np.sum(b * b, axis=-1)
    # (a - i b.gamma) acting on spin
    bg = np.einsum("...m,mst->...st", b, GAMMA)
    Minv = (a[..., None, None] * np.eye(4) - 1j * bg) / den[..., None, None]
    G = np.einsum("...st,...tc->...sc", Minv, F)
    psi = np.fft.ifftn(G, axes=(0, 1, 2, 3)) / tw
    return np.ascontiguousarray(psi.reshape(-1, 4, 3)).view(np.float64).reshape(-1, 4, 3, 2)
