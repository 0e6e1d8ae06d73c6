"""Dirac matrices of the paper's Appendix A (Conventions).

gamma_mu for mu = 0, 1, 2, 3 act on the spinor index alpha = 0..3; mu runs
over the lattice directions in the order x, y, z, t (Sec. 2.1 labels the four
link matrices U_mu, mu = 0..3, and Sec. 6.2 names the link arrays U_x, U_y,
U_z, U_t).  gamma_5 is the diagonal matrix printed beside them.
"""
import numpy as np

_i = 1j

GAMMA = np.array([
    # gamma_0
    [[0, 0, 0, _i],
     [0, 0, _i, 0],
     [0, -_i, 0, 0],
     [-_i, 0, 0, 0]],
    # gamma_1
    [[0, 0, 0, -1],
     [0, 0, 1, 0],
     [0, 1, 0, 0],
     [-1, 0, 0, 0]],
    # gamma_2
    [[0, 0, _i, 0],
     [0, 0, 0, -_i],
     [-_i, 0, 0, 0],
     [0, _i, 0, 0]],
    # gamma_3
    [[0, 0, 1, 0],
     [0, 0, 0, 1],
     [1, 0, 0, 0],
     [0, 1, 0, 0]],
], dtype=np.complex128)

GAMMA5 = np.diag([1, 1, -1, -1]).astype(np.complex128)

IDENTITY4 = np.eye(4, dtype=np.complex128)


def projector(mu: int, sign: int) -> np.ndarray:
    """P^{sign mu} = 1 + sign * gamma_mu (Sec. 2.1, the projector definition)."""
    return IDENTITY4 + sign * GAMMA[mu]
