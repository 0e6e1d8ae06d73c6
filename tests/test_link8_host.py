"""CPU study of the 8-real binary16 link form (lattice flag WD_F16_LINKS_8).

A NumPy model of the format the library's binary16 8-real links use (its
layout is described where the library defines the form): row 0 led by its
largest entry (columns relabelled cyclically), two of its entries and one
component of the leading one stored; rows 1 and 2 as alpha e1 + beta e2 and
conj(alpha) e2 - conj(beta) e1 in a frame (e1, e2) orthogonal to row 0,
pivoted on the smaller stored entry; the smaller of alpha, beta and one
component of the other stored; eight choice bits in the last significand
bit of the eight halves.

The checks:
* without rounding the decoded matrix is the link itself (1e-13), for
  near-identity exp(i eps H) links and for Haar links, which exercise every
  relabelling and pivot;
* with binary16 rounding the largest entry error stays within a few units
  of binary16 rounding (2e-3), close to that of 12 stored reals, where the
  form that divides by 1 - |U_00|^2 loses an order of magnitude on the same
  near-identity links (the reason for the pivoted form).
"""
import numpy as np
import pytest

import synth


def _links(dims, seed, kind):
    U = synth.gauge(dims, seed, kind, 0.3)
    return synth.as_complex(U).reshape(-1, 3, 3)


def _half_with_bit(x, bit):
    """binary16 nearest to x whose last significand bit is `bit` (arrays)."""
    h = np.asarray(x, np.float64).astype(np.float16)
    b = h.view(np.uint16)
    ok = (b & 1) == bit
    sgn, mag = b & 0x8000, b & 0x7FFF
    dn = (sgn | np.maximum(mag, 1) - 1).astype(np.uint16)
    up = (sgn | (mag + 1)).astype(np.uint16)
    vd, vu = dn.view(np.float16).astype(np.float64), up.view(np.float16).astype(np.float64)
    pick = np.where((mag == 0) | (np.abs(vu - x) < np.abs(vd - x)), up, dn)
    return np.where(ok, b, pick).astype(np.uint16)


def _derive(stored, comp, im, neg):
    m = 1.0 - (np.sum(stored ** 2, axis=0) + comp ** 2)
    d = np.sqrt(np.maximum(m, 0.0)) * np.where(neg, -1.0, 1.0)
    return np.where(im, comp + 1j * d, d + 1j * comp)


def _frame(r0, kq):
    """e1 = conj(r0 x e_k) / |.|, e2 = conj(r0 x e1); r0 (N, 3) relabelled."""
    z = np.zeros_like(r0[:, 0])
    c = np.where(kq[:, None], np.stack([r0[:, 1], -r0[:, 0], z], 1),
                 np.stack([-r0[:, 2], z, r0[:, 0]], 1))
    ak2 = np.where(kq, np.abs(r0[:, 2]) ** 2, np.abs(r0[:, 1]) ** 2)
    e1 = np.conj(c) / np.sqrt(1.0 - ak2)[:, None]
    e2 = np.conj(np.cross(r0, e1))
    return e1, e2


def encode(U, rounding=True):
    """(vals (N, 8) float64, bits (N, 8) int).  Without rounding the values
    are kept exact (and the bits kept apart) to check the algebra."""
    N = U.shape[0]
    mags = np.abs(U[:, 0, :]) ** 2
    j = np.argmax(mags, axis=1)  # first of equal maxima
    idx = (j[:, None] + np.arange(3)[None, :]) % 3
    r0 = np.take_along_axis(U[:, 0, :], idx, 1)
    r1 = np.take_along_axis(U[:, 1, :], idx, 1)
    bits = np.zeros((N, 8), int)
    vals = np.zeros((N, 8))
    bits[:, 0], bits[:, 1] = j & 1, j >> 1
    bits[:, 2] = np.abs(r0[:, 0].imag) > np.abs(r0[:, 0].real)
    dv = np.where(bits[:, 2] == 1, r0[:, 0].imag, r0[:, 0].real)
    bits[:, 3] = dv < 0

    def put(k, x):
        vals[:, k] = (_half_with_bit(x, bits[:, k]).view(np.float16).astype(np.float64)
                      if rounding else x)

    put(0, r0[:, 1].real)
    put(1, r0[:, 1].imag)
    put(2, r0[:, 2].real)
    put(3, r0[:, 2].imag)
    bits[:, 4] = vals[:, 2] ** 2 + vals[:, 3] ** 2 < vals[:, 0] ** 2 + vals[:, 1] ** 2
    put(4, np.where(bits[:, 2] == 1, r0[:, 0].real, r0[:, 0].imag))
    d0 = np.stack([_derive(vals[:, :4].T, vals[:, 4], bits[:, 2] == 1, bits[:, 3] == 1),
                   vals[:, 0] + 1j * vals[:, 1], vals[:, 2] + 1j * vals[:, 3]], 1)
    e1, e2 = _frame(d0, bits[:, 4] == 1)
    al = np.sum(np.conj(e1) * r1, 1)
    be = np.sum(np.conj(e2) * r1, 1)
    bits[:, 5] = np.abs(al) ** 2 < np.abs(be) ** 2
    gs = np.where(bits[:, 5] == 1, al, be)
    dl = np.where(bits[:, 5] == 1, be, al)
    bits[:, 6] = np.abs(dl.imag) > np.abs(dl.real)
    bits[:, 7] = np.where(bits[:, 6] == 1, dl.imag, dl.real) < 0
    put(5, gs.real)
    put(6, gs.imag)
    put(7, np.where(bits[:, 6] == 1, dl.real, dl.imag))
    return vals, bits


def decode(vals, bits, dtype=np.float32):
    f = vals.astype(dtype).astype(np.float64) if dtype == np.float32 else vals
    b = bits == 1
    r0 = np.stack([_derive(f[:, :4].T, f[:, 4], b[:, 2], b[:, 3]),
                   f[:, 0] + 1j * f[:, 1], f[:, 2] + 1j * f[:, 3]], 1)
    e1, e2 = _frame(r0, b[:, 4])
    g = f[:, 5] + 1j * f[:, 6]
    d = _derive(np.stack([f[:, 5], f[:, 6]]), f[:, 7], b[:, 6], b[:, 7])
    al = np.where(b[:, 5], g, d)
    be = np.where(b[:, 5], d, g)
    r1 = al[:, None] * e1 + be[:, None] * e2
    r2 = np.conj(al)[:, None] * e2 - np.conj(be)[:, None] * e1
    W = np.stack([r0, r1, r2], 1)
    j = bits[:, 0] | (bits[:, 1] << 1)
    inv = (np.arange(3)[None, :] - j[:, None]) % 3  # column c of U = column c - j of W
    return np.take_along_axis(W, inv[:, None, :].repeat(3, 1), 2)


@pytest.mark.parametrize("kind", [synth.EXP, synth.HAAR])
def test_exact_without_rounding(kind):
    U = _links((4, 4, 4, 4), 11, kind)
    vals, bits = encode(U, rounding=False)
    got = decode(vals, bits, dtype=np.float64)
    assert np.max(np.abs(got - U)) < 1e-13
    if kind == synth.HAAR:  # every relabelling and both pivots occur
        j = bits[:, 0] | (bits[:, 1] << 1)
        assert set(j) == {0, 1, 2} and set(bits[:, 4]) == {0, 1} and set(bits[:, 5]) == {0, 1}


def _err12(U):
    """largest entry error of the 12-real binary16 form (rows 0, 1 rounded,
    row 2 = conj(row0 x row1) in float32)."""
    r = U[:, :2, :]
    rr = (r.real.astype(np.float16).astype(np.float32)
          + 1j * r.imag.astype(np.float16).astype(np.float32))
    r2 = np.conj(np.cross(rr[:, 0], rr[:, 1]))
    W = np.concatenate([rr, r2[:, None, :]], 1)
    return np.max(np.abs(W - U))


def _err_divided(U):
    """largest entry error of the 8-real form that rebuilds rows 1, 2 through
    a division by 1 - |U_00|^2 (row 0 and column 0 stored, binary16)."""
    q = lambda z: z.real.astype(np.float16).astype(np.float64) + 1j * z.imag.astype(
        np.float16).astype(np.float64)
    a2, a3, b1 = q(U[:, 0, 1]), q(U[:, 0, 2]), q(U[:, 1, 0])
    th_a1 = np.angle(U[:, 0, 0]).astype(np.float16).astype(np.float64)
    th_c1 = np.angle(U[:, 2, 0]).astype(np.float16).astype(np.float64)
    a1 = np.sqrt(np.maximum(1 - np.abs(a2) ** 2 - np.abs(a3) ** 2, 0)) * np.exp(1j * th_a1)
    c1 = np.sqrt(np.maximum(1 - np.abs(a1) ** 2 - np.abs(b1) ** 2, 0)) * np.exp(1j * th_c1)
    n = np.abs(a2) ** 2 + np.abs(a3) ** 2
    b2 = -(np.conj(a3) * np.conj(c1) + np.conj(a1) * a2 * b1) / n
    return np.max(np.abs(b2 - U[:, 1, 1]))


@pytest.mark.parametrize("kind", [synth.EXP, synth.HAAR])
def test_binary16_rounding_error(kind):
    U = _links((8, 8, 8, 8), 12, kind)
    vals, bits = encode(U)
    got = decode(vals, bits)
    err8 = np.max(np.abs(got - U))
    err12 = _err12(U)
    assert err8 <= 2e-3, err8
    assert err8 <= 4 * err12 + 1e-4, (err8, err12)
    # the decoded matrices stay unitary to the same order
    I = np.einsum("nab,ncb->nac", got, np.conj(got))
    assert np.max(np.abs(I - np.eye(3))) <= 4e-3
    if kind == synth.EXP:
        # near-identity links: dividing by 1 - |U_00|^2 amplifies the rounding
        assert _err_divided(U) > 5 * err8
