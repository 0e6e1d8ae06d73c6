"""Helpers shared by the GPU tests (inputs from synth, no method arithmetic)."""
import numpy as np

import synth


def site_rel_err(got, want):
    """max over sites (and rhs) of |got - want| / |want| per site."""
    g = np.asarray(got).reshape(-1, 24)
    w = np.asarray(want).reshape(-1, 24)
    num = np.linalg.norm(g - w, axis=1)
    den = np.linalg.norm(w, axis=1)
    return float(np.max(num / den))


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gauge(dims, seed, kind="exp"):
    return synth.gauge(dims, seed, synth.EXP if kind == "exp" else synth.HAAR, 0.3)


def vol(dims):
    return int(np.prod(dims))


def assert_same_count_parity(x, xo_n, bound=1e-9):
    """A float64 GPU solution against the oracle's iterate after the same
    number of CG steps: relative 2-norm and largest element difference (as a
    fraction of the largest element) both within `bound`."""
    a = np.asarray(x).ravel()
    b = np.asarray(xo_n).ravel()
    r = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    e = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    assert r <= bound and e <= bound, (r, e)
    return r, e
