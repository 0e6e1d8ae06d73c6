"""Seeded synthetic inputs shared by the oracle's tests and the GPU path.

Nothing here computes the Dirac operator or any solver step; the module only
draws gauge fields, sources and gauge rotations (see ``gen.c`` for the
generator definitions: SplitMix64, Box-Muller, Haar-QR SU(3) and
exp(i eps H) SU(3) links).  The C part is compiled with gcc on first use
(or by the package build step) into ``_libsynth.so`` next to this file.

Canonical array shapes (float64, last axis = (re, im)):
  gauge  (V, 4, 3, 3, 2)   U_mu(s)[a][b], mu = 0..3 = x, y, z, t
  spinor (V, 4, 3, 2)      psi(s)[spin][colour]
  site s = x + Lx*(y + Ly*(z + Lz*t))
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "_libsynth.so")
_lock = threading.Lock()
_lib = None

HAAR = 0
EXP = 1


def build(force: bool = False) -> str:
    """Compile gen.c into _libsynth.so (gcc, OpenMP, strict FP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-std=c99", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i32p = ctypes.POINTER(ctypes.c_int32)
            dp = ctypes.POINTER(ctypes.c_double)
            lib.synth_gauge.argtypes = [i32p, ctypes.c_uint64, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int32, ctypes.c_int32, dp]
            lib.synth_gauge_unit.argtypes = [i32p, dp]
            lib.synth_gaussian_spinor.argtypes = [ctypes.c_uint64, ctypes.c_int64,
                                                  ctypes.c_int64, dp]
            lib.synth_gauge_rotation.argtypes = [ctypes.c_uint64, ctypes.c_int64, dp]
            lib.synth_splitmix_stream.argtypes = [ctypes.c_uint64, ctypes.c_int64,
                                                  ctypes.POINTER(ctypes.c_uint64)]
            for f in (lib.synth_gauge, lib.synth_gauge_unit, lib.synth_gaussian_spinor,
                      lib.synth_gauge_rotation, lib.synth_splitmix_stream):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    if d.shape != (4,) or np.any(d < 1):
        raise ValueError("dims must be four positive extents (Lx, Ly, Lz, Lt)")
    return d


def volume(dims) -> int:
    d = _dims(dims)
    return int(np.prod(d.astype(np.int64)))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gauge(dims, seed: int, kind: int = EXP, eps: float = 0.3, t0: int = 0, t1=None,
          out: np.ndarray | None = None) -> np.ndarray:
    """SU(3) links for time slices [t0, t1): Haar-QR (kind=HAAR) or exp(i eps H).

    Returns float64 (n_sites, 4, 3, 3, 2).  ``out`` may be any C-contiguous
    float64 buffer of that size (e.g. a pinned host tensor's numpy view).
    """
    d = _dims(dims)
    if t1 is None:
        t1 = int(d[3])
    if not (0 <= t0 <= t1 <= d[3]):
        raise ValueError("bad t-slab range")
    n = int(d[0]) * int(d[1]) * int(d[2]) * (t1 - t0)
    if out is None:
        out = np.empty((n, 4, 3, 3, 2), dtype=np.float64)
    if out.dtype != np.float64 or not out.flags.c_contiguous or out.size != n * 72:
        raise ValueError("out must be C-contiguous float64 with n*72 elements")
    rc = _load().synth_gauge(d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), kind, float(eps),
                             t0, t1, _dp(out))
    if rc != 0:
        raise ValueError("synth_gauge failed")
    return out


def gauge_unit(dims) -> np.ndarray:
    d = _dims(dims)
    out = np.empty((volume(d), 4, 3, 3, 2), dtype=np.float64)
    _load().synth_gauge_unit(d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(out))
    return out


def gaussian_spinor(dims, seed: int, s0: int = 0, s1=None, out=None) -> np.ndarray:
    """Spinor with every component N(0,1); sites [s0, s1).  (n, 4, 3, 2)."""
    v = volume(dims)
    if s1 is None:
        s1 = v
    if not (0 <= s0 <= s1 <= v):
        raise ValueError("bad site range")
    n = s1 - s0
    if out is None:
        out = np.empty((n, 4, 3, 2), dtype=np.float64)
    if out.dtype != np.float64 or not out.flags.c_contiguous or out.size != n * 24:
        raise ValueError("out must be C-contiguous float64 with n*24 elements")
    _load().synth_gaussian_spinor(ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), s0, s1, _dp(out))
    return out


def gaussian_sources(dims, seeds) -> np.ndarray:
    """Several Gaussian sources stacked: (nrhs, V, 4, 3, 2)."""
    v = volume(dims)
    out = np.empty((len(seeds), v, 4, 3, 2), dtype=np.float64)
    for k, s in enumerate(seeds):
        gaussian_spinor(dims, s, out=out[k])
    return out


def point_source(dims, spin: int = 0, colour: int = 0, site: int = 0) -> np.ndarray:
    """Single entry set to 1 + 0i (spin, colour) at one site."""
    v = volume(dims)
    out = np.zeros((v, 4, 3, 2), dtype=np.float64)
    out[site, spin, colour, 0] = 1.0
    return out


def spin_colour_point_sources(dims, site: int = 0) -> np.ndarray:
    """The 12 point sources k = 3*spin + colour at one site: (12, V, 4, 3, 2)."""
    v = volume(dims)
    out = np.zeros((12, v, 4, 3, 2), dtype=np.float64)
    for k in range(12):
        out[k, site, k // 3, k % 3, 0] = 1.0
    return out


def gauge_rotation(dims, seed: int) -> np.ndarray:
    """Haar SU(3) matrix per site (random gauge transformation): (V, 3, 3, 2)."""
    v = volume(dims)
    out = np.empty((v, 3, 3, 2), dtype=np.float64)
    _load().synth_gauge_rotation(ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), v, _dp(out))
    return out


def splitmix_stream(key: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().synth_splitmix_stream(ctypes.c_uint64(key & 0xFFFFFFFFFFFFFFFF), n,
                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def as_complex(a: np.ndarray) -> np.ndarray:
    """View a (..., 2) float64 array as complex128 (...)."""
    a = np.ascontiguousarray(a)
    return a.view(np.complex128)[..., 0]


def as_real(c: np.ndarray) -> np.ndarray:
    """complex128 (...) -> float64 (..., 2)."""
    c = np.ascontiguousarray(c, dtype=np.complex128)
    return c.view(np.float64).reshape(c.shape + (2,))
