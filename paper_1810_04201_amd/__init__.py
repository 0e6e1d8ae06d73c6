"""Python binding of libwdirac (the MI355X Wilson-Dirac solver library).

Argument marshalling only: every step of the operator and the solve runs in
the HIP kernels of ``libwdirac.so``; torch supplies device memory and
streams.  The functions keep the C names of ``include/wd.h`` (``wd_apply_D``,
``wd_cg_solve``, ``wd_submit`` ...) and take torch tensors where the C call
takes device pointers.  Small classes (``Lattice``, ``Field``, ``Server``)
own the opaque handles.

Canonical tensors are float64 on the GPU:
  gauge  (V, 4, 3, 3, 2)            U_mu(s)[a][b] (re, im)
  spinor (V, 4, 3, 2) or (nrhs, V, 4, 3, 2)
with site s = x + Lx*(y + Ly*(z + Lz*t)).

If the library is missing or fails to load, importing this package raises:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# WDIRAC_LIB may point at another build of the same library (tuning variants)
LIB_PATH = os.environ.get("WDIRAC_LIB") or os.path.join(HERE, "libwdirac.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "wd.h")

WD_OK = 0
WD_PENDING = 1
WD_ERR_ARG = -1
WD_ERR_NOMEM = -2
WD_ERR_HIP = -3
WD_ERR_NOCONV = -4
WD_ERR_NUMERIC = -5
WD_ERR_NOGAUGE = -6
WD_ERR_NOTFOUND = -7
WD_ERR_STATE = -8
WD_F64, WD_F32, WD_F16 = 0, 1, 2
WD_BC_ANTIPERIODIC_T = 1
WD_SIGN_PLUS_KAPPA = 2
WD_F16_LINKS_8 = 4
WD_FORM_CGNR, WD_FORM_CGNE = 0, 1
WD_SOLVE_EVEN_ODD = 1 << 8
WD_HALO_FIRST, WD_HALO_LAST, WD_HALO_INTERIOR, WD_HALO_ENDS = 1, 2, 4, 8
HALO_REGION = {"all": 0, "interior": WD_HALO_INTERIOR, "ends": WD_HALO_ENDS}
FORM = {"cgnr": WD_FORM_CGNR, "cgne": WD_FORM_CGNE, WD_FORM_CGNR: WD_FORM_CGNR,
        WD_FORM_CGNE: WD_FORM_CGNE}

PREC = {"f64": WD_F64, "f32": WD_F32, "f16": WD_F16, WD_F64: WD_F64, WD_F32: WD_F32,
        WD_F16: WD_F16}


class WdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"wd error {code}: {msg}")
        self.code = code


class wd_solve_params(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("prec_inner", ctypes.c_int32),
                ("nrhs", ctypes.c_int32), ("reliable_max_iter", ctypes.c_int32),
                ("reliable_delta", ctypes.c_double), ("x0_given", ctypes.c_int32),
                ("form", ctypes.c_int32)]


class wd_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("reliable_updates", ctypes.c_int32), ("true_rel_resid", ctypes.c_double),
                ("rel_resid_D", ctypes.c_double), ("seconds", ctypes.c_double),
                ("queued_seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class wd_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("chunk_iters", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("streams", ctypes.POINTER(ctypes.c_void_p))]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_SIGS = {
    "wd_create_lattice": [ctypes.POINTER(ctypes.c_int32), ctypes.c_uint32, ctypes.POINTER(_vp)],
    "wd_destroy_lattice": [_vp],
    "wd_lattice_volume": [_vp, ctypes.POINTER(ctypes.c_int64)],
    "wd_set_gauge": [_vp, _vp, _vp],
    "wd_lattice_gauge_bytes": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "wd_lattice_links_info": [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)],
    "wd_apply_D": [_vp, ctypes.c_double, _i32, _vp, _vp, _vp],
    "wd_apply_Ddag": [_vp, ctypes.c_double, _i32, _vp, _vp, _vp],
    "wd_apply": [_vp, ctypes.c_double, _i32, _i32, _i32, _vp, _vp, _vp],
    "wd_apply_schur": [_vp, ctypes.c_double, _i32, _i32, _i32, _vp, _vp, _vp],
    "wd_apply_noalloc": [_vp, ctypes.c_double, _i32, _i32, _i32, _vp, _vp, _vp],
    "wd_set_halo_gauge": [_vp, _vp, _vp],
    "wd_halo_pack": [_vp, _i32, _vp, _vp, _vp, _vp],
    "wd_dslash_halo": [_vp, ctypes.c_double, _i32, _vp, _vp, _vp, _vp, ctypes.c_uint32, _vp],
    "wd_field_create": [_vp, _i32, _i32, ctypes.POINTER(_vp)],
    "wd_field_destroy": [_vp],
    "wd_field_import": [_vp, _vp, _vp],
    "wd_field_export": [_vp, _vp, _vp],
    "wd_dslash": [_vp, ctypes.c_double, _i32, _vp, _vp, _vp],
    "wd_cg_solve": [_vp, ctypes.POINTER(wd_solve_params), _vp, _vp,
                    ctypes.POINTER(wd_solve_info), _vp],
    "wd_server_create": [ctypes.POINTER(wd_server_config), ctypes.POINTER(_vp)],
    "wd_submit": [_vp, _vp, ctypes.POINTER(wd_solve_params), _vp, _vp,
                  ctypes.POINTER(ctypes.c_uint64)],
    "wd_poll": [_vp, ctypes.c_uint64, ctypes.POINTER(wd_solve_info)],
    "wd_server_stats": [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(ctypes.c_double)],
    "wd_server_peak_bytes": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "wd_server_destroy": [_vp],
    "wd_stream_probe": [ctypes.POINTER(_vp), _i32, _vp, ctypes.c_size_t, _vp],
    "wd_last_error": [],
    "wd_timing_enable": [_i32],
    "wd_timing_reset": [],
    "wd_timing_read": [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_int64)],
}


def header_functions(path: str = HEADER):
    """Names of the functions include/wd.h declares."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wd_[A-Za-z0-9_]+)\s*\(", txt)))


def _load():
    # PyTorch ships its own libamdhip64.so.7 (same soname as the system one).
    # Import it first so that the library binds to the runtime torch already
    # uses: one HIP runtime per process, or neither sees the GPU.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "wd_last_error" else ctypes.c_int
    return lib


lib = _load()


def last_error() -> str:
    return (lib.wd_last_error() or b"").decode()


def _check(rc: int, allow=(WD_OK,)) -> int:
    if rc not in allow:
        raise WdError(rc, last_error())
    return rc


# ------------------------------------------------------------------ torch helpers

def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return _vp(stream)
    return _vp(stream.cuda_stream)


def _dptr(t, numel=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return _vp(t.data_ptr())


# ------------------------------------------------------------------ C names

def wd_create_lattice(dims, antiperiodic_t: bool = True, plus_kappa: bool = False,
                      f16_links8: bool = False):
    d = (ctypes.c_int32 * 4)(*[int(v) for v in dims])
    h = _vp()
    flags = ((WD_BC_ANTIPERIODIC_T if antiperiodic_t else 0) |
             (WD_SIGN_PLUS_KAPPA if plus_kappa else 0) | (WD_F16_LINKS_8 if f16_links8 else 0))
    _check(lib.wd_create_lattice(d, flags, ctypes.byref(h)))
    return h


def wd_destroy_lattice(h):
    _check(lib.wd_destroy_lattice(h))


def wd_set_gauge(h, U, volume, stream=None):
    _check(lib.wd_set_gauge(h, _dptr(U, volume * 72, "U"), _stream(stream)))


def wd_apply(h, kappa, prec, dagger, nrhs, inp, out, volume, stream=None):
    n = volume * 24 * nrhs
    _check(lib.wd_apply(h, float(kappa), PREC[prec], int(dagger), int(nrhs),
                        _dptr(inp, n, "in"), _dptr(out, n, "out"), _stream(stream)))


def wd_apply_schur(h, kappa, prec, dagger, nrhs, inp, out, volume, stream=None):
    n = volume * 24 * nrhs
    _check(lib.wd_apply_schur(h, float(kappa), PREC[prec], int(dagger), int(nrhs),
                              _dptr(inp, n, "in"), _dptr(out, n, "out"), _stream(stream)))


def face_numel(lattice, nrhs=1):
    """float64 elements of one halo face buffer (96 bytes per face site)."""
    return nrhs * 12 * (lattice.volume // lattice.dims[3])


def wd_set_halo_gauge(lattice, U_prev, stream=None):
    n = 18 * (lattice.volume // lattice.dims[3])
    _check(lib.wd_set_halo_gauge(lattice.handle, _dptr(U_prev, n, "U_prev"), _stream(stream)))


def wd_halo_pack(lattice, field, send_prev, send_next, dagger=False, stream=None):
    n = face_numel(lattice, field.nrhs)
    _check(lib.wd_halo_pack(lattice.handle, 1 if dagger else 0, field.handle,
                            _dptr(send_prev, n, "send_prev"), _dptr(send_next, n, "send_next"),
                            _stream(stream)))


def wd_dslash_halo(lattice, kappa, fin, fout, recv_prev, recv_next, first, last, dagger=False,
                   stream=None, region="all"):
    """region: "all", "interior" (no face read; recv_* may be None) or
    "ends" (the chunks holding the slab's first and last slices)."""
    n = face_numel(lattice, fin.nrhs)
    flags = (WD_HALO_FIRST if first else 0) | (WD_HALO_LAST if last else 0) | HALO_REGION[region]
    rp = None if recv_prev is None else _dptr(recv_prev, n, "recv_prev")
    rn = None if recv_next is None else _dptr(recv_next, n, "recv_next")
    _check(lib.wd_dslash_halo(lattice.handle, float(kappa), 1 if dagger else 0, fin.handle,
                              fout.handle, rp, rn, flags, _stream(stream)))


def wd_apply_D(h, kappa, prec, inp, out, volume, stream=None):
    _check(lib.wd_apply_D(h, float(kappa), PREC[prec], _dptr(inp, volume * 24, "in"),
                          _dptr(out, volume * 24, "out"), _stream(stream)))


def wd_apply_Ddag(h, kappa, prec, inp, out, volume, stream=None):
    _check(lib.wd_apply_Ddag(h, float(kappa), PREC[prec], _dptr(inp, volume * 24, "in"),
                             _dptr(out, volume * 24, "out"), _stream(stream)))


def make_params(kappa, tol=1e-10, max_iter=20000, prec="f64", nrhs=1, reliable_max_iter=50,
                reliable_delta=0.1, x0_given=False, form="cgnr", even_odd=False):
    f = FORM[form] if form in FORM else int(form)
    if even_odd:
        f |= WD_SOLVE_EVEN_ODD
    return wd_solve_params(float(kappa), float(tol), int(max_iter), PREC[prec], int(nrhs),
                           int(reliable_max_iter), float(reliable_delta), 1 if x0_given else 0, f)


def wd_cg_solve(h, params: wd_solve_params, b, x, volume, stream=None):
    """Blocking solve; returns (rc, [info dict per rhs])."""
    n = volume * 24 * params.nrhs
    infos = (wd_solve_info * params.nrhs)()
    rc = lib.wd_cg_solve(h, ctypes.byref(params), _dptr(b, n, "b"), _dptr(x, n, "x"), infos,
                         _stream(stream))
    if rc in (WD_ERR_ARG, WD_ERR_NOMEM, WD_ERR_HIP, WD_ERR_NOGAUGE, WD_ERR_STATE):
        raise WdError(rc, last_error())
    return rc, [i.as_dict() for i in infos]


def wd_stream_probe(srcs, dst, stream=None):
    """dst = the element-wise sum of the tensors in srcs (1..4 contiguous
    float64 device tensors of dst's size) through the library's streaming
    probe kernel."""
    nb = dst.numel() * dst.element_size()
    for t in list(srcs) + [dst]:
        if not (t.is_cuda and t.is_contiguous()) or t.numel() * t.element_size() != nb:
            raise ValueError("sources and dst must be contiguous device tensors of one size")
    arr = (_vp * len(srcs))(*[s.data_ptr() for s in srcs])
    _check(lib.wd_stream_probe(arr, len(srcs), _vp(dst.data_ptr()), nb, _stream(stream)))


def wd_timing_enable(on=True):
    _check(lib.wd_timing_enable(1 if on else 0))


def wd_timing_reset():
    _check(lib.wd_timing_reset())


def wd_timing_read(name: str):
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(lib.wd_timing_read(name.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


# ------------------------------------------------------------------ objects

class Lattice:
    """Owns a wd_lattice handle: geometry plus resident packed gauge forms."""

    def __init__(self, dims, antiperiodic_t: bool = True, plus_kappa: bool = False,
                 f16_links8: bool = False):
        """f16_links8: binary16 links stored as 8 reals (WD_F16_LINKS_8)."""
        self.dims = tuple(int(v) for v in dims)
        self.volume = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.handle = wd_create_lattice(self.dims, antiperiodic_t, plus_kappa, f16_links8)

    def set_gauge(self, U, stream=None):
        wd_set_gauge(self.handle, U, self.volume, stream)

    def links_info(self):
        """(float64 link reals 12 or 18, largest row-2 deviation from special
        unitary measured by set_gauge, -1 if unchecked)."""
        n = ctypes.c_int()
        d = ctypes.c_double()
        _check(lib.wd_lattice_links_info(self.handle, ctypes.byref(n), ctypes.byref(d)))
        return n.value, d.value

    def gauge_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib.wd_lattice_gauge_bytes(self.handle, ctypes.byref(b)))
        return b.value

    def apply(self, kappa, inp, out, prec="f64", dagger=False, nrhs=1, stream=None):
        wd_apply(self.handle, kappa, prec, dagger, nrhs, inp, out, self.volume, stream)

    def apply_schur(self, kappa, inp, out, prec="f64", dagger=False, nrhs=1, stream=None):
        wd_apply_schur(self.handle, kappa, prec, dagger, nrhs, inp, out, self.volume, stream)

    def solve(self, b, x, kappa, tol=1e-10, prec="f64", nrhs=1, max_iter=20000,
              reliable_max_iter=50, reliable_delta=0.1, x0_given=False, form="cgnr",
              even_odd=False, stream=None):
        p = make_params(kappa, tol, max_iter, prec, nrhs, reliable_max_iter, reliable_delta,
                        x0_given, form, even_odd)
        return wd_cg_solve(self.handle, p, b, x, self.volume, stream)

    def close(self):
        if self.handle:
            wd_destroy_lattice(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Field:
    """A spinor field in the kernels' internal layout (wd_field)."""

    def __init__(self, lattice: Lattice, prec="f64", nrhs=1):
        self.lattice = lattice
        self.nrhs = int(nrhs)
        self.prec = PREC[prec]
        h = _vp()
        _check(lib.wd_field_create(lattice.handle, self.prec, self.nrhs, ctypes.byref(h)))
        self.handle = h

    def load(self, canon, stream=None):
        n = self.lattice.volume * 24 * self.nrhs
        _check(lib.wd_field_import(self.handle, _dptr(canon, n, "canon"), _stream(stream)))

    def store(self, canon, stream=None):
        n = self.lattice.volume * 24 * self.nrhs
        _check(lib.wd_field_export(self.handle, _dptr(canon, n, "canon"), _stream(stream)))

    def close(self):
        if self.handle:
            _check(lib.wd_field_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wd_dslash(lattice: Lattice, kappa, dagger, fin: Field, fout: Field, stream=None):
    _check(lib.wd_dslash(lattice.handle, float(kappa), int(dagger), fin.handle, fout.handle,
                         _stream(stream)))


class Server:
    """Continuous-batching solve server (wd_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 8, chunk_iters: int = 0,
                 streams=None):
        """streams: optional torch streams (or raw hipStream_t ints) for the
        slots; the server then runs len(streams) requests at once on them."""
        self._streams = list(streams or [])
        arr = (ctypes.c_void_p * max(1, len(self._streams)))(
            *[s if isinstance(s, int) else s.cuda_stream for s in self._streams])
        self._stream_arr = arr
        cfg = wd_server_config(int(hbm_budget_bytes), int(max_active), int(chunk_iters),
                               len(self._streams),
                               ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
                               if self._streams else None)
        h = _vp()
        _check(lib.wd_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, lattice: Lattice, b, x, kappa, tol=1e-10, prec="f32", nrhs=1,
               max_iter=20000, reliable_max_iter=50, reliable_delta=0.1, form="cgnr",
               even_odd=False) -> int:
        p = make_params(kappa, tol, max_iter, prec, nrhs, reliable_max_iter, reliable_delta,
                        form=form, even_odd=even_odd)
        n = lattice.volume * 24 * nrhs
        # the server reads b on its own stream: make the caller's writes visible
        _torch().cuda.current_stream().synchronize()
        t = ctypes.c_uint64()
        _check(lib.wd_submit(self.handle, lattice.handle, ctypes.byref(p), _dptr(b, n, "b"),
                             _dptr(x, n, "x"), ctypes.byref(t)))
        self._keep[t.value] = (b, x, nrhs)
        return t.value

    def poll(self, ticket: int):
        nrhs = self._keep.get(ticket, (None, None, 1))[2]
        infos = (wd_solve_info * nrhs)()
        rc = lib.wd_poll(self.handle, ctypes.c_uint64(ticket), infos)
        if rc == WD_ERR_NOTFOUND:
            raise WdError(rc, last_error())
        return rc, [i.as_dict() for i in infos]

    def stats(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib.wd_server_stats(self.handle, ctypes.byref(a), ctypes.byref(b),
                                   ctypes.byref(c)))
        return {"solves_per_s": a.value, "p50_s": b.value, "p99_s": c.value}

    def peak_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib.wd_server_peak_bytes(self.handle, ctypes.byref(b)))
        return b.value

    def close(self):
        if self.handle:
            _check(lib.wd_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
