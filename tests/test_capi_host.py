"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/wd.h declares, and rejects invalid arguments before
any HIP call."""
import ctypes
import subprocess

import pytest

import paper_1810_04201_amd as wd


def test_header_symbols_exported():
    names = wd.header_functions()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", wd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(wd.lib, n)


def test_binding_covers_header():
    assert set(wd.header_functions()) == set(wd._SIGS)


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 0, 4), (4, 4, 4, 1), (-2, 4, 4, 4)])
def test_bad_dims_rejected(dims):
    d = (ctypes.c_int32 * 4)(*dims)
    h = ctypes.c_void_p()
    rc = wd.lib.wd_create_lattice(d, 1, ctypes.byref(h))
    assert rc == wd.WD_ERR_ARG
    assert "even" in wd.last_error()
    assert not h.value


def test_solve_params_layout():
    # the form field fills the struct's tail padding: every earlier offset
    # and the size match the header's natural C layout
    P = wd.wd_solve_params
    assert ctypes.sizeof(P) == 48
    assert [getattr(P, f).offset for f in ("kappa", "tol", "max_iter", "prec_inner", "nrhs",
            "reliable_max_iter", "reliable_delta", "x0_given", "form")] == \
        [0, 8, 16, 20, 24, 28, 32, 40, 44]


def test_plus_kappa_flag_accepted():
    d = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    h = ctypes.c_void_p()
    assert wd.lib.wd_create_lattice(d, wd.WD_BC_ANTIPERIODIC_T | wd.WD_SIGN_PLUS_KAPPA,
                                    ctypes.byref(h)) == wd.WD_OK
    assert wd.lib.wd_destroy_lattice(h) == wd.WD_OK


def test_volume_limit():
    # 64^3 x 64 (16.8 M sites) is accepted; beyond 2^28 sites is not
    d = (ctypes.c_int32 * 4)(64, 64, 64, 64)
    h = ctypes.c_void_p()
    assert wd.lib.wd_create_lattice(d, 1, ctypes.byref(h)) == wd.WD_OK
    v = ctypes.c_int64()
    assert wd.lib.wd_lattice_volume(h, ctypes.byref(v)) == 0 and v.value == 64 ** 4
    assert wd.lib.wd_destroy_lattice(h) == wd.WD_OK
    d = (ctypes.c_int32 * 4)(256, 256, 64, 128)
    assert wd.lib.wd_create_lattice(d, 1, ctypes.byref(h)) == wd.WD_ERR_ARG
    assert "2^28" in wd.last_error()


def test_bad_flags_and_null():
    d = (ctypes.c_int32 * 4)(4, 4, 4, 4)
    h = ctypes.c_void_p()
    assert wd.lib.wd_create_lattice(d, 0x10, ctypes.byref(h)) == wd.WD_ERR_ARG
    assert wd.lib.wd_create_lattice(None, 1, ctypes.byref(h)) == wd.WD_ERR_ARG
    assert wd.lib.wd_destroy_lattice(None) == wd.WD_ERR_ARG
    assert wd.lib.wd_poll(None, 1, None) in (wd.WD_ERR_ARG, wd.WD_ERR_STATE)


def test_lattice_lifecycle_host_only():
    lat = wd.Lattice((4, 6, 8, 10))
    assert lat.volume == 1920
    v = ctypes.c_int64()
    assert wd.lib.wd_lattice_volume(lat.handle, ctypes.byref(v)) == 0 and v.value == 1920
    assert lat.gauge_bytes() == 0
    # no gauge yet: 18-real float64 links, deviation unchecked
    assert lat.links_info() == (18, -1.0)
    n = ctypes.c_int(7)
    assert wd.lib.wd_lattice_links_info(lat.handle, ctypes.byref(n), None) == 0 and n.value == 18
    assert wd.lib.wd_lattice_links_info(None, None, None) == wd.WD_ERR_ARG
    lat.close()


def test_solve_rejected_without_gauge_and_bad_params():
    lat = wd.Lattice((4, 4, 4, 4))
    infos = (wd.wd_solve_info * 1)()
    p = wd.make_params(0.12, tol=1e-10)
    dummy = ctypes.c_void_p(16)
    assert wd.lib.wd_cg_solve(lat.handle, ctypes.byref(p), dummy, ctypes.c_void_p(32), infos,
                              None) == wd.WD_ERR_NOGAUGE
    for bad in (wd.make_params(0.12, tol=0.0), wd.make_params(0.12, nrhs=13),
                wd.make_params(0.12, nrhs=0), wd.make_params(float("nan")),
                wd.make_params(0.12, max_iter=0), wd.make_params(0.12, prec=2),
                wd.make_params(0.12, form=2), wd.make_params(0.12, form="cgne", x0_given=True)):
        if bad.prec_inner == 2:
            bad.prec_inner = 7
        assert wd.lib.wd_cg_solve(lat.handle, ctypes.byref(bad), dummy, ctypes.c_void_p(32),
                                  infos, None) == wd.WD_ERR_ARG
    lat.close()


def test_apply_rejects_bad_args_before_gpu():
    lat = wd.Lattice((4, 4, 4, 4))
    a, b = ctypes.c_void_p(16), ctypes.c_void_p(32)
    assert wd.lib.wd_apply(lat.handle, 0.1, 9, 0, 1, a, b, None) == wd.WD_ERR_ARG
    assert wd.lib.wd_apply(lat.handle, 0.1, 0, 0, 13, a, b, None) == wd.WD_ERR_ARG
    assert wd.lib.wd_apply(lat.handle, 0.1, 0, 2, 1, a, b, None) == wd.WD_ERR_ARG
    assert wd.lib.wd_apply(lat.handle, float("inf"), 0, 0, 1, a, b, None) == wd.WD_ERR_ARG
    assert wd.lib.wd_apply(lat.handle, 0.1, 0, 0, 1, a, a, None) == wd.WD_ERR_ARG
    # no gauge yet: refused before any device work
    assert wd.lib.wd_apply(lat.handle, 0.1, 0, 0, 1, a, b, None) == wd.WD_ERR_NOGAUGE
    lat.close()


def test_no_unresolved_library_symbols():
    out = subprocess.run(["nm", "-D", "--undefined-only", wd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    own = [line for line in out.splitlines() if "_ZN2wd" in line or " wd_" in line]
    assert not own, own


def test_even_odd_needs_even_x_bricks(monkeypatch):
    # an odd brick x extent (forced) cannot pair x neighbours into halves:
    # refused before any device work, for the solve and the Schur operator
    monkeypatch.setenv("WD_BRICK", "3,4,4")
    lat = wd.Lattice((6, 4, 4, 4))
    infos = (wd.wd_solve_info * 1)()
    p = wd.make_params(0.12, even_odd=True)
    a, b = ctypes.c_void_p(16), ctypes.c_void_p(32)
    assert wd.lib.wd_cg_solve(lat.handle, ctypes.byref(p), a, b, infos, None) == wd.WD_ERR_ARG
    assert "even x extent" in wd.last_error()
    assert wd.lib.wd_apply_schur(lat.handle, 0.12, 0, 0, 1, a, b, None) == wd.WD_ERR_ARG
    lat.close()


def test_bad_form_flags_rejected():
    lat = wd.Lattice((4, 4, 4, 4))
    infos = (wd.wd_solve_info * 1)()
    a, b = ctypes.c_void_p(16), ctypes.c_void_p(32)
    for form in (2, 1 << 9, wd.WD_SOLVE_EVEN_ODD | 3):
        p = wd.make_params(0.12, form=form)
        assert wd.lib.wd_cg_solve(lat.handle, ctypes.byref(p), a, b, infos, None) == wd.WD_ERR_ARG
    lat.close()
