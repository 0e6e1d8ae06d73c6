"""Parity of the HIP stencil (wd_apply / wd_dslash) with the CPU oracle.

Tolerances: FP64 <= 1e-13 per site (relative, Gaussian inputs so that no
site is near zero), FP32 <= 1e-5, FP16 with 12-real links <= 5e-3.  Lattice
extents are distinct (4x6x8x10) to catch axis mix-ups, 2^4 has coinciding
forward/backward neighbours, and the grid always ends in a partial block.
"""
import numpy as np
import pytest

import synth
from oracle import gauge as ogauge
from oracle import wilson
from gpu_util import gauge, rel, site_rel_err, vol

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-5, "f16": 5e-3}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def wd():
    import paper_1810_04201_amd as wd
    return wd


def _apply(wd, torch, dev, dims, U, psi, kappa, prec, dagger, nrhs=1):
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    pd = torch.from_numpy(np.ascontiguousarray(psi)).to(dev)
    od = torch.full_like(pd, float("nan"))
    lat.apply(kappa, pd, od, prec=prec, dagger=dagger, nrhs=nrhs)
    torch.cuda.synchronize()
    out = od.cpu().numpy()
    lat.close()
    return out


DIMS = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 6, 8, 10), (2, 4, 6, 8), (8, 8, 8, 8)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("dagger", [0, 1])
def test_dslash_parity(torch_dev, wd, dims, prec, dagger):
    torch, dev = torch_dev
    print(f"dslash parity dims={dims} prec={prec} dagger={dagger}", flush=True)
    U = gauge(dims, 11, "exp")
    psi = synth.gaussian_spinor(dims, 12)
    k = 0.1245
    got = _apply(wd, torch, dev, dims, U, psi, k, prec, dagger)
    want = (wilson.apply_Ddag if dagger else wilson.apply_D)(U, psi, dims, k)
    assert site_rel_err(got, want) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_dslash_haar_links(torch_dev, wd, prec):
    torch, dev = torch_dev
    dims = (4, 6, 8, 10)
    U = gauge(dims, 3, "haar")
    psi = synth.gaussian_spinor(dims, 4)
    got = _apply(wd, torch, dev, dims, U, psi, 0.2, prec, 0)
    assert site_rel_err(got, wilson.apply_D(U, psi, dims, 0.2)) <= TOL[prec]


def test_dslash_periodic_t(torch_dev, wd):
    torch, dev = torch_dev
    dims = (4, 4, 4, 6)
    U = gauge(dims, 5)
    psi = synth.gaussian_spinor(dims, 6)
    lat = wd.Lattice(dims, antiperiodic_t=False)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    pd = torch.from_numpy(psi).to(dev)
    od = torch.empty_like(pd)
    lat.apply(0.13, pd, od)
    torch.cuda.synchronize()
    want = wilson.apply_D(U, psi, dims, 0.13, antiperiodic_t=False)
    assert site_rel_err(od.cpu().numpy(), want) <= 1e-13
    lat.close()


def test_dslash_16x32_config2_fields(torch_dev, wd):
    """16^3 x 32, eps = 0.3 links seed 2, Gaussian source seed 102."""
    torch, dev = torch_dev
    dims = (16, 16, 16, 32)
    U = gauge(dims, 2)
    psi = synth.gaussian_spinor(dims, 102)
    for dagger in (0, 1):
        got = _apply(wd, torch, dev, dims, U, psi, 0.124, "f64", dagger)
        want = (wilson.apply_Ddag if dagger else wilson.apply_D)(U, psi, dims, 0.124)
        assert site_rel_err(got, want) <= 1e-13


@pytest.mark.parametrize("nrhs", [2, 5, 12])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_dslash_multi_rhs(torch_dev, wd, nrhs, prec):
    torch, dev = torch_dev
    dims = (4, 6, 4, 8)
    U = gauge(dims, 21)
    psis = synth.gaussian_sources(dims, [100 + k for k in range(nrhs)])
    for dagger in (0, 1):
        got = _apply(wd, torch, dev, dims, U, psis, 0.124, prec, dagger, nrhs=nrhs)
        want = wilson.apply_D_multi(U, psis, dims, 0.124, dagger=bool(dagger))
        assert site_rel_err(got, want) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("nrhs", [1, 3])
def test_dslash_384_site_bricks(torch_dev, wd, monkeypatch, prec, nrhs):
    """Bricks of 8x8x6 = 384 sites: every precision marches two 192-site
    parts of each brick slice (neighbours across the parts come from memory).
    Full parity with the oracle, D and D^dag, 1 and 3 rhs."""
    torch, dev = torch_dev
    monkeypatch.setenv("WD_BRICK", "8,8,6")
    dims = (8, 8, 12, 6)
    print(f"384-site bricks prec={prec} nrhs={nrhs}", flush=True)
    U = gauge(dims, 21, "exp")
    psi = synth.gaussian_sources(dims, [22 + k for k in range(nrhs)])
    for dagger in (0, 1):
        got = _apply(wd, torch, dev, dims, U, psi if nrhs > 1 else psi[0], 0.1245, prec, dagger,
                     nrhs=nrhs)
        got = got.reshape(psi.shape)
        op = wilson.apply_Ddag if dagger else wilson.apply_D
        for k in range(nrhs):
            assert site_rel_err(got[k], op(U, psi[k], dims, 0.1245)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_dslash_ragged_last_chunk_twelve_rhs(torch_dev, wd, prec):
    """4x20x20x20 with 12 rhs: the marching stencil takes chunks of 3 time
    slices, so the last chunk of every column has 2 (20 = 6 x 3 + 2; the host
    layout check pins this chunk length).  D and D^dag against the oracle
    for every rhs."""
    torch, dev = torch_dev
    dims = (4, 20, 20, 20)
    print(f"ragged last chunk, 12 rhs, prec={prec}", flush=True)
    U = gauge(dims, 29, "exp")
    psi = synth.gaussian_sources(dims, [30 + k for k in range(12)])
    for dagger in (0, 1):
        got = _apply(wd, torch, dev, dims, U, psi, 0.1245, prec, dagger, nrhs=12)
        got = got.reshape(psi.shape)
        op = wilson.apply_Ddag if dagger else wilson.apply_D
        for k in range(12):
            assert site_rel_err(got[k], op(U, psi[k], dims, 0.1245)) <= TOL[prec], (dagger, k)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_dslash_bricks_larger_than_a_workgroup(torch_dev, wd, monkeypatch, prec):
    """Bricks of 16x8x6 = 768 sites: every precision marches the brick slice
    in several parts (float64 four of 192, the float kernels three of 256),
    neighbours across parts and faces from memory.  Parity with the oracle,
    D and D^dag, 2 rhs."""
    torch, dev = torch_dev
    monkeypatch.setenv("WD_BRICK", "16,8,6")
    dims = (16, 8, 12, 4)
    U = gauge(dims, 25, "exp")
    psi = synth.gaussian_sources(dims, [26, 27])
    for dagger in (0, 1):
        got = _apply(wd, torch, dev, dims, U, psi, 0.1245, prec, dagger, nrhs=2).reshape(psi.shape)
        op = wilson.apply_Ddag if dagger else wilson.apply_D
        for k in range(2):
            assert site_rel_err(got[k], op(U, psi[k], dims, 0.1245)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_plus_kappa_lattice(torch_dev, wd, prec):
    """WD_SIGN_PLUS_KAPPA: D = 1 + kappa (hops) as printed in Eq. (1)."""
    torch, dev = torch_dev
    dims = (4, 6, 8, 10)
    U = gauge(dims, 35)
    psi = synth.gaussian_spinor(dims, 36)
    lat = wd.Lattice(dims, plus_kappa=True)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    pd = torch.from_numpy(psi).to(dev)
    for dagger in (0, 1):
        od = torch.full_like(pd, float("nan"))
        lat.apply(0.1245, pd, od, prec=prec, dagger=dagger)
        torch.cuda.synchronize()
        op = wilson.apply_Ddag if dagger else wilson.apply_D
        assert site_rel_err(od.cpu().numpy(), op(U, psi, dims, 0.1245, hop_sign=+1)) <= TOL[prec]
    lat.close()


def test_point_source_zero_sites_exact(torch_dev, wd):
    torch, dev = torch_dev
    dims = (4, 6, 8, 10)
    U = gauge(dims, 7)
    psi = synth.point_source(dims, 2, 1, site=123)
    got = _apply(wd, torch, dev, dims, U, psi, 0.124, "f64", 0)
    want = wilson.apply_D(U, psi, dims, 0.124)
    zero = np.all(want.reshape(vol(dims), -1) == 0, axis=1)
    assert zero.sum() == vol(dims) - 9
    assert np.all(got.reshape(vol(dims), -1)[zero] == 0)
    assert site_rel_err(got.reshape(vol(dims), -1)[~zero], want.reshape(vol(dims), -1)[~zero]) <= 1e-13


def test_kappa_zero_identity(torch_dev, wd):
    torch, dev = torch_dev
    dims = (4, 4, 2, 4)
    U = gauge(dims, 8)
    psi = synth.gaussian_spinor(dims, 9)
    got = _apply(wd, torch, dev, dims, U, psi, 0.0, "f64", 0)
    assert np.array_equal(got, psi)


def test_adjoint_and_gamma5_on_gpu(torch_dev, wd):
    torch, dev = torch_dev
    dims = (8, 4, 6, 8)
    U = gauge(dims, 31, "haar")
    phi = synth.gaussian_spinor(dims, 32)
    psi = synth.gaussian_spinor(dims, 33)
    k = 0.13
    Dphi = _apply(wd, torch, dev, dims, U, phi, k, "f64", 0)
    Ddpsi = _apply(wd, torch, dev, dims, U, psi, k, "f64", 1)
    lhs = wilson.dot(phi, Ddpsi)
    rhs = wilson.dot(Dphi, psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13
    g5 = np.array([1, 1, -1, -1], dtype=np.float64)[None, :, None, None]
    g = g5 * _apply(wd, torch, dev, dims, U, g5 * psi, k, "f64", 0)
    assert site_rel_err(g, Ddpsi) < 1e-14


def test_gauge_covariance_on_gpu(torch_dev, wd):
    torch, dev = torch_dev
    dims = (4, 6, 8, 10)
    U = gauge(dims, 41)
    psi = synth.gaussian_spinor(dims, 42)
    G = synth.gauge_rotation(dims, 43)
    Up = ogauge.transform_gauge(U, G, dims)
    a = _apply(wd, torch, dev, dims, Up, ogauge.transform_spinor(psi, G), 0.125, "f64", 0)
    b = ogauge.transform_spinor(_apply(wd, torch, dev, dims, U, psi, 0.125, "f64", 0), G)
    assert site_rel_err(a, b) < 1e-13


def test_field_roundtrip_and_dslash_on_fields(torch_dev, wd):
    torch, dev = torch_dev
    dims = (4, 6, 8, 10)
    U = gauge(dims, 51)
    psi = synth.gaussian_sources(dims, [1, 2, 3])
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    pd = torch.from_numpy(psi).to(dev)
    f = wd.Field(lat, "f64", nrhs=3)
    g = wd.Field(lat, "f64", nrhs=3)
    f.load(pd)
    back = torch.empty_like(pd)
    f.store(back)
    torch.cuda.synchronize()
    assert torch.equal(back, pd)  # bitwise round trip
    wd.wd_dslash(lat, 0.12, 1, f, g)
    out = torch.empty_like(pd)
    g.store(out)
    torch.cuda.synchronize()
    want = wilson.apply_D_multi(U, psi, dims, 0.12, dagger=True)
    assert site_rel_err(out.cpu().numpy(), want) <= 1e-13
    # fp16 round trip stays within the format's rounding
    h = wd.Field(lat, "f16", nrhs=3)
    h.load(pd)
    h.store(back)
    torch.cuda.synchronize()
    assert site_rel_err(back.cpu().numpy(), psi) < 1e-3
    for x in (f, g, h):
        x.close()
    lat.close()


def test_free_field_plane_wave_full_size(torch_dev, wd):
    """48^3 x 96, U = 1: a plane wave is mapped to D(p) times itself (closed form)."""
    torch, dev = torch_dev
    dims = (48, 48, 48, 96)
    L = dims
    V = vol(dims)
    print("plane wave 48^3x96", flush=True)
    Ud = torch.zeros((V, 4, 3, 3, 2), dtype=torch.float64, device=dev)
    for a in range(3):
        Ud[:, :, a, a, 0] = 1.0
    lat = wd.Lattice(dims)
    lat.set_gauge(Ud)
    del Ud
    p = np.array([2 * np.pi * 3 / L[0], 2 * np.pi * 5 / L[1], 2 * np.pi * 1 / L[2],
                  (2 * 7 + 1) * np.pi / L[3]])
    rng = np.random.default_rng(3)
    chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
    t = torch.arange(L[3], device=dev, dtype=torch.float64)
    z = torch.arange(L[2], device=dev, dtype=torch.float64)
    y = torch.arange(L[1], device=dev, dtype=torch.float64)
    x = torch.arange(L[0], device=dev, dtype=torch.float64)
    ph = (p[3] * t[:, None, None, None] + p[2] * z[None, :, None, None] +
          p[1] * y[None, None, :, None] + p[0] * x[None, None, None, :]).reshape(-1)
    wave = torch.polar(torch.ones_like(ph), ph)
    chi_t = torch.from_numpy(chi).to(dev)
    psi = torch.view_as_real((wave[:, None, None] * chi_t[None]).contiguous()).contiguous()
    k = 0.1245
    a = 1 - 2 * k * np.sum(np.cos(p))
    b = 2 * k * np.sin(p)
    from oracle.gamma import GAMMA, IDENTITY4
    Dp = a * IDENTITY4 + 1j * np.einsum("m,mst->st", b, GAMMA)
    want = torch.view_as_real((wave[:, None, None] *
                               torch.from_numpy(Dp @ chi).to(dev)[None]).contiguous())
    out = torch.empty_like(psi)
    lat.apply(k, psi, out)
    torch.cuda.synchronize()
    d = (out - want).reshape(V, -1).norm(dim=1) / want.reshape(V, -1).norm(dim=1)
    assert float(d.max()) < 1e-13
    lat.close()


def test_full_size_sampled_parity(torch_dev, wd):
    """48^3 x 96 eps = 0.3 links: oracle at sampled sites (all boundary cases)."""
    torch, dev = torch_dev
    dims = (48, 48, 48, 96)
    V = vol(dims)
    print("full-size sampled parity 48^3x96: generating links", flush=True)
    U = gauge(dims, 3)
    psi = synth.gaussian_spinor(dims, 103)
    lat = wd.Lattice(dims)
    Ud = torch.from_numpy(U).to(dev)
    lat.set_gauge(Ud)
    del Ud
    pd = torch.from_numpy(psi).to(dev)
    od = torch.empty_like(pd)
    Uc = wilson.to_complex(U)
    pc = wilson.to_complex(psi)
    rng = np.random.default_rng(7)
    corners = [0, V - 1, 47, 48 * 47, 48 * 48 * 47, 48 ** 3 * 95, 48 ** 3 - 1, 48 ** 3]
    sites = np.concatenate([corners, rng.integers(0, V, 300)])
    for dagger, prec in ((0, "f64"), (1, "f64"), (0, "f32"), (1, "f16")):
        print(f"  dagger={dagger} prec={prec}", flush=True)
        lat.apply(0.1245, pd, od, prec=prec, dagger=dagger)
        torch.cuda.synchronize()
        got = od.cpu().numpy().reshape(V, 4, 3, 2)[sites]
        want = wilson.apply_D_sites(lambda s: Uc[s], lambda s: pc[s], dims, 0.1245, sites,
                                    dagger=bool(dagger))
        assert site_rel_err(got, wilson.to_real(want)) <= TOL[prec]
    lat.close()


def test_f64_12_real_links_chosen_for_special_unitary(torch_dev, wd, monkeypatch):
    """Special unitary links are also kept as 12 reals in float64 and the
    float64 stencil reads them (results differ from the 18-real ones in the
    last bits, both within 1e-13 of the oracle); WD_LINKS64_12=0 keeps
    18 reals only.  Extra memory: the F64-12 form, 2/3 of F64-18."""
    torch, dev = torch_dev
    dims = (8, 8, 8, 8)
    U = gauge(dims, 141, "exp")
    psi = synth.gaussian_spinor(dims, 142)
    want = wilson.apply_D(U, psi, dims, 0.1245)
    outs = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("WD_LINKS64_12", mode)
        lat = wd.Lattice(dims)
        lat.set_gauge(torch.from_numpy(U).to(dev))
        n, d = lat.links_info()
        b18 = vol(dims) * 576
        if mode == "1":
            assert n == 12 and 0.0 <= d <= 1e-14
            assert lat.gauge_bytes() == b18 + vol(dims) * 384
        else:
            assert n == 18 and d == -1.0
            assert lat.gauge_bytes() == b18
        pd = torch.from_numpy(psi).to(dev)
        od = torch.full_like(pd, float("nan"))
        lat.apply(0.1245, pd, od)
        torch.cuda.synchronize()
        outs[mode] = od.cpu().numpy()
        lat.close()
        assert site_rel_err(outs[mode], want) <= 1e-13
    assert not np.array_equal(outs["1"], outs["0"])


def test_f64_links_not_special_unitary_stay_18_real(torch_dev, wd):
    """Links off the group (scaled by 1 + 1e-9, and random complex matrices)
    fail the check: 18 reals only, and the stencil still matches the oracle
    (a rebuilt row 2 would be wrong at O(1e-9) or O(1)).  A later
    wd_set_gauge with special unitary links switches the form back on."""
    torch, dev = torch_dev
    dims = (4, 6, 8, 10)
    rng = np.random.default_rng(143)
    U = gauge(dims, 144, "exp")
    psi = synth.gaussian_spinor(dims, 145)
    lat = wd.Lattice(dims)
    for Ux, n_want in ((U * (1 + 1e-9), 18), (rng.standard_normal(U.shape), 18), (U, 12)):
        lat.set_gauge(torch.from_numpy(np.ascontiguousarray(Ux)).to(dev))
        n, d = lat.links_info()
        assert n == n_want, (n, d)
        assert (d > 1e-14) == (n_want == 18)
        pd = torch.from_numpy(psi).to(dev)
        od = torch.full_like(pd, float("nan"))
        lat.apply(0.1245, pd, od, dagger=1)
        torch.cuda.synchronize()
        assert site_rel_err(od.cpu().numpy(), wilson.apply_Ddag(Ux, psi, dims, 0.1245)) <= 1e-13
    lat.close()


@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (8, 8, 8, 8)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_wd_apply_D_and_Ddag_by_name(torch_dev, wd, dims, prec):
    """The two operator entry points of the boundary, called by their own C
    names through ctypes (wd.lib.wd_apply_D / wd.lib.wd_apply_Ddag), against
    the oracle's D and D^dag of Eq. (1) site by site; (8,8,8,8) runs the
    marching stencil, (4,6,8,10) the one-lane-per-site one."""
    import ctypes
    torch, dev = torch_dev
    U = gauge(dims, 41)
    psi = synth.gaussian_spinor(dims, 42)
    k = 0.1245
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    pd = torch.from_numpy(psi).to(dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for name, ref in (("wd_apply_D", wilson.apply_D), ("wd_apply_Ddag", wilson.apply_Ddag)):
        od = torch.full_like(pd, float("nan"))
        rc = getattr(wd.lib, name)(lat.handle, ctypes.c_double(k), wd.PREC[prec],
                                   ctypes.c_void_p(pd.data_ptr()),
                                   ctypes.c_void_p(od.data_ptr()), stream)
        assert rc == wd.WD_OK, wd.last_error()
        torch.cuda.synchronize()
        assert site_rel_err(od.cpu().numpy(), ref(U, psi, dims, k)) <= TOL[prec], name
    lat.close()
