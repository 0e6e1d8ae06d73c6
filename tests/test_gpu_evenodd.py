"""Even-odd (Schur complement) path on the GPU against the oracle.

wd_apply_schur against the oracle's M = 1 - D_eo D_oe (per-site tolerances
as for the stencil; odd sites exactly zero), and solves with
WD_SOLVE_EVEN_ODD against the oracle's even-odd solve: FP64 within +-1
iterations and within 1e-9 of the oracle's iterate after the same number of
steps, mixed precision within the condition-number bound, the CGNE
form, the +kappa sign, batched = single bit for bit, 384-site bricks, and
the 16^3 x 32 configuration against the GPU's own full-lattice solve.
"""
import numpy as np
import pytest

import synth
from oracle import cg, evenodd, wilson
from gpu_util import assert_same_count_parity, gauge, rel, site_rel_err, vol

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-5, "f16": 5e-3}


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1810_04201_amd as wd
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0"), wd


def _schur(env, dims, U, psi, kappa, prec, dagger, nrhs=1, plus_kappa=False):
    torch, dev, wd = env
    lat = wd.Lattice(dims, plus_kappa=plus_kappa)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    pd = torch.from_numpy(np.ascontiguousarray(psi)).to(dev)
    od = torch.full_like(pd, float("nan"))
    lat.apply_schur(kappa, pd, od, prec=prec, dagger=dagger, nrhs=nrhs)
    torch.cuda.synchronize()
    out = od.cpu().numpy()
    lat.close()
    return out


def _check_schur(got, U, psi, dims, kappa, prec, dagger, hop_sign=-1):
    par = evenodd.parity(dims)
    want = evenodd.apply_M(U, psi, dims, kappa, dagger=bool(dagger), hop_sign=hop_sign)
    ev = par == 0
    assert np.all(got[~ev] == 0.0)
    assert site_rel_err(got[ev], want[ev]) <= TOL[prec]


@pytest.mark.parametrize("dims", [(4, 6, 8, 10), (2, 4, 2, 6), (4, 4, 4, 4), (8, 8, 8, 8)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("dagger", [0, 1])
def test_schur_operator_parity(env, dims, prec, dagger):
    print(f"schur dims={dims} prec={prec} dagger={dagger}", flush=True)
    U = gauge(dims, 81)
    psi = synth.gaussian_spinor(dims, 82)
    got = _schur(env, dims, U, psi, 0.1245, prec, dagger)
    _check_schur(got, U, psi, dims, 0.1245, prec, dagger)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_schur_ragged_last_chunk_twelve_rhs(env, prec):
    """8x20x20x20 with 12 rhs: the marching half-field stencil takes chunks of
    3 time slices, the last one 2 (the host layout check pins this).  M and
    M^dag against the oracle for every rhs."""
    dims = (8, 20, 20, 20)
    print(f"schur ragged last chunk, 12 rhs, prec={prec}", flush=True)
    U = gauge(dims, 87)
    psi = synth.gaussian_sources(dims, [88 + k for k in range(12)])
    for dagger in (0, 1):
        got = _schur(env, dims, U, psi, 0.1245, prec, dagger, nrhs=12).reshape(psi.shape)
        for k in range(12):
            _check_schur(got[k], U, psi[k], dims, 0.1245, prec, dagger)


@pytest.mark.parametrize("prec", ["f64", "f16"])
def test_schur_multi_rhs_and_384_site_bricks(env, monkeypatch, prec):
    monkeypatch.setenv("WD_BRICK", "8,8,6")
    dims = (8, 8, 12, 6)
    U = gauge(dims, 83)
    psi = synth.gaussian_sources(dims, [84, 85, 86])
    got = _schur(env, dims, U, psi, 0.1245, prec, 0, nrhs=3).reshape(psi.shape)
    for k in range(3):
        _check_schur(got[k], U, psi[k], dims, 0.1245, prec, 0)


def test_schur_plus_kappa(env):
    dims = (4, 6, 8, 10)
    U = gauge(dims, 87)
    psi = synth.gaussian_spinor(dims, 88)
    got = _schur(env, dims, U, psi, 0.1245, "f64", 1, plus_kappa=True)
    _check_schur(got, U, psi, dims, 0.1245, "f64", 1, hop_sign=+1)


def _solve(env, dims, U, b, kappa, nrhs=1, plus_kappa=False, **kw):
    torch, dev, wd = env
    lat = wd.Lattice(dims, plus_kappa=plus_kappa)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    bd = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    xd = torch.zeros_like(bd)
    rc, info = lat.solve(bd, xd, kappa, nrhs=nrhs, even_odd=True, **kw)
    torch.cuda.synchronize()
    x = xd.cpu().numpy()
    lat.close()
    return rc, info, x


@pytest.mark.parametrize("dims,seed,kind,kappa,src", [
    ((4, 4, 4, 4), 1, "haar", 0.12, "point"),
    ((4, 6, 8, 10), 5, "exp", 0.124, "gauss"),
    ((8, 8, 8, 8), 6, "exp", 0.124, "gauss"),
    ((2, 4, 2, 6), 7, "haar", 0.15, "gauss"),
])
def test_evenodd_fp64_solve_matches_oracle(env, dims, seed, kind, kappa, src):
    print(f"eo solve dims={dims}", flush=True)
    U = gauge(dims, seed, kind)
    b = synth.point_source(dims) if src == "point" else synth.gaussian_spinor(dims, seed + 100)
    rc, info, x = _solve(env, dims, U, b, kappa, tol=1e-10)
    assert rc == 0, info
    assert info[0]["true_rel_resid"] <= 1e-10
    xo, it, oinfo = evenodd.solve(U, b, dims, kappa, tol=1e-10)
    assert abs(info[0]["iters"] - it) <= 1
    n = info[0]["iters"]
    xo_n, itn, _ = evenodd.solve(U, b, dims, kappa, tol=1e-30, max_iter=n)
    assert itn == n
    assert_same_count_parity(x, xo_n)
    # the full system: ||b - D x|| / ||b||
    assert rel(wilson.apply_D(U, x, dims, kappa), b) == pytest.approx(info[0]["rel_resid_D"],
                                                                      rel=1e-3, abs=1e-13)


@pytest.mark.parametrize("prec", ["f32", "f16"])
@pytest.mark.parametrize("form", ["cgnr", "cgne"])
def test_evenodd_mixed_and_cgne(env, prec, form):
    dims = (4, 6, 8, 10)
    print(f"eo mixed prec={prec} form={form}", flush=True)
    U = gauge(dims, 91)
    b = synth.gaussian_spinor(dims, 92)
    rc, info, x = _solve(env, dims, U, b, 0.124, tol=1e-10, prec=prec, form=form)
    assert rc == 0, info
    assert info[0]["true_rel_resid"] <= 1e-10
    xo, it, oinfo = evenodd.solve(U, b, dims, 0.124, tol=1e-12)
    cond = cg.lanczos_condition(oinfo["alphas"], oinfo["betas"])
    assert rel(x, xo) <= max(1e-9, 2e-10 * cond)


def test_evenodd_plus_kappa_solve(env):
    dims = (4, 4, 4, 8)
    U = gauge(dims, 93)
    b = synth.gaussian_spinor(dims, 94)
    rc, info, x = _solve(env, dims, U, b, 0.124, tol=1e-10, plus_kappa=True)
    assert rc == 0
    xo, it, oinfo = evenodd.solve(U, b, dims, 0.124, tol=1e-10, hop_sign=+1)
    assert abs(info[0]["iters"] - it) <= 1
    n = info[0]["iters"]
    xo_n, itn, _ = evenodd.solve(U, b, dims, 0.124, tol=1e-30, hop_sign=+1, max_iter=n)
    assert itn == n
    assert_same_count_parity(x, xo_n)


@pytest.mark.parametrize("prec", ["f64", "f16"])
@pytest.mark.parametrize("dims", [(4, 4, 4, 8), (8, 8, 8, 8)])
def test_evenodd_batched_equals_single_bitwise(env, prec, dims):
    """(4,4,4,8) runs the one-lane-per-site half stencil, (8,8,8,8) the
    marching one in float64."""
    U = gauge(dims, 95)
    B = synth.gaussian_sources(dims, [96, 97, 98, 99])
    rc, info, X = _solve(env, dims, U, B, 0.124, nrhs=4, tol=1e-11, prec=prec)
    assert rc == 0
    for k in (0, 3):
        rc1, info1, x1 = _solve(env, dims, U, B[k], 0.124, tol=1e-11, prec=prec)
        assert rc1 == 0 and np.array_equal(X[k], x1)
        assert info[k]["iters"] == info1[0]["iters"]


def test_evenodd_384_site_bricks(env, monkeypatch):
    monkeypatch.setenv("WD_BRICK", "8,8,6")
    dims = (8, 8, 12, 6)
    U = gauge(dims, 101)
    b = synth.gaussian_spinor(dims, 102)
    rc, info, x = _solve(env, dims, U, b, 0.124, tol=1e-10, prec="f32")
    assert rc == 0
    xo, it, oinfo = evenodd.solve(U, b, dims, 0.124, tol=1e-12)
    cond = cg.lanczos_condition(oinfo["alphas"], oinfo["betas"])
    assert rel(x, xo) <= max(1e-9, 2e-10 * cond)


def test_evenodd_config2_against_full_solve(env):
    """16^3 x 32, kappa 0.124, eps = 0.3 links seed 2, Gaussian source seed 102:
    the even-odd FP64 and mixed FP16 solutions against the full-lattice FP64
    solve, with fewer iterations."""
    torch, dev, wd = env
    dims = (16, 16, 16, 32)
    U = gauge(dims, 2)
    b = synth.gaussian_spinor(dims, 102)
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    bd = torch.from_numpy(b).to(dev)
    xf = torch.zeros_like(bd)
    rcf, inff = lat.solve(bd, xf, 0.124, tol=1e-10)
    res = {}
    for prec in ("f64", "f16"):
        xe = torch.zeros_like(bd)
        rc, inf = lat.solve(bd, xe, 0.124, tol=1e-10, prec=prec, even_odd=True)
        assert rc == 0 and inf[0]["true_rel_resid"] <= 1e-10
        assert inf[0]["iters"] < inff[0]["iters"]
        res[prec] = xe
    torch.cuda.synchronize()
    x_full = xf.cpu().numpy()
    for prec, xe in res.items():
        assert rel(xe.cpu().numpy(), x_full) < 1e-8
    assert rcf == 0
    lat.close()


def test_evenodd_served_equals_alone(env):
    torch, dev, wd = env
    dims = (8, 8, 8, 8)
    U = gauge(dims, 103)
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    B = torch.from_numpy(synth.gaussian_sources(dims, [104, 105])).to(dev)
    xa = torch.zeros_like(B)
    rc, _ = lat.solve(B, xa, 0.124, tol=1e-10, prec="f32", nrhs=2, even_odd=True)
    assert rc == 0
    srv = wd.Server(8 << 30, max_active=4)
    xs = torch.zeros_like(B)
    t = srv.submit(lat, B, xs, 0.124, tol=1e-10, prec="f32", nrhs=2, even_odd=True)
    while True:
        rc2, info = srv.poll(t)
        if rc2 != wd.WD_PENDING:
            break
    srv.close()
    torch.cuda.synchronize()
    assert rc2 == 0 and torch.equal(xa, xs)
    lat.close()


@pytest.mark.parametrize("prec", ["f64", "f16"])
def test_evenodd_fused_update_and_link_forms(env, monkeypatch, prec):
    """The even-odd iteration's last half-field launch updates x and r where
    it forms q (WD_FUSE_XR=0: q stored, separate update), on float64 halves
    of 12 or 18 reals (WD_LINKS64_12).  Every combination reaches the
    oracle's solution; the fused runs launch the x/r-updating kernel."""
    torch, dev, wd = env
    dims = (4, 6, 8, 10)
    U = gauge(dims, 151)
    b = synth.gaussian_spinor(dims, 152)
    xo, _, oinfo = evenodd.solve(U, b, dims, 0.124, tol=1e-12)
    cond = cg.lanczos_condition(oinfo["alphas"], oinfo["betas"])
    _, it, _ = evenodd.solve(U, b, dims, 0.124, tol=1e-10)
    for fuse in ("1", "0"):
        for r12 in ("1", "0"):
            monkeypatch.setenv("WD_FUSE_XR", fuse)
            monkeypatch.setenv("WD_LINKS64_12", r12)
            print(f"eo fuse={fuse} r12={r12} prec={prec}", flush=True)
            lat = wd.Lattice(dims)
            lat.set_gauge(torch.from_numpy(U).to(dev))
            assert lat.links_info()[0] == (12 if r12 == "1" else 18)
            bd = torch.from_numpy(b).to(dev)
            xd = torch.zeros_like(bd)
            wd.wd_timing_reset()
            wd.wd_timing_enable(True)
            rc, info = lat.solve(bd, xd, 0.124, tol=1e-10, prec=prec, even_odd=True)
            torch.cuda.synchronize()
            wd.wd_timing_enable(False)
            assert rc == 0 and info[0]["true_rel_resid"] <= 1e-10
            assert (wd.wd_timing_read("eo_xr_" + prec)[1] > 0) == (fuse == "1")
            if prec == "f64":
                n = info[0]["iters"]
                assert abs(n - it) <= 1
                xo_n = evenodd.solve(U, b, dims, 0.124, tol=1e-30, max_iter=n)[0]
                assert_same_count_parity(xd.cpu().numpy(), xo_n)
            else:
                assert rel(xd.cpu().numpy(), xo) <= max(1e-9, 2e-10 * cond)
            lat.close()


def test_schur_after_gauge_form_changes(env):
    """Float64 halves built on special unitary links (12 reals) are dropped
    and rebuilt with 18 when wd_set_gauge gets links off the group, and
    back: M stays equal to the oracle's in every case."""
    torch, dev, wd = env
    dims = (4, 4, 4, 8)
    U = gauge(dims, 153)
    psi = synth.gaussian_spinor(dims, 154)
    lat = wd.Lattice(dims)
    bytes_seen = []
    for Ux, n in ((U, 12), (U * (1 + 1e-9), 18), (U, 12)):
        lat.set_gauge(torch.from_numpy(np.ascontiguousarray(Ux)).to(dev))
        assert lat.links_info()[0] == n
        pd = torch.from_numpy(psi).to(dev)
        od = torch.full_like(pd, float("nan"))
        lat.apply_schur(0.1245, pd, od, prec="f64")
        torch.cuda.synchronize()
        _check_schur(od.cpu().numpy(), Ux, psi, dims, 0.1245, "f64", 0)
        bytes_seen.append(lat.gauge_bytes())
    lat.close()
    V = vol(dims)
    # F64-18 + F64-12 + 12-real halves; F64-18 + 18-real halves
    assert bytes_seen[0] == bytes_seen[2] == V * 576 + V * 384 + V * 384
    assert bytes_seen[1] == V * 576 + V * 576


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dims,brick", [((8, 8, 8, 8), None), ((8, 8, 12, 6), "8,8,6"),
                                        ((16, 8, 8, 4), "16,8,2"), ((16, 8, 8, 4), "16,8,8")])
def test_marching_half_stencil_equals_site_form(env, monkeypatch, prec, dims, brick):
    """The marching half-field stencil (half slices of 64-multiples staged in
    LDS; float64 and float32) against the one-lane-per-site form
    (WD_EO_SITE=1): the same hops in the same order, so M and M^dag agree to
    the last bits, with 3 rhs.  16x8x8 bricks (512 sites per parity) take two
    parts per half slice."""
    torch, dev, wd = env
    if brick:
        monkeypatch.setenv("WD_BRICK", brick)
    U = gauge(dims, 161)
    psi = synth.gaussian_sources(dims, [162, 163, 164])
    res = {}
    for site in ("0", "1"):
        monkeypatch.setenv("WD_EO_SITE", site)
        for dagger in (0, 1):
            res[site, dagger] = _schur(env, dims, U, psi, 0.1245, prec, dagger, nrhs=3)
    ev = evenodd.parity(dims) == 0
    for dagger in (0, 1):
        a, b = res["0", dagger], res["1", dagger]
        assert site_rel_err(a[:, ev], b[:, ev]) <= {"f64": 1e-15, "f32": 1e-6}[prec]
        for k in range(3):
            _check_schur(a[k], U, psi[k], dims, 0.1245, prec, dagger)
