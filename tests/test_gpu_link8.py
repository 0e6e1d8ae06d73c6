"""The 8-real binary16 link form (lattice flag WD_F16_LINKS_8) on the GPU.

The binary16 stencil, the even-odd operator and the mixed-precision solve
with 8-real links against the oracle, to the same bars as the 12-real
binary16 form: 5e-3 per site for the operators (Gaussian inputs), an FP64
true residual of 1e-10 and the condition-number bound for solutions.  Haar
links exercise every column relabelling and frame pivot of the form,
exp(i eps H) links the near-identity fields of the workloads.
"""
import numpy as np
import pytest

import synth
from oracle import cg, evenodd, wilson
from gpu_util import gauge, rel, site_rel_err, vol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1810_04201_amd as wd
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0"), wd


def _lat(env, dims, U):
    torch, dev, wd = env
    lat = wd.Lattice(dims, f16_links8=True)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    return lat


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 6, 8, 10), (8, 8, 8, 8), (4, 4, 4, 4)])
@pytest.mark.parametrize("kind", ["exp", "haar"])
@pytest.mark.parametrize("dagger", [0, 1])
def test_f16_links8_stencil_parity(env, dims, kind, dagger):
    torch, dev, wd = env
    print(f"f16-8 stencil dims={dims} kind={kind} dagger={dagger}", flush=True)
    U = gauge(dims, 301, kind)
    psi = synth.gaussian_spinor(dims, 302)
    lat = _lat(env, dims, U)
    pd = torch.from_numpy(psi).to(dev)
    od = torch.full_like(pd, float("nan"))
    lat.apply(0.1245, pd, od, prec="f16", dagger=dagger)
    torch.cuda.synchronize()
    # F64-18, F64-12 and F16-8 tiles of 64 sites
    assert lat.gauge_bytes() == -(-vol(dims) // 64) * 64 * (576 + 384 + 64)
    lat.close()
    want = (wilson.apply_Ddag if dagger else wilson.apply_D)(U, psi, dims, 0.1245)
    assert site_rel_err(od.cpu().numpy(), want) <= 5e-3


def test_f16_links8_error_close_to_12_real_form(env):
    """On the same inputs the 8-real form's per-site error stays within a
    small factor of the 12-real form's (both bound by binary16 rounding)."""
    torch, dev, wd = env
    dims = (8, 8, 8, 8)
    U = gauge(dims, 303)
    psi = synth.gaussian_spinor(dims, 304)
    want = wilson.apply_D(U, psi, dims, 0.1245)
    errs = {}
    for r8 in (False, True):
        lat = wd.Lattice(dims, f16_links8=r8)
        lat.set_gauge(torch.from_numpy(U).to(dev))
        pd = torch.from_numpy(psi).to(dev)
        od = torch.full_like(pd, float("nan"))
        lat.apply(0.1245, pd, od, prec="f16")
        torch.cuda.synchronize()
        errs[r8] = site_rel_err(od.cpu().numpy(), want)
        lat.close()
    assert errs[True] <= 2.0 * errs[False] + 1e-4, errs


@pytest.mark.parametrize("dagger", [0, 1])
def test_f16_links8_schur_parity(env, dagger):
    torch, dev, wd = env
    dims = (4, 6, 8, 10)
    U = gauge(dims, 305, "haar")
    psi = synth.gaussian_spinor(dims, 306)
    lat = _lat(env, dims, U)
    pd = torch.from_numpy(psi).to(dev)
    od = torch.full_like(pd, float("nan"))
    lat.apply_schur(0.1245, pd, od, prec="f16", dagger=dagger)
    torch.cuda.synchronize()
    lat.close()
    got = od.cpu().numpy()
    par = evenodd.parity(dims)
    want = evenodd.apply_M(U, psi, dims, 0.1245, dagger=bool(dagger))
    assert np.all(got[par == 1] == 0.0)
    assert site_rel_err(got[par == 0], want[par == 0]) <= 5e-3


@pytest.mark.parametrize("dims,even_odd", [((8, 8, 8, 8), False), ((4, 6, 8, 10), False),
                                           ((8, 8, 8, 8), True)])
def test_f16_links8_mixed_solve(env, dims, even_odd):
    torch, dev, wd = env
    print(f"f16-8 mixed solve dims={dims} even_odd={even_odd}", flush=True)
    U = gauge(dims, 307)
    b = synth.gaussian_spinor(dims, 308)
    lat = _lat(env, dims, U)
    bd = torch.from_numpy(b).to(dev)
    x = torch.zeros_like(bd)
    rc, info = lat.solve(bd, x, 0.124, tol=1e-10, prec="f16", even_odd=even_odd)
    torch.cuda.synchronize()
    lat.close()
    assert rc == 0 and info[0]["true_rel_resid"] <= 1e-10, info
    xo, it, oinfo = cg.cgnr(lambda v: wilson.apply_D(U, v, dims, 0.124),
                            lambda v: wilson.apply_Ddag(U, v, dims, 0.124), b, tol=1e-12)
    cond = cg.lanczos_condition(oinfo["alphas"], oinfo["betas"])
    assert rel(x.cpu().numpy(), xo) <= max(1e-9, 2e-10 * cond)


def test_f16_links8_batched_equals_single_bitwise(env):
    torch, dev, wd = env
    dims = (4, 4, 4, 8)
    U = gauge(dims, 309)
    B = synth.gaussian_sources(dims, [310, 311, 312])
    lat = _lat(env, dims, U)
    Bd = torch.from_numpy(B).to(dev)
    X = torch.zeros_like(Bd)
    rc, info = lat.solve(Bd, X, 0.124, tol=1e-11, prec="f16", nrhs=3)
    assert rc == 0
    for k in (0, 2):
        x1 = torch.zeros_like(Bd[k])
        rc1, info1 = lat.solve(Bd[k].contiguous(), x1, 0.124, tol=1e-11, prec="f16")
        assert rc1 == 0 and torch.equal(X[k], x1)
        assert info[k]["iters"] == info1[0]["iters"]
    lat.close()
