"""wd_apply_noalloc: the operator application for callers that cannot
allocate, against wd_apply through the C ABI.

Both run the same kernels on the same inputs, so the outputs must agree bit
for bit.  Two calls in a row share the library's fixed scratch buffer, the
second on a smaller input; a size beyond the scratch and a link form that is
not built yet are refused before any GPU work.
"""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import gauge

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1810_04201_amd as wd
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0"), wd


def _noalloc(wd, torch, lat, kappa, prec, dagger, nrhs, pd, od):
    f = wd.lib.wd_apply_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return f(lat.handle, ctypes.c_double(kappa), wd.PREC[prec], int(dagger), int(nrhs),
             ctypes.c_void_p(pd.data_ptr()), ctypes.c_void_p(od.data_ptr()), stream)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
def test_noalloc_equals_wd_apply_two_calls(env, prec):
    torch, dev, wd = env
    cases = [((8, 8, 8, 8), 3, 0, 201), ((4, 6, 8, 10), 1, 1, 202)]  # second is smaller
    for dims, nrhs, dagger, seed in cases:
        print(f"noalloc prec={prec} dims={dims} nrhs={nrhs} dagger={dagger}", flush=True)
        lat = wd.Lattice(dims)
        lat.set_gauge(torch.from_numpy(gauge(dims, seed)).to(dev))
        src = synth.gaussian_sources(dims, [seed * 10 + k for k in range(nrhs)])
        pd = torch.from_numpy(src if nrhs > 1 else src[0]).to(dev)
        want = torch.full_like(pd, float("nan"))
        lat.apply(0.1245, pd, want, prec=prec, dagger=dagger, nrhs=nrhs)  # builds the form
        got = torch.full_like(pd, float("nan"))
        rc = _noalloc(wd, torch, lat, 0.1245, prec, dagger, nrhs, pd, got)
        assert rc == wd.WD_OK, wd.last_error()
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        lat.close()


def test_noalloc_refusals(env):
    torch, dev, wd = env
    dims = (8, 8, 8, 8)
    lat = wd.Lattice(dims)
    pd = torch.from_numpy(synth.gaussian_spinor(dims, 5)).to(dev)
    od = torch.zeros_like(pd)
    assert _noalloc(wd, torch, lat, 0.12, "f64", 0, 1, pd, od) == wd.WD_ERR_NOGAUGE
    lat.set_gauge(torch.from_numpy(gauge(dims, 6)).to(dev))
    # the float32 form is built on first use by an allocating call only
    rc = _noalloc(wd, torch, lat, 0.12, "f32", 0, 1, pd, od)
    assert rc == wd.WD_ERR_STATE and "not built" in wd.last_error()
    lat.close()
    # 24^3 x 48 float64 with 2 rhs needs two 255 MB fields: beyond the scratch
    big = wd.Lattice((24, 24, 24, 48))
    x = torch.zeros(2 * 24 * 24 * 24 * 48 * 24, dtype=torch.float64, device=dev)
    y = torch.zeros_like(x)
    rc = _noalloc(wd, torch, big, 0.12, "f64", 0, 2, x, y)
    assert rc == wd.WD_ERR_ARG and "scratch" in wd.last_error()
    big.close()
