"""Translation covariance of the HIP operators, GPU against GPU.

Shifting the links and the source together by a spatial vector shifts D psi
by the same vector (the lattice is periodic in x, y, z; the antiperiodic t
boundary is not moved).  Each site's arithmetic is the same wherever the
site sits, so the shifted inputs give the shifted output up to the order of
a few float operations at most, while the site moves between brick
interiors, brick faces and the parts of a brick slice that different
workgroups stage.  This pins the layout's neighbour and face indexing at
every position of sizes the oracle could not afford at all shifts.  The
even-odd operator keeps the parity of a site only under even shifts.
"""
import functools

import numpy as np
import pytest

import synth
from gpu_util import gauge, site_rel_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-14, "f32": 1e-6, "f16": 2e-3}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def wd():
    import paper_1810_04201_amd as wd
    return wd


def shift(a, dims, s):
    """Canonical field (site = x + Lx (y + Ly (z + Lz t)), then per-site
    entries) moved by the spatial vector s: out(x + s) = a(x)."""
    Lx, Ly, Lz, Lt = dims
    tail = a.shape[1:]
    f = a.reshape((Lt, Lz, Ly, Lx) + tail)
    f = np.roll(f, (s[2], s[1], s[0]), axis=(1, 2, 3))
    return np.ascontiguousarray(f.reshape(a.shape))


@functools.lru_cache(maxsize=4)
def _inputs(dims, seed):
    U = gauge(dims, seed)
    psi = synth.gaussian_spinor(dims, seed + 1)
    U.setflags(write=False)
    psi.setflags(write=False)
    return U, psi


def _run(wd, torch, dev, dims, U, psi, op, prec, dagger):
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(np.array(U)).to(dev))
    pd = torch.from_numpy(np.array(psi)).to(dev)
    od = torch.full_like(pd, float("nan"))
    getattr(lat, op)(0.1245, pd, od, prec=prec, dagger=dagger)
    torch.cuda.synchronize()
    out = od.cpu().numpy()
    lat.close()
    return out


# 48^3 spatial extent with few slices: the 48x2x8 bricks and 192-site parts
# of the large lattice; 16^3 x 8 and 24 x 12 x 20 x 4: other brick shapes
CASES = [((48, 48, 48, 4), [(1, 0, 0), (0, 1, 0), (0, 0, 1), (5, 3, 7)]),
         ((16, 16, 16, 8), [(1, 1, 1), (0, 3, 2)]),
         ((24, 12, 20, 4), [(1, 0, 0), (0, 1, 1), (7, 5, 3)])]


@pytest.mark.parametrize("dims,shifts", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16"])
@pytest.mark.parametrize("dagger", [0, 1])
def test_stencil_translation_covariant(torch_dev, wd, dims, shifts, prec, dagger):
    torch, dev = torch_dev
    print(f"translation dims={dims} prec={prec} dagger={dagger}", flush=True)
    U, psi = _inputs(dims, 21)
    base = _run(wd, torch, dev, dims, U, psi, "apply", prec, dagger)
    for s in shifts:
        got = _run(wd, torch, dev, dims, shift(U, dims, s), shift(psi, dims, s), "apply",
                   prec, dagger)
        err = site_rel_err(got, shift(base, dims, s))
        assert err <= TOL[prec], (s, err)


@pytest.mark.parametrize("dims,shifts", [((48, 48, 48, 4), [(2, 0, 0), (0, 2, 0), (0, 0, 2),
                                                            (4, 2, 6)]),
                                         ((16, 16, 16, 8), [(2, 2, 0), (0, 4, 2)])])
@pytest.mark.parametrize("prec", ["f64", "f16"])
def test_schur_translation_covariant_even_shifts(torch_dev, wd, dims, shifts, prec):
    torch, dev = torch_dev
    print(f"schur translation dims={dims} prec={prec}", flush=True)
    U, psi = _inputs(dims, 23)
    base = _run(wd, torch, dev, dims, U, psi, "apply_schur", prec, 0)
    even = base.reshape(-1, 24).any(axis=1)
    assert even.sum() == base.shape[0] // 2
    for s in shifts:
        got = _run(wd, torch, dev, dims, shift(U, dims, s), shift(psi, dims, s), "apply_schur",
                   prec, 0)
        want = shift(base, dims, s)
        m = want.reshape(-1, 24).any(axis=1)
        assert np.array_equal(m, even), s  # even sites stay even
        assert not got.reshape(-1, 24)[~m].any(), s
        err = site_rel_err(got.reshape(-1, 24)[m], want.reshape(-1, 24)[m])
        assert err <= TOL[prec], (s, err)
