"""Halo exchange across t-slabs (the single-GPU half of the sharded design).

A lattice cut into slabs along t, each slab its own wd_lattice holding its
part of the gauge and spinor fields; faces packed by wd_halo_pack are handed
to the neighbouring slabs (here by passing the buffers: the transfer a
multi-GPU run does over xGMI), and wd_dslash_halo on every slab must give
the global stencil: against the oracle, and bit for bit against the plain
stencil for a single slab that receives its own faces.
"""
import numpy as np
import pytest

import synth
from oracle import wilson
from gpu_util import gauge, site_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1810_04201_amd as wd
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0"), wd


def _slabs(env, dims, U, psis, nslab, kappa, dagger):
    """D (or D^dag) of the global lattice computed slab by slab."""
    torch, dev, wd = env
    lx, ly, lz, lt = dims
    lts = lt // nslab
    vs = lx * ly * lz
    nrhs = psis.shape[0]
    lats, fins, fouts = [], [], []
    for r in range(nslab):
        sl = slice(r * lts * vs, (r + 1) * lts * vs)
        lat = wd.Lattice((lx, ly, lz, lts))
        lat.set_gauge(torch.from_numpy(np.ascontiguousarray(U[sl])).to(dev))
        # links entering from the previous slab: its U_t on its last slice
        tprev = (r * lts - 1) % lt
        up = np.ascontiguousarray(U[tprev * vs:(tprev + 1) * vs, 3])
        wd.wd_set_halo_gauge(lat, torch.from_numpy(up).to(dev))
        fi = wd.Field(lat, "f64", nrhs=nrhs)
        fi.load(torch.from_numpy(np.ascontiguousarray(psis[:, sl])).to(dev).squeeze(0)
                if nrhs == 1 else torch.from_numpy(np.ascontiguousarray(psis[:, sl])).to(dev))
        lats.append(lat)
        fins.append(fi)
        fouts.append(wd.Field(lat, "f64", nrhs=nrhs))
    n = wd.face_numel(lats[0], nrhs)
    to_prev = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(nslab)]
    to_next = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(nslab)]
    for r in range(nslab):
        wd.wd_halo_pack(lats[r], fins[r], to_prev[r], to_next[r], dagger=dagger)
    out = []
    for r in range(nslab):
        # from the previous slab: what it sent to its next; from the next: its to_prev
        wd.wd_dslash_halo(lats[r], kappa, fins[r], fouts[r], to_next[(r - 1) % nslab],
                          to_prev[(r + 1) % nslab], first=(r == 0), last=(r == nslab - 1),
                          dagger=dagger)
        o = torch.empty((nrhs, lts * vs, 4, 3, 2), dtype=torch.float64, device=dev)
        fouts[r].store(o if nrhs > 1 else o[0])
        out.append(o)
    torch.cuda.synchronize()
    res = torch.cat(out, dim=1).cpu().numpy()
    for f in fins + fouts:
        f.close()
    for lat in lats:
        lat.close()
    return res


@pytest.mark.parametrize("dims,nslab", [((4, 4, 4, 8), 2), ((8, 8, 8, 16), 4), ((8, 4, 8, 12), 3)])
@pytest.mark.parametrize("dagger", [False, True])
def test_slabs_equal_global_stencil(env, dims, nslab, dagger):
    print(f"halo dims={dims} slabs={nslab} dagger={dagger}", flush=True)
    U = gauge(dims, 111)
    psi = synth.gaussian_sources(dims, [112])
    got = _slabs(env, dims, U, psi, nslab, 0.1245, dagger)[0]
    want = (wilson.apply_Ddag if dagger else wilson.apply_D)(U, psi[0], dims, 0.1245)
    assert site_rel_err(got, want) <= 1e-13


def test_slabs_multi_rhs(env):
    dims = (4, 4, 4, 8)
    U = gauge(dims, 113)
    psis = synth.gaussian_sources(dims, [114, 115, 116])
    got = _slabs(env, dims, U, psis, 2, 0.1245, False)
    for k in range(3):
        assert site_rel_err(got[k], wilson.apply_D(U, psis[k], dims, 0.1245)) <= 1e-13


def test_slabs_twelve_rhs_ragged_chunks(env):
    """Two 4x20x20x20 slabs of 4x20x20x40 with 12 rhs: each slab marches
    chunks of 3 time slices, the last one 2, so the chunk holding the slab's
    last slice (and the next slab's face) is the ragged one.  Against the
    global oracle stencil, every rhs."""
    dims = (4, 20, 20, 40)
    print("halo 12 rhs ragged chunks", flush=True)
    U = gauge(dims, 117)
    psis = synth.gaussian_sources(dims, [130 + k for k in range(12)])
    for dagger in (False, True):
        got = _slabs(env, dims, U, psis, 2, 0.1245, dagger)
        op = wilson.apply_Ddag if dagger else wilson.apply_D
        for k in range(12):
            assert site_rel_err(got[k], op(U, psis[k], dims, 0.1245)) <= 1e-13, (dagger, k)


@pytest.mark.parametrize("links12", ["1", "0"])
def test_single_slab_equals_plain_stencil_bitwise(env, monkeypatch, links12):
    """One slab receiving its own faces is the whole (antiperiodic) lattice:
    bit for bit the plain marching stencil, with float64 links of 12 reals
    (the entering links keep 18, which rebuild to the same values only up to
    rounding: they are the same special unitary links, so the first slice's
    backward hop may differ in the last bit; compared to 1e-15 there) or
    18."""
    torch, dev, wd = env
    monkeypatch.setenv("WD_LINKS64_12", links12)
    dims = (8, 8, 8, 8)
    U = gauge(dims, 117)
    psi = synth.gaussian_spinor(dims, 118)
    got = _slabs(env, dims, U, psi[None], 1, 0.1245, False)[0]
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(U).to(dev))
    fa, fb = wd.Field(lat, "f64"), wd.Field(lat, "f64")
    fa.load(torch.from_numpy(psi).to(dev))
    wd.wd_dslash(lat, 0.1245, 0, fa, fb)
    o = torch.empty_like(torch.from_numpy(psi)).to(dev)
    fb.store(o)
    torch.cuda.synchronize()
    want = o.cpu().numpy()
    if links12 == "0":
        assert np.array_equal(got, want)
    else:
        # sites of slice t = 0 take the entering links' 18 reals
        vs = dims[0] * dims[1] * dims[2]
        assert np.array_equal(got[vs:], want[vs:])
        assert site_rel_err(got[:vs], want[:vs]) <= 1e-15
    fa.close()
    fb.close()
    lat.close()


def test_halo_argument_errors(env):
    torch, dev, wd = env
    lat = wd.Lattice((4, 4, 4, 4))
    f = wd.Field(lat, "f64")
    g = wd.Field(lat, "f32")
    n = wd.face_numel(lat)
    a = torch.zeros(n, dtype=torch.float64, device=dev)
    b = torch.zeros(n, dtype=torch.float64, device=dev)
    with pytest.raises(wd.WdError):
        wd.wd_halo_pack(lat, g, a, b)  # float32 field
    lat.set_gauge(torch.from_numpy(gauge((4, 4, 4, 4), 1)).to(dev))
    with pytest.raises(wd.WdError):
        wd.wd_dslash_halo(lat, 0.1, f, wd.Field(lat, "f64"), a, b, True, True)  # links not set
    f.close()
    g.close()
    lat.close()


@pytest.mark.parametrize("dims,nslab", [((8, 8, 8, 32), 2), ((4, 4, 8, 16), 1)])
def test_interior_then_ends_equals_whole_slab_bitwise(env, dims, nslab):
    """The interior chunks (computed with no faces at all) and then the end
    chunks write exactly what one whole-slab call writes, and NaN faces given
    to the interior call cannot reach its output."""
    torch, dev, wd = env
    lx, ly, lz, lt = dims
    lts = lt // nslab
    vs = lx * ly * lz
    U = gauge(dims, 119)
    psi = synth.gaussian_spinor(dims, 120)
    sl = slice(0, lts * vs)
    lat = wd.Lattice((lx, ly, lz, lts))
    lat.set_gauge(torch.from_numpy(np.ascontiguousarray(U[sl])).to(dev))
    tprev = lt - 1
    wd.wd_set_halo_gauge(lat, torch.from_numpy(
        np.ascontiguousarray(U[tprev * vs:(tprev + 1) * vs, 3])).to(dev))
    fi = wd.Field(lat, "f64")
    fi.load(torch.from_numpy(np.ascontiguousarray(psi[sl])).to(dev))
    n = wd.face_numel(lat)
    sp = torch.empty(n, dtype=torch.float64, device=dev)
    sn = torch.empty(n, dtype=torch.float64, device=dev)
    wd.wd_halo_pack(lat, fi, sp, sn)
    outs = []
    for split in (False, True):
        fo = wd.Field(lat, "f64")
        o = torch.full((lts * vs, 4, 3, 2), float("nan"), dtype=torch.float64, device=dev)
        fo.load(o)
        if split:
            nan = torch.full_like(sp, float("nan"))
            wd.wd_dslash_halo(lat, 0.1245, fi, fo, None, nan, True, nslab == 1,
                              region="interior")
            wd.wd_dslash_halo(lat, 0.1245, fi, fo, sn, sp, True, nslab == 1, region="ends")
        else:
            wd.wd_dslash_halo(lat, 0.1245, fi, fo, sn, sp, True, nslab == 1)
        fo.store(o)
        torch.cuda.synchronize()
        outs.append(o.cpu().numpy())
        fo.close()
    assert np.all(np.isfinite(outs[1]))
    assert np.array_equal(outs[0], outs[1])
    fo = wd.Field(lat, "f64")
    with pytest.raises(wd.WdError, match="exclude"):
        wd.wd_dslash_halo(lat, 0.1, fi, fo, None, None, True, True, region="interior")
        wd._check(wd.lib.wd_dslash_halo(lat.handle, 0.1, 0, fi.handle, fo.handle, None, None,
                                        wd.WD_HALO_INTERIOR | wd.WD_HALO_ENDS, None))
    with pytest.raises(wd.WdError, match="null"):
        wd._check(wd.lib.wd_dslash_halo(lat.handle, 0.1, 0, fi.handle, fo.handle, None, None,
                                        wd.WD_HALO_ENDS, None))
    fo.close()
    fi.close()
    lat.close()
