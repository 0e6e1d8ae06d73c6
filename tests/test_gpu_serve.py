"""Solve serving (wd_server_*): continuous batching over streams.

Every request served in a mix of lattice sizes, kappa, precisions and rhs
counts returns bitwise the same solution as the same request solved alone
(deterministic kernels, per-request reductions); requests overlap in time;
the HBM budget is never exceeded; failures stay with their own ticket.
Latency percentiles use the nearest-rank definition (parity unpinned: there
is no reference implementation to compare with).
"""
import time

import numpy as np
import pytest

import synth
from gpu_util import gauge, vol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1810_04201_amd as wd
    assert torch.cuda.is_available()
    return torch, torch.device("cuda:0"), wd


def _lattices(env, specs):
    torch, dev, wd = env
    lats = {}
    for name, dims, seed in specs:
        lat = wd.Lattice(dims)
        lat.set_gauge(torch.from_numpy(gauge(dims, seed)).to(dev))
        lats[name] = lat
    return lats


REQS = [  # lattice, kappa, prec, nrhs, source seed
    ("a", 0.121, "f32", 1, 1), ("b", 0.124, "f16", 3, 2), ("a", 0.118, "f64", 1, 3),
    ("c", 0.1245, "f32", 12, 4), ("b", 0.115, "f64", 2, 5), ("a", 0.123, "f16", 5, 6),
    ("c", 0.12, "f16", 1, 7), ("b", 0.122, "f32", 1, 8), ("d", 0.124, "f32", 2, 9),
    ("e", 0.1245, "f16", 1, 10), ("d", 0.119, "f16", 3, 11),
]
# the serving mix's lattice sizes: 8^4, 12^4, 16^3 x 32 and 24^3 x 48 (plus a
# lattice whose extents all differ)
SPECS = [("a", (8, 8, 8, 8), 31), ("b", (4, 6, 8, 10), 32), ("c", (12, 12, 12, 12), 33),
         ("d", (16, 16, 16, 32), 34), ("e", (24, 24, 24, 48), 35)]


def _sources(torch, dev, lat, nrhs, seed):
    dims = lat.dims
    b = synth.gaussian_sources(dims, [seed * 100 + k for k in range(nrhs)])
    return torch.from_numpy(b if nrhs > 1 else b[0]).to(dev)


def test_served_equals_alone_bitwise_and_overlaps(env):
    torch, dev, wd = env
    lats = _lattices(env, SPECS)
    alone = []
    for name, k, prec, nrhs, seed in REQS:
        lat = lats[name]
        b = _sources(torch, dev, lat, nrhs, seed)
        x = torch.zeros_like(b)
        rc, info = lat.solve(b, x, k, tol=1e-10, prec=prec, nrhs=nrhs)
        assert rc == 0, (name, prec, info)
        alone.append(x.cpu())
    srv = wd.Server(hbm_budget_bytes=8 << 30, max_active=4)
    tickets, xs, t_sub = [], [], []
    for name, k, prec, nrhs, seed in REQS:
        lat = lats[name]
        b = _sources(torch, dev, lat, nrhs, seed)
        x = torch.full_like(b, float("nan"))
        t_sub.append(time.time())
        tickets.append(srv.submit(lat, b, x, k, tol=1e-10, prec=prec, nrhs=nrhs))
        xs.append((b, x))
    infos = {}
    deadline = time.time() + 120
    while len(infos) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t in infos:
                continue
            rc, info = srv.poll(t)
            if rc != wd.WD_PENDING:
                infos[t] = (rc, info, time.time())
        time.sleep(0.002)
    assert len(infos) == len(tickets)
    for t, (b, x), want in zip(tickets, xs, alone):
        rc, info, _ = infos[t]
        assert rc == 0, info
        assert torch.equal(x.cpu(), want)  # bitwise: alone == in the mix
        assert all(i["true_rel_resid"] <= 1e-10 for i in info)
    # requests ran concurrently: some request was admitted before another finished
    spans = []
    for t, ts in zip(tickets, t_sub):
        info = infos[t][1][0]
        spans.append((ts + info["queued_seconds"], ts + info["seconds"]))
    overlaps = sum(1 for i in range(len(spans)) for j in range(len(spans))
                   if i != j and spans[i][0] < spans[j][1] and spans[j][0] < spans[i][1])
    assert overlaps > 0
    st = srv.stats()
    assert st["solves_per_s"] > 0 and 0 < st["p50_s"] <= st["p99_s"]
    assert srv.peak_bytes() <= 8 << 30
    srv.close()
    for lat in lats.values():
        lat.close()


def test_tight_budget_queues_and_respects_limit(env):
    torch, dev, wd = env
    lats = _lattices(env, [("a", (8, 8, 8, 8), 41)])
    lat = lats["a"]
    # room for the gauge forms and about two f32 requests at a time
    one = 4096 * (6 * 192 + 5 * 96 + 64) + 4096 * (576 + 192)
    budget = int(2.5 * one)
    srv = wd.Server(hbm_budget_bytes=budget, max_active=8)
    outs = []
    for seed in range(6):
        b = _sources(torch, dev, lat, 1, 50 + seed)
        x = torch.zeros_like(b)
        outs.append((srv.submit(lat, b, x, 0.12, prec="f32"), b, x))
    done = 0
    deadline = time.time() + 120
    while done < len(outs) and time.time() < deadline:
        done = sum(1 for t, _, _ in outs if srv.poll(t)[0] != wd.WD_PENDING)
        time.sleep(0.002)
    assert done == len(outs)
    for t, b, x in outs:
        rc, info = srv.poll(t)
        assert rc == 0 and info[0]["true_rel_resid"] <= 1e-10
    assert 0 < srv.peak_bytes() <= budget
    srv.close()
    lat.close()


def test_failures_stay_with_their_ticket(env):
    torch, dev, wd = env
    lats = _lattices(env, [("a", (4, 4, 4, 4), 51)])
    lat = lats["a"]
    srv = wd.Server(hbm_budget_bytes=1 << 30, max_active=4)
    good = _sources(torch, dev, lat, 1, 1)
    bad = good.clone()
    bad[7, 2, 1, 0] = float("nan")
    xg, xb, xn = torch.zeros_like(good), torch.zeros_like(good), torch.zeros_like(good)
    tg = srv.submit(lat, good, xg, 0.12, prec="f32")
    tb = srv.submit(lat, bad, xb, 0.12, prec="f32")
    tn = srv.submit(lat, good, xn, 0.12, prec="f64", max_iter=1)
    res = {}
    deadline = time.time() + 60
    while len(res) < 3 and time.time() < deadline:
        for t in (tg, tb, tn):
            if t not in res:
                rc, info = srv.poll(t)
                if rc != wd.WD_PENDING:
                    res[t] = rc
        time.sleep(0.002)
    assert res[tg] == 0 and res[tb] == wd.WD_ERR_NUMERIC and res[tn] == wd.WD_ERR_NOCONV
    with pytest.raises(wd.WdError):
        srv.poll(987654)
    # a request larger than the whole budget is refused at submission
    tiny = wd.Server(hbm_budget_bytes=64 << 10, max_active=2)
    with pytest.raises(wd.WdError) as e:
        tiny.submit(lat, good, xg, 0.12)
    assert e.value.code == wd.WD_ERR_NOMEM
    tiny.close()
    srv.close()
    lat.close()


def _wait_all(srv, wd, tickets, limit=120):
    res = {}
    deadline = time.time() + limit
    while len(res) < len(tickets) and time.time() < deadline:
        for t in tickets:
            if t not in res:
                rc, info = srv.poll(t)
                if rc != wd.WD_PENDING:
                    res[t] = (rc, info)
        time.sleep(0.002)
    assert len(res) == len(tickets)
    return res


def test_budget_holds_resident_forms_of_two_lattices(env):
    """Two 8^4 lattices alternate float32 requests under a budget with room
    for one lattice's float64 links, one request's workspace and one and a
    half float32 link forms.  A retired request's float32 form stays
    allocated and charged, so before the other lattice builds its own the
    server must release it: the two forms never coexist, the charge never
    exceeds the budget, and every result is bitwise the one solved alone
    (a released form is rebuilt bit for bit)."""
    torch, dev, wd = env
    # the same two gauge fields twice: solved alone, and served
    ref = _lattices(env, [("a", (8, 8, 8, 8), 61), ("b", (8, 8, 8, 8), 62)])
    lats = _lattices(env, [("a", (8, 8, 8, 8), 61), ("b", (8, 8, 8, 8), 62)])
    V = 4096
    master = lats["a"].gauge_bytes()  # float64 links only, right after set_gauge
    assert master == lats["b"].gauge_bytes() == V * (576 + 384)
    f32 = V * 192
    # CG workspace of one float32 request on 8^4 (6 float64 fields, 4 float32
    # fields, partial sums, solver state; each field padded by 256 bytes)
    ws = 6 * (V * 192 + 256) + 4 * (V * 96 + 256) + 768 + 1536 + 256
    budget = master + ws + f32 + f32 // 2
    order = ["a", "b", "a", "b", "a", "b"]
    srcs = [_sources(torch, dev, lats[n], 1, 70 + k) for k, n in enumerate(order)]
    alone = []
    for n, b in zip(order, srcs):
        x = torch.zeros_like(b)
        rc, _ = ref[n].solve(b, x, 0.12, tol=1e-10, prec="f32")
        assert rc == 0
        alone.append(x.cpu())
    srv = wd.Server(hbm_budget_bytes=budget, max_active=4)
    xs = [torch.full_like(b, float("nan")) for b in srcs]
    tickets = [srv.submit(lats[n], b, x, 0.12, prec="f32") for n, b, x in zip(order, srcs, xs)]
    res = _wait_all(srv, wd, tickets)
    for t, x, want in zip(tickets, xs, alone):
        rc, info = res[t]
        assert rc == 0 and info[0]["true_rel_resid"] <= 1e-10
        assert torch.equal(x.cpu(), want)
    assert 0 < srv.peak_bytes() <= budget
    # the last request ran on b: a's float32 form was released for it
    assert lats["a"].gauge_bytes() == master
    assert lats["b"].gauge_bytes() == master + f32
    srv.close()
    for lat in list(lats.values()) + list(ref.values()):
        lat.close()


def test_server_on_caller_streams(env):
    """wd_server_config.streams: the slots run on the caller's torch streams
    (two of them, so two requests at a time); results are bitwise the ones
    solved alone, and the streams stay usable after the server is gone."""
    torch, dev, wd = env
    lats = _lattices(env, [("a", (8, 8, 8, 8), 81), ("b", (4, 6, 8, 10), 82)])
    reqs = [("a", "f32", 1, 1), ("b", "f16", 2, 2), ("a", "f64", 1, 3), ("b", "f32", 3, 4)]
    alone = []
    for n, prec, nrhs, seed in reqs:
        b = _sources(torch, dev, lats[n], nrhs, seed)
        x = torch.zeros_like(b)
        rc, _ = lats[n].solve(b, x, 0.124, tol=1e-10, prec=prec, nrhs=nrhs)
        assert rc == 0
        alone.append(x.cpu())
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    srv = wd.Server(hbm_budget_bytes=4 << 30, streams=streams)
    xs, tickets = [], []
    for n, prec, nrhs, seed in reqs:
        b = _sources(torch, dev, lats[n], nrhs, seed)
        x = torch.full_like(b, float("nan"))
        tickets.append(srv.submit(lats[n], b, x, 0.124, tol=1e-10, prec=prec, nrhs=nrhs))
        xs.append((b, x))
    res = _wait_all(srv, wd, tickets)
    srv.close()
    for t, (b, x), want in zip(tickets, xs, alone):
        assert res[t][0] == 0
        assert torch.equal(x.cpu(), want)
    for s in streams:
        with torch.cuda.stream(s):
            y = torch.ones(16, device=dev) * 2
        s.synchronize()
        assert float(y.sum()) == 32.0
    for lat in lats.values():
        lat.close()
