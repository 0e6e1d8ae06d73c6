"""Benchmark: Wilson-Dirac CG to a 1e-10 true residual, FP64 versus mixed
precision, on the 48^3 x 96 lattice (kappa 0.1245, exp(i eps H) links with
eps = 0.3, Gaussian source), on one MI355X.

One step = gauge ingest (canonical -> packed forms) + the plain FP64 CG solve
+ the mixed-precision solve (FP16-12 inner, FP64 reliable updates) of the
same source, every kernel in libwdirac.  `value` is the FP64 stencil's
throughput inside the FP64 solve: 1320 flop x V over its average launch
time (HIP events recorded on its launch stream in an instrumented re-run of
the step).  The JSON line also carries the time to solution of each solver
from the timed region, the dominant kernel's roofline (traffic from the
committed counter summary when it matches the current kernel source), the
stencil alone per precision, streaming ceilings (the library's probe with
the stencils' read/write mix, and torch's device copy), the 4^4 and
16^3 x 32 configurations, the 12-source batched solve on 24^3 x 48, Poisson
request streams through the solve server, and the CPU oracle on a sample of
the same workload.  Inputs are synthetic and resident in HBM before timing.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
    python bench.py --probe                  # workload for rocprofv3 counter runs
    python bench.py --pmc-summary FETCH.csv WRITE.csv --out profiles/X.json --cmd "..."
    python bench.py --trace-summary STATS.csv --out profiles/X.md --cmd "..." [--match RE]
    python bench.py --valu-summary PMC.csv --out profiles/X.md --cmd "..."
    python bench.py --only multi_rhs         # one extra workload alone (profiling)
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_SITE = 1320
# algorithmic bytes per site of one stencil application: spinor in once,
# four links per site (each read once), spinor out once
BYTES_PER_SITE = {"f64": 192 + 576 + 192, "f32": 96 + 192 + 96, "f16": 52 + 96 + 52}
LINK_BYTES = {"f64": 576, "f32": 192, "f16": 96}
# the CG's second stencil with the r update fused: links and spinor in as
# above, r read and written (F64, or F32 beside an F32/F16 stencil); q itself
# is never stored (x follows in the p update)
XR_BYTES_PER_SITE = {"f64": 576 + 192 + 2 * 192,
                     "f32": 192 + 96 + 2 * 96,
                     "f16": 96 + 52 + 2 * 96}
FUSED_XR = os.environ.get("WD_FUSE_XR", "1") != "0"


def f64_bytes(lat):
    """Per-site algorithmic bytes of the float64 marching stencil and of its
    r-updating form on this lattice: its links are read as 12 reals (384
    bytes per site) when wd_set_gauge found them special unitary, else 18
    (576)."""
    link = 384 if lat.links_info()[0] == 12 else 576
    return 192 + link + 192, link + 192 + 2 * 192
SPINOR_BYTES = {"f64": 192, "f32": 96, "f16": 52}
HBM_PEAK_GBS = 8000.0
METRIC = "dslash GFLOP/s & HBM GB/s; CG time-to-1e-10 residual, mixed vs FP64"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_traffic_48x48x48x96.json")
KERNEL_SOURCES = ["dslash.hip", "device.hpp", "wd_internal.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", default="48x48x48x96")
    ap.add_argument("--kappa", type=float, default=0.1245)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--mixed", default="f16", choices=["f32", "f16"])
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--probe", action="store_true")
    ap.add_argument("--probe-multi", action="store_true",
                    help="workload for counter runs of the 12-source batch (24^3 x 48)")
    ap.add_argument("--multi-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "TRACE_CSV"))
    ap.add_argument("--only", choices=["multi_rhs", "small_configs", "serving", "slab_share"],
                    help="run one of the extra workloads alone and print its JSON (profiling)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--trace-summary", metavar="STATS_CSV")
    ap.add_argument("--valu-summary", metavar="PMC_CSV")
    ap.add_argument("--sq-summary", nargs="+", metavar="PMC_CSV",
                    help="wave occupancy and wait counters of the probe's stencil launches")
    ap.add_argument("--out")
    ap.add_argument("--cmd", default="")
    ap.add_argument("--match", default="", help="--trace-summary: only kernels matching")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1810_04201_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def applications(info, prec_inner):
    """Stencil applications a solve performed, by kernel and precision (no-op
    launches enqueued after convergence do no work and are not counted).  An
    iteration applies the plain stencil once and, with the fused update, the
    r-updating stencil once ("xr_" keys)."""
    it, up = info["iters"], info["reliable_updates"]
    out = {"f64": 1 + 2 * max(up - 1, 0) + 1}  # D^dag b, reliable updates, final D x
    out[prec_inner] = out.get(prec_inner, 0) + (it if FUSED_XR else 2 * it)
    if FUSED_XR:
        out["xr_" + prec_inner] = it
    return out


def load_traffic(key):
    """HBM traffic per launch of the stencil kernel `key` ("f64", "xr_f64",
    ...) from the committed counter summary, or None if it is missing or was
    taken on a different stencil source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(f"dslash_{key}")
    return None if k is None else k.get("traffic_bytes")


# ------------------------------------------------------------------ main bench

def main():
    args = parse()
    if args.pmc_summary:
        return pmc_summary(args)
    if args.trace_summary:
        return trace_summary(args)
    if args.valu_summary:
        return valu_summary(args)
    if args.multi_summary:
        return multi_summary(args)
    if args.sq_summary:
        return sq_summary(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                          "(no collective exchange is built; one GPU's share of a t-slab "
                          "split is measured under extras.slab_share)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    import paper_1810_04201_amd as wd

    if args.probe:
        return probe(np, torch, synth, wd)
    if args.probe_multi:
        return probe_multi(np, torch, synth, wd)
    if args.only:
        fn = {"multi_rhs": lambda: multi_rhs(np, torch, synth, wd),
              "small_configs": lambda: small_configs(np, torch, synth, wd),
              "serving": lambda: serving(np, torch, synth, wd, args.serve_requests),
              "slab_share": lambda: slab_share(np, torch, synth, wd)}[args.only]
        print(json.dumps({args.only: fn()}))
        return

    dims = tuple(int(v) for v in args.dims.split("x"))
    V = int(np.prod(dims))
    kappa = args.kappa
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    copy_gbs = copy_bandwidth(torch, wd)

    t0 = time.time()
    Uh = torch.empty((V, 4, 3, 3, 2), dtype=torch.float64, pin_memory=True)
    synth.gauge(dims, 3, synth.EXP, 0.3, out=Uh.numpy())
    bh = torch.empty((V, 4, 3, 2), dtype=torch.float64, pin_memory=True)
    synth.gaussian_spinor(dims, 103, out=bh.numpy())
    Ud = Uh.to(dev)
    bd = bh.to(dev)
    del Uh
    log(f"inputs {dims}: {time.time() - t0:.1f}s")
    lat = wd.Lattice(dims)
    xd = torch.zeros_like(bd)
    xm = torch.zeros_like(bd)

    def step():
        with torch.cuda.stream(stream):
            lat.set_gauge(Ud, stream=stream)
            xd.zero_()
            xm.zero_()
            rc1, i1 = lat.solve(bd, xd, kappa, tol=args.tol, prec="f64", stream=stream)
            rc2, i2 = lat.solve(bd, xm, kappa, tol=args.tol, prec=args.mixed, stream=stream)
        if rc1 != 0 or rc2 != 0:
            raise RuntimeError(f"solve failed: {rc1} {i1} {rc2} {i2}")
        return i1[0], i2[0]

    for w in range(args.warmup):
        step()
        log(f"warmup {w} done")
    # the timed region: K steps on the default solver path (chunks of CG
    # iterations replayed from HIP graphs, no event timing)
    torch.cuda.synchronize()
    t_start = time.time()
    per_step = []
    for k in range(args.steps):
        ts = time.time()
        i1, i2 = step()
        torch.cuda.synchronize()
        per_step.append({"t": time.time() - ts, "fp64": i1, "mixed": i2})
        log(f"step {k}: {per_step[-1]['t']:.2f}s fp64 {i1['seconds']:.2f}s/{i1['iters']} it, "
            f"{args.mixed} {i2['seconds']:.2f}s/{i2['iters']} it/{i2['reliable_updates']} upd")
    torch.cuda.synchronize()
    elapsed = time.time() - t_start
    # kernel timing: the same step again (up to 3 times) with HIP events
    # recorded on the launch stream around every stencil launch (the solver
    # launches eagerly while events are recorded)
    n_timed = min(args.steps, 3)
    apps = {k: 0 for k in ("f64", "f32", "f16", "xr_f64", "xr_f32", "xr_f16")}
    wd.wd_timing_reset()
    wd.wd_timing_enable(True)
    for k in range(n_timed):
        i1, i2 = step()
        for info, p in ((i1, "f64"), (i2, args.mixed)):
            for key, n in applications(info, p).items():
                apps[key] += n
    torch.cuda.synchronize()
    wd.wd_timing_enable(False)
    log(f"kernel timing: {n_timed} instrumented steps")
    ms = {k: wd.wd_timing_read("dslash_" + k)[0] for k in apps}
    BYTES_PER_SITE["f64"], XR_BYTES_PER_SITE["f64"] = f64_bytes(lat)
    f64_link_reals = lat.links_info()[0]
    msl, cntl = wd.wd_timing_read("dslash_" + args.mixed)

    # the headline: the FP64 stencil's GFLOP/s (1320 flop per site) over its
    # average launch time inside the FP64 CG (t = D p, and D^dag b, the
    # reliable updates and the final residual)
    f64_ms = ms["f64"] / apps["f64"]
    value = V * FLOP_PER_SITE / (f64_ms * 1e-3) / 1e9
    t_fp64 = statistics.median(s["fp64"]["seconds"] for s in per_step)
    t_mix = statistics.median(s["mixed"]["seconds"] for s in per_step)
    s0 = per_step[-1]
    full = dims == (48, 48, 48, 96)

    def roof(key, what):
        """HBM roofline of one stencil kernel: average over its working
        launches in the instrumented steps."""
        avg_ms = ms[key] / apps[key]
        prec = key[-3:]
        bps = XR_BYTES_PER_SITE[prec] if key.startswith("xr_") else BYTES_PER_SITE[prec]
        achieved = V * bps / (avg_ms * 1e-3) / 1e9
        traffic = load_traffic(key) if full else None
        mix = "probe_4r1w" if key.startswith("xr_") else "probe_3r1w"
        return {
            "kernel": what,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": (round(traffic / (avg_ms * 1e-3) / 1e9, 1) if traffic else None),
            "traffic_bytes_per_launch": traffic,
            "algorithmic_bytes_per_launch": V * bps,
            "avg_launch_ms": round(avg_ms, 4),
            "launches": apps[key],
            "bytes_per_site": bps,
            "sites_per_launch": V,
            "copy_GBps": copy_gbs["probe"],
            "frac_of_copy": round(achieved / copy_gbs["probe"], 4),
            # the probe with the kernel's own read/write mix
            "stream_GBps": copy_gbs[mix],
            "frac_of_stream": round(achieved / copy_gbs[mix], 4),
        }

    plain = roof("f64", f"dslash_f64 (k_dslash_tm<F64>, time-marching stencil, "
                        f"F64-{f64_link_reals} links)")
    # dominant kernel: whichever FP64 stencil kernel took the most time
    if FUSED_XR and apps["xr_f64"] and ms["xr_f64"] > ms["f64"]:
        roofline = roof("xr_f64", f"dslash_xr_f64 (k_dslash_tm<F64, XR>, time-marching stencil "
                                  f"with the fused CG update r -= alpha D^dag D p, "
                                  f"F64-{f64_link_reals} links)")
        roofline["plain_stencil"] = plain
    else:
        roofline = plain
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"FP64 Wilson-Dirac dslash (1320 flop/site, F64-{f64_link_reals} links) "
                        f"inside CGNR on {'x'.join(map(str, dims))}, kappa={kappa}, "
                        f"exp(i*0.3*H) SU(3) links seed 3, Gaussian source seed 103; one step = "
                        f"gauge ingest + FP64 CG + mixed {args.mixed.upper()}-12 CG to a true "
                        f"relative residual of {args.tol}",
            "lattice": "x".join(map(str, dims)),
            "kappa": kappa,
            "tol": args.tol,
            "parallelism": "single GPU",
        },
        "value_source": (f"1320 flop x {V} sites over the average launch time of the FP64 "
                         f"stencil (t = D p) measured with HIP events on its launch stream over "
                         f"{apps['f64']} launches in {n_timed} instrumented steps"),
        "dslash_f64": {"GFLOPs": round(value, 1), "avg_launch_ms": round(f64_ms, 4),
                       "GBps_algorithmic": round(V * BYTES_PER_SITE["f64"] / f64_ms / 1e6, 1),
                       "bytes_per_site": BYTES_PER_SITE["f64"], "launches": apps["f64"]},
        "cg": {
            "timing": "median over the timed steps, default solver path (HIP graph replays)",
            "fp64_s": round(t_fp64, 3),
            "fp64_iters": s0["fp64"]["iters"],
            "fp64_true_rel_resid": s0["fp64"]["true_rel_resid"],
            f"mixed_{args.mixed}_s": round(t_mix, 3),
            f"mixed_{args.mixed}_iters": s0["mixed"]["iters"],
            f"mixed_{args.mixed}_reliable_updates": s0["mixed"]["reliable_updates"],
            f"mixed_{args.mixed}_true_rel_resid": s0["mixed"]["true_rel_resid"],
            "speedup_mixed_vs_fp64": round(t_fp64 / t_mix, 3),
        },
        "roofline": roofline,
        "copy_ceiling": copy_gbs,
    }
    if cntl:
        ml = msl / apps[args.mixed]
        out["roofline_" + args.mixed] = {
            "kernel": f"dslash_{args.mixed} (the mixed CG's inner stencil)",
            "avg_launch_ms": round(ml, 4),
            "achieved_GBps": round(V * BYTES_PER_SITE[args.mixed] / (ml * 1e-3) / 1e9, 1),
            "GFLOPs": round(V * FLOP_PER_SITE / (ml * 1e-3) / 1e9, 1),
        }
        if apps["xr_" + args.mixed]:
            mx = ms["xr_" + args.mixed] / apps["xr_" + args.mixed]
            out["roofline_" + args.mixed]["xr"] = {
                "avg_launch_ms": round(mx, 4),
                "achieved_GBps": round(V * XR_BYTES_PER_SITE[args.mixed] / (mx * 1e-3) / 1e9, 1),
                "bytes_per_site": XR_BYTES_PER_SITE[args.mixed]}
    if not args.no_extras:
        ex = {}
        ex.update(stencil_alone(wd, torch, lat, bd, V, kappa, stream))
        ex.update(other_mixed(args, lat, bd, kappa, stream, torch))
        ex["even_odd"] = even_odd(args, wd, lat, bd, kappa, stream, torch, V)
        lat.close()
        ex["f16_links8"] = f16_links8(wd, torch, dims, Ud, bd, V, kappa, args.tol, stream)
        del Ud
        torch.cuda.empty_cache()
        ex["slab_share"] = slab_share(np, torch, synth, wd)
        ex["small_configs"] = small_configs(np, torch, synth, wd)
        ex["multi_rhs"] = multi_rhs(np, torch, synth, wd)
        ex["serving"] = serving(np, torch, synth, wd, args.serve_requests)
        out["extras"] = ex
    else:
        lat.close()
    if not args.no_cpu:
        it16 = (out.get("extras", {}).get("small_configs", {}).get("16x16x16x32", {})
                .get("cg_f64_iters"))
        out["cpu_baseline"] = cpu_baseline(np, it16, s0["fp64"]["iters"] if full else None)
    print(json.dumps(out))


def copy_bandwidth(torch, wd):
    """Streaming ceilings, median of 5 (bytes read plus written over the kernel
    time, HIP events), from the library's streaming probe (wd_stream_probe,
    16-byte non-temporal loads and stores) on 1 GiB arrays: a copy (1 read
    per write), the stencil's mix (3 reads per write: 576 / 192 bytes per
    site) and the r-updating stencil's (4 per write: 768 / 192); torch's
    device copy beside them."""
    n = 128 * 1024 * 1024
    src = [torch.full((n,), float(k + 1), dtype=torch.float64, device="cuda:0")
           for k in range(4)]
    b = torch.empty_like(src[0])

    def med(fn, nread):
        for _ in range(2):
            fn()
        ts = []
        for _ in range(5):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return round((nread + 1) * n * 8 / statistics.median(ts) / 1e6, 1)

    res = {"probe": med(lambda: wd.wd_stream_probe(src[:1], b), 1)}
    assert torch.equal(b, src[0])
    res["probe_3r1w"] = med(lambda: wd.wd_stream_probe(src[:3], b), 3)
    assert float(b[0]) == 6.0
    res["probe_4r1w"] = med(lambda: wd.wd_stream_probe(src, b), 4)
    res["torch_copy"] = med(lambda: b.copy_(src[0]), 1)
    res.update({"array_bytes": n * 8, "peak": HBM_PEAK_GBS})
    for k in ("probe", "probe_3r1w", "probe_4r1w"):
        res[k + "_frac_of_peak"] = round(res[k] / HBM_PEAK_GBS, 4)
    del src, b
    torch.cuda.empty_cache()
    log(f"streaming ceilings: {res}")
    return res


def slab_share(np, torch, synth, wd):
    """One GPU's share of 48^3 x 96 cut into 8 t-slabs (48^3 x 12, slab 0 of
    the seed-3 configuration): the plain stencil on the slab against the
    halo path (faces packed, staged and read across the slab ends; the slab
    receives its own faces in place of its neighbours').  The transfer time
    of a face over one xGMI link (~153 GB/s) is an estimate, not measured."""
    dev = torch.device("cuda:0")
    full = (48, 48, 48, 96)
    dims = (48, 48, 48, 12)
    V = int(np.prod(dims))
    vs = 48 ** 3
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(synth.gauge(full, 3, synth.EXP, 0.3, t0=0, t1=12)).to(dev))
    up = synth.gauge(full, 3, synth.EXP, 0.3, t0=95, t1=96)[:, 3]
    wd.wd_set_halo_gauge(lat, torch.from_numpy(np.ascontiguousarray(up)).to(dev))
    psi = torch.from_numpy(synth.gaussian_spinor(dims, 103)).to(dev)
    fa, fb = wd.Field(lat, "f64"), wd.Field(lat, "f64")
    fa.load(psi)
    n = wd.face_numel(lat)
    sp = torch.empty(n, dtype=torch.float64, device=dev)
    sn = torch.empty(n, dtype=torch.float64, device=dev)

    def timeit(fn, reps=20):
        for _ in range(3):
            fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    plain = timeit(lambda: wd.wd_dslash(lat, 0.1245, 0, fa, fb))
    pack = timeit(lambda: wd.wd_halo_pack(lat, fa, sp, sn))
    halo = timeit(lambda: wd.wd_dslash_halo(lat, 0.1245, fa, fb, sn, sp, False, False))
    # the split a multi-GPU run overlaps with the face transfer: interior
    # chunks first (no face read), then the chunks holding the slab ends
    inner = timeit(lambda: wd.wd_dslash_halo(lat, 0.1245, fa, fb, None, None, False, False,
                                             region="interior"))
    ends = timeit(lambda: wd.wd_dslash_halo(lat, 0.1245, fa, fb, sn, sp, False, False,
                                            region="ends"))
    face_bytes = n * 8
    res = {"lattice": "48x48x48x12 (one of 8 t-slabs of 48x48x48x96)",
           "dslash_plain_ms": round(plain, 4), "halo_pack_ms": round(pack, 4),
           "dslash_halo_ms": round(halo, 4),
           "dslash_halo_interior_ms": round(inner, 4), "dslash_halo_ends_ms": round(ends, 4),
           "dslash_halo_GBps_algorithmic": round(V * f64_bytes(lat)[0] / halo / 1e6, 1),
           "face_bytes_per_direction": face_bytes,
           "face_over_xgmi_link_us_estimate": round(face_bytes / 153e9 * 1e6, 1)}
    fa.close()
    fb.close()
    lat.close()
    log(f"slab share: {res}")
    return res


def small_configs(np, torch, synth, wd):
    """The 4^4 configuration (Haar links seed 1, kappa 0.12, point source)
    and 16^3 x 32 (eps = 0.3 links seed 2, kappa 0.124, Gaussian source seed
    102): FP64 and mixed time to a 1e-10 true residual (median of 5 on 4^4,
    of 3 on 16^3 x 32) and, on 16^3 x 32, the stencil per precision (its
    fields fit in the 256 MB Infinity Cache: an L2-miss rate, not HBM)."""
    dev = torch.device("cuda:0")
    res = {}
    for name, dims, seed, kind, kappa, src, reps in (
            ("4x4x4x4", (4, 4, 4, 4), 1, synth.HAAR, 0.12, "point", 5),
            ("16x16x16x32", (16, 16, 16, 32), 2, synth.EXP, 0.124, "gauss", 3)):
        V = int(np.prod(dims))
        lat = wd.Lattice(dims)
        lat.set_gauge(torch.from_numpy(synth.gauge(dims, seed, kind, 0.3)).to(dev))
        b = synth.point_source(dims) if src == "point" else synth.gaussian_spinor(dims, 102)
        bd = torch.from_numpy(b).to(dev)
        x = torch.zeros_like(bd)
        r = {}
        for prec in ("f64", "f32", "f16"):
            lat.solve(bd, x, kappa, tol=1e-10, prec=prec)  # warm
            ts, info = [], None
            for _ in range(reps):
                x.zero_()
                torch.cuda.synchronize()
                t = time.time()
                rc, info = lat.solve(bd, x, kappa, tol=1e-10, prec=prec)
                ts.append(time.time() - t)
            r[f"cg_{prec}_s"] = round(statistics.median(ts), 5)
            r[f"cg_{prec}_iters"] = info[0]["iters"]
            r[f"cg_{prec}_true_rel_resid"] = info[0]["true_rel_resid"]
        if V >= 1 << 17:
            for prec in ("f64", "f32", "f16"):
                fa, fb = wd.Field(lat, prec), wd.Field(lat, prec)
                fa.load(bd)
                for _ in range(3):
                    wd.wd_dslash(lat, kappa, 0, fa, fb)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(20):
                    wd.wd_dslash(lat, kappa, 0, fa, fb)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / 20
                r[f"dslash_{prec}_ms"] = round(ms, 4)
                r[f"dslash_{prec}_GFLOPs"] = round(V * FLOP_PER_SITE / ms / 1e6, 1)
                bps = f64_bytes(lat)[0] if prec == "f64" else BYTES_PER_SITE[prec]
                r[f"dslash_{prec}_GBps_l2_miss"] = round(V * bps / ms / 1e6, 1)
                fa.close()
                fb.close()
        lat.close()
        res[name] = r
    log(f"small configs: {res}")
    return res


def stencil_alone(wd, torch, lat, bd, V, kappa, stream):
    """The stencil alone on resident fields, per precision (HIP events)."""
    res = {}
    for prec in ("f64", "f32", "f16"):
        fa = wd.Field(lat, prec)
        fb = wd.Field(lat, prec)
        with torch.cuda.stream(stream):
            fa.load(bd, stream=stream)
            for _ in range(3):
                wd.wd_dslash(lat, kappa, 0, fa, fb, stream=stream)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            n = 20
            e0.record(stream)
            for i in range(n):
                wd.wd_dslash(lat, kappa, i & 1, fa, fb, stream=stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        bps = f64_bytes(lat)[0] if prec == "f64" else BYTES_PER_SITE[prec]
        res[f"dslash_{prec}"] = {"ms": round(ms, 4),
                                 "GFLOPs": round(V * FLOP_PER_SITE / ms / 1e6, 1),
                                 "GBps_algorithmic": round(V * bps / ms / 1e6, 1),
                                 "bytes_per_site": bps}
        fa.close()
        fb.close()
    log(f"stencil alone: {res}")
    return res


def f16_links8(wd, torch, dims, Ud, bd, V, kappa, tol, stream):
    """The same system on a lattice whose binary16 links are stored as 8
    reals (16 bytes per link, WD_F16_LINKS_8): the binary16 stencil alone
    (algorithmic bytes 52 + 64 + 52 per site) and the mixed FP16-8 CG."""
    lat = wd.Lattice(dims, f16_links8=True)
    with torch.cuda.stream(stream):
        lat.set_gauge(Ud, stream=stream)
        fa, fb = wd.Field(lat, "f16"), wd.Field(lat, "f16")
        fa.load(bd, stream=stream)
        for _ in range(3):
            wd.wd_dslash(lat, kappa, 0, fa, fb, stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(20):
            wd.wd_dslash(lat, kappa, i & 1, fa, fb, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    fa.close()
    fb.close()
    x = torch.zeros_like(bd)
    with torch.cuda.stream(stream):
        lat.solve(bd, x, kappa, tol=tol, prec="f16", stream=stream)  # warm
        x.zero_()
        rc, info = lat.solve(bd, x, kappa, tol=tol, prec="f16", stream=stream)
    torch.cuda.synchronize()
    bps = 52 + 64 + 52
    res = {"dslash_f16_8_ms": round(ms, 4),
           "dslash_f16_8_GFLOPs": round(V * FLOP_PER_SITE / ms / 1e6, 1),
           "dslash_f16_8_GBps_algorithmic": round(V * bps / ms / 1e6, 1),
           "bytes_per_site": bps,
           "mixed_f16_8_s": round(info[0]["seconds"], 3), "mixed_f16_8_iters": info[0]["iters"],
           "mixed_f16_8_reliable_updates": info[0]["reliable_updates"],
           "mixed_f16_8_true_rel_resid": info[0]["true_rel_resid"], "rc": rc}
    lat.close()
    log(f"f16 links8: {res}")
    return res


def other_mixed(args, lat, bd, kappa, stream, torch):
    other = "f32" if args.mixed == "f16" else "f16"
    xo = torch.zeros_like(bd)
    with torch.cuda.stream(stream):
        rc, info = lat.solve(bd, xo, kappa, tol=args.tol, prec=other, stream=stream)
    return {f"mixed_{other}_s": round(info[0]["seconds"], 3),
            f"mixed_{other}_iters": info[0]["iters"],
            f"mixed_{other}_true_rel_resid": info[0]["true_rel_resid"]}


def even_odd(args, wd, lat, bd, kappa, stream, torch, V):
    """The same system through the even-odd Schur complement (FP64 and mixed
    FP16-12), with the half-field stencil's average launch time."""
    res = {}
    for prec in ("f64", args.mixed):
        x = torch.zeros_like(bd)
        wd.wd_timing_reset()
        wd.wd_timing_enable(True)
        with torch.cuda.stream(stream):
            rc, info = lat.solve(bd, x, kappa, tol=args.tol, prec=prec, even_odd=True,
                                 stream=stream)
        torch.cuda.synchronize()
        wd.wd_timing_enable(False)
        ms, _ = wd.wd_timing_read("eo_" + prec)
        ms_xr, n_xr = wd.wd_timing_read("eo_xr_" + prec)
        it, up = info[0]["iters"], info[0]["reliable_updates"]
        res[f"{prec}_s"] = round(info[0]["seconds"], 3)
        res[f"{prec}_iters"] = it
        res[f"{prec}_true_rel_resid"] = info[0]["true_rel_resid"]
        res[f"{prec}_rel_resid_D"] = info[0]["rel_resid_D"]
        # half-field launches that did work in this precision (gated launches
        # that found nothing to do are timed too, so the average is an upper
        # bound): 4 per inner iteration, the last of them r-updating when
        # fused; in float64 also b^ and M^dag b^ (3), 4 per reliable update
        # after the first, and the odd half and the final residual (3)
        fused = n_xr > 0
        n = (3 if fused else 4) * it
        if prec == "f64":
            n += 3 + 4 * max(up - 1, 0) + 3
        # float64 halves are read as 12 reals when the links are special unitary
        link = LINK_BYTES[prec]
        if prec == "f64" and lat.links_info()[0] == 12:
            link = 384
        if n:
            # one launch writes half the sites and reads every link once
            # (forward links of its parity, backward of the other) and the
            # other half's spinors; the c field some launches add is not counted
            avg = ms / n
            per_site = 2 * link + 2 * SPINOR_BYTES[prec]
            res[f"hop_{prec}_avg_ms"] = round(avg, 4)
            res[f"hop_{prec}_GBps_algorithmic"] = round((V // 2) * per_site / avg / 1e6, 1)
        if fused and it:
            # plus c read, r (float64, else float32) read and written; q not
            # stored
            xs = 192 if prec == "f64" else 96
            avg = ms_xr / it
            per_site = 2 * link + 2 * SPINOR_BYTES[prec] + 2 * xs
            res[f"hop_xr_{prec}_avg_ms"] = round(avg, 4)
            res[f"hop_xr_{prec}_GBps_algorithmic"] = round((V // 2) * per_site / avg / 1e6, 1)
    log(f"even-odd: {res}")
    return res


def multi_rhs(np, torch, synth, wd):
    """24^3 x 48, kappa 0.124, eps = 0.3 links seed 4: the 12 spin-colour point
    sources at the origin solved in one batched call (FP32-12 inner, FP64
    reliable updates) versus 12 single solves; and the batched stencil."""
    dims = (24, 24, 24, 48)
    V = int(np.prod(dims))
    dev = torch.device("cuda:0")
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(synth.gauge(dims, 4, synth.EXP, 0.3)).to(dev))
    B = torch.from_numpy(synth.spin_colour_point_sources(dims)).to(dev)
    X = torch.zeros_like(B)
    lat.solve(B, X, 0.124, tol=1e-10, prec="f32", nrhs=12)  # warm
    torch.cuda.synchronize()
    t = time.time()
    rc, info = lat.solve(B, X, 0.124, tol=1e-10, prec="f32", nrhs=12)
    torch.cuda.synchronize()
    t12 = time.time() - t
    Xs = torch.zeros_like(B)
    t = time.time()
    single = []
    for k in range(12):
        r1, i1 = lat.solve(B[k], Xs[k], 0.124, tol=1e-10, prec="f32")
        single.append(i1[0])
    torch.cuda.synchronize()
    t1 = time.time() - t
    # batched stencil versus one source, FP32-12
    res = {"lattice": "24x24x24x48", "rhs": 12, "batched_s": round(t12, 3),
           "sequential_12_s": round(t1, 3), "speedup": round(t1 / t12, 3),
           "max_iters": max(i["iters"] for i in info),
           "sum_iters": sum(i["iters"] for i in info),
           "max_true_rel_resid": max(i["true_rel_resid"] for i in info),
           "batched_bitwise_equal_to_single": bool(torch.equal(X, Xs))}
    for nrhs in (1, 12):
        fa = wd.Field(lat, "f32", nrhs=nrhs)
        fb = wd.Field(lat, "f32", nrhs=nrhs)
        fa.load(B[:nrhs].contiguous() if nrhs > 1 else B[0].contiguous())
        for _ in range(3):
            wd.wd_dslash(lat, 0.124, 0, fa, fb)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            wd.wd_dslash(lat, 0.124, 0, fa, fb)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        alg = V * (LINK_BYTES["f32"] + nrhs * 2 * SPINOR_BYTES["f32"])
        res[f"dslash_f32_nrhs{nrhs}_ms"] = round(ms, 4)
        res[f"dslash_f32_nrhs{nrhs}_bytes_per_rhs_site"] = round(alg / (V * nrhs), 1)
        res[f"dslash_f32_nrhs{nrhs}_GBps_algorithmic"] = round(alg / ms / 1e6, 1)
        res[f"dslash_f32_nrhs{nrhs}_GFLOPs"] = round(V * nrhs * FLOP_PER_SITE / ms / 1e6, 1)
        fa.close()
        fb.close()
    lat.close()
    log(f"multi-rhs: {res}")
    return res


def serving(np, torch, synth, wd, n_requests):
    """Poisson request stream through the solve server: lattices uniform over
    {8^4, 12^4, 16^3x32, 24^3x48} (two eps = 0.3 gauge fields each), kappa
    uniform in [0.115, 0.1245], 1-12 sources, tol 1e-10, mixed FP32-12;
    64 GiB budget.  The arrival rate is 0.7 x the closed-loop rate measured
    first with 16 requests submitted at once; shorter streams at 0.4x and
    1.0x sweep the rate."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    sizes = [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 32), (24, 24, 24, 48)]
    lats, srcs = [], {}
    for d in sizes:
        for seed in (61, 62):
            lat = wd.Lattice(d)
            lat.set_gauge(torch.from_numpy(synth.gauge(d, seed + 10 * len(lats), synth.EXP, 0.3)).to(dev))
            lats.append(lat)
        srcs[d] = torch.from_numpy(synth.gaussian_sources(d, [500 + k for k in range(12)])).to(dev)

    def draw():
        lat = lats[rng.integers(len(lats))]
        return lat, float(rng.uniform(0.115, 0.1245)), int(rng.integers(1, 13))

    def run(srv, reqs, arrivals):
        live, done = {}, {}
        t0 = time.time()
        k = 0
        while len(done) < len(reqs):
            now = time.time() - t0
            while k < len(reqs) and arrivals[k] <= now:
                lat, kap, nrhs = reqs[k]
                b = srcs[lat.dims][:nrhs]
                b = b[0] if nrhs == 1 else b
                x = torch.empty_like(b)
                live[srv.submit(lat, b, x, kap, tol=1e-10, prec="f32", nrhs=nrhs)] = (b, x)
                k += 1
            for t in list(live):
                rc, info = srv.poll(t)
                if rc != wd.WD_PENDING:
                    done[t] = (rc, info)
                    del live[t]
            time.sleep(0.0005)
        return done

    budget = 64 << 30
    srv = wd.Server(budget, max_active=8)
    closed = [draw() for _ in range(16)]
    t = time.time()
    d0 = run(srv, closed, [0.0] * 16)
    rate = 16 / (time.time() - t)
    srv.close()

    def stream_at(factor, n):
        lam = factor * rate
        reqs = [draw() for _ in range(n)]
        arrivals = np.cumsum(rng.exponential(1.0 / lam, n))
        srv = wd.Server(budget, max_active=8)
        d = run(srv, reqs, arrivals)
        st = srv.stats()
        peak = srv.peak_bytes()
        srv.close()
        ok = sum(1 for rc, _ in d.values() if rc == 0)
        worst = max(max(i["true_rel_resid"] for i in info) for rc, info in d.values())
        return {"requests": n, "arrival_rate_per_s": round(lam, 2),
                "solves_per_s": round(st["solves_per_s"], 2),
                "p50_latency_s": round(st["p50_s"], 4), "p99_latency_s": round(st["p99_s"], 4),
                "succeeded": ok, "max_true_rel_resid": worst, "peak_bytes": peak}

    res = stream_at(0.7, n_requests)
    res.update({"closed_loop_solves_per_s": round(rate, 2), "budget_bytes": budget,
                "closed_loop_ok": sum(1 for rc, _ in d0.values() if rc == 0)})
    res["rate_sweep"] = {f"{f}x": stream_at(f, max(16, n_requests // 4)) for f in (0.4, 1.0)}
    for lat in lats:
        lat.close()
    log(f"serving: {res}")
    return res


def cpu_baseline(np, iters_16=None, iters_48=None):
    """The CPU oracle (NumPy, complex128, one thread), timed on this host.

    The headline `value` is the oracle on a bounded sample of the benchmark
    workload itself: one D^dag D application (apply_D then apply_Ddag) on a
    48^3 x 6 t-slab of the 48^3 x 96 configuration (links seed 3 for t = 0..5,
    the Gaussian source seed 103 on those sites; the slab's t ends wrap, so
    this is a timing sample, not a result), in GFLOP/s at 1320 flop per site
    and application.  From it, the FP64 CG on 48^3 x 96 is extrapolated: the
    sampled D^dag D time per site x V x the GPU solve's iteration count
    (vector updates not counted), labelled as extrapolated.  Also: the
    oracle's stencil on 16^3 x 32 (median of 5), its CG to solution on the
    4^4 configuration, and 3 CG iterations on 16^3 x 32 extrapolated to the
    GPU's iteration count."""
    import synth
    from oracle import cg, wilson
    full = (48, 48, 48, 96)
    ts_ = 6
    slab = (48, 48, 48, ts_)
    vs = 48 ** 3 * ts_
    Us = synth.gauge(full, 3, synth.EXP, 0.3, t0=0, t1=ts_)
    ps = synth.gaussian_spinor(full, 103, s0=0, s1=vs)
    t = time.time()
    y = wilson.apply_D(Us, ps, slab, 0.1245)
    t_d = time.time() - t
    t = time.time()
    wilson.apply_Ddag(Us, y, slab, 0.1245)
    t_dd = time.time() - t
    del Us, ps, y
    gflops = 2 * vs * FLOP_PER_SITE / (t_d + t_dd) / 1e9
    out = {"value": round(gflops, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
           "sample": (f"oracle apply_D + apply_Ddag (NumPy einsum stencil, complex128) on a "
                      f"48^3x{ts_} t-slab of the 48^3x96 workload: {t_d:.2f}s + {t_dd:.2f}s; "
                      f"1 thread used (einsum is single-threaded), {os.cpu_count()} cores "
                      f"present"),
           "DdagD_48x48x48x96_s_per_site": (t_d + t_dd) / vs}
    if iters_48:
        out["cg_48x48x48x96_fp64_extrapolated_s"] = round((t_d + t_dd) / vs * 48 ** 3 * 96 *
                                                          iters_48, 1)
        out["cg_48x48x48x96_note"] = (f"extrapolated: the sampled D^dag D time per site x "
                                      f"{48 ** 3 * 96} sites x the GPU solve's {iters_48} "
                                      f"iterations (vector updates not counted)")
    dims = (16, 16, 16, 32)
    V = int(np.prod(dims))
    U = synth.gauge(dims, 2, synth.EXP, 0.3)
    psi = synth.gaussian_spinor(dims, 102)
    ts = []
    for _ in range(5):
        t = time.time()
        wilson.apply_D(U, psi, dims, 0.124)
        ts.append(time.time() - t)
    t16 = statistics.median(ts)
    out["stencil_16x16x16x32_GFLOPs"] = round(V * FLOP_PER_SITE / t16 / 1e9, 3)
    out["stencil_16x16x16x32_note"] = f"median of 5 runs of {t16:.3f}s"
    d4 = (4, 4, 4, 4)
    U4 = synth.gauge(d4, 1, synth.HAAR, 0.3)
    b4 = synth.point_source(d4)
    tc = time.time()
    _, it4, _ = cg.cgnr(lambda v: wilson.apply_D(U4, v, d4, 0.12),
                        lambda v: wilson.apply_Ddag(U4, v, d4, 0.12), b4, tol=1e-10)
    out["cg_4x4x4x4_s"] = round(time.time() - tc, 4)
    out["cg_4x4x4x4_iters"] = it4
    if iters_16:
        b16 = synth.gaussian_spinor(dims, 102)
        t3 = time.time()
        cg.cgnr(lambda v: wilson.apply_D(U, v, dims, 0.124),
                lambda v: wilson.apply_Ddag(U, v, dims, 0.124), b16, tol=1e-30, max_iter=3)
        t3 = (time.time() - t3) / 3
        out["cg_16x16x16x32_extrapolated_s"] = round(t3 * iters_16, 1)
        out["cg_16x16x16x32_note"] = (f"extrapolated: 3 oracle CG iterations ({t3:.2f} s each, "
                                      f"D^dag b included) times the GPU solve's {iters_16}")
    log(f"cpu baseline: {out}")
    return out


# ------------------------------------------------------------------ profiling helpers

def probe(np, torch, synth, wd):
    """Workload for counter runs: a plain 2 GiB copy (calibration), then three
    stencil sweeps per precision at 48^3 x 96."""
    dev = torch.device("cuda:0")
    n = 256 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    dims = (48, 48, 48, 96)
    V = int(np.prod(dims))
    U = torch.empty((V, 4, 3, 3, 2), dtype=torch.float64, pin_memory=True)
    synth.gauge(dims, 3, synth.EXP, 0.3, out=U.numpy())
    lat = wd.Lattice(dims)
    Ud = U.to(dev)
    lat.set_gauge(Ud)
    del Ud
    psi = torch.from_numpy(synth.gaussian_spinor(dims, 103)).to(dev)
    for prec in ("f64", "f32", "f16"):
        fa = wd.Field(lat, prec)
        fb = wd.Field(lat, prec)
        fa.load(psi)
        for _ in range(3):
            wd.wd_dslash(lat, 0.1245, 0, fa, fb)
        torch.cuda.synchronize()
        fa.close()
        fb.close()
        print(f"probe {prec} done", flush=True)
    # the even-odd Schur operator: two half-field stencil launches each
    out = torch.empty_like(psi)
    for prec in ("f64", "f16"):
        for _ in range(3):
            lat.apply_schur(0.1245, psi, out, prec=prec)
        torch.cuda.synchronize()
        print(f"probe schur {prec} done", flush=True)
    # CG iterations (the stencil with the fused r update), FP64 and mixed;
    # eager launches (no graph replay) for the counters
    os.environ["WD_GRAPH"] = "0"
    x = torch.zeros_like(psi)
    for prec in ("f64", "f16"):
        x.zero_()
        lat.solve(psi, x, 0.1245, tol=1e-10, prec=prec, max_iter=4)
        torch.cuda.synchronize()
        print(f"probe cg {prec} done", flush=True)
    lat.close()
    del psi, out, x
    torch.cuda.empty_cache()
    # the batched stencil: 12 sources on 24^3 x 48, FP32-12
    dims = (24, 24, 24, 48)
    V = int(np.prod(dims))
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(synth.gauge(dims, 4, synth.EXP, 0.3)).to(dev))
    B = torch.from_numpy(synth.gaussian_sources(dims, list(range(200, 212)))).to(dev)
    fa = wd.Field(lat, "f32", nrhs=12)
    fb = wd.Field(lat, "f32", nrhs=12)
    fa.load(B)
    for _ in range(3):
        wd.wd_dslash(lat, 0.124, 0, fa, fb)
    torch.cuda.synchronize()
    fa.close()
    fb.close()
    lat.close()
    print("probe nrhs=12 done", flush=True)


MULTI_DIMS = (24, 24, 24, 48)


def probe_multi(np, torch, synth, wd):
    """Workload for counter and trace runs of the 12-source batch on 24^3 x 48
    (FP32-12): one source, then all 12, each as five stencil sweeps and six
    eager CG iterations (FP32 inner).  A tiny streaming-probe launch marks
    the start and end of each phase in the dispatch order."""
    dev = torch.device("cuda:0")
    dims = MULTI_DIMS
    lat = wd.Lattice(dims)
    lat.set_gauge(torch.from_numpy(synth.gauge(dims, 4, synth.EXP, 0.3)).to(dev))
    B = torch.from_numpy(synth.gaussian_sources(dims, list(range(200, 212)))).to(dev)
    tick_src = torch.zeros(4096, dtype=torch.float64, device=dev)
    tick_dst = torch.empty_like(tick_src)
    os.environ["WD_GRAPH"] = "0"

    def marker():
        torch.cuda.synchronize()
        wd.wd_stream_probe([tick_src], tick_dst)
        torch.cuda.synchronize()

    for nrhs in (1, 12):
        marker()
        src = B[:nrhs].contiguous() if nrhs > 1 else B[0].contiguous()
        fa = wd.Field(lat, "f32", nrhs=nrhs)
        fb = wd.Field(lat, "f32", nrhs=nrhs)
        fa.load(src)
        for _ in range(5):
            wd.wd_dslash(lat, 0.124, 0, fa, fb)
        torch.cuda.synchronize()
        fa.close()
        fb.close()
        x = torch.zeros_like(src)
        lat.solve(src, x, 0.124, tol=1e-10, prec="f32", nrhs=nrhs, max_iter=6)
        torch.cuda.synchronize()
        print(f"probe-multi nrhs={nrhs} done", flush=True)
    marker()
    lat.close()


def multi_summary(args):
    """Per-kernel time and HBM traffic of --probe-multi, one source against
    twelve: time per launch from a kernel trace, FETCH_SIZE / WRITE_SIZE per
    launch from two counter runs (scaled as the stencil summary is), both as
    per-rhs-site figures."""
    fetch = _pmc_rows(args.multi_summary[0])
    write = _pmc_rows(args.multi_summary[1])
    # fetch/write factors of this chip's counters (2 GiB copies calibrate the
    # stencil summary; the same factors hold here)
    try:
        with open(TRAFFIC_FILE) as f:
            cal = json.load(f)["copy_calibration"]
        ff, wf = cal["fetch_factor"], cal["write_factor"]
    except (OSError, ValueError, KeyError):
        ff, wf = 2.0, 1.0
    trace = []
    with open(args.multi_summary[2]) as f:
        for r in csv.DictReader(f):
            trace.append({"id": int(r["Dispatch_Id"]), "name": r["Kernel_Name"],
                          "grid": int(r["Grid_Size"]) if "Grid_Size" in r else
                          int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]),
                          "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
    trace.sort(key=lambda r: r["id"])

    def phases(rows):
        """rows between the probe's markers: [nrhs 1 rows, nrhs 12 rows]"""
        cut = [k for k, r in enumerate(rows) if "k_stream_probe" in r["name"]]
        return [rows[cut[0] + 1:cut[1]], rows[cut[1] + 1:cut[2]]]

    V = 1
    for d in MULTI_DIMS:
        V *= d
    short = lambda n: re.sub(r"\(.*", "", n.replace("void ", "")).replace("wd::", "")
    lines = ["# 12-source batch against one source: kernel time and HBM traffic (24^3 x 48, FP32-12)",
             "", f"Command: `{args.cmd}`", "",
             "Per launch: median over the launches of the phase that did work; bytes are "
             "FETCH_SIZE and WRITE_SIZE scaled by the copy calibration "
             f"(x{ff} and x{wf}), per rhs-site (V = {V} sites).", "",
             "| kernel | nrhs | launches | us per launch | us per rhs | fetch B/rhs-site | "
             "write B/rhs-site | TB/s |", "|---|---|---|---|---|---|---|---|"]
    per_iter = {}
    for nrhs, fr, wr, tr in zip((1, 12), phases(fetch), phases(write), phases(trace)):
        groups = {}
        for r in tr:
            groups.setdefault((r["name"], r["grid"]), {"ns": [], "f": [], "w": []})["ns"].append(r["ns"])
        for r in fr:
            g = groups.get((r["name"], r["grid"]))
            if g is not None:
                g["f"].append(r.get("FETCH_SIZE", 0.0))
        for r in wr:
            g = groups.get((r["name"], r["grid"]))
            if g is not None:
                g["w"].append(r.get("WRITE_SIZE", 0.0))
        rows = []
        for (name, grid), g in groups.items():
            m = max(g["ns"])
            ns = statistics.median(d for d in g["ns"] if d > 0.5 * m)
            if ns < 2000:
                continue  # finalizers, status copies
            # launches enqueued past the iteration limit return at once
            fk = statistics.median(v for v in g["f"] if v >= 0.5 * max(g["f"])) if g["f"] else 0.0
            wk = statistics.median(v for v in g["w"] if v >= 0.5 * max(g["w"])) if g["w"] else 0.0
            fb, wb = fk * 1024 * ff, wk * 1024 * wf
            rows.append((short(name), len(g["ns"]), ns, fb, wb))
        rows.sort(key=lambda r: -r[2])
        for name, n, ns, fb, wb in rows:
            lines.append(f"| `{name}` | {nrhs} | {n} | {ns / 1e3:.1f} | {ns / 1e3 / nrhs:.1f} | "
                         f"{fb / (V * nrhs):.0f} | {wb / (V * nrhs):.0f} | "
                         f"{(fb + wb) / ns / 1e3:.2f} |")
        # one inner CG iteration: the reducing stencil (q = D p), the
        # r-updating one and the x/p update
        pats = (r"k_dslash_tm<1, false, true, \d+, false, false, 1>",
                r"k_dslash_tm<1, true, true, \d+, false, true, 1>", r"k_update_xp<1, 1>")
        it = [r for r in rows if any(re.fullmatch(p, r[0]) for p in pats)]
        if len(it) == 3:
            ns = sum(r[2] for r in it)
            b = sum(r[3] + r[4] for r in it)
            per_iter[nrhs] = (ns / nrhs, b / (V * nrhs), b / ns / 1e3)
    lines += ["", "One inner CG iteration (reducing stencil + r-updating stencil + x/p update):", "",
              "| nrhs | us per rhs | bytes per rhs-site | TB/s |", "|---|---|---|---|"]
    for nrhs, (us, bps, tbs) in sorted(per_iter.items()):
        lines.append(f"| {nrhs} | {us / 1e3:.1f} | {bps:.0f} | {tbs:.2f} |")
    if 1 in per_iter and 12 in per_iter:
        lines += ["", f"Batch speed-up per iteration: {per_iter[1][0] / per_iter[12][0]:.3f}; "
                  f"bytes per rhs-site {per_iter[12][1] / per_iter[1][1]:.3f} of one source's, "
                  f"streamed at {per_iter[12][2] / per_iter[1][2]:.3f} of its rate."]
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _pmc_rows(path):
    rows = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            key = int(r["Dispatch_Id"])
            e = rows.setdefault(key, {"name": r["Kernel_Name"], "grid": int(r["Grid_Size"])})
            e[r["Counter_Name"]] = float(r["Counter_Value"])
    return [rows[k] for k in sorted(rows)]


def pmc_summary(args):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the probe, scaled by
    what the same counters read for the plain copy of known size."""
    fetch = _pmc_rows(args.pmc_summary[0])
    write = _pmc_rows(args.pmc_summary[1])
    copy_bytes = 256 * 1024 * 1024 * 8
    # the 2 GiB calibration copies: the largest copy dispatches (small copies
    # of status words run too)
    cf = [r for r in fetch if "copyBuffer" in r["name"]]
    cw = [r for r in write if "copyBuffer" in r["name"]]
    cf = [r for r in cf if r["grid"] == max(q["grid"] for q in cf)]
    cw = [r for r in cw if r["grid"] == max(q["grid"] for q in cw)]
    ff = copy_bytes / (statistics.median(r["FETCH_SIZE"] for r in cf) * 1024)
    wf = copy_bytes / (statistics.median(r["WRITE_SIZE"] for r in cw) * 1024)
    V = 48 * 48 * 48 * 96
    out = {"command": args.cmd, "source_sha256": kernel_source_hash(),
           "copy_calibration": {"bytes_read": copy_bytes, "bytes_written": copy_bytes,
                                "fetch_factor": round(ff, 4), "write_factor": round(wf, 4)},
           "kernels": {}}
    # kernel names carry the hop scheduling group (a tuning constant) in the
    # fourth template argument: match any
    def named(rows, i, dag, red, xr, lf):
        pat = re.compile(rf"k_dslash_tm<{i}, {dag}, {red}, \d+, false, {xr}, {lf}>")
        return [r for r in rows if pat.search(r["name"])]

    kinds = []
    for i, prec in enumerate(("f64", "f32", "f16")):
        # the plain stencil (D, no reduction) and the CG's r-updating D^dag;
        # float64 with its 12-real (form 3) or 18-real links
        forms = ((3, 384), (0, 576)) if prec == "f64" else ((i, None),)
        for lf, link in forms:
            b, bx = BYTES_PER_SITE[prec], XR_BYTES_PER_SITE[prec]
            if link is not None:
                b, bx = b - 576 + link, bx - 576 + link
            kinds.append((prec, (i, "false", "false", "false", lf), b))
            kinds.append(("xr_" + prec, (i, "true", "true", "true", lf), bx))
    for key, sig, bps in kinds:
        fr = named(fetch, *sig)
        wr = named(write, *sig)
        if not fr or not wr:
            continue
        # the 48^3 x 96 launches (the batched probe on 24^3 x 48 has another
        # launch shape and comes later)
        fr = [r for r in fr if r["grid"] == fr[0]["grid"]]
        wr = [r for r in wr if r["grid"] == wr[0]["grid"]]
        # launches that did work (a solve's launches after it stopped return
        # at once)
        fm = max(r["FETCH_SIZE"] for r in fr)
        wm = max(r["WRITE_SIZE"] for r in wr)
        fk = statistics.median(r["FETCH_SIZE"] for r in fr if r["FETCH_SIZE"] > 0.5 * fm)
        wk = statistics.median(r["WRITE_SIZE"] for r in wr if r["WRITE_SIZE"] > 0.5 * wm)
        traffic = fk * 1024 * ff + wk * 1024 * wf
        alg = V * bps
        if f"dslash_{key}" in out["kernels"]:
            continue  # a probe runs one link form per precision
        out["kernels"][f"dslash_{key}"] = {
            "FETCH_SIZE_KiB": fk, "WRITE_SIZE_KiB": wk, "traffic_bytes": round(traffic),
            "algorithmic_bytes": alg, "algorithmic_bytes_per_site": bps,
            "traffic_over_algorithmic": round(traffic / alg, 3),
            "traffic_bytes_per_site": round(traffic / V, 1)}
    # the batched FP32 stencil, 12 sources on 24^3 x 48: bytes per rhs-site
    fr = named(fetch, 1, "false", "false", "false", 1)
    wr = named(write, 1, "false", "false", "false", 1)
    if fr and wr and fr[-1]["grid"] != fr[0]["grid"]:
        g12 = fr[-1]["grid"]
        fk = statistics.median(r["FETCH_SIZE"] for r in fr if r["grid"] == g12)
        wk = statistics.median(r["WRITE_SIZE"] for r in wr if r["grid"] == g12)
        n = 24 * 24 * 24 * 48 * 12
        out["kernels"]["dslash_f32_nrhs12_24x24x24x48"] = {
            "FETCH_SIZE_KiB": fk, "WRITE_SIZE_KiB": wk,
            "traffic_bytes": round(fk * 1024 * ff + wk * 1024 * wf),
            "algorithmic_bytes_per_rhs_site": 208,
            "fetch_bytes_per_rhs_site": round(fk * 1024 * ff / n, 1),
            "write_bytes_per_rhs_site": round(wk * 1024 * wf / n, 1)}
    # even-odd half-field stencil (k_hop_half): a launch writes V/2 sites,
    # reads every link once and the other half's spinors, and (every second
    # launch of M) a c field
    for prec, i in (("f64", 0), ("f16", 2)):
        # the marching form where the probe ran it, else one lane per site
        for tag in (f"k_hop_half_tm<{i}", f"k_hop_half<{i}"):
            fr = [r for r in fetch if tag in r["name"]]
            wr = [r for r in write if tag in r["name"]]
            if fr and wr:
                break
        if not fr or not wr:
            continue
        fk = statistics.mean(r["FETCH_SIZE"] for r in fr)
        wk = statistics.mean(r["WRITE_SIZE"] for r in wr)
        traffic = fk * 1024 * ff + wk * 1024 * wf
        # the last template argument is the link form (3: float64, 12 reals)
        link = 384 if prec == "f64" and fr[0]["name"].split(">")[0].endswith(", 3") else \
            LINK_BYTES[prec]
        per_site = 2 * link + 2.5 * SPINOR_BYTES[prec]
        alg = V // 2 * per_site
        out["kernels"][f"hop_half_{prec}"] = {
            "kernel": tag.split("<")[0],
            "FETCH_SIZE_KiB": fk, "WRITE_SIZE_KiB": wk, "traffic_bytes": round(traffic),
            "algorithmic_bytes": alg, "traffic_over_algorithmic": round(traffic / alg, 3),
            "traffic_bytes_per_output_site": round(traffic / (V // 2), 1)}
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def valu_summary(args):
    """Vector-ALU instructions of the probe's stencil launches (SQ_INSTS_VALU,
    wave instructions) and the time the chip needs just to issue them: four
    cycles per wave64 instruction on each of 1024 SIMDs at 2.4 GHz (no packed
    FP32).  Compared with a launch's duration this says how close to
    ALU-bound it is."""
    rows = _pmc_rows(args.valu_summary)
    lines = ["# Vector-ALU work of the stencil launches", "", f"Command: `{args.cmd}`", "",
             "Issue time: SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz), the least time "
             "the chip needs to issue the launch's vector instructions; the launch durations "
             "are in the kernel statistics and the bench line (e.g. FP64 stencil 1.86 ms, "
             "binary16 0.55 ms, the 12-source FP32 stencil 0.54 ms).", "",
             "| kernel | launch shape (threads) | VALU wave-instr. | issue time ms |",
             "|---|---|---|---|"]
    # per kernel and launch shape, the launch that did the most work (a
    # solve's launches after it stopped return at once)
    best = {}
    for r in rows:
        if "k_dslash_tm" not in r["name"] and "k_hop_half" not in r["name"]:
            continue
        key = (r["name"], r["grid"])
        if r.get("SQ_INSTS_VALU", 0.0) >= best.get(key, {}).get("SQ_INSTS_VALU", -1.0):
            best[key] = r
    for (_, _), r in best.items():
        valu = r.get("SQ_INSTS_VALU", 0.0)
        name = r["name"].split("(")[0].replace("void wd::", "")
        lines.append(f"| `{name}` | {r['grid']} | {valu / 1e6:.1f} M | "
                     f"{valu * 4 / (1024 * 2.4e9) * 1e3:.3f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def sq_summary(args):
    """Wave counters of the probe's stencil launches, from one or more
    counter runs of `bench.py --probe` (each run holds a few SQ counters; the
    k-th launch of a kernel is the same launch in every run).  Per kernel and
    launch shape, the launch with the most wave-cycles: waves, their average
    lifetime, and the share of that lifetime spent issuing (any, vector ALU,
    vector memory) and waiting (for any instruction's dependencies)."""
    merged = {}
    for path in args.sq_summary:
        seen = {}
        for r in _pmc_rows(path):
            if "k_dslash_tm" not in r["name"] and "k_hop_half" not in r["name"]:
                continue
            key = (r["name"], r["grid"])
            k = seen.get(key, 0)
            seen[key] = k + 1
            e = merged.setdefault((key, k), {"name": r["name"], "grid": r["grid"]})
            e.update({c: v for c, v in r.items() if c.startswith("SQ_")})
    best = {}
    for (key, _), e in merged.items():
        if e.get("SQ_WAVE_CYCLES", 0.0) >= best.get(key, {}).get("SQ_WAVE_CYCLES", -1.0):
            best[key] = e
    cols = [("SQ_ACTIVE_INST_ANY", "issuing"), ("SQ_ACTIVE_INST_VALU", "VALU"),
            ("SQ_ACTIVE_INST_VMEM", "VMEM"), ("SQ_WAIT_INST_ANY", "waiting"),
            ("SQ_WAIT_ANY", "wait (any)")]
    lines = ["# Wave counters of the stencil launches", "", f"Command: `{args.cmd}`", "",
             "Shares are of SQ_WAVE_CYCLES (the waves' summed lifetime, same units): "
             "issuing = SQ_ACTIVE_INST_ANY, VALU = SQ_ACTIVE_INST_VALU, VMEM = "
             "SQ_ACTIVE_INST_VMEM, waiting = SQ_WAIT_INST_ANY (a wave held by an "
             "instruction dependency, e.g. a memory wait), wait (any) = SQ_WAIT_ANY.", "",
             "| kernel | threads | SQ_WAVES | wave-cycles per wave | SQ_BUSY_CYCLES | " +
             " | ".join(h for _, h in cols) + " |",
             "|---|---|---|---|---|" + "---|" * len(cols)]
    for (_, _), e in best.items():
        wc = e.get("SQ_WAVE_CYCLES", 0.0)
        nw = e.get("SQ_WAVES", 0.0)
        name = e["name"].split("(")[0].replace("void wd::", "")
        share = [f"{e[c] / wc:.2f}" if c in e and wc > 0 else "" for c, _ in cols]
        lines.append(f"| `{name}` | {e['grid']} | {nw:.0f} | "
                     f"{wc / nw if nw else 0:.0f} | {e.get('SQ_BUSY_CYCLES', 0.0):.0f} | " +
                     " | ".join(share) + " |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def trace_summary(args):
    """Short markdown table of a rocprofv3 --stats kernel summary.  With the
    sibling *_kernel_trace.csv it also averages only the launches that did
    work (over 1% of the kernel's longest): iterations enqueued after a solve
    converged return at once and would dilute the plain average."""
    with open(args.trace_summary) as f:
        rows = list(csv.DictReader(f))
    if args.match:
        rows = [r for r in rows if re.search(args.match, r["Name"])]
    rows.sort(key=lambda r: -float(r.get("TotalDurationNs", 0)))
    busy = {}
    tr = args.trace_summary.replace("_kernel_stats.csv", "_kernel_trace.csv")
    wl = os.path.join(os.path.dirname(args.trace_summary), "working_launches.json")
    if os.path.exists(wl):
        # the same averages, computed where the (large) trace was taken:
        # {kernel: [calls, working launches, average ns of those]}
        with open(wl) as f:
            for name, (_, n, ns) in json.load(f).items():
                busy[name] = (n, ns / 1e6)
    elif os.path.exists(tr):
        durs = {}
        with open(tr) as f:
            for r in csv.DictReader(f):
                d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                durs.setdefault(r["Kernel_Name"], []).append(d)
        for name, ds in durs.items():
            m = max(ds)
            real = [d for d in ds if d > 0.01 * m]
            busy[name] = (len(real), sum(real) / len(real) / 1e6)
    lines = [f"# rocprofv3 kernel statistics", "", f"Command: `{args.cmd}`", "",
             "| kernel | calls | total ms | avg ms | working launches | avg ms (working) | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows[:20]:
        name = r["Name"].replace("|", "/")
        n, a = busy.get(r["Name"], ("", None))
        short = name if len(name) <= 90 else name[:87] + "..."
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e6:.4f} | {n} | "
                     f"{'' if a is None else f'{a:.4f}'} | {float(r['Percentage']):.1f} |")
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
