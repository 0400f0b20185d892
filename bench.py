"""Benchmark of the HISQ Dslash + CG hot path on one MI355X.

Default (the headline line): the 16^3x32 workload (eps 0.2, m 0.02), links
already resident in HBM.  One step is one pass of the hot path:
  * half-lattice Dslash D_eo and D_oe in FP32 recon-18, FP32 recon-12,
    FP16 recon-12 and FP64 recon-18 on device vectors;
  * CG to FP64 true residual 1e-10 from the same source: plain FP64, mixed
    FP32 (recon-18), mixed FP16 storage (recon-12), and the flexible CG with
    the learned preconditioner (trained before the timed region on pairs
    the solver harvests from two other sources).
value = FP32 recon-18 Dslash throughput in algorithmic GB/s (16 links + one
input + one output colour vector per output site) from HIP events recorded on
the stream the kernels run on.  Reported beside it: the other formats, a 32^4
lattice whose links exceed the 256 MB Infinity Cache, the solver times, and
the FP64 CPU oracle timed on the host cores over a bounded sample.

Other workloads (--workload): c0 (4^4 plain FP64 CG), c2 (24^3x48
multi-shift, 12 shifts x 4 sources), c3 (64 uneven solves in one batch),
c4 (16^4 learned preconditioner: 32 training fields, 8 held-out fields).
Each prints one JSON line of its own.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "Dslash GB/s (% HBM peak); CG time-to-1e-10: plain vs mixed/learned"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def site_bytes(prec, recon):
    """Algorithmic bytes per half-Dslash output site."""
    el = {0: 8, 1: 4, 2: 2}[prec]
    spin = {0: 48, 1: 24, 2: 16}[prec]          # FP16: 12 B + 4 B scale
    return 16 * recon * el + 2 * spin


def kernel_hash():
    h = hashlib.sha256()
    for f in ["dslash.hip", "fields.h", "hisq_dev.h", "reduce.h", "finish.h", "launch.h"]:
        with open(os.path.join(ROOT, "paper_1712_00143_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_entry():
    """Measured HBM bytes per launch from the committed counter summary, if it
    was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "dslash_f32r18_16x16x16x32_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def _vec(torch, prec, h, seed):
    dt = {0: torch.float64, 1: torch.float32, 2: torch.float16}[prec]
    n = {0: 6 * h, 1: 6 * h, 2: 8 * h}[prec]     # FP16: 6h halves + h float scales
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn(n, device="cuda", dtype=torch.float32, generator=g).to(dt)
    if prec == 2:
        x[6 * h:] = 1.0
    return x


def timed_dslash(torch, lat, prec, recon, h, stream, reps):
    """Average duration (s) of one half-Dslash launch (both parities alternate),
    as (graph, eager).  The 2*reps launches are captured once in a HIP graph on
    the library's stream and replayed there between two events, so host launch
    gaps do not count; the same launches issued eagerly are timed too.  graph
    is None where capture fails."""
    x = _vec(torch, prec, h, 7)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    lat.dslash(0, prec, recon, x, y)      # tunes the block shape before any capture
    lat.dslash(1, prec, recon, y, x)
    torch.cuda.synchronize()

    def body():
        for _ in range(reps):
            lat.dslash(0, prec, recon, x, y)
            lat.dslash(1, prec, recon, y, x)

    graph = None
    try:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            body()
        with torch.cuda.stream(stream):
            graph.replay()
        torch.cuda.synchronize()
    except Exception as exc:   # pragma: no cover - capture not supported
        log(f"graph capture unavailable ({exc}); timing eager launches")
        graph = None
    def run(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            fn()
            e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / 1000.0 / (2 * reps)

    t_eager = run(body)
    t_graph = run(graph.replay) if graph is not None else None
    return t_graph, t_eager


def timed_ceilings(H, stream):
    """Practical HBM ceilings on the same stream, in GB/s, from the library's
    streaming kernels over 1 GiB: a read-only pass (the half-Dslash is
    96-98 % reads) and a copy (read + written bytes)."""
    return H.stream_bandwidth(0, H.ctypes.c_void_p(stream.cuda_stream), 1 << 30, 10)


def cpu_baseline(dims, fat, lng, budget_s=12.0):
    """The FP64 oracle Dslash on the same lattice: as many half-Dslash
    applications as fit in budget_s seconds of host time."""
    import oracle
    from paper_1712_00143_amd import synth
    psi = synth.gaussian_even(dims, 99)
    h = psi.shape[0]
    oracle.dslash_half(dims, fat, lng, 0, psi)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        psi = oracle.dslash_half(dims, fat, lng, n % 2, psi)
        psi /= np.linalg.norm(psi)
        n += 1
    dt = time.perf_counter() - t0
    gbs = n * h * site_bytes(0, 18) / dt / 1e9
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} FP64 half-Dslash applications on {'x'.join(map(str, dims))} in {dt:.1f} s "
                      f"(plain C oracle, OpenMP over sites, same byte model)"}


def solve_timed(torch, stream, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def train_preconditioner(H, synth, dims, eps, mass, seed0, nfield, nsrc, steps, chans=(1, 4, 4, 1),
                         every=10, maxpairs=60, batch=8, lr=3e-3, init="poly"):
    """Harvest (residual, error) pairs with the solver on nfield seeded fields
    and train the network on the GPU, starting from the polynomial weights
    (init "poly") or small random ones ("random").  Returns (net, lattices,
    seconds, losses)."""
    t0 = time.perf_counter()
    lats, net = [], None
    for j in range(nfield):
        fat, lng = synth.make_links(dims, eps, seed=seed0 + j)
        L = H.Lattice(dims)
        L.load_links(fat, lng)
        L.prepare_links(1, 18)
        lats.append(L)
        if net is None:
            net = H.PTC(L, chans)
            if init == "poly":
                lam = net.init_polynomial(a=4.0, c=1.2)
                log(f"polynomial start: lambda_max(-D_f^2) ~ {lam:.4f}")
            else:
                rng = np.random.default_rng(seed0)
                net.set_weights([0.05 * (rng.standard_normal((b, a, 9)) + 1j * rng.standard_normal((b, a, 9)))
                                 for a, b in zip(chans[:-1], chans[1:])])
        for s in range(nsrc):
            net.harvest(L, mass, synth.gaussian_even(dims, seed0 + j + 500 + 100 * s), every=every,
                        maxpairs=maxpairs)
        log(f"harvested field {j + 1}/{nfield}: {net.pair_count()} pairs")
    t1 = time.perf_counter()
    losses = net.train(steps, batch=batch, lr=lr, seed=seed0)
    t2 = time.perf_counter()
    log(f"trained {steps} steps: loss {losses[:10].mean():.4f} -> {losses[-50:].mean():.4f}")
    times = {"total_s": round(t2 - t0, 2), "harvest_s": round(t1 - t0, 2), "train_s": round(t2 - t1, 2),
             "pairs": net.pair_count()}
    return net, lats, times, losses


# ----------------------------------------------------------------- headline

def run_headline(args):
    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth

    w = synth.C1
    fat, lng = w.links()
    b = w.sources()[0]
    h = synth.volume(w.dims) // 2
    stream = torch.cuda.Stream()
    sp = H.ctypes.c_void_p(stream.cuda_stream)
    lat = H.Lattice(w.dims, stream=sp)
    lat.load_links(fat, lng)
    formats = [(1, 18), (1, 12), (2, 12), (0, 18)]
    for p, r in formats:
        lat.prepare_links(p, r)
    bd = torch.from_numpy(b.view(np.float64)).cuda()
    solves = {
        "plain_f64": H.hisq_default_params(tol=1e-10, sloppy=0, recon=18, flags=H.HISQ_USE_GRAPH),
        "mixed_f32_r18": H.hisq_default_params(tol=1e-10, sloppy=1, recon=18, flags=H.HISQ_USE_GRAPH),
        "mixed_f16_r12": H.hisq_default_params(tol=1e-10, sloppy=2, recon=12, flags=H.HISQ_USE_GRAPH),
    }
    net = None
    train_info = None
    if not args.no_learned and not args.dslash_only:
        # trained outside the timed region, on pairs from two other sources
        net = H.PTC(lat, (1, 2, 1))
        t0 = time.perf_counter()
        net.init_polynomial(a=4.0, c=1.2)
        srcs = w.sources()
        npair = sum(net.harvest(lat, w.mass, srcs[k], every=20, maxpairs=60) for k in (1, 2))
        losses = net.train(300, batch=8, lr=3e-3, seed=1)
        train_info = {"network": "1-2-1 PTC, polynomial start, energy-norm loss",
                      "pairs": npair, "steps": 300, "seconds": round(time.perf_counter() - t0, 3),
                      "loss_first10": round(float(losses[:10].mean()), 4),
                      "loss_last50": round(float(losses[-50:].mean()), 4)}

    def step():
        res = {"dslash_s": {}, "cg": {}}
        for p, r in formats:
            res["dslash_s"][(p, r)] = timed_dslash(torch, lat, p, r, h, stream, args.reps)
        if not args.dslash_only:
            for name, prm in solves.items():
                xd = torch.zeros_like(bd)
                (_, info), dt = solve_timed(torch, stream, lambda: lat.cg(w.mass, bd, x=xd, params=prm))
                info["wall_s"] = dt
                res["cg"][name] = info
            if net is not None:
                xd = torch.zeros_like(bd)
                prm = H.hisq_default_params(tol=1e-10, sloppy=1, recon=18, flags=H.HISQ_USE_GRAPH)
                (_, info), dt = solve_timed(torch, stream, lambda: net.cg_learned(lat, w.mass, bd, x=xd, params=prm))
                info["wall_s"] = dt
                res["cg"]["learned_fcg_f32"] = info
        return res

    for _ in range(args.warmup):
        step()
    log("warm-up done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for k in range(args.steps):
        results.append(step())
        log(f"step {k + 1}/{args.steps}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0

    def avg(key, which):
        ts = [r["dslash_s"][key][which] for r in results]
        return None if any(t is None for t in ts) else float(np.mean(ts))

    def dtime(key):
        """Graph-replay time where capture worked, else the eager time."""
        tg = avg(key, 0)
        return (tg, "graph") if tg is not None else (avg(key, 1), "eager")

    dsl = {}
    for p, r in formats:
        t, how = dtime((p, r))
        gbs = h * site_bytes(p, r) / t / 1e9
        dsl[f"{['f64', 'f32', 'f16'][p]}_r{r}"] = {
            "us": round(t * 1e6, 3), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
            "GFLOP/s": round(1146.0 * h / t / 1e9, 1), "timing": how,
            "us_eager_launches": round(avg((p, r), 1) * 1e6, 3)}
    t32, how32 = dtime((1, 18))
    achieved = h * site_bytes(1, 18) / t32 / 1e9

    cg = {}
    if not args.dslash_only:
        for name in results[0]["cg"]:
            infos = [r["cg"][name] for r in results]
            cg[name] = {"time_s": round(float(np.median([i["wall_s"] for i in infos])), 5),
                        "iters": infos[-1]["iters"], "reliable_updates": infos[-1]["reliable_updates"],
                        "true_residual_fp64": float(f"{infos[-1]['true_residual']:.3e}"),
                        "converged": bool(infos[-1]["converged"])}
            if name.startswith("learned"):
                cg[name]["fell_back"] = bool(infos[-1]["fell_back"])
                cg[name]["training"] = train_info

    read_gbs, copy_gbs = timed_ceilings(H, stream)
    # the same FP32 half-Dslash called on host FP64 vectors: the library
    # stages them over PCIe and converts on the device (a rate that includes
    # the host link, reported beside the device-resident one, never as it)
    psi_h = b.copy()
    out_h = np.zeros_like(psi_h)
    lat.dslash(0, 1, 18, psi_h, out_h)
    t0 = time.perf_counter()
    nh = 20
    for k in range(nh):
        lat.dslash(k & 1, 1, 18, psi_h, out_h)
    t_host = (time.perf_counter() - t0) / nh
    host_path = {"us": round(t_host * 1e6, 1),
                 "what": "hisq_dslash on host FP64 vectors (copy in, convert, FP32 Dslash, convert, copy out, "
                         "synchronised), per call"}
    hbm = None
    if not args.no_hbm:
        dims = (32, 32, 32, 32)
        f2, l2 = synth.make_links(dims, 0.2, seed=1900)
        lat2 = H.Lattice(dims, stream=sp)
        lat2.load_links(f2, l2)
        del f2, l2
        hbm = {}
        h2 = synth.volume(dims) // 2
        for p, r in formats:
            lat2.prepare_links(p, r)
            tg, te = timed_dslash(torch, lat2, p, r, h2, stream, 20)
            t = tg if tg is not None else te
            gbs = h2 * site_bytes(p, r) / t / 1e9
            hbm[f"{['f64', 'f32', 'f16'][p]}_r{r}"] = {"us": round(t * 1e6, 2), "GB/s": round(gbs, 1),
                                                       "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)}
        lat2.close()

    out = {
        "metric": METRIC,
        "value": round(achieved, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * t_total / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "HISQ even-odd Dslash (FP32 recon-18) + CG to 1e-10, 16^3x32, eps 0.2, m 0.02",
                   "lattice": list(w.dims), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_entry(),
                     "kernel": "k_dslash<float,18,float,float,W,EPI_PLAIN,CP>",
                     "bytes_per_launch": h * site_bytes(1, 18),
                     "launch_us": round(t32 * 1e6, 3), "timing": f"HIP events around a {how32} of "
                     f"{2 * args.reps} launches on the library stream",
                     "read_ceiling": {"GB/s": round(read_gbs, 1), "frac_of_peak": round(read_gbs / PEAK_HBM_GBS, 4),
                                      "what": "library streaming read of 1 GiB (non-temporal 16-byte loads)",
                                      "dslash_frac_of_read_ceiling": round(achieved / read_gbs, 4)},
                     "copy_ceiling": {"GB/s": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / PEAK_HBM_GBS, 4),
                                      "what": "library copy of 1 GiB, read + written bytes"},
                     "cache": "both parities' FP32 links (151 MB) fit the 256 MB Infinity Cache; the tuner times "
                              "streamed, cached (and, beyond the cache, partly cached) link loads and keeps the "
                              "fastest, so part of the link stream may come from the cache at this size (the 32^4 "
                              "lines are beyond it)"},
        "dslash": dsl,
        "dslash_32^4_beyond_infinity_cache": hbm,
        "dslash_host_buffers": host_path,
        "cg_time_to_1e-10": cg,
    }
    if "plain_f64" in cg:
        out["cg_speedup_vs_plain_f64"] = {k: round(cg["plain_f64"]["time_s"] / v["time_s"], 3)
                                          for k, v in cg.items()}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w.dims, fat, lng)
    if net is not None:
        net.close()
    lat.close()
    print(json.dumps(out), flush=True)


# ------------------------------------------------------- other workloads

def run_c0(args):
    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    w = synth.C0
    fat, lng = w.links()
    b = w.sources()[0]
    lat = H.Lattice(w.dims)
    lat.load_links(fat, lng)
    res = {}
    for name, fl in (("eager", 0), ("graph", H.HISQ_USE_GRAPH)):
        prm = H.hisq_default_params(tol=1e-10, sloppy=0, flags=fl)
        lat.cg(w.mass, b, params=prm)
        ts = []
        for _ in range(5):
            (_, info), dt = solve_timed(torch, None, lambda: lat.cg(w.mass, b, params=prm))
            ts.append(dt)
        res[name] = {"time_s": round(float(np.median(ts)), 6), "iters": info["iters"],
                     "true_residual_fp64": float(f"{info['true_residual']:.3e}")}
    print(json.dumps({"workload": "plain FP64 CG 4^4, eps 0.3, m 0.1, tol 1e-10", "results": res}), flush=True)


def run_c2(args):
    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    w = synth.C2
    fat, lng = w.links()
    b = w.sources()
    shifts = synth.shifts_log(12)
    stream = torch.cuda.Stream()
    lat = H.Lattice(w.dims, stream=H.ctypes.c_void_p(stream.cuda_stream))
    lat.load_links(fat, lng)
    lat.prepare_links(1, 18)
    h = synth.volume(w.dims) // 2
    # multi-RHS Dslash throughput (4 right-hand sides share the link stream)
    x = torch.randn(4 * 6 * h, device="cuda")
    y = torch.empty_like(x)
    lat.dslash(0, 1, 18, x, y, nrhs=4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(20):
        lat.dslash(0, 1, 18, x, y, nrhs=4)
        lat.dslash(1, 1, 18, y, x, nrhs=4)
    e1.record(stream)
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1000.0 / 40
    mrhs_bytes = h * (16 * 18 * 4 + 4 * 2 * 24)
    # 48 right-hand sides (all 12 x 4 problems of the refinement) in one
    # launch: 12 groups of four whose blocks share each tile's link reads
    x48 = torch.randn(48 * 6 * h, device="cuda")
    y48 = torch.empty_like(x48)
    lat.dslash(0, 1, 18, x48, y48, nrhs=48)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(5):
        lat.dslash(0, 1, 18, x48, y48, nrhs=48)
        lat.dslash(1, 1, 18, y48, x48, nrhs=48)
    e1.record(stream)
    e1.synchronize()
    t48 = e0.elapsed_time(e1) / 1000.0 / 10
    del x48, y48
    mrhs = {"mrhs_dslash_f32_r18_nrhs4": {"us": round(t * 1e6, 2), "GB/s": round(mrhs_bytes / t / 1e9, 1),
                                          "frac_hbm": round(mrhs_bytes / t / 1e9 / PEAK_HBM_GBS, 4)},
            "mrhs_dslash_f32_r18_nrhs48": {"us": round(t48 * 1e6, 2), "groups": 12,
                                           "us_per_group": round(t48 * 1e6 / 12, 2),
                                           "what": "one launch over 12 groups of four right-hand sides"}}
    if args.dslash_only:
        print(json.dumps({"workload": "multi-RHS Dslash 24^3x48, FP32 recon-18", **mrhs}), flush=True)
        return
    prm = H.hisq_default_params(tol=1e-8, sloppy=1, flags=H.HISQ_USE_GRAPH)
    # sources and solutions resident in HBM (device pointers)
    bd = torch.from_numpy(np.ascontiguousarray(b).view(np.float64).ravel()).cuda()
    xd = torch.zeros(len(b) * len(shifts) * h * 6, dtype=torch.float64, device="cuda")
    lat.multishift_cg(w.mass, shifts, bd, x=xd, params=prm)
    (xs, infos), dt = solve_timed(torch, stream, lambda: lat.multishift_cg(w.mass, shifts, bd, x=xd, params=prm))
    worst = max(i["true_residual"] for i in infos)
    print(json.dumps({
        "workload": "multi-shift CG 24^3x48, 12 shifts in [1e-4, 1], 4 sources, m 0.01, FP32 + FP64 recurrences, tol 1e-8",
        **mrhs,
        "time_s": round(dt, 4), "krylov_phase_s": round(infos[0]["t_done_s"], 4),
        "iters_per_shift_rhs0": [i["iters"] for i in infos[:12]],
        "refine_iters_per_shift_rhs0": [i["refine_iters"] for i in infos[:12]],
        "worst_true_residual_fp64": float(f"{worst:.3e}"),
        "all_converged": all(i["converged"] for i in infos)}), flush=True)


def run_c3(args):
    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    ws = synth.batch_workload(nper=args.nper)
    lats, bs, ms = [], [], []
    for q, wk in enumerate(ws):
        if q % 16 == 0:
            log(f"generating batch problem {q}/{len(ws)}")
        fat, lng = wk.links()
        L = H.Lattice(wk.dims)
        L.load_links(fat, lng)
        L.prepare_links(1, 18)
        lats.append(L)
        bs.append(wk.sources()[0])
        ms.append(wk.mass)
    prm = H.hisq_default_params(tol=1e-10, sloppy=1, flags=H.HISQ_USE_GRAPH)
    H.hisq_batch_cg(lats, ms, bs, params=prm)          # warm-up: tuning, graph capture
    (xs, infos), dt = solve_timed(torch, None, lambda: H.hisq_batch_cg(lats, ms, bs, params=prm))
    tdone = np.array([i["t_done_s"] for i in infos])
    total_bytes = sum(i["dslash_bytes"] for i in infos)
    # the same solves one after another, for comparison
    t_seq = 0.0
    for L, m, bb in zip(lats, ms, bs):
        (_, _), d1 = solve_timed(torch, None, lambda: L.cg(m, bb, params=prm))
        t_seq += d1
    print(json.dumps({
        "workload": f"batched CG: {len(ws)} solves, {args.nper} each of 8^4, 12^4, 16^4, 16^3x32; eps~U[0.1,0.4], m~logU[0.005,0.2]; FP32 + FP64 reliable, tol 1e-10",
        "time_s": round(dt, 4), "aggregate_dslash_GB/s": round(total_bytes / dt / 1e9, 1),
        "time_to_solution_p50_s": round(float(np.percentile(tdone, 50)), 5),
        "time_to_solution_p99_s": round(float(np.percentile(tdone, 99)), 5),
        "iters_min_max": [min(i["iters"] for i in infos), max(i["iters"] for i in infos)],
        "all_converged": all(i["converged"] for i in infos),
        "sequential_time_s": round(t_seq, 4), "batch_speedup": round(t_seq / dt, 3)}), flush=True)


def run_c4(args):
    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    w = synth.C4
    # the 1 -> 4 -> 4 -> 1 network, trained from small random weights
    net, tl, t_train, losses = train_preconditioner(H, synth, w.dims, w.eps, w.mass, 4000, args.nfield,
                                                    args.nsrc, args.train_steps, init="random")
    # the two-layer 1 -> 2 -> 1 network (the smallest that holds the polynomial
    # preconditioner), on a quarter of the fields, from random weights and
    # from the polynomial start
    nq, sq = max(1, args.nfield // 4), max(1, args.nsrc // 2)
    net2, tl2, t_train2, losses2 = train_preconditioner(H, synth, w.dims, w.eps, w.mass, 4000, nq, sq,
                                                        args.train_steps, chans=(1, 2, 1), init="random")
    net3, tl3, t_train3, losses3 = train_preconditioner(H, synth, w.dims, w.eps, w.mass, 4000, nq, sq,
                                                        args.train_steps, chans=(1, 2, 1), init="poly")
    res = {"plain_f64": [], "mixed_f32": [], "mixed_f16_r12": [], "learned_fcg": [], "learned_fcg_121": [],
           "learned_fcg_121_random_start": [], "untrained_fcg": [], "poly_fcg": [], "poly_fcg_121": []}
    untrained = None
    for j in range(args.nheld):
        fat, lng = synth.make_links(w.dims, w.eps, seed=4900 + j)
        L = H.Lattice(w.dims)
        L.load_links(fat, lng)
        L.prepare_links(1, 18)
        L.prepare_links(2, 12)
        if untrained is None:
            untrained = H.PTC(L, (1, 4, 4, 1))
        # the polynomial start alone, on this field's own spectrum estimate
        # (set up outside the timed solves)
        poly = H.PTC(L, (1, 4, 4, 1))
        poly.init_polynomial(a=4.0, c=1.2)
        poly2 = H.PTC(L, (1, 2, 1))
        poly2.init_polynomial(a=4.0, c=1.2)
        for s in range(2):
            b = synth.gaussian_even(w.dims, 5400 + 10 * j + s)
            for name, fn in (
                    ("plain_f64", lambda: L.cg(w.mass, b, params=H.hisq_default_params(sloppy=0, flags=H.HISQ_USE_GRAPH))),
                    ("mixed_f32", lambda: L.cg(w.mass, b, params=H.hisq_default_params(sloppy=1, flags=H.HISQ_USE_GRAPH))),
                    ("mixed_f16_r12", lambda: L.cg(w.mass, b, params=H.hisq_default_params(sloppy=2, recon=12, flags=H.HISQ_USE_GRAPH))),
                    ("learned_fcg", lambda: net.cg_learned(L, w.mass, b, params=H.hisq_default_params(sloppy=1, flags=H.HISQ_USE_GRAPH))),
                    ("learned_fcg_121_random_start", lambda: net2.cg_learned(L, w.mass, b, params=H.hisq_default_params(sloppy=1, flags=H.HISQ_USE_GRAPH))),
                    ("learned_fcg_121", lambda: net3.cg_learned(L, w.mass, b, params=H.hisq_default_params(sloppy=1, flags=H.HISQ_USE_GRAPH))),
                    ("untrained_fcg", lambda: untrained.cg_learned(L, w.mass, b, params=H.hisq_default_params(sloppy=1, flags=H.HISQ_USE_GRAPH))),
                    ("poly_fcg", lambda: poly.cg_learned(L, w.mass, b, params=H.hisq_default_params(sloppy=1, flags=H.HISQ_USE_GRAPH))),
                    ("poly_fcg_121", lambda: poly2.cg_learned(L, w.mass, b, params=H.hisq_default_params(sloppy=1, flags=H.HISQ_USE_GRAPH)))):
                (_, info), dt = solve_timed(torch, None, fn)
                res[name].append((info["iters"], dt, info["true_residual"], info.get("fell_back", 0)))
            log(f"held-out field {j}, source {s}: " + ", ".join(f"{k} {v[-1][0]} it {v[-1][1]:.3f}s" for k, v in res.items()))
        poly.close()
        poly2.close()
        L.close()
    summ = {k: {"iters_mean": round(float(np.mean([r[0] for r in v])), 1),
                "time_s_mean": round(float(np.mean([r[1] for r in v])), 5),
                "worst_true_residual": float(f"{max(r[2] for r in v):.3e}"),
                "fell_back": int(sum(r[3] for r in v))} for k, v in res.items()}
    print(json.dumps({
        "workload": f"learned PTC preconditioner 16^4, eps 0.25, m 0.005: trained on {args.nfield} fields x {args.nsrc} sources, tested on {args.nheld} held-out fields x 2 sources",
        "training": {"seconds": t_train, "steps": args.train_steps,
                     "start": "small random weights (learned_fcg, learned_fcg_121_random_start); polynomial "
                              "K = 4 (1 + 1.2 D_f^2 / lambda) for learned_fcg_121 and the untrained poly_* nets",
                     "what": "harvest_s: synthetic fields generated on the host, loaded, and plain CG to 1e-12 per source; "
                             "train_s: the Adam steps on the GPU",
                     "loss": "energy norm of the error (HISQ_LOSS_ENERGY)",
                     "loss_first10": round(float(losses[:10].mean()), 4),
                     "loss_last50": round(float(losses[-50:].mean()), 4),
                     "net_121_random_start": {"seconds": t_train2, "fields": max(1, args.nfield // 4),
                                 "sources": max(1, args.nsrc // 2),
                                 "loss_first10": round(float(losses2[:10].mean()), 4),
                                 "loss_last50": round(float(losses2[-50:].mean()), 4)},
                     "net_121": {"seconds": t_train3, "fields": max(1, args.nfield // 4),
                                            "sources": max(1, args.nsrc // 2),
                                          "loss_first10": round(float(losses3[:10].mean()), 4),
                                          "loss_last50": round(float(losses3[-50:].mean()), 4)}},
        "solves": summ,
        "learned_iteration_gain_vs_plain": round(summ["plain_f64"]["iters_mean"] / summ["learned_fcg"]["iters_mean"], 3),
        "learned_time_gain_vs_plain": round(summ["plain_f64"]["time_s_mean"] / summ["learned_fcg"]["time_s_mean"], 3),
        "learned_121_time_gain_vs_plain": round(summ["plain_f64"]["time_s_mean"] / summ["learned_fcg_121"]["time_s_mean"], 3),
        "learned_121_time_gain_vs_mixed_f32": round(summ["mixed_f32"]["time_s_mean"] / summ["learned_fcg_121"]["time_s_mean"], 3)}),
        flush=True)


def run_copy(args):
    """Calibration for the HBM byte counters: the library's streaming kernels
    over 512 MiB (k_stream_read reads 512 MiB per launch, k_stream_copy reads
    and writes 512 MiB), one warm-up and three timed launches each."""
    import torch
    from paper_1712_00143_amd import hisq as H
    stream = torch.cuda.Stream()
    r, c = H.stream_bandwidth(0, H.ctypes.c_void_p(stream.cuda_stream), 512 << 20, 3)
    print(json.dumps({"workload": "streaming calibration", "bytes_read_per_launch": 512 << 20,
                      "copy_bytes_written_per_launch": 512 << 20, "launches_each": 4,
                      "read_GB/s": round(r, 1), "copy_GB/s": round(c, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--reps", type=int, default=50, help="Dslash launches per parity per step")
    ap.add_argument("--workload", default="c1", choices=["c0", "c1", "c2", "c3", "c4", "copy"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm", action="store_true", help="skip the 32^4 (beyond-cache) lattice")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--dslash-only", action="store_true", help="time only the Dslash")
    ap.add_argument("--nper", type=int, default=16, help="c3: solves per lattice size")
    ap.add_argument("--nfield", type=int, default=32, help="c4: training fields")
    ap.add_argument("--nsrc", type=int, default=4, help="c4: sources per training field")
    ap.add_argument("--nheld", type=int, default=8, help="c4: held-out fields")
    ap.add_argument("--train-steps", type=int, default=600)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU halo-exchange design is documented, not built)", file=sys.stderr)
        sys.exit(2)
    {"c0": run_c0, "c1": run_headline, "c2": run_c2, "c3": run_c3, "c4": run_c4,
     "copy": run_copy}[args.workload](args)


if __name__ == "__main__":
    main()
