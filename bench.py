"""Benchmark of the HISQ Dslash + CG hot path on one MI355X.

Default (the headline line).  One step is one pass of the hot path on inputs
already resident in HBM:
  * the half-lattice Dslash D_eo / D_oe on a 32^4 lattice (eps 0.2) whose
    links (1.2 GB per half-Dslash in FP64) are far beyond the 256 MB Infinity
    Cache: FP64 recon-18 (the paper's precision), FP32 recon-18, FP32 recon-12
    and FP16 recon-12 with every link streamed past the caches, and FP64 /
    FP32 recon-18 in the autotuner's choice (part of the links may be kept in
    the Infinity Cache: an effective rate);
  * the 16^3x32 workload (eps 0.2, m 0.02): the half-Dslash in every format,
    and CG to FP64 true residual 1e-10 from one source: plain FP64, mixed
    FP32 (recon-18), mixed FP16 storage (recon-12), and the flexible CG with
    the learned preconditioner (a 1-4-1 network trained from small random
    weights before the timed region, on pairs the solver harvests on four
    other fields of the same size and recipe; its untrained start is solved
    once for comparison);
  * the HISQ smearing, the Symanzik gauge force and the HISQ fermion force
    on 32^4 (outside the timed steps, each checked against the oracle on
    sampled links).
value = FP64 recon-18 streamed half-Dslash throughput on 32^4 in algorithmic
GB/s (16 links + one input + one output colour vector per output site) from
HIP events recorded on the stream the kernels run on.  Reported beside it:
the other formats, link load / pack times, each solve's error against the
oracle's solution and the oracle's recomputed true residual, the practical
HBM ceilings, and (outside the timed steps) one multi-shift solve on 24^3x48
(12 shifts x 4 sources) and one batch of 64 uneven solves, each with oracle
true residuals of a sample of its solutions; the FP64 CPU oracle is timed on
the host cores over a bounded sample.

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
    """Measured HBM bytes per launch of the headline kernel (FP64 recon-18,
    streamed links, 32^4) from the committed counter summary, if it was taken
    on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "dslash_f64r18_streamed_32x32x32x32_traffic.json")
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


def timed_dslash(torch, lat, prec, recon, h, stream, reps, flags=0):
    """Average duration (s) of one half-Dslash launch (both parities alternate),
    as (graph, eager).  The 2*reps launches are captured once in a HIP graph on
    the library's stream and replayed there between two events, so host launch
    gaps do not count; the same launches issued eagerly are timed too.  graph
    is None where capture fails.  flags: hisq_dslash flags (HISQ_STREAM_LINKS)."""
    x = _vec(torch, prec, h, 7)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    lat.dslash(0, prec, recon, x, y, flags=flags)      # tunes the block shape before any capture
    lat.dslash(1, prec, recon, y, x, flags=flags)
    torch.cuda.synchronize()

    def body():
        for _ in range(reps):
            lat.dslash(0, prec, recon, x, y, flags=flags)
            lat.dslash(1, prec, recon, y, x, flags=flags)

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


def random_start(chans, seed, scale=0.05):
    """Small random complex starting weights of a network (one array per layer)."""
    rng = np.random.default_rng(seed)
    return [scale * (rng.standard_normal((b, a, 9)) + 1j * rng.standard_normal((b, a, 9)))
            for a, b in zip(chans[:-1], chans[1:])]


def train_preconditioner(H, synth, dims, eps, mass, seed0, nfield, nsrc, steps, chans=(1, 4, 4, 1),
                         every=10, maxpairs=60, batch=8, lr=3e-3, init="poly", transport=(1, 18), act16=False):
    """Harvest (residual, error) pairs with the solver on nfield seeded fields
    and train the network on the GPU, starting from the polynomial weights
    (init "poly") or small random ones ("random", random_start(chans, seed0)).
    transport: the network's link format, used by training and inference
    alike; act16: FP16 activation storage at inference.  Returns (net,
    lattices, seconds, losses)."""
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
            net.set_transport(*transport)
            if act16:
                net.set_activations(2)
            if init == "poly":
                lam = net.init_polynomial(a=4.0, c=1.2)
                log(f"polynomial start: lambda_max(-D_f^2) ~ {lam:.4f}")
            else:
                net.set_weights(random_start(chans, seed0))
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

HEAD_DIMS = (32, 32, 32, 32)
FMT_NAME = {(0, 18): "f64_r18", (1, 18): "f32_r18", (1, 12): "f32_r12", (2, 12): "f16_r12"}


def timed_call(torch, fn):
    """(result, seconds) of fn() between two device synchronisations."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def shape_name(prec, recon, shape):
    W, remap, cpol = shape
    lt = {0: "double", 1: "float", 2: "__half"}[prec]
    st, ot = lt, lt
    cp = 0 if cpol <= 0 else 1 if cpol >= 16 else 2
    kern = "k_dslash_lo" if W & 256 else "k_dslash"
    return f"{kern}<{lt},{recon},{st},{ot},{W & 255},EPI_PLAIN,{cp}>"


def run_headline(args):
    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    import oracle

    stream = torch.cuda.Stream()
    sp = H.ctypes.c_void_p(stream.cuda_stream)
    formats = [(1, 18), (1, 12), (2, 12), (0, 18)]
    setup = {}

    # ---- the headline lattice, 32^4: 1.2 GB of FP64 links per half-Dslash,
    # far beyond the 256 MB Infinity Cache
    t0 = time.perf_counter()
    fh, lh = synth.make_links(HEAD_DIMS, 0.2, seed=1900)
    setup["32^4_link_generation_host_s"] = round(time.perf_counter() - t0, 2)
    log(f"32^4 links generated in {setup['32^4_link_generation_host_s']} s")
    latH = H.Lattice(HEAD_DIMS, stream=sp)
    _, dt = timed_call(torch, lambda: latH.load_links(fh, lh))
    setup["32^4_load_links_s"] = round(dt, 4)
    del fh, lh
    for p, r in formats[:3]:
        _, dt = timed_call(torch, lambda: latH.prepare_links(p, r))
        setup[f"32^4_prepare_{FMT_NAME[(p, r)]}_s"] = round(dt, 4)
    hH = synth.volume(HEAD_DIMS) // 2

    if args.head_only:
        run_head_only(args, torch, H, latH, hH, stream, setup)
        return
    # ---- the 16^3x32 workload (eps 0.2, m 0.02): Dslash formats and solvers
    w = synth.C1
    fat, lng = w.links()
    b = w.sources()[0]
    h = synth.volume(w.dims) // 2
    lat = H.Lattice(w.dims, stream=sp)
    _, dt = timed_call(torch, lambda: lat.load_links(fat, lng))
    setup["16^3x32_load_links_s"] = round(dt, 4)
    for p, r in formats[:3]:
        _, dt = timed_call(torch, lambda: lat.prepare_links(p, r))
        setup[f"16^3x32_prepare_{FMT_NAME[(p, r)]}_s"] = round(dt, 4)
    bd = torch.from_numpy(b.view(np.float64)).cuda()
    solves = {
        "plain_f64": H.hisq_default_params(tol=1e-10, sloppy=0, recon=18, flags=H.HISQ_USE_GRAPH),
        "mixed_f32_r18": H.hisq_default_params(tol=1e-10, sloppy=1, recon=18, delta=args.delta,
                                               flags=H.HISQ_USE_GRAPH),
        "mixed_f16_r12": H.hisq_default_params(tol=1e-10, sloppy=2, recon=12, flags=H.HISQ_USE_GRAPH),
    }
    x_oracle = None
    if not args.dslash_only:
        # the oracle's solution of the same system, solved beyond the target,
        # for the per-solve error (host FP64, outside the timed region)
        t0 = time.perf_counter()
        x_oracle, it_or, tr_or, ok_or = oracle.cg(w.dims, fat, lng, w.mass, b, tol=1e-12)
        setup["oracle_solution"] = {"seconds": round(time.perf_counter() - t0, 2), "iters": it_or,
                                    "true_residual": float(f"{tr_or:.3e}"), "converged": bool(ok_or)}
        log(f"oracle solution: {it_or} iterations in {setup['oracle_solution']['seconds']} s")
    net = None
    train_info = None
    train_lats = []
    if not args.no_learned and not args.dslash_only:
        # trained outside the timed region from small random weights, on pairs
        # the solver harvests on four other fields of the same size and recipe
        chans = (1, 4, 1)
        t0 = time.perf_counter()
        net = H.PTC(lat, chans)
        net.set_transport(2, 12)       # FP16 recon-12 transports, training and inference alike
        net.set_activations(2)         # FP16 activation storage at inference
        net.set_weights(random_start(chans, w.seed))
        for j in range(4):
            tf, tg = synth.make_links(w.dims, w.eps, seed=w.seed + 100 + j)
            TL = H.Lattice(w.dims)
            TL.load_links(tf, tg)
            TL.prepare_links(1, 18)
            train_lats.append(TL)
            for k in range(2):
                net.harvest(TL, w.mass, synth.gaussian_even(w.dims, w.seed + 700 + 10 * j + k), every=10,
                            maxpairs=60)
        npair = net.pair_count()
        steps = 600
        losses = net.train(steps, batch=8, lr=3e-3, seed=1)
        t_train = time.perf_counter() - t0
        # the same network at its random start, on the test system
        start = H.PTC(lat, chans)
        start.set_transport(2, 12)
        start.set_activations(2)
        start.set_weights(random_start(chans, w.seed))
        _, info0 = start.cg_learned(lat, w.mass, b, params=H.hisq_default_params(tol=1e-10, sloppy=1, recon=18,
                                                                                  delta=args.delta))
        start.close()
        train_info = {"network": "1-4-1 PTC trained from small random weights, energy-norm loss, FP16 recon-12 "
                                 "transports, FP16 inference activations; pairs from four other fields of the "
                                 "same size and recipe, two sources each",
                      "pairs": npair, "steps": steps, "seconds": round(t_train, 3),
                      "loss_first10": round(float(losses[:10].mean()), 4),
                      "loss_last50": round(float(losses[-50:].mean()), 4),
                      "untrained_start_iters": int(info0["iters"])}
        log(f"learned preconditioner: {npair} pairs, loss {train_info['loss_first10']} -> "
            f"{train_info['loss_last50']}, untrained start {info0['iters']} iterations")

    head_fmts = [((0, 18), H.HISQ_STREAM_LINKS), ((1, 18), H.HISQ_STREAM_LINKS),
                 ((1, 12), H.HISQ_STREAM_LINKS), ((2, 12), H.HISQ_STREAM_LINKS), ((0, 18), 0), ((1, 18), 0)]

    def step():
        res = {"head": {}, "dslash_s": {}, "cg": {}, "x": {}}
        for (p, r), fl in head_fmts:
            res["head"][(p, r, fl)] = timed_dslash(torch, latH, p, r, hH, stream, args.head_reps, fl)
        for p, r in formats:
            res["dslash_s"][(p, r)] = timed_dslash(torch, lat, p, r, h, stream, args.reps)
        if not args.dslash_only:
            for name, prm in solves.items():
                xd = torch.zeros_like(bd)
                (_, info), dt = solve_timed(torch, stream, lambda: lat.cg(w.mass, bd, x=xd, params=prm))
                info["wall_s"] = dt
                res["cg"][name] = info
                res["x"][name] = xd
            if net is not None:
                xd = torch.zeros_like(bd)
                prm = H.hisq_default_params(tol=1e-10, sloppy=1, recon=18, delta=args.delta, flags=H.HISQ_USE_GRAPH)
                (_, info), dt = solve_timed(torch, stream, lambda: net.cg_learned(lat, w.mass, bd, x=xd, params=prm))
                info["wall_s"] = dt
                res["cg"]["learned_fcg_f32"] = info
                res["x"]["learned_fcg_f32"] = xd
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

    def avg(group, key, which):
        ts = [r[group][key][which] for r in results]
        return None if any(t is None for t in ts) else float(np.mean(ts))

    def dtime(group, key):
        """Graph-replay time where capture worked, else the eager time."""
        tg = avg(group, key, 0)
        return (tg, "graph") if tg is not None else (avg(group, key, 1), "eager")

    # 32^4 lines
    head = {}
    for (p, r), fl in head_fmts:
        t, how = dtime("head", (p, r, fl))
        gbs = hH * site_bytes(p, r) / t / 1e9
        shape = latH.dslash_shape(p, r, fl)
        head[FMT_NAME[(p, r)] + ("_streamed" if fl else "_tuned")] = {
            "us": round(t * 1e6, 3), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
            "GFLOP/s": round(1146.0 * hH / t / 1e9, 1), "timing": how, "kernel": shape_name(p, r, shape),
            "link_blocks_cached": shape[2],
            "links": "all streamed past the caches (an HBM rate)" if fl else
                     ("tuned: part of the links kept in the Infinity Cache (an effective rate, not an HBM rate)"
                      if shape[2] else "tuned: all streamed")}
    t64, how64 = dtime("head", (0, 18, H.HISQ_STREAM_LINKS))
    achieved = hH * site_bytes(0, 18) / t64 / 1e9
    shape64 = latH.dslash_shape(0, 18, H.HISQ_STREAM_LINKS)

    dsl = {}
    for p, r in formats:
        t, how = dtime("dslash_s", (p, r))
        gbs = h * site_bytes(p, r) / t / 1e9
        shape = lat.dslash_shape(p, r, 0)
        dsl[FMT_NAME[(p, r)]] = {
            "us": round(t * 1e6, 3), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
            "GFLOP/s": round(1146.0 * h / t / 1e9, 1), "timing": how, "kernel": shape_name(p, r, shape),
            "link_blocks_cached": shape[2],
            "us_eager_launches": round(avg("dslash_s", (p, r), 1) * 1e6, 3)}

    cg = {}
    if not args.dslash_only:
        last = results[-1]
        for name in results[0]["cg"]:
            infos = [r["cg"][name] for r in results]
            xh = last["x"][name].cpu().numpy().view(np.complex128).reshape(-1, 3)
            err = float(np.linalg.norm(xh - x_oracle) / np.linalg.norm(x_oracle))
            tr_or = oracle.true_residual(w.dims, fat, lng, w.mass, b, xh)
            cg[name] = {"time_s": round(float(np.median([i["wall_s"] for i in infos])), 5),
                        "iters": infos[-1]["iters"], "reliable_updates": infos[-1]["reliable_updates"],
                        "true_residual_fp64": float(f"{infos[-1]['true_residual']:.3e}"),
                        "oracle_true_residual": float(f"{tr_or:.3e}"),
                        "error_vs_oracle_solution": float(f"{err:.3e}"),
                        "converged": bool(infos[-1]["converged"])}
            if name == "mixed_f32_r18" or name.startswith("learned"):
                cg[name]["reliable_update_delta"] = args.delta
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
                 "what": "hisq_dslash on host FP64 vectors, 16^3x32 (copy in, convert, FP32 Dslash, convert, "
                         "copy out, synchronised), per call"}
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "HISQ even-odd half-Dslash D_eo/D_oe in FP64 recon-18 (the paper's precision) with "
                               "every link streamed past the caches, 32^4 (eps 0.2); in the same step the "
                               "16^3x32 workload (eps 0.2, m 0.02): Dslash in every format and CG to FP64 true "
                               "residual 1e-10 plain / mixed / learned",
                   "lattice": list(HEAD_DIMS), "solver_lattice": list(w.dims), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic_entry(),
                     "kernel": shape_name(0, 18, shape64),
                     "bytes_per_launch": hH * site_bytes(0, 18),
                     "bytes_per_site": site_bytes(0, 18), "sites_per_launch": hH,
                     "launch_us": round(t64 * 1e6, 3), "timing": f"HIP events around a {how64} of "
                     f"{2 * args.head_reps} launches (parities alternating) on the library stream",
                     "read_ceiling": {"GB/s": round(read_gbs, 1), "frac_of_peak": round(read_gbs / PEAK_HBM_GBS, 4),
                                      "what": "library streaming read of 1 GiB (non-temporal 16-byte loads)",
                                      "dslash_frac_of_read_ceiling": round(achieved / read_gbs, 4)},
                     "copy_ceiling": {"GB/s": round(copy_gbs, 1), "frac_of_peak": round(copy_gbs / PEAK_HBM_GBS, 4),
                                      "what": "library copy of 1 GiB, read + written bytes"},
                     "cache": "links streamed with non-temporal loads; both parities' FP64 links take 2.4 GB "
                              "against a 256 MB Infinity Cache, so the rate is an HBM rate"},
        "dslash_32^4": head,
        "dslash_16^3x32": dsl,
        "dslash_host_buffers": host_path,
        "cg_time_to_1e-10_16^3x32": cg,
        "setup": setup,
    }
    if "plain_f64" in cg:
        out["cg_speedup_vs_plain_f64"] = {k: round(cg["plain_f64"]["time_s"] / v["time_s"], 3)
                                          for k, v in cg.items()}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w.dims, fat, lng)
    if net is not None:
        net.close()
    for TL in train_lats:
        TL.close()
    lat.close()
    latH.close()
    if not args.dslash_only and not args.no_c2:
        out["c2_multishift_24^3x48"] = c2_summary(args, oracle_sample=8)
    if not args.dslash_only and not args.no_c3:
        out["c3_batched_64_solves"] = c3_summary(args, oracle_sample=8)
    if not args.dslash_only and not args.no_smear:
        out["smear_32^4"] = smear_summary(args)
        out["gauge_force_32^4"] = gforce_summary(args)
        out["fermion_force_32^4"] = fforce_summary(args)
    print(json.dumps(out), flush=True)


def smear_summary(args):
    """HISQ link smearing at 32^4: thin links are a 16^4 random SU(3) field
    (eps 0.4, plaquette about 0.65) repeated twice along each axis, so that
    the oracle's smearing of the 16^4 field, repeated the same way, is the
    exact answer for every link; a sample of links is compared."""
    import torch
    import oracle
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    small, dims = (16, 16, 16, 16), (32, 32, 32, 32)
    u16 = synth.thin_links(small, 0.4, 7000)
    t0 = time.perf_counter()
    fat_ref, lng_ref = oracle.hisq_smear(small, u16)
    t_oracle = time.perf_counter() - t0
    thin = torch.from_numpy(synth.tile_field(u16, small, (2, 2, 2, 2)).view(np.float64)).cuda()
    lat = H.Lattice(dims)
    fat = torch.empty_like(thin)
    lng = torch.empty_like(thin)
    lat.smear_links(thin)                      # workspace allocation
    times = []
    for _ in range(max(3, args.steps)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fat, lng = lat.smear_links(thin)       # synchronous
        times.append(time.perf_counter() - t1)
    t = float(np.median(times))
    V = synth.volume(dims)
    rng = np.random.default_rng(7001)
    idx = rng.choice(V, 4096, replace=False)
    c = synth.coords(dims)[idx] % 16
    j = c[:, 0] + 16 * (c[:, 1] + 16 * (c[:, 2] + 16 * c[:, 3]))
    sel = torch.from_numpy(idx).cuda()
    f = fat.view(V, 4, 3, 6)[sel].cpu().numpy().view(np.complex128).reshape(-1, 4, 3, 3)
    l = lng.view(V, 4, 3, 6)[sel].cpu().numpy().view(np.complex128).reshape(-1, 4, 3, 3)
    err = max(float(np.abs(f - fat_ref[j]).max() / np.abs(fat_ref).max()),
              float(np.abs(l - lng_ref[j]).max() / np.abs(lng_ref).max()))
    lat.close()
    return {"ms": round(t * 1e3, 3), "links_per_s": round(4 * V / t, 1),
            "what": "hisq_smear_links on device arrays, 32^4: fat7 level 1, U(3) projection, fat7 level 2 "
                    "with Lepage, Naik, phases; synchronous call, median of the timed calls",
            "sample_max_rel_error_vs_oracle": float(f"{err:.3e}"), "sample_links": 4 * len(idx),
            "oracle_s_16^4": round(t_oracle, 2)}


def run_smear(args):
    print(json.dumps({"smear_32^4": smear_summary(args)}), flush=True)


GF_FLOP_PER_LINK = 145 * 198 + 60   # 3x3 complex products per link (see gforce.hip) and the projection


def one_loop_coefs(u0):
    """Tadpole-improved one-loop Luescher-Weisz weights (plaquette,
    rectangle, parallelogram) for the mean link u0."""
    a_s = -4.0 * math.log(u0) / 3.0684
    return (1.0, -(1.0 + 0.4805 * a_s) / (20.0 * u0 * u0), -0.03325 * a_s / (u0 * u0))


def gforce_summary(args):
    """Symanzik gauge force and action at 32^4 on a 16^4 random field
    (eps 0.5) repeated twice per axis; a sample of force links and the
    action (16 times the 16^4 value) are compared with the oracle."""
    import torch
    import oracle
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    small, dims = (16, 16, 16, 16), (32, 32, 32, 32)
    u16 = synth.thin_links(small, 0.5, 7100)
    # tadpole factor u0 = (mean plaquette)^(1/4), the plaquette from the
    # plaquette-only action: S = sum over the 6 V plaquettes of 1 - Re Tr / 3
    plaq = 1.0 - oracle.gauge_action(small, u16, 1.0, (1.0, 0.0, 0.0)) / (6 * synth.volume(small))
    beta, coefs = 6.0, one_loop_coefs(plaq ** 0.25)
    t0 = time.perf_counter()
    f_ref = oracle.gauge_force(small, u16, beta, coefs)
    t_oracle = time.perf_counter() - t0
    s_ref = 16 * oracle.gauge_action(small, u16, beta, coefs)
    thin = torch.from_numpy(synth.tile_field(u16, small, (2, 2, 2, 2)).view(np.float64)).cuda()
    lat = H.Lattice(dims)
    F = lat.gauge_force(thin, beta, coefs)
    times = []
    for _ in range(max(3, args.steps)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        F = lat.gauge_force(thin, beta, coefs)
        times.append(time.perf_counter() - t1)
    t = float(np.median(times))
    S = lat.gauge_action(thin, beta, coefs)
    V = synth.volume(dims)
    idx = np.random.default_rng(7101).choice(V, 4096, replace=False)
    c = synth.coords(dims)[idx] % 16
    j = c[:, 0] + 16 * (c[:, 1] + 16 * (c[:, 2] + 16 * c[:, 3]))
    f = F.view(V, 4, 3, 6)[torch.from_numpy(idx).cuda()].cpu().numpy().view(np.complex128).reshape(-1, 4, 3, 3)
    err = float(np.abs(f - f_ref[j]).max() / np.abs(f_ref).max())
    lat.close()
    gflops = 4 * V * GF_FLOP_PER_LINK / t / 1e9
    return {"ms": round(t * 1e3, 3), "GFLOP/s": round(gflops, 1), "frac_fp64_peak": round(gflops / 78600.0, 4),
            "flop_per_link": GF_FLOP_PER_LINK, "beta": beta, "plaquette": round(plaq, 5),
            "coefs": [round(x, 6) for x in coefs],
            "what": "hisq_gauge_force on device arrays, 32^4 (plaquette, rectangle and parallelogram loops); "
                    "synchronous call incl. the layout conversions, median of the timed calls",
            "sample_max_rel_error_vs_oracle": float(f"{err:.3e}"), "sample_links": 4 * len(idx),
            "action_rel_error_vs_oracle": float(f"{abs(S - s_ref) / abs(s_ref):.3e}"),
            "oracle_s_16^4": round(t_oracle, 2)}


FF_TERMS = 12   # rational-approximation terms of the RHMD pseudofermion action


def fforce_summary(args):
    """HISQ fermion force at 32^4 for FF_TERMS solution vectors: an 8^4
    random field and 8^4 Gaussian vectors (standing in for the multi-shift
    solutions) repeated 4 times per axis, so that the oracle's force on the
    8^4 field, repeated, is the exact answer; a sample of links is compared.
    The call includes the smearing (the force smears and loads the links)."""
    import torch
    import oracle
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    small, dims, reps = (8, 8, 8, 8), (32, 32, 32, 32), (4, 4, 4, 4)
    u8 = synth.thin_links(small, 0.4, 7200)
    alphas = list(np.random.default_rng(7201).uniform(0.01, 1.0, FF_TERMS))
    xs8 = [synth.gaussian_even(small, 7300 + k) for k in range(FF_TERMS)]
    t0 = time.perf_counter()
    f_ref = oracle.hisq_fermion_force(small, u8, alphas, xs8)
    t_oracle = time.perf_counter() - t0
    ev8, ev = synth.even_sites(small), synth.even_sites(dims)
    xs = np.empty((FF_TERMS, len(ev), 3), dtype=np.complex128)
    for k, x8 in enumerate(xs8):
        full = np.zeros((synth.volume(small), 3), dtype=np.complex128)
        full[ev8] = x8
        xs[k] = synth.tile_field(full, small, reps)[ev]
    thin = torch.from_numpy(synth.tile_field(u8, small, reps).view(np.float64)).cuda()
    xt = torch.from_numpy(xs.view(np.float64)).cuda()
    del xs
    lat = H.Lattice(dims)
    F = lat.fermion_force(thin, alphas, xt)
    times = []
    for _ in range(max(3, args.steps)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        F = lat.fermion_force(thin, alphas, xt)
        times.append(time.perf_counter() - t1)
    t = float(np.median(times))
    V = synth.volume(dims)
    idx = np.random.default_rng(7202).choice(V, 4096, replace=False)
    c = synth.coords(dims)[idx] % 8
    j = c[:, 0] + 8 * (c[:, 1] + 8 * (c[:, 2] + 8 * c[:, 3]))
    f = F.view(V, 4, 3, 6)[torch.from_numpy(idx).cuda()].cpu().numpy().view(np.complex128).reshape(-1, 4, 3, 3)
    err = float(np.abs(f - f_ref[j]).max() / np.abs(f_ref).max())
    lat.close()
    return {"ms": round(t * 1e3, 3), "terms": FF_TERMS,
            "what": "hisq_fermion_force on device arrays, 32^4, 12 solution vectors: smearing and loading the links, "
                    "D_oe of each vector, outer products, Naik / fat7 level 2 / projection / fat7 level 1 adjoints, "
                    "projection onto su(3); synchronous call, median of the timed calls",
            "sample_max_rel_error_vs_oracle": float(f"{err:.3e}"), "sample_links": 4 * len(idx),
            "oracle_s_8^4": round(t_oracle, 2)}


def run_fforce(args):
    print(json.dumps({"fermion_force_32^4": fforce_summary(args)}), flush=True)


def run_gforce(args):
    print(json.dumps({"gauge_force_32^4": gforce_summary(args)}), flush=True)


def run_head_only(args, torch, H, latH, hH, stream, setup):
    """Only the 32^4 headline launches (FP64 and FP32 recon-18, streamed
    links), for profiling them alone; one JSON line."""
    res = {}
    for _ in range(args.warmup):
        for p, r in ((0, 18), (1, 18)):
            timed_dslash(torch, latH, p, r, hH, stream, args.head_reps, H.HISQ_STREAM_LINKS)
    t0 = time.perf_counter()
    for k in range(args.steps):
        for p, r in ((0, 18), (1, 18)):
            tg, te = timed_dslash(torch, latH, p, r, hH, stream, args.head_reps, H.HISQ_STREAM_LINKS)
            res.setdefault((p, r), []).append(tg if tg is not None else te)
        log(f"step {k + 1}/{args.steps}")
    t_total = time.perf_counter() - t0
    lines = {}
    for (p, r), ts in res.items():
        t = float(np.mean(ts))
        gbs = hH * site_bytes(p, r) / t / 1e9
        lines[FMT_NAME[(p, r)] + "_streamed"] = {
            "us": round(t * 1e6, 3), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
            "kernel": shape_name(p, r, latH.dslash_shape(p, r, H.HISQ_STREAM_LINKS)),
            "launches_per_step": 2 + 6 * args.head_reps}
    print(json.dumps({"workload": "32^4 half-Dslash, recon-18, streamed links (headline launches only)",
                      "steps": args.steps, "ms_per_step": round(1000 * t_total / args.steps, 2),
                      "dslash_32^4": lines, "setup": setup}), flush=True)
    latH.close()


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


def c2_summary(args, oracle_sample=0):
    """One multi-shift CG solve on the 24^3x48 workload (12 shifts in
    [1e-4, 1], 4 sources batched through the multi-RHS Dslash, m 0.01, FP32
    with FP64 recurrences and refinement, tol 1e-8) after one warm-up solve,
    plus the multi-RHS Dslash rates.  oracle_sample > 0: the oracle recomputes
    the FP64 true residual of that many solutions (both ends of the shift range
    for each source first)."""
    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    import oracle
    w = synth.C2
    t0 = time.perf_counter()
    fat, lng = w.links()
    gen_s = time.perf_counter() - t0
    b = w.sources()
    shifts = synth.shifts_log(12)
    stream = torch.cuda.Stream()
    lat = H.Lattice(w.dims, stream=H.ctypes.c_void_p(stream.cuda_stream))
    _, load_s = timed_call(torch, lambda: lat.load_links(fat, lng))
    _, prep_s = timed_call(torch, lambda: lat.prepare_links(1, 18))
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
    out = {"workload": "multi-shift CG 24^3x48, 12 shifts in [1e-4, 1], 4 sources, m 0.01, FP32 + FP64 "
                       "recurrences, tol 1e-8",
           "mrhs_dslash_f32_r18_nrhs4": {"us": round(t * 1e6, 2), "GB/s": round(mrhs_bytes / t / 1e9, 1),
                                         "frac_hbm": round(mrhs_bytes / t / 1e9 / PEAK_HBM_GBS, 4)},
           "mrhs_dslash_f32_r18_nrhs48": {"us": round(t48 * 1e6, 2), "groups": 12,
                                          "us_per_group": round(t48 * 1e6 / 12, 2),
                                          "what": "one launch over 12 groups of four right-hand sides"},
           "link_generation_host_s": round(gen_s, 2), "load_links_s": round(load_s, 4),
           "prepare_f32_r18_s": round(prep_s, 4)}
    if args.dslash_only:
        lat.close()
        return out
    prm = H.hisq_default_params(tol=1e-8, sloppy=1, flags=H.HISQ_USE_GRAPH)
    # sources and solutions resident in HBM (device pointers)
    bd = torch.from_numpy(np.ascontiguousarray(b).view(np.float64).ravel()).cuda()
    xd = torch.zeros(len(b) * len(shifts) * h * 6, dtype=torch.float64, device="cuda")
    lat.multishift_cg(w.mass, shifts, bd, x=xd, params=prm)          # warm-up: tuning, graph capture
    xd.zero_()
    (xs, infos), dt = solve_timed(torch, stream, lambda: lat.multishift_cg(w.mass, shifts, bd, x=xd, params=prm))
    worst = max(i["true_residual"] for i in infos)
    out.update({
        "time_s": round(dt, 4), "krylov_phase_s": round(infos[0]["t_done_s"], 4),
        "iters_per_shift_rhs0": [i["iters"] for i in infos[:12]],
        "refine_iters_per_shift_rhs0": [i["refine_iters"] for i in infos[:12]],
        "worst_true_residual_fp64": float(f"{worst:.3e}"),
        "all_converged": all(i["converged"] for i in infos)})
    if oracle_sample > 0:
        xh = xd.cpu().numpy().view(np.complex128).reshape(len(b), len(shifts), h, 3)
        picks = [(j, k) for j in range(len(b)) for k in (0, len(shifts) - 1)]
        picks += [(j, k) for j in range(len(b)) for k in range(1, len(shifts) - 1)]
        t0 = time.perf_counter()
        checked = []
        for j, k in picks[:oracle_sample]:
            tr = oracle.true_residual(w.dims, fat, lng, w.mass, b[j], xh[j, k], shifts[k])
            checked.append({"rhs": j, "shift": float(f"{shifts[k]:.4e}"), "oracle_true_residual": float(f"{tr:.3e}")})
        out["oracle_check"] = {"solutions": checked, "all_within_tol": all(c["oracle_true_residual"] <= 1e-8
                                                                          for c in checked),
                               "seconds": round(time.perf_counter() - t0, 2)}
    lat.close()
    return out


def run_c2(args):
    print(json.dumps(c2_summary(args, oracle_sample=args.oracle_sample)), flush=True)


def c3_summary(args, oracle_sample=0):
    """One batch of 64 uneven solves (16 each of 8^4, 12^4, 16^4, 16^3x32,
    eps ~ U[0.1, 0.4], m ~ logU[0.005, 0.2]; FP32 with FP64 reliable updates,
    tol 1e-10) in one set of launches, after a warm-up batch, and the same
    solves one after another.  oracle_sample > 0: the oracle recomputes the
    FP64 true residual of that many solutions, spread over the four sizes."""
    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    import oracle
    ws = synth.batch_workload(nper=args.nper)
    lats, bs, ms, links = [], [], [], []
    t0 = time.perf_counter()
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
        links.append((wk.dims, fat, lng) if oracle_sample > 0 else None)
    setup_s = time.perf_counter() - t0
    prm = H.hisq_default_params(tol=1e-10, sloppy=1, delta=args.delta, flags=H.HISQ_USE_GRAPH)
    H.hisq_batch_cg(lats, ms, bs, params=prm)          # warm-up: tuning, graph capture
    (xs, infos), dt = solve_timed(torch, None, lambda: H.hisq_batch_cg(lats, ms, bs, params=prm))
    tdone = np.array([i["t_done_s"] for i in infos])
    total_bytes = sum(i["dslash_bytes"] for i in infos)
    # the same solves one after another, for comparison
    t_seq = 0.0
    for L, m, bb in zip(lats, ms, bs):
        (_, _), d1 = solve_timed(torch, None, lambda: L.cg(m, bb, params=prm))
        t_seq += d1
    out = {
        "workload": f"batched CG: {len(ws)} solves, {args.nper} each of 8^4, 12^4, 16^4, 16^3x32; eps~U[0.1,0.4], "
                    f"m~logU[0.005,0.2]; FP32 + FP64 reliable, tol 1e-10",
        "time_s": round(dt, 4), "aggregate_dslash_GB/s": round(total_bytes / dt / 1e9, 1),
        "time_to_solution_p50_s": round(float(np.percentile(tdone, 50)), 5),
        "time_to_solution_p99_s": round(float(np.percentile(tdone, 99)), 5),
        "iters_min_max": [min(i["iters"] for i in infos), max(i["iters"] for i in infos)],
        "all_converged": all(i["converged"] for i in infos),
        "worst_true_residual_fp64": float(f"{max(i['true_residual'] for i in infos):.3e}"),
        "sequential_time_s": round(t_seq, 4), "batch_speedup": round(t_seq / dt, 3),
        "setup_s": round(setup_s, 2), "reliable_update_delta": args.delta,
        "reliable_updates_mean": round(float(np.mean([i["reliable_updates"] for i in infos])), 2)}
    if oracle_sample > 0:
        n = len(ws)
        # interleave the four sizes: problems are ordered size by size
        order = [q for k in range(args.nper) for q in range(k, n, args.nper)]
        t0 = time.perf_counter()
        checked = []
        for q in order[:oracle_sample]:
            dims, fat, lng = links[q]
            tr = oracle.true_residual(dims, fat, lng, ms[q], bs[q], xs[q])
            checked.append({"problem": q, "lattice": list(dims), "oracle_true_residual": float(f"{tr:.3e}")})
        out["oracle_check"] = {"solutions": checked, "all_within_tol": all(c["oracle_true_residual"] <= 1e-10
                                                                          for c in checked),
                               "seconds": round(time.perf_counter() - t0, 2)}
    for L in lats:
        L.close()
    return out


def run_c3(args):
    print(json.dumps(c3_summary(args, oracle_sample=args.oracle_sample)), flush=True)


def run_c4(args):
    """Learned preconditioner on 16^4 (eps 0.25, m 0.005): networks trained on
    the GPU from pairs the solver harvests on `nfield` training fields, tested
    against plain and mixed CG on `nheld` held-out fields x 2 sources.  Every
    network runs its transports on FP16 recon-12 fat links (training and
    inference) and stores its inference activations in FP16; each trained
    network is also run from its own untrained starting weights.  Every
    solution's FP64 true residual is recomputed by the oracle."""
    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth
    import oracle
    w = synth.C4
    fmt = dict(transport=(2, 12), act16=True)
    chans = (1, 4, 4, 1)
    # the specified 1 -> 4 -> 4 -> 1 network, trained from small random weights
    net, tl, t_train, losses = train_preconditioner(H, synth, w.dims, w.eps, w.mass, 4000, args.nfield,
                                                    args.nsrc, args.train_steps, chans=chans, init="random", **fmt)
    # the two-layer 1 -> 4 -> 1 network (the specified one without its middle
    # layer: four layer applications per iteration instead of six), trained
    # from small random weights on the same fields
    chans4 = (1, 4, 1)
    net4, tl4, t_train4, losses4 = train_preconditioner(H, synth, w.dims, w.eps, w.mass, 4000, args.nfield,
                                                        args.nsrc, args.train_steps, chans=chans4, init="random",
                                                        **fmt)
    # the two-layer 1 -> 2 -> 1 network (the smallest that holds the polynomial
    # preconditioner), on a quarter of the fields, from random weights and
    # from the polynomial start
    nq, sq = max(1, args.nfield // 4), max(1, args.nsrc // 2)
    net2, tl2, t_train2, losses2 = train_preconditioner(H, synth, w.dims, w.eps, w.mass, 4000, nq, sq,
                                                        args.train_steps, chans=(1, 2, 1), init="random", **fmt)
    net3, tl3, t_train3, losses3 = train_preconditioner(H, synth, w.dims, w.eps, w.mass, 4000, nq, sq,
                                                        args.train_steps, chans=(1, 2, 1), init="poly", **fmt)
    names = ["plain_f64", "mixed_f32", "mixed_f16_r12", "learned_fcg", "learned_fcg_untrained_start",
             "learned_fcg_141_random", "learned_fcg_141_random_untrained_start",
             "learned_fcg_121_random", "learned_fcg_121_random_untrained_start", "learned_fcg_121_poly",
             "poly_fcg_121_untrained", "identity_fcg"]
    res = {k: [] for k in names}
    for j in range(args.nheld):
        fat, lng = synth.make_links(w.dims, w.eps, seed=4900 + j)
        L = H.Lattice(w.dims)
        L.load_links(fat, lng)
        L.prepare_links(1, 18)
        L.prepare_links(2, 12)
        nets = {}
        for name, ch, wts in (("learned_fcg_untrained_start", chans, random_start(chans, 4000)),
                              ("learned_fcg_141_random_untrained_start", chans4, random_start(chans4, 4000)),
                              ("learned_fcg_121_random_untrained_start", (1, 2, 1), random_start((1, 2, 1), 4000)),
                              ("identity_fcg", chans, None)):
            n = H.PTC(L, ch)
            n.set_transport(2, 12)
            n.set_activations(2)
            if wts is not None:
                n.set_weights(wts)
            nets[name] = n
        # the polynomial start alone, on this field's own spectrum estimate
        # (set up outside the timed solves)
        poly = H.PTC(L, (1, 2, 1))
        poly.set_transport(2, 12)
        poly.set_activations(2)
        poly.init_polynomial(a=4.0, c=1.2)
        nets["poly_fcg_121_untrained"] = poly
        nets["learned_fcg"] = net
        nets["learned_fcg_141_random"] = net4
        nets["learned_fcg_121_random"] = net2
        nets["learned_fcg_121_poly"] = net3
        for s in range(2):
            b = synth.gaussian_even(w.dims, 5400 + 10 * j + s)
            bd = torch.from_numpy(b.view(np.float64)).cuda()
            for name in names:
                if name == "plain_f64":
                    fn = lambda xd: L.cg(w.mass, bd, x=xd, params=H.hisq_default_params(sloppy=0, flags=H.HISQ_USE_GRAPH))
                elif name == "mixed_f32":
                    fn = lambda xd: L.cg(w.mass, bd, x=xd, params=H.hisq_default_params(sloppy=1, delta=args.delta,
                                                                                        flags=H.HISQ_USE_GRAPH))
                elif name == "mixed_f16_r12":
                    fn = lambda xd: L.cg(w.mass, bd, x=xd,
                                         params=H.hisq_default_params(sloppy=2, recon=12, flags=H.HISQ_USE_GRAPH))
                else:
                    nn = nets[name]
                    fn = lambda xd: nn.cg_learned(L, w.mass, bd, x=xd,
                                                  params=H.hisq_default_params(sloppy=1, delta=args.delta,
                                                                               flags=H.HISQ_USE_GRAPH))
                xd = torch.zeros_like(bd)
                fn(xd)                                 # warm-up: tuning, graph capture
                xd = torch.zeros_like(bd)
                (_, info), dt = solve_timed(torch, None, lambda: fn(xd))
                xh = xd.cpu().numpy().view(np.complex128).reshape(-1, 3)
                tr = oracle.true_residual(w.dims, fat, lng, w.mass, b, xh)
                res[name].append((info["iters"], dt, tr, info.get("fell_back", 0)))
            log(f"held-out field {j}, source {s}: " + ", ".join(f"{k} {v[-1][0]} it {v[-1][1]:.4f}s" for k, v in res.items()))
        for name in ("learned_fcg_untrained_start", "learned_fcg_141_random_untrained_start",
                     "learned_fcg_121_random_untrained_start", "identity_fcg", "poly_fcg_121_untrained"):
            nets[name].close()
        L.close()
    summ = {k: {"iters_mean": round(float(np.mean([r[0] for r in v])), 1),
                "time_s_mean": round(float(np.mean([r[1] for r in v])), 5),
                "worst_oracle_true_residual": float(f"{max(r[2] for r in v):.3e}"),
                "fell_back": int(sum(r[3] for r in v))} for k, v in res.items()}
    plain = summ["plain_f64"]["time_s_mean"]

    def loss_info(ls, t):
        return {"seconds": t, "loss_first10": round(float(ls[:10].mean()), 4),
                "loss_last50": round(float(ls[-50:].mean()), 4)}
    print(json.dumps({
        "workload": f"learned PTC preconditioner 16^4, eps 0.25, m 0.005: trained on {args.nfield} fields x "
                    f"{args.nsrc} sources, tested on {args.nheld} held-out fields x 2 sources; FP16 recon-12 "
                    f"transports (training and inference), FP16 inference activations, FP64 true residual 1e-10",
        "reliable_update_delta": {"mixed_f32_and_learned": args.delta, "mixed_f16_r12": 0.1},
        "training": {"steps": args.train_steps, "loss": "energy norm of the error (HISQ_LOSS_ENERGY)",
                     "learned_fcg (1-4-4-1, random start)": loss_info(losses, t_train),
                     "learned_fcg_141_random (1-4-1, random start)": loss_info(losses4, t_train4),
                     "learned_fcg_121_random (1-2-1, random start)": loss_info(losses2, t_train2),
                     "learned_fcg_121_poly (1-2-1, polynomial start)": loss_info(losses3, t_train3),
                     "what": "harvest_s: synthetic fields generated on the host, loaded, and plain CG to 1e-12 per "
                             "source; train_s: the Adam steps on the GPU"},
        "solves": summ,
        "time_gain_vs_plain_f64": {k: round(plain / v["time_s_mean"], 3) for k, v in summ.items()},
        "iteration_gain_of_training": {
            "1-4-4-1": round(summ["learned_fcg_untrained_start"]["iters_mean"] / summ["learned_fcg"]["iters_mean"], 3),
            "1-4-1 random start": round(summ["learned_fcg_141_random_untrained_start"]["iters_mean"]
                                        / summ["learned_fcg_141_random"]["iters_mean"], 3),
            "1-2-1 random start": round(summ["learned_fcg_121_random_untrained_start"]["iters_mean"]
                                        / summ["learned_fcg_121_random"]["iters_mean"], 3),
            "1-2-1 polynomial start": round(summ["poly_fcg_121_untrained"]["iters_mean"]
                                            / summ["learned_fcg_121_poly"]["iters_mean"], 3)}}), flush=True)
    for n in (net, net4, net2, net3):
        n.close()
    for L in tl + tl4 + tl2 + tl3:
        L.close()


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
    ap.add_argument("--reps", type=int, default=50, help="16^3x32 Dslash launches per parity per step")
    ap.add_argument("--head-reps", type=int, default=20, help="32^4 Dslash launches per parity per step")
    ap.add_argument("--head-only", action="store_true", help="only the 32^4 headline launches (for profiling)")
    ap.add_argument("--no-c2", action="store_true", help="headline: skip the multi-shift summary")
    ap.add_argument("--no-c3", action="store_true", help="headline: skip the batched-solve summary")
    ap.add_argument("--no-smear", action="store_true", help="headline: skip the smearing, gauge- and fermion-force summaries")
    ap.add_argument("--oracle-sample", type=int, default=8, help="c2/c3: solutions checked by the oracle")
    ap.add_argument("--workload", default="c1", choices=["c0", "c1", "c2", "c3", "c4", "copy", "smear", "gforce", "fforce"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--delta", type=float, default=0.01,
                    help="reliable-update threshold of the FP32-sloppy solvers (mixed FP32 CG, learned FCG)")
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
     "copy": run_copy, "smear": run_smear, "gforce": run_gforce, "fforce": run_fforce}[args.workload](args)


if __name__ == "__main__":
    main()
