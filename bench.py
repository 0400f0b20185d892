"""Benchmark of the HISQ Dslash + CG hot path on one MI355X.

One step = one pass of the hot path over the 16^3x32 workload (eps 0.2,
m 0.02, links already resident in HBM):
  * half-lattice Dslash D_eo and D_oe in FP32 recon-18, FP32 recon-12,
    FP16 recon-12 and FP64 recon-18 (device vectors);
  * CG to FP64 true residual 1e-10: plain FP64, mixed FP32 (recon-18) and
    mixed FP16 storage (recon-12), all from the same source.
value = FP32 recon-18 Dslash throughput in algorithmic GB/s (16 links +
1 input + 1 output colour vector per output site), from HIP events recorded
on the stream the kernels run on.  The CG times-to-solution, the other
storage formats and a 32^4 lattice whose links do not fit the 256 MB
Infinity Cache are reported beside it, with the FP64 CPU oracle timed on the
host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


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
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "dslash_f32r18_16x16x16x32_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def timed_dslash(H, torch, lat, prec, recon, h, stream, reps):
    """Average duration (s) of one half-Dslash launch, both parities,
    measured with events on the library's stream."""
    dt = {0: torch.float64, 1: torch.float32, 2: torch.float16}[prec]
    nreal = {0: 6 * h, 1: 6 * h, 2: 8 * h}[prec]    # FP16: 6h halves + h float scales (= 2h halves)
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.randn(nreal, device="cuda", dtype=torch.float32, generator=g).to(dt)
    if prec == 2:
        x[6 * h:] = 1.0
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    lat.dslash(0, prec, recon, x, y)
    lat.dslash(1, prec, recon, y, x)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(reps):
            lat.dslash(0, prec, recon, x, y)
            lat.dslash(1, prec, recon, y, x)
        e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1000.0 / (2 * reps)


def cpu_baseline(w, fat, lng, budget_s=12.0):
    """The FP64 oracle Dslash on the same lattice, as many half-Dslash
    applications as fit in budget_s seconds of host time."""
    import oracle
    from paper_1712_00143_amd import synth
    psi = synth.gaussian_even(w.dims, 99)
    h = psi.shape[0]
    oracle.dslash_half(w.dims, fat, lng, 0, psi)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        psi = oracle.dslash_half(w.dims, fat, lng, n % 2, psi)
        psi /= np.linalg.norm(psi)
        n += 1
    dt = time.perf_counter() - t0
    gbs = n * h * site_bytes(0, 18) / dt / 1e9
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} FP64 half-Dslash applications on {w.dims} in {dt:.1f} s "
                      f"(plain C oracle, OpenMP over sites)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--reps", type=int, default=50, help="Dslash launches per parity per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm", action="store_true", help="skip the 32^4 (beyond-cache) lattice")
    ap.add_argument("--dslash-only", action="store_true", help="time only the Dslash (profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU halo-exchange design is documented, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1712_00143_amd import hisq as H
    from paper_1712_00143_amd import synth

    w = synth.C1
    fat, lng = w.links()
    b = w.sources()[0]
    h = synth.volume(w.dims) // 2
    stream = torch.cuda.Stream()
    lat = H.Lattice(w.dims, stream=H.ctypes.c_void_p(stream.cuda_stream))
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

    def step():
        res = {"dslash_s": {}, "cg": {}}
        for p, r in formats:
            res["dslash_s"][(p, r)] = timed_dslash(H, torch, lat, p, r, h, stream, args.reps)
        if not args.dslash_only:
            for name, prm in solves.items():
                xd = torch.zeros_like(bd)
                with torch.cuda.stream(stream):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, info = lat.cg(w.mass, bd, x=xd, params=prm)
                    t1 = time.perf_counter()
                info["wall_s"] = t1 - t0
                res["cg"][name] = (info, xd)
        return res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0

    def avg(key):
        return float(np.mean([r["dslash_s"][key] for r in results]))

    dsl = {}
    for p, r in formats:
        t = avg((p, r))
        gbs = h * site_bytes(p, r) / t / 1e9
        dsl[f"{['f64', 'f32', 'f16'][p]}_r{r}"] = {
            "us": round(t * 1e6, 3), "GB/s": round(gbs, 1), "frac_hbm": round(gbs / PEAK_HBM_GBS, 4),
            "GFLOP/s": round(1146.0 * h / t / 1e9, 1)}
    t32 = avg((1, 18))
    achieved = h * site_bytes(1, 18) / t32 / 1e9

    cg = {}
    if not args.dslash_only:
        for name in solves:
            infos = [r["cg"][name][0] for r in results]
            cg[name] = {"time_s": round(float(np.median([i["wall_s"] for i in infos])), 4),
                        "iters": infos[-1]["iters"], "reliable_updates": infos[-1]["reliable_updates"],
                        "true_residual_fp64": float(f"{infos[-1]['true_residual']:.3e}"),
                        "converged": bool(infos[-1]["converged"])}

    hbm = None
    if not args.no_hbm:
        dims = (32, 32, 32, 32)
        f2, l2 = synth.make_links(dims, 0.2, seed=1900)
        lat2 = H.Lattice(dims, stream=H.ctypes.c_void_p(stream.cuda_stream))
        lat2.load_links(f2, l2)
        del f2, l2
        hbm = {}
        h2 = synth.volume(dims) // 2
        for p, r in formats:
            lat2.prepare_links(p, r)
            t = timed_dslash(H, torch, lat2, p, r, h2, stream, 20)
            gbs = h2 * site_bytes(p, r) / t / 1e9
            hbm[f"{['f64', 'f32', 'f16'][p]}_r{r}"] = {"us": round(t * 1e6, 2), "GB/s": round(gbs, 1),
                                                       "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)}
        lat2.close()

    out = {
        "metric": "Dslash GB/s (% HBM peak); CG time-to-1e-10: plain vs mixed/learned",
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
                     "kernel": "k_dslash<float,18,float,float,W,EPI_PLAIN>",
                     "bytes_per_launch": h * site_bytes(1, 18)},
        "dslash": dsl,
        "dslash_32^4_beyond_infinity_cache": hbm,
        "cg_time_to_1e-10": cg,
    }
    if cg:
        out["cg_speedup_vs_plain_f64"] = {k: round(cg["plain_f64"]["time_s"] / v["time_s"], 2)
                                          for k, v in cg.items()}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, fat, lng)
    lat.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
