"""Benchmark of the two-component Shan-Chen step on one MI355X.

Workload: D3Q19 two-component Shan-Chen BGK, 256^3 periodic, spinodal
decomposition from rho_A = rho_B = 0.5 with seeded U(-0.01, 0.01) noise
(seed 3), G = 1.6, tau_A = tau_B = 1.0.  A step is one full lattice time step
(moments, force gather, force shift, collision, streaming) of both species.

Prints one JSON line: MLUPS of the FP64 step (value), its HBM roofline
fraction from algorithmic bytes (2 species x 19 populations x read+write x
8 B = 608 B per site update) over the step kernel's average duration timed
with HIP events on the lattice's stream, the FP32-shifted step's figures, a
streaming-copy ceiling, and the FP64 CPU oracle timed on the host on the
same lattice (all cores and one thread) and on the full 64^2 D2Q9 drop run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E
Q19 = 19
L = 256
G, TAU = 1.6, 1.0
WORKLOAD = ("D3Q19 two-component Shan-Chen BGK 256^3 periodic, spinodal from rho_A=rho_B=0.5 "
            "+ U(-0.01,0.01) noise (seed 3), G=1.6, tau=1.0")


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
# the step kernels and the runtime that lays out their buffers (array stride):
# recorded traffic is valid only for these exact sources
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1112_5547_amd", "csrc", f)
                  for f in ("sc_device.h", "sc_steps.h", "sc_kernels.hip", "sc_runtime.hip")]
COPY_BYTES = 2 << 30  # the copy-ceiling leg moves this many bytes each way per launch


def progress(msg: str):
    """One line on stderr as each leg of the run ends (stdout keeps the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def record_traffic(fetch_csv: str, write_csv: str):
    """Turns two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, then
    WRITE_SIZE, KiB per dispatch) into per-launch HBM bytes of each step
    kernel, scaled by what the same counters read for the copy kernel of
    known size, and stores them with a hash of the kernel sources."""
    import csv
    import re

    def per_kernel(path):
        acc = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                k = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").strip()
                acc.setdefault(k, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    F, W = per_kernel(fetch_csv), per_kernel(write_csv)
    copy = [k for k in F if k.endswith("k_copy")][0]
    fscale = COPY_BYTES / 1024.0 / F[copy]
    wscale = COPY_BYTES / 1024.0 / W[copy]
    out = {"sources_sha256": kernel_sources_sha(), "fetch_scale": fscale, "write_scale": wscale,
           "kernels": {}}
    for k in F:
        if "k_step" in k:
            out["kernels"][k] = {"fetch_kib": F[k], "write_kib": W.get(k),
                                 "read_bytes": F[k] * 1024.0 * fscale,
                                 "write_bytes": W.get(k, 0.0) * 1024.0 * wscale}
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


def traffic_for(kernel_name: str, kernel_ms: float):
    """Measured HBM GB/s of a step kernel from the committed counters, or None
    if they are missing or were taken on different kernel sources."""
    try:
        with open(TRAFFIC_JSON) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None, None
    if t.get("sources_sha256") != kernel_sources_sha():
        return None, None
    e = t["kernels"].get(kernel_name)
    if not e:
        return None, None
    b = e["read_bytes"] + e["write_bytes"]
    return b / (kernel_ms * 1e-3) / 1e9, b


def kernel_symbol(kern, precision: str, forcing: str = "shift", trt: bool = False) -> str:
    variant, tx, ty, _ = kern
    name = {0: "k_step_fused", 2: "k_step_pipe", 3: "k_step_repull"}.get(variant, "k_collide2")
    pr = "sc::PF64" if precision == "fp64" else "sc::PF32S"
    if forcing == "guo":
        pr += "G"
    if trt:
        pr += "T"
    if variant == 1:
        return f"sc::k_collide2<19, {pr}>"
    return f"sc::{name}<19, {pr}, {tx}, {ty}>"


def b_alg(q: int, esize: int) -> int:
    """Algorithmic bytes per site update: 2 species x Q x (read + write)."""
    return 2 * q * 2 * esize


def time_lattice(fields, precision, steps, warmup, kernel=None, forcing="shift", tau_minus=None,
                 repeats=0):
    import torch
    from paper_1112_5547_amd import Lattice, autotune
    lat = Lattice(Q19, L, L, L, tau_A=TAU, tau_B=TAU, G=G, precision=precision, forcing=forcing,
                  tau_minus=tau_minus)
    if kernel:
        lat.set_kernel(*kernel)
    else:
        autotune.apply(lat)  # tuned tile / march chunk when the table has one
    lat.init(fields.rho_A, fields.rho_B)
    T0 = lat.totals()
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_events = lat.time_steps(steps)     # HIP events on the lattice's stream
    lat.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T = lat.totals()
    # further samples of the same number of steps after the timed region (the
    # spread of the step time on this machine; value and roofline keep the first)
    again = [lat.time_steps(steps) / steps for _ in range(repeats)]
    kern = lat.kernel
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return {"wall_s": wall, "kernel_ms": ms_events / steps, "T0": T0, "T": T, "kernel": kern,
            "repeats_ms": again}


def repeat_summary(r) -> dict:
    import statistics
    ms = [r["kernel_ms"]] + r["repeats_ms"]
    return {"samples": len(ms), "kernel_ms": [round(v, 4) for v in ms],
            "median_ms": round(statistics.median(ms), 4),
            "spread": round((max(ms) - min(ms)) / statistics.median(ms), 4)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(fields):
    """The FP64 oracle (plain C, -O2, no FMA contraction) timed on the host:
    the same source built with OpenMP over lattice planes on every core this
    process may use (the headline value), one thread, and the full 2000-step
    run of the 64^2 D2Q9 drop."""
    import oracle
    import sc_inputs
    host_cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS") or host_cores)
    os.environ["OMP_NUM_THREADS"] = str(threads)
    oracle.build(force=False)
    n = L ** 3
    f0 = oracle.init(Q19, fields.rho_A, fields.rho_B)
    steps_mt = 2
    t0 = time.perf_counter()
    oracle.run(f0, TAU, TAU, G, steps_mt, all_cores=True)
    dt_mt = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.run(f0, TAU, TAU, G, 1)
    dt_1 = time.perf_counter() - t0
    del f0
    fl = sc_inputs.drop(64, 64, 1, radius=16, rho_in=1.0, rho_out=0.05, noise=1e-3, seed=1)
    g0 = oracle.init(9, fl.rho_A, fl.rho_B)
    t0 = time.perf_counter()
    oracle.run(g0, 1.0, 1.0, 1.3, 2000)
    dt_cfg1 = time.perf_counter() - t0
    return {"value": round(n * steps_mt / dt_mt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps_mt} full time steps of the 256^3 D3Q19 lattice "
                      f"({n * steps_mt} site updates, {dt_mt:.1f} s) on {threads} OpenMP threads "
                      "(the C oracle, -O2, no FMA contraction, per-site loops shared over "
                      "lattice planes)",
            "host_cores": host_cores, "cpu_model": cpu_model(),
            "single_thread": {"value": round(n / dt_1 / 1e6, 3), "unit": "MLUPS",
                              "sample": f"1 full time step of the 256^3 lattice, {dt_1:.1f} s"},
            "cfg1_full_run": {"seconds": round(dt_cfg1, 3), "threads": 1,
                              "workload": "D2Q9 64x64 drop R=16, tau=1, G=1.3, 2000 steps "
                                          "(8.19M site updates)",
                              "mlups": round(64 * 64 * 2000 / dt_cfg1 / 1e6, 3)}}


def batch_leg(n_jobs: int, steps: int, epoch: int):
    """64 independent D2Q9 drop lattices (L ~ U{64..512}, seed 4), FP32 shifted,
    advanced `steps` steps each: one launch per lattice per step (each lattice
    with its own autotuned kernel), one launch per step for all lattices
    (graph-replayed; the batch form the library and the server use), and one
    persistent launch per epoch (reported beside it), each form with the block
    shape and march chunks the batch autotuner picked for it."""
    import torch
    import sc_inputs
    from paper_1112_5547_amd import Batch, Lattice, autotune
    jobs = sc_inputs.batch_jobs(n_jobs, seed=4, steps=steps)
    tuned = {m: autotune.tune_batch(jobs, precision="fp32_shifted", mode=m, epoch=50)
             for m in ("fused", "persistent")}
    tuned["per_lattice"] = tuned["fused"]
    work = sum(j.sites * j.steps for j in jobs)
    out = {"workload": f"{n_jobs} D2Q9 drop lattices L~U{{64..512}} (seed 4), FP32 shifted, "
                       f"{steps} steps each, epochs of {epoch}",
           "site_updates": work, "tiles": tuned["fused"], "tiles_persistent": tuned["persistent"]}
    for mode in ("per_lattice", "fused", "persistent"):
        lats = []
        for j in jobs:
            lat = Lattice(9, j.nx, j.ny, 1, tau_A=j.tau, G=j.G, precision="fp32_shifted")
            if mode == "per_lattice":
                autotune.apply(lat)
            fl = j.fields()
            lat.init(fl.rho_A, fl.rho_B)
            lats.append(lat)
        b = Batch()
        t = tuned[mode]
        b.set_tiles(t["tx9"], t["tx19"], t["ty19"], t["mb9"], t["mb19"])
        for lat, j in zip(lats, jobs):
            b.add(lat, j.steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while len(b.poll()) < len(lats):
            b.run(epoch, mode)
        dt = time.perf_counter() - t0
        out[mode] = {"seconds": round(dt, 4), "mlups": round(work / dt / 1e6, 1)}
        for lat in lats:
            b.remove(lat)
            lat.close()
        b.close()
    out["speedup_fused_vs_per_lattice"] = round(
        out["fused"]["mlups"] / out["per_lattice"]["mlups"], 2)
    out["persistent_vs_fused"] = round(out["persistent"]["mlups"] / out["fused"]["mlups"], 2)
    return out


def serve_leg(n_jobs: int, budgets_gb, epoch: int):
    """Poisson stream of drop / spinodal jobs (seed 5): 70 % D2Q9 drops
    L~U{64..512}, 30 % D3Q19 L~U{64..256} (half drops, half spinodal), steps
    U{500..5000}, FP32 shifted.  The arrival rate offers 0.7 x the measured
    batched capacity of this job mix (the server's site updates per second
    with every job present from the start and a tenth of the steps).  Served
    with continuous batching, shortest remaining work first (work priced by
    the measured solo step time of each lattice shape; device-filling
    lattices and lone jobs step with their tuned solo kernels), under each
    memory budget, and sequentially (one job at a time, one lattice per
    launch, arrival order) on the same arrivals."""
    import sc_inputs
    from paper_1112_5547_amd import autotune
    from paper_1112_5547_amd.serve import (GpuBackend, Server, batched_capacity, offered_rate,
                                           sequential_baseline, solo_capacity, solo_step_seconds)
    probe = sc_inputs.serving_jobs(n_jobs, seed=5, rate=1.0)
    be = GpuBackend("fp32_shifted")
    step_s = solo_step_seconds(probe, be)
    solo = solo_capacity(probe, step_s)
    # batch tile shape for the job mix, timed on the 8 smallest jobs of each
    # lattice type; the march chunks stay each lattice's own tuned chunk (a
    # chunk tuned on the smallest jobs alone can be a single-chunk march that
    # leaves the large members a few long work items per step)
    sample = (sorted([j for j in probe if j.lattice == 9], key=lambda j: j.sites)[:8]
              + sorted([j for j in probe if j.lattice == 19], key=lambda j: j.sites)[:8])
    tiles = autotune.tune_batch(sample, precision="fp32_shifted", mode="fused", epoch=20,
                                mbs=(0,))
    capacity = batched_capacity(probe, backend=be, tiles=tiles, epoch_steps=epoch)
    progress(f"serving: solo capacity {solo:.0f} MLUPS, batched capacity {capacity:.0f} MLUPS")
    rate = offered_rate(probe, capacity, load=0.7)
    jobs = sc_inputs.serving_jobs(n_jobs, seed=5, rate=rate)
    r3 = lambda v: round(v, 3) if isinstance(v, float) else v
    out = {"workload": f"{n_jobs} Poisson jobs (seed 5), 70% D2Q9 64^2-512^2 drops, 30% D3Q19 "
                       f"64^3-256^3 drops/spinodal, 500-5000 steps, FP32 shifted, offered load "
                       f"0.7 x {capacity:.0f} MLUPS (measured batched capacity of this mix)",
           "arrival_rate_per_s": round(rate, 4), "batched_capacity_mlups": round(capacity, 1),
           "solo_capacity_mlups": round(solo, 1),
           "sequential_offered_load": round(0.7 * capacity / solo, 3),
           "batch_tiles": tiles, "mode": "fused", "epoch_steps": epoch, "runs": []}
    for gb in budgets_gb:
        server = Server(hbm_budget=int(gb * 1e9), epoch_steps=epoch, mode="fused", backend=be,
                        tiles=tiles, policy="srpt", aging=0.0, nominal_rate=solo * 1e6,
                        step_seconds=step_s)
        rep = server.run(jobs)
        served = rep.summary()
        progress(f"serving: {gb:g} GB budget: p50 {served['p50_latency_s']:.2f} s, "
                 f"p99 {served['p99_latency_s']:.2f} s, max queue {served['max_queue']}")
        out["runs"].append({
            "budget_gb": gb, "policy": server.policy, "sat_sites": server.sat_sites,
            "guard_s": server.guard,
            "nonfinite_jobs": [{"job": j.job_id, "tau": round(j.tau, 3), "G": round(j.G, 3)}
                               for j in jobs if j.job_id in served["nonfinite_jobs"]],
            "served": {k: r3(v) for k, v in served.items()}})
    seq = sequential_baseline(jobs, backend=be)
    progress(f"serving: sequential p50 {seq['p50_latency_s']:.2f} s, "
             f"p99 {seq['p99_latency_s']:.2f} s")
    out["sequential"] = {k: r3(v) for k, v in seq.items()}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-schemes", action="store_true",
                    help="skip the Guo-forcing and two-relaxation-time legs")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-ceiling leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-lattices leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-jobs leg")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--serve-jobs", type=int, default=200)
    ap.add_argument("--kernel", type=str, default=None,
                    help="variant,tx,ty,mb of the FP64 step (default: tuned table)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="store per-launch HBM bytes from two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(*args.record_traffic)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not a built path", file=sys.stderr)
        sys.exit(2)

    import torch
    import sc_inputs
    from paper_1112_5547_amd import copy_bench

    torch.cuda.set_device(0)
    fields = sc_inputs.spinodal(L, L, L, rho0=0.5, noise=0.01, seed=3)
    n = L ** 3

    kernel = tuple(int(v) for v in args.kernel.split(",")) if args.kernel else None
    r64 = time_lattice(fields, "fp64", args.steps, args.warmup, kernel, repeats=4)
    mlups = n * args.steps / r64["wall_s"] / 1e6
    ach = b_alg(Q19, 8) * n / (r64["kernel_ms"] * 1e-3) / 1e9
    sym64 = kernel_symbol(r64["kernel"], "fp64")
    traffic64, tbytes64 = traffic_for(sym64, r64["kernel_ms"])
    progress(f"fp64 step {r64['kernel_ms']:.4f} ms")
    out = {
        "metric": "MLUPS + % HBM roofline, D3Q19 2-comp SC 256^3; served-job p50/p99 latency",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["wall_s"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "lattice": "D3Q19", "size": [L, L, L],
                   "precision": "fp64", "kernel": list(r64["kernel"])},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBPS, 4),
                     "traffic": None if traffic64 is None else round(traffic64, 1),
                     "traffic_bytes_per_launch": tbytes64,
                     "kernel": sym64, "kernel_ms": round(r64["kernel_ms"], 4),
                     "bytes_per_site": b_alg(Q19, 8)},
        "checks": {"mass_drift_A": (r64["T"]["mass_A"] - r64["T0"]["mass_A"]) / r64["T0"]["mass_A"],
                   "mom_x": r64["T"]["mom_x"], "max_u": r64["T"]["max_u"]},
        "repeats": repeat_summary(r64),
    }
    if not args.no_fp32:
        r32 = time_lattice(fields, "fp32_shifted", args.steps, args.warmup, repeats=4)
        ach32 = b_alg(Q19, 4) * n / (r32["kernel_ms"] * 1e-3) / 1e9
        sym32 = kernel_symbol(r32["kernel"], "fp32_shifted")
        traffic32, tbytes32 = traffic_for(sym32, r32["kernel_ms"])
        progress(f"fp32_shifted step {r32['kernel_ms']:.4f} ms")
        out["fp32_shifted"] = {
            "value": round(n * args.steps / r32["wall_s"] / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(r32["wall_s"] * 1e3 / args.steps, 4),
            "roofline": {"bound": "hbm", "achieved": round(ach32, 1), "peak": PEAK_HBM_GBPS,
                         "unit": "GB/s", "frac": round(ach32 / PEAK_HBM_GBPS, 4),
                         "traffic": None if traffic32 is None else round(traffic32, 1),
                         "traffic_bytes_per_launch": tbytes32, "kernel": sym32,
                         "kernel_ms": round(r32["kernel_ms"], 4), "bytes_per_site": b_alg(Q19, 4)},
            "kernel": list(r32["kernel"]), "repeats": repeat_summary(r32),
            "mass_drift_A": (r32["T"]["mass_A"] - r32["T0"]["mass_A"]) / r32["T0"]["mass_A"],
        }
    if not args.no_schemes:
        # the same workload with the Guo discrete forcing and with two
        # relaxation times (tau- = 0.8), each its own kernel instantiation
        out["schemes"] = {}
        for scheme, forcing, tm in (("guo", "guo", None), ("trt", "shift", (0.8, 0.8))):
            out["schemes"][scheme] = {}
            for prec, esize in (("fp64", 8), ("fp32_shifted", 4)):
                rg = time_lattice(fields, prec, args.steps, args.warmup, forcing=forcing,
                                  tau_minus=tm)
                achg = b_alg(Q19, esize) * n / (rg["kernel_ms"] * 1e-3) / 1e9
                out["schemes"][scheme][prec] = {
                    "value": round(n * args.steps / rg["wall_s"] / 1e6, 1), "unit": "MLUPS",
                    "ms_per_step": round(rg["wall_s"] * 1e3 / args.steps, 4),
                    "roofline": {"bound": "hbm", "achieved": round(achg, 1),
                                 "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                                 "frac": round(achg / PEAK_HBM_GBPS, 4),
                                 "kernel": kernel_symbol(rg["kernel"], prec, forcing, tm is not None),
                                 "kernel_ms": round(rg["kernel_ms"], 4),
                                 "bytes_per_site": b_alg(Q19, esize)},
                    "kernel": list(rg["kernel"]),
                    "mass_drift_A": (rg["T"]["mass_A"] - rg["T0"]["mass_A"]) / rg["T0"]["mass_A"],
                }
                progress(f"{scheme} {prec} step {rg['kernel_ms']:.4f} ms")
    if not args.no_batch:
        out["batched"] = batch_leg(64, args.batch_steps, epoch=250)
        progress("batch leg done")
    if not args.no_serve:
        # 96 GB holds every job that is ever resident at once; 8 GB holds one of
        # the largest lattices (about 5.6 GB) beside small ones, so a second
        # large job queues for memory
        out["served"] = serve_leg(args.serve_jobs, budgets_gb=(96.0, 8.0), epoch=250)
        main_run = out["served"]["runs"][0]["served"]
        out["metric_served"] = {"p50_latency_s": main_run["p50_latency_s"],
                                "p99_latency_s": main_run["p99_latency_s"],
                                "aggregate_mlups": main_run["aggregate_mlups"],
                                "budget_gb": out["served"]["runs"][0]["budget_gb"],
                                "sequential_p50_latency_s":
                                    out["served"]["sequential"]["p50_latency_s"],
                                "sequential_p99_latency_s":
                                    out["served"]["sequential"]["p99_latency_s"]}
        progress("serving leg done")
    if not args.no_copy:
        out["copy_ceiling_GBps"] = round(copy_bench(COPY_BYTES, reps=10), 1)
        progress(f"copy ceiling {out['copy_ceiling_GBps']} GB/s")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(fields)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
