#!/usr/bin/env python3
"""Coupled-step throughput of the MI355X central-moment LB step.

One step = one pass of the whole hot path (pull-streaming, moments, LDS halo,
gradients, forces, the four central-moment collisions, store) over every
lattice of the workload.  Prints ONE JSON line on stdout:

  value        whole-job MLUPS (lattice-node updates of all four sets / s / 1e6),
               inputs resident in HBM, timed over exactly --steps steps
  roofline     the step kernel's algorithmic HBM bytes (36 population loads +
               36 stores per node) per step / the average step duration over
               the timed region (HIP events on the launch stream around each
               launched graph of 100 steps), against 8 TB/s
  cpu_baseline the FP64 oracle timed on the host cores over a bounded sample

Default workload: the four 1024x512 FP32 channels (NF and SRF at beta_s 0 and
0.2), advanced together in one launch per step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {0: 576, 1: 288, 2: 144}  # 72 populations x storage bytes
DTYPE = {0: "f64", 1: "f32", 2: "f16-storage/f32"}


def workload(name: str):
    from paper_2408_00146_amd import cases

    if name == "fp32_1024x512x4":
        return cases.config_fp32_runs()
    if name == "fp32_1024x512":
        return cases.config_fp32_runs()[3:]
    if name == "fp64_128x64":
        return [cases.config_small_fp64()]
    if name.startswith(("fp16s_", "fp32_", "fp64_")) and name.endswith("2048x1024"):
        prec = {"fp16s": cases.FP16S, "fp32": cases.FP32, "fp64": cases.FP64}[name.split("_")[0]]
        return [cases.config_precision(prec)]
    if name == "batched64":
        return cases.config_batched()
    if name == "large_plus_small":
        return cases.config_large_plus_small()
    if name == "srf_600x300x4":
        # the paper's migration problem (Sec. 6): four 600x300 channels, M2 5 / 1.25, beta 0 / 0.4
        return [cases.srf_channel(M2=m2, beta=b, psi_L=pl, rho_ratio=10.0)
                for m2, b, pl in ((5.0, 0.0, 0.4), (5.0, 0.4, 0.4), (5.0, 0.4, 0.6), (1.25, 0.4, 0.4))]
    raise SystemExit(f"unknown workload {name}")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_2408_00146_amd/csrc/lbm.hip", "paper_2408_00146_amd/csrc/lbm_device.hpp", "include/lbm.h")


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and whitespace removed, so
    that a measured traffic figure stays tied to the code, not its comments."""
    import hashlib
    import re

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            src = re.sub(r"/\*.*?\*/|//[^\n]*", " ", f.read(), flags=re.S)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def config_tag(config: str) -> str:
    """File-name form of a configuration name ("tile 64x8/512" -> "tile64x8-512")."""
    return config.replace(" ", "").replace("/", "-")


def measured_traffic(workload: str, config: str) -> int | None:
    """HBM bytes per step launch from the committed counter summary of this
    workload and kernel configuration ("tile 64x4/256", "tile 64x8/512"), or
    None when there is none or the kernel sources have changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", f"k_step_{workload}_{config_tag(config)}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                kv[k.strip()] = v.strip().strip("`")
    if kv.get("kernel_source_sha256") != kernel_source_hash() or kv.get("config") != config:
        return None
    try:
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(params: dict, budget_s: float = 15.0) -> dict:
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O

    o = O.Oracle(params)
    t = time.perf_counter()
    o.step(2)
    per = max((time.perf_counter() - t) / 2, 1e-6)
    n = max(2, min(2000, int(budget_s / per)))
    t = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t
    cells = params["nx"] * params["ny"]
    return {"value": cells * n / dt / 1e6, "unit": "MLUPS", "cores": O.threads(), "kind": "oracle",
            "sample": f"one {params['nx']}x{params['ny']} channel of the workload, {n} steps from the "
                      f"initial state, FP64, {dt:.1f} s"}


COMPARE = ("fp32_1024x512", "fp16s_2048x1024", "fp32_2048x1024", "fp64_2048x1024", "batched64",
           "large_plus_small", "srf_600x300x4")


def measure(name: str, steps: int, warmup: int) -> dict:
    """MLUPS and roofline fraction of one workload (autotuned configuration,
    graph launches for the rate, HIP events for the step-kernel duration)."""
    import torch

    from paper_2408_00146_amd import lbm

    ps = workload(name)
    cells = sum(p["nx"] * p["ny"] for p in ps)
    alg = sum(p["nx"] * p["ny"] * BYTES_PER_NODE[p["precision"]] for p in ps)
    s = lbm.Solver(ps)
    s.autotune(5)
    warm_graphs(s, steps, warmup)
    s.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.synchronize()
    dt = time.perf_counter() - t0
    s.set_kernel_timing(2)
    s.step(min(steps, 100))
    kms, _ = s.kernel_time_ms()
    config = lbm.config_name(s.tile)
    s.close()
    del s
    torch.cuda.empty_cache()
    return {"workload": name, "cases": len(ps), "nodes": cells, "MLUPS": round(cells * steps / dt / 1e6, 1),
            "frac": round(alg / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "config": config}


CHUNK = 100  # steps per captured graph (lbm_step)


def warm_graphs(s, steps: int, warmup: int):
    """Untimed warm-up: `warmup` steps, then one step chunk of every size the
    timed `steps` will launch, so that no graph is captured or instantiated
    inside the timed region."""
    s.step(warmup)
    for k in sorted({min(steps, CHUNK), steps % CHUNK} - {0}):
        s.step(k)


def calibrate_counters(mib: int = 1024, reps: int = 5):
    """A plain elementwise kernel of known size for calibrating the HBM byte
    counters: y = x + 1 over float32 tensors of `mib` MiB, `reps` dispatches,
    each reading and writing exactly `mib` MiB.  Under rocprofv3 --pmc
    FETCH_SIZE (then WRITE_SIZE) the known bytes over the counted bytes of
    this kernel are the factors that convert the step kernel's counters."""
    import torch

    if not torch.cuda.is_available():
        raise SystemExit("--calibrate-counters needs a GPU")
    n = mib * (1 << 20) // 4
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.add(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"kernel": "elementwise add (float32)", "bytes_read_per_dispatch": n * 4,
                      "bytes_written_per_dispatch": n * 4, "dispatches": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="fp32_1024x512x4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tile", type=int, default=None)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the comparison workloads (plain FP32 single channel, FP16 storage, batched)")
    ap.add_argument("--calibrate-counters", action="store_true",
                    help="run only the elementwise kernel of known size that calibrates FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()

    if args.calibrate_counters:
        calibrate_counters()
        return

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design, not code)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2408_00146_amd import lbm

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    ps = workload(args.workload)
    cells = sum(p["nx"] * p["ny"] for p in ps)
    alg_bytes = sum(p["nx"] * p["ny"] * BYTES_PER_NODE[p["precision"]] for p in ps)
    precs = sorted({p["precision"] for p in ps})

    s = lbm.Solver(ps)
    if args.tile is not None:
        s.set_tile(args.tile)
    elif not args.no_autotune:
        s.autotune(10)
    config = lbm.config_name(s.tile)
    log(f"workload {args.workload}: {len(ps)} case(s), {cells} nodes, {config}")

    warm_graphs(s, args.steps, args.warmup)
    s.synchronize()
    # timed region: the production path (captured graphs of 100 steps), HIP
    # events on the launch stream around each launched chunk
    s.set_kernel_timing(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, nlaunch = s.kernel_time_ms()
    # the step kernels alone (each step launched between two events), for
    # comparison with the profiler's kernel durations
    s.set_kernel_timing(1)
    s.step(min(args.steps, 200))
    kms_only, _ = s.kernel_time_ms()
    s.set_kernel_timing(0)
    for i in range(min(len(ps), 4)):
        d = s.reduce(i)
        log(f"case {i}: step {d['step']} xc {d['xc']:.3f} ux {d['ux']:.3e} nonfinite {d['nonfinite']}")

    mlups = cells * args.steps / dt / 1e6
    achieved = alg_bytes / (kms * 1e-3) / 1e9
    line = {
        "metric": "coupled-step MLUPS + % HBM roofline; batched/FP16-store vs plain FP32",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "+".join(DTYPE[p] for p in precs),
        "data": "synthetic",
        "config": {"workload": args.workload, "cases": len(ps), "nodes": cells,
                   "grids": sorted({f"{p['nx']}x{p['ny']}" for p in ps}),
                   "kernel_config": config, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.workload, config),
                     "kernel": "k_step", "avg_launch_ms": round(kms, 5),
                     "launches": nlaunch, "kernel_only_ms": round(kms_only, 5),
                     "alg_bytes_per_launch": alg_bytes},
    }
    s.close()
    del s
    torch.cuda.empty_cache()
    if not args.no_compare:
        # the metric compares batching and FP16 storage against the plain FP32 path
        line["compare"] = []
        for name in COMPARE:
            line["compare"].append(measure(name, 300, 30))
            log(f"compare {line['compare'][-1]}")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(ps[0])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
