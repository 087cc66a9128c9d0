#!/usr/bin/env python3
"""Write the long-run oracle references under tests/golden/.

Calls only the FP64 oracle (oracle/) and the parameter-only case module; no
value here comes from the GPU library.  For each run it stores, in one
compressed .npz:

  diag_steps, diag       the oracle diagnostics (Sigma phi, Sigma psi,
                         phi-weighted centroid and velocity, p_in, p_out,
                         extrema) every `every` steps, step 0 included;
  fields, stride         phi, p, ux, uy, T, psi at the last step on the nodes
                         (y, x) with y % stride == x % stride == 0;
  row, col               the same six fields at the last step along the row
                         and the column through the initial bubble centre,
                         at every node;
  steps, oracle_sha256   the run length and the oracle source it came from;
  spread_fields, spread_row, spread_col
                         (the shorter runs) the same samples from the
                         oracle's source built with FMA contraction
                         (-mfma -ffp-contract=fast): the same arithmetic
                         rounded differently, whose distance from the strict
                         build is the method's own rounding spread over the
                         run.

Runs (lattice units; the workloads of the parity tests):
  fp32_runs   the four 1024x512 channels (NF and SRF at beta_s 0 and 0.2,
              R = 80, W = 5), 20000 steps, diagnostics every 100 steps;
  precision   the 2048x1024 channel (R = 128, W = 5, sigma_TT = 1e-4,
              beta_s = 0.3), 10000 steps, diagnostics every 500 steps;
  batched64   the smallest of the 64 seeded uneven channels (256x128),
              5000 steps, diagnostics every 100 steps;
  large_plus_small
              the first of the 256 seeded 128x64 channels that run beside
              the 4096x2048 one, 2000 steps, diagnostics every 100 steps.

The full set takes hours on an 8-core host.  Progress is checkpointed to
--ckpt (populations every --ckpt-every steps), so an interrupted run resumes.

    python tests/golden/make_long_runs.py --runs fp32_runs precision batched64 large_plus_small
"""
from __future__ import annotations

import argparse
import hashlib
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "oracle"))

import oracle as O  # noqa: E402

from paper_2408_00146_amd import cases  # noqa: E402

FIELDS = ("phi", "p", "ux", "uy", "T", "psi")


def oracle_sha() -> str:
    h = hashlib.sha256()
    for name in ("lbm_oracle.c", "lbm_oracle.h"):
        with open(os.path.join(ROOT, "oracle", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def runs() -> dict:
    """name -> (parameters, steps, diagnostics interval, field stride, with the rounding spread)"""
    out = {}
    for c in cases.config_fp32_runs():
        out[f"fp32_runs_{c['label']}"] = (c, 20000, 100, 4, False)
    out["precision_2048x1024"] = (cases.config_precision(cases.FP64), 10000, 500, 8, False)
    cb = cases.config_batched()
    k = int(np.argmin([c["nx"] * c["ny"] for c in cb]))
    out[f"batched64_case{k}"] = (cb[k], 5000, 100, 2, True)
    out["large_plus_small_case1"] = (cases.config_large_plus_small()[1], 2000, 100, 1, True)
    return out


def contracted_fields(params: dict, steps: int) -> dict:
    """Fields after `steps` steps from the oracle's source built with FMA
    contraction, loaded in place of the strict build for this call only."""
    strict = O.LIB_PATH
    with tempfile.TemporaryDirectory() as tmp:
        so = os.path.join(tmp, "liblbm_oracle.so")
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-fopenmp", "-mfma", "-ffp-contract=fast", "-shared",
                        "-o", so, os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-lm"], check=True)
        O.LIB_PATH, O._lib = so, None
        try:
            o = O.Oracle(params)
            o.step(steps)
            f = o.fields()
            del o
        finally:
            O.LIB_PATH, O._lib = strict, None
    return f


def diag_vec(o) -> np.ndarray:
    d = o.diag()
    return np.array([d[k] for k in O.DIAG_NAMES], dtype=np.float64)


def run_one(name: str, params: dict, steps: int, every: int, stride: int, spread: bool, ckpt_dir: str,
            ckpt_every: int):
    dst = os.path.join(HERE, f"long_{name}.npz")
    o = O.Oracle(params)
    ck = os.path.join(ckpt_dir, f"{name}.npz")
    diags, dsteps = [], []
    start = 0
    if os.path.exists(ck):
        z = np.load(ck)
        if str(z["oracle_sha256"]) == oracle_sha():
            o.set_populations(z["pops"])
            start = int(z["step"])
            diags = list(z["diag"])
            dsteps = list(z["diag_steps"])
            print(f"{name}: resumed at step {start}", flush=True)
    if start == 0:
        diags, dsteps = [diag_vec(o)], [0]
    t0 = time.time()
    s = start
    while s < steps:
        k = min(every - s % every, steps - s)
        o.step(k)
        s += k
        if s % every == 0 or s == steps:
            diags.append(diag_vec(o))
            dsteps.append(s)
        if s % ckpt_every == 0 and s < steps:
            np.savez(ck + ".tmp.npz", pops=o.populations(), step=s, diag=np.array(diags),
                     diag_steps=np.array(dsteps), oracle_sha256=oracle_sha())
            os.replace(ck + ".tmp.npz", ck)
            rate = params["nx"] * params["ny"] * (s - start) / (time.time() - t0) / 1e6
            print(f"{name}: step {s}/{steps}  {rate:.2f} MLUPS  xc {diags[-1][2]:.4f}", flush=True)
    f = o.fields()
    del o
    yc, xc = int(round(params["yc"])), int(round(params["xc"]))
    extra = {}
    if spread:
        g = contracted_fields(params, steps)
        extra = dict(spread_fields=np.stack([g[k][::stride, ::stride] for k in FIELDS]),
                     spread_row=np.stack([g[k][yc, :] for k in FIELDS]),
                     spread_col=np.stack([g[k][:, xc] for k in FIELDS]))
    np.savez_compressed(
        dst,
        diag_steps=np.array(dsteps, dtype=np.int64), diag=np.array(diags), diag_names=np.array(O.DIAG_NAMES),
        fields=np.stack([f[k][::stride, ::stride] for k in FIELDS]), stride=stride,
        field_names=np.array(FIELDS), row=np.stack([f[k][yc, :] for k in FIELDS]), row_y=yc,
        col=np.stack([f[k][:, xc] for k in FIELDS]), col_x=xc, steps=steps, oracle_sha256=oracle_sha(), **extra,
    )
    print(f"{name}: wrote {dst} after {time.time() - t0:.0f} s", flush=True)
    if os.path.exists(ck):
        os.remove(ck)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--runs", nargs="*", default=["fp32_runs", "precision", "batched64", "large_plus_small"])
    ap.add_argument("--ckpt", default=os.path.join(ROOT, "_work", "golden_ckpt"))
    ap.add_argument("--ckpt-every", type=int, default=2000)
    args = ap.parse_args()
    os.makedirs(args.ckpt, exist_ok=True)
    O.build()
    todo = []
    for r in args.runs:  # in the order given
        todo += [n for n in runs() if n.startswith(r) and n not in todo]
    for name in todo:
        p, steps, every, stride, spread = runs()[name]
        if os.path.exists(os.path.join(HERE, f"long_{name}.npz")):
            print(f"{name}: present, skipped", flush=True)
            continue
        run_one(name, p, steps, every, stride, spread, args.ckpt, args.ckpt_every)


if __name__ == "__main__":
    main()
