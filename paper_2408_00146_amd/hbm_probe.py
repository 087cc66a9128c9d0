"""Plain streaming kernel of known size, for calibrating HBM byte counters.

Runs ``y = x + 1`` over float32 tensors of ``--mib`` MiB each, ``--reps``
times, so that one dispatch reads and writes exactly ``--mib`` MiB.  Under
``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``) the counter value of
that elementwise kernel, divided into the known byte count, is the factor
that converts the same counter of the step kernel into bytes.
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()

    import torch

    if not torch.cuda.is_available():
        raise SystemExit("hbm_probe needs a GPU")
    n = args.mib * (1 << 20) // 4
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.reps):
        torch.add(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"kernel": "elementwise add (float32)", "bytes_read_per_dispatch": n * 4,
                      "bytes_written_per_dispatch": n * 4, "dispatches": args.reps}), flush=True)


if __name__ == "__main__":
    main()
