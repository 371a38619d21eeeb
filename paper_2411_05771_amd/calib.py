"""Reference traffic for HBM byte counters: an elementwise device pass that
reads and writes a known number of bytes.

    python -m paper_2411_05771_amd.calib [--mib 512] [--reps 5]

Each of `reps` launches reads `mib` MiB and writes `mib` MiB (out = -in on
float32), so a profiler's fetch / write byte counters for these dispatches
can be compared with the exact figures to scale the counters of other
kernels.  Prints one JSON line with the bytes per launch.
"""
from __future__ import annotations

import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("needs a HIP device")
    n = args.mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.reps):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"kernel": "neg (elementwise)", "read_bytes_per_launch": 4 * n, "write_bytes_per_launch": 4 * n,
                      "launches": args.reps}))


if __name__ == "__main__":
    main()
