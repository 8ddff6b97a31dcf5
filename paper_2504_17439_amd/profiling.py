"""Profiling helpers for rocprofv3 runs.

    python -m paper_2504_17439_amd.profiling copy --gib 4

copies a float32 device buffer of the given size three times with a plain
device-to-device copy kernel, so that the HBM counters of a profiled kernel
(FETCH_SIZE, WRITE_SIZE, KiB per dispatch) can be scaled by what the same
counters read for a copy whose traffic is known (size read + size written).
"""
from __future__ import annotations

import argparse
import sys


def copy(gib: float, reps: int = 3):
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {n * 4} bytes x {reps}", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--gib", type=float, default=4.0)
    args = ap.parse_args(argv)
    if args.cmd == "copy":
        copy(args.gib)
    return 0


if __name__ == "__main__":
    sys.exit(main())
