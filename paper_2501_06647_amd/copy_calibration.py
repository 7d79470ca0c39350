"""Reference copy for HBM counter calibration.

Runs a device-to-device copy of a known size (a plain PyTorch copy kernel)
so that rocprofv3's FETCH_SIZE / WRITE_SIZE counters, read per dispatch for
it, give the factor between counter units and bytes moved:
    rocprofv3 --pmc FETCH_SIZE -- python3 paper_2501_06647_amd/copy_calibration.py
    rocprofv3 --pmc WRITE_SIZE -- python3 paper_2501_06647_amd/copy_calibration.py
Each copy reads and writes MIB mebibytes.
"""

import argparse
import sys

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    n = args.mib * (1 << 20) // 4
    src = torch.randn(n, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d x %d MiB" % (args.reps, args.mib), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
