"""Calibration run for HBM byte counters: one device-to-device copy of a known
size, so that a profiler's FETCH_SIZE / WRITE_SIZE readings can be scaled to
bytes.  ``python calib_copy.py [GiB]``"""
import sys

import torch


def main():
    gib = float(sys.argv[1]) if len(sys.argv) > 1 else 4.0
    n = int(gib * (1 << 30)) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copy of %d bytes x3 done" % (4 * n), flush=True)


if __name__ == "__main__":
    main()
