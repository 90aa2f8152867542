"""Plain device-to-device copy of a known size, for calibrating rocprofv3's
FETCH_SIZE / WRITE_SIZE counters: run it under the same counter as the
kernel being measured; the ratio of known bytes to counted bytes is the
scale factor applied to that kernel's counts.

Usage: python -m paper_1508_03452_amd.copy_probe [GiB] [repeats]
"""
import sys

import torch


def main():
    gib = float(sys.argv[1]) if len(sys.argv) > 1 else 2.0
    reps = int(sys.argv[2]) if len(sys.argv) > 2 else 3
    n = int(gib * (1 << 30) // 8)
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy_probe: {reps} copies of {n * 8} bytes ({n * 8 / 1024:.0f} KiB read and written per dispatch)",
          flush=True)


if __name__ == "__main__":
    main()
