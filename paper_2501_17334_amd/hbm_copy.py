"""Calibration kernel for HBM byte counters: a plain device-to-device copy of
a known size.

Run under `rocprofv3 --pmc FETCH_SIZE` (then `WRITE_SIZE`), the copy's
dispatch reads `nbytes` and writes `nbytes`; the ratio of the counter to
that figure is the factor by which the same counter is scaled for another
kernel on the same machine.

    python3 -m paper_2501_17334_amd.hbm_copy [MiB] [repeats]
"""
from __future__ import annotations

import sys


def main(argv):
    import torch
    mib = int(argv[1]) if len(argv) > 1 else 1024
    reps = int(argv[2]) if len(argv) > 2 else 3
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    for r in range(reps):
        ev[2 * r].record()
        dst.copy_(src)
        ev[2 * r + 1].record()
    torch.cuda.synchronize()
    for r in range(reps):
        ms = ev[2 * r].elapsed_time(ev[2 * r + 1])
        print(f"copy {r}: {n * 8} bytes read + {n * 8} written in {ms:.3f} ms "
              f"({2 * n * 8 / ms / 1e6:.1f} GB/s)", flush=True)


if __name__ == "__main__":
    main(sys.argv)
