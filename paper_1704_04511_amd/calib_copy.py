"""Plain device-to-device copy of a known size, for calibrating HBM counters.

Run it under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``): the counter
values of this copy, whose traffic is exactly ``--mb`` MiB read and written
per launch, give the scale between counter units and bytes on this GPU.

Usage: ``python -m paper_1704_04511_amd.calib_copy --mb 256 --reps 3``
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mb", type=int, default=256)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = a.mb * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for i in range(a.reps):
        ev0.record()
        dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        print(f"copy {a.mb} MiB: {ms:.3f} ms, {2 * a.mb * (1 << 20) / ms / 1e6:.1f} GB/s (read+write)", flush=True)


if __name__ == "__main__":
    main()
