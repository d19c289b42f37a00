"""Plain device copy of a known size, used to calibrate HBM traffic counters.

    python -m paper_2410_19993_amd.copy_probe [GiB]

Copies a float64 buffer of the given size (default 1 GiB) to another with
torch's elementwise copy kernel, three times, so that a counter run can
compare what FETCH_SIZE / WRITE_SIZE report against the bytes moved.
"""
import sys

import torch


def main():
    gib = float(sys.argv[1]) if len(sys.argv) > 1 else 1.0
    n = int(gib * (1 << 30)) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {n * 8} bytes x3")


if __name__ == "__main__":
    main()
