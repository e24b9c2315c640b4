"""Plain device-to-device copy of a known size, used to calibrate the HBM
byte counters (FETCH_SIZE, WRITE_SIZE) of rocprofv3 against known traffic.

    python -m paper_0904_0232_amd.hbm_copy [MiB] [repeats]
"""
import sys

import torch


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    reps = int(sys.argv[2]) if len(sys.argv) > 2 else 3
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d MiB x %d (read %d bytes and write %d bytes per copy)" % (mib, reps, n * 4, n * 4), flush=True)


if __name__ == "__main__":
    main()
