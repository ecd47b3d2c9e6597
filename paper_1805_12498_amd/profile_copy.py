"""Device copy of a known size, for calibrating hardware byte counters.

    python -m paper_1805_12498_amd.profile_copy [MiB]

Allocates MiB mebibytes on the current device, then copies them once into a
second buffer (one read and one write of MiB each); a counter that sums the
bytes a kernel reads from or writes to HBM should report about MiB * 1024 KiB
for the copy kernel.
"""
import sys

import torch


def main(mib: int = 1024) -> None:
    src = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print("copied %d MiB" % mib, flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 1024)
