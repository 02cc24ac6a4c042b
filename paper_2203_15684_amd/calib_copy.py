"""Plain device-to-device copy of a known size, used to calibrate the HBM byte
counters (FETCH_SIZE / WRITE_SIZE) of the profiler: the counters read for this
copy are compared with the bytes it must move (size read + size written)."""
import sys

import torch


def main():
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 1 << 30
    a = torch.empty(n // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {n} bytes x 3")


if __name__ == "__main__":
    main()
