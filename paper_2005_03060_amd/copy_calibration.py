"""Copy of a known size, the calibration run for the HBM-traffic counters.

    rocprofv3 --pmc FETCH_SIZE -- python3 paper_2005_03060_amd/copy_calibration.py

Copies a 256 MiB float32 tensor three times; FETCH_SIZE and WRITE_SIZE of
the copy kernel against the bytes it must move give the scale applied to a
kernel's counters (part of the source may be served by the device's last-
level cache, which the counters do not see as memory traffic).
"""
import torch


def main():
    n = 256 * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x", n * 4, "bytes", flush=True)


if __name__ == "__main__":
    main()
