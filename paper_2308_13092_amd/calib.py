"""Plain device copy of a known size, the reference for HBM byte counters.

Run under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``): a copy of B
bytes should fetch and write B bytes, so the counter it reports, divided by
B, is the factor that converts the counter into HBM bytes.
"""
import argparse


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    import torch
    n = a.mib * (1 << 20)
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {n} bytes x {a.reps}")


if __name__ == "__main__":
    main()
