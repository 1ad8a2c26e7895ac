"""Plain device-to-device copy of a known size, used to calibrate the HBM
byte counters (FETCH_SIZE, WRITE_SIZE) read by rocprofv3: a copy of B bytes
must fetch B and write B, so the counters' ratio to B is the scale applied
to the same counters read on the library's kernels.

    python paper_1809_05334_amd/hbm_copy.py --mib 1024 --reps 3
"""
import argparse


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch

    n = args.mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {args.reps} x {args.mib} MiB", flush=True)


if __name__ == "__main__":
    main()
