"""A plain device-to-device copy of known size, for calibrating HBM traffic
counters: FETCH_SIZE / WRITE_SIZE of this copy against its byte count give
the scale applied to the same counters of the library's kernels.

    python -m paper_2606_10477_amd.hbm_copy [--mib 512] [--reps 5]
"""
import argparse
import json


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    n = args.mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"bytes_read_per_copy": n, "bytes_written_per_copy": n, "copies": args.reps}), flush=True)


if __name__ == "__main__":
    main()
