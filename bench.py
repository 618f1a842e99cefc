"""Benchmark: encrypted inverse square roots per second at N = 2^16.

One step = CryptoInvSqrt (paper Alg. 1: Chebyshev initial value, Newton
steps, bootstrapping when levels run out) over a batch of ciphertexts already
resident in HBM.  Prints one JSON line (see the contract in the design notes):
value = ciphertexts/s for the whole job, plus the roofline of the dominant
kernel family measured live with HIP events on the library's stream, the MRE
of the result against FP64, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
P16 = dict(log_n=16, max_level=27, num_special=7, digit_size=10, hamming_weight=192)
LO, HI = 2.0 ** -10, 1.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=1, help="ciphertexts per step")
    ap.add_argument("--degree", type=int, default=31)
    ap.add_argument("--iters", type=int, default=3)
    ap.add_argument("--level", type=int, default=13, help="input level")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=1)
    return ap.parse_args()


def cpu_baseline(args, x_list):
    """The oracle, as it stands, on the same chain for `cpu_samples` ciphertexts."""
    from oracle import oracle as O
    o = O.Context(16, 27, 7, 10, h=192)
    o.keygen(9)
    cts = [o.encrypt(x, args.level, 2.0 ** 50, 100 + i) for i, x in enumerate(x_list[:args.cpu_samples])]
    t0 = time.perf_counter()
    for ct in cts:
        o.invsqrt(ct, args.degree, args.iters, LO, HI)
    dt = time.perf_counter() - t0
    return {"value": len(cts) / dt, "unit": "ciphertexts/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(cts)} full invsqrt (degree {args.degree}, {args.iters} Newton steps) "
                      f"at N=2^16 from level {args.level}, single-threaded, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2606_10477_amd import ckks, inputs

    torch.cuda.set_device(0)
    ctx = ckks.Context(**P16)
    ctx.keygen(9)
    xs = [inputs.log_uniform(ctx.n, LO, HI, 1 + i) for i in range(args.batch)]
    cts = [ctx.encrypt(x, args.level, 2.0 ** 50, 3 + i) for i, x in enumerate(xs)]
    ctx.sync()

    def step():
        if args.batch == 1:
            return [ctx.invsqrt(cts[0], args.degree, args.iters, a=LO, b=HI)]
        return ctx.invsqrt_batch(cts, args.degree, args.iters, a=LO, b=HI)

    for _ in range(args.warmup):
        out = step()
        del out
    ctx.sync()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    ctx.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fam = {}
    for name in ("ntt", "keyswitch"):
        n, ms, by = ctx.profile_read(name)
        fam[name] = (n, ms, by)
    ctx.profile(False)

    ref = 1 / np.sqrt(xs[0])
    z = ctx.decrypt(out[0]).real
    mre = float(np.mean(np.abs(z - ref) / ref))
    out_level = out[0].level

    # dominant kernel family: the one with the most GPU time
    dom = max(fam, key=lambda k: fam[k][1])
    n, ms, by = fam[dom]
    achieved = (by / (ms / 1e3)) / 1e9 if ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
            "launches": n, "avg_launch_us": round(ms * 1e3 / max(n, 1), 2),
            "share_of_step": round(ms / 1e3 / dt, 3) if dt > 0 else None}
    others = {k: {"calls": v[0], "gpu_ms": round(v[1], 3),
                  "GB/s": round((v[2] / (v[1] / 1e3)) / 1e9, 1) if v[1] > 0 else None}
              for k, v in fam.items()}
    total = args.batch * args.steps
    res = {
        "metric": "invsqrt ciphertexts/s at N=2^16, MRE<=3.1e-8",
        "value": round(total / dt, 3),
        "unit": "ciphertexts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"CryptoInvSqrt degree {args.degree}, {args.iters} Newton steps, "
                               f"x log-uniform in [2^-10,1], input level {args.level} (no bootstrap needed)",
                   "ring_degree": 65536, "slots": 32768, "batch": args.batch,
                   "params": "q0 60-bit + 27 x 40-bit, 7 x 60-bit special, dnum 3, h 192",
                   "output_level": out_level},
        "mre": mre,
        "roofline": roof,
        "kernel_families": others,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args, xs if len(xs) >= args.cpu_samples else
                                           [inputs.log_uniform(ctx.n, LO, HI, 1 + i) for i in range(args.cpu_samples)])
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
