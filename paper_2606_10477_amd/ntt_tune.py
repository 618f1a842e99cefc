"""Tuner of the N = 2^16 transform schedule: times forward and inverse NTT
calls of several sizes with 4 (4 or 16 sub-transforms per workgroup), 8 and
16 words per thread on this GPU and picks the limb-count bounds for
ckks_ntt_schedule (the largest call sizes at which the smaller variants are
still the fastest).  Results are identical
under every schedule; only the time changes.

    python -m paper_2606_10477_amd.ntt_tune [--limbs 1,2,4,...] [--json PATH]

With --chain it times the benchmarked chain (bootstrapping set, degree 31,
3 Newton steps, one ciphertext) under the listed schedules instead:

    python -m paper_2606_10477_amd.ntt_tune --chain "s32:32,32,32;s128:128,128,128"

With --calls K it only issues K forward and K inverse transforms at each
size under the library's schedule, untimed, for a counter profiler to
attribute per dispatch (each dispatch's grid gives its limb count):

    python -m paper_2606_10477_amd.ntt_tune --limbs 1,8,43,96 --calls 20

With --word-size it measures the butterfly rate of each word form in
registers (ckks_butterfly_rate): 64-bit words on the chain's 60- and 52-bit
primes, binary64 on its 40-bit primes, and 32-bit words on a 30-bit prime
= 1 mod 2N (the alternative design), and states each form's modulus bits
transformed per second and per byte of HBM traffic:

    python -m paper_2606_10477_amd.ntt_tune --word-size [--json PATH]

From a counter run of the same command (rocprofv3 --pmc ... -o run, the SQ
instruction counters), VALU wave instructions per butterfly of each form and
the rate they allow at the VALU peak (256 CUs x 2.4 GHz, one wave
instruction per CU per cycle):

    python -m paper_2606_10477_amd.ntt_tune --word-size-counters PMC_DIR --json WORD_SIZE.json
"""
import argparse
import csv
import json
import os
import time

SIZES = (1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 24, 28, 32, 40, 48, 64, 96)
BIG = 1 << 20
VARIANTS = (("4s4", (BIG, BIG, BIG)), (4, (BIG, BIG, 0)), (8, (0, BIG, 0)), (16, (0, 0, 0)))


def time_calls(ctx, x, n, idx, inverse, reps):
    ctx.ntt_device(x.data_ptr(), n, idx, inverse=inverse)
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.ntt_device(x.data_ptr(), n, idx, inverse=inverse)
    ctx.sync()
    return (time.perf_counter() - t0) / reps


def scan(ctx, sizes, nprimes):
    import numpy as np
    import torch
    rows = []
    for n in sizes:
        # a mix of all primes of the chain (40/52/60-bit), as in the key switch
        idx = np.array([(7 * i) % nprimes for i in range(n)], dtype=np.uint32)
        x = torch.randint(0, 1 << 30, (n, 1 << 16), dtype=torch.int64, device="cuda")
        reps = max(10, 600 // n)
        row = {"limbs": n}
        for R, sched in VARIANTS:
            ctx.ntt_schedule(*sched)
            row[f"fwd_R{R}_us"] = 1e6 * time_calls(ctx, x, n, idx, False, reps)
            row[f"inv_R{R}_us"] = 1e6 * time_calls(ctx, x, n, idx, True, reps)
        rows.append(row)
        print(json.dumps({k: round(v, 1) if isinstance(v, float) else v for k, v in row.items()}), flush=True)
    ctx.ntt_schedule(-1, -1, -1)
    return rows


def issue(ctx, sizes, nprimes, calls):
    """`calls` forward and inverse transforms at each size (default schedule)."""
    import numpy as np
    import torch
    for n in sizes:
        idx = np.array([(7 * i) % nprimes for i in range(n)], dtype=np.uint32)
        x = torch.randint(0, 1 << 30, (n, 1 << 16), dtype=torch.int64, device="cuda")
        for _ in range(calls):
            ctx.ntt_device(x.data_ptr(), n, idx, inverse=False)
            ctx.ntt_device(x.data_ptr(), n, idx, inverse=True)
        ctx.sync()
        print(json.dumps({"limbs": n, "calls": calls}), flush=True)


def choose(rows, tol=0.01):
    """Bounds (r4_max, r8_max, s4_max): every call size up to s4_max is fastest
    (fwd + inv) with 4 words per thread and 4 sub-transforms per workgroup, up
    to r4_max with 4 words, up to r8_max with 4 or 8.  A variant within `tol`
    (relative) of the fastest counts as fastest, preferring the smaller
    workgroups, so that timing noise at near-ties does not end a run early."""
    rank = {R: k for k, (R, _) in enumerate(VARIANTS)}
    best = []
    for r in rows:
        t = {R: r[f"fwd_R{R}_us"] + r[f"inv_R{R}_us"] for R, _ in VARIANTS}
        tmin = min(t.values())
        best.append((r["limbs"], min((R for R in t if t[R] <= tmin * (1 + tol)), key=rank.get)))

    def run_of(allowed, start):
        b = start
        for n, R in best:
            if n <= start:
                continue
            if R not in allowed:
                break
            b = n
        return b
    s4 = run_of({"4s4"}, 0)
    r4 = run_of({"4s4", 4}, s4)
    r8 = run_of({8}, r4)
    return r4, r8, s4, best


def chain_times(schedules, reps=3, runs=10):
    """The benchmarked chain (bootstrapping set, degree 31, 3 Newton steps,
    one ciphertext from the top level) under each (name, (r4, r8, s4))
    schedule: the best of `reps` means over `runs` calls, in ms; the result
    words are checked equal across schedules."""
    import numpy as np
    from . import ckks, inputs
    ctx = ckks.Context.from_set("p16b")
    ctx.keygen(9, ctx.bts_galois())
    x = inputs.log_uniform(ctx.n, 2.0 ** -10, 1.0, 1)
    ct = ctx.encrypt(x, ctx.l_after, 2.0 ** 50, 3)
    out, ref = [], None
    for name, sc in schedules:
        ctx.ntt_schedule(*sc)
        w = ctx.invsqrt(ct, 31, 3, 2.0 ** -10, 1.0).words()
        if ref is None:
            ref = w
        if not np.array_equal(w, ref):
            raise RuntimeError(f"schedule {name} changed the result words")
        best = float("inf")
        for _ in range(reps):
            ctx.sync()
            t0 = time.perf_counter()
            for _ in range(runs):
                ctx.invsqrt(ct, 31, 3, 2.0 ** -10, 1.0)
            ctx.sync()
            best = min(best, (time.perf_counter() - t0) / runs)
        out.append({"schedule": name, "bounds": list(sc), "ms": 1e3 * best})
        print(json.dumps(out[-1]), flush=True)
    ctx.ntt_schedule(-1, -1, -1)
    ctx.close()
    return out


def _is_prime(n):
    """Deterministic Miller-Rabin for n < 3.3e24 (the first 12 prime bases)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, r = n - 1, 0
    while d % 2 == 0:
        d, r = d // 2, r + 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def prime_below(bits, two_n):
    """The largest prime q < 2^bits with q = 1 mod two_n."""
    q = ((1 << bits) - 1) // two_n * two_n + 1
    while q >= (1 << bits) or not _is_prime(q):
        q -= two_n
    return q


WS_THREADS, WS_ROUNDS, WS_LAUNCHES = 2048 * 256, 128, 20
VALU_WAVE_INSTR_PER_S = 256 * 2.4e9


def word_size_counters(pmc_dir, cases, rounds=WS_ROUNDS, launches=WS_LAUNCHES, threads=WS_THREADS):
    """Per case of word_size(): counters per butterfly, averaged over the timed
    dispatches (each case issues one warm-up and `launches` timed dispatches,
    in case order)."""
    by = {}
    with open(os.path.join(pmc_dir, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if "k_butterfly_rate" not in r["Kernel_Name"]:
                continue
            c = by.setdefault(int(r["Dispatch_Id"]), {})
            c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    ids = sorted(by)
    if len(ids) != len(cases) * (launches + 1):
        raise SystemExit(f"expected {len(cases) * (launches + 1)} probe dispatches, found {len(ids)}")
    per = threads * rounds * 12       # butterflies per dispatch: 3 stages of 4 per round
    out = []
    for i, case in enumerate(cases):
        grp = ids[i * (launches + 1) + 1:(i + 1) * (launches + 1)]
        mean = {k: sum(by[d].get(k, 0.0) for d in grp) / len(grp) for k in by[grp[0]]}
        row = dict(case)
        row.update({f"{k}_per_butterfly": v * 64 / per for k, v in sorted(mean.items()) if k.startswith("SQ_INSTS")})
        ipb = mean.get("SQ_INSTS_VALU", 0.0) * 64 / per
        if ipb > 0:
            row["valu_bound_butterflies_per_s"] = VALU_WAVE_INSTR_PER_S * 64 / ipb
            row["valu_issue_pct"] = 100 * case["butterflies_per_s"] / row["valu_bound_butterflies_per_s"]
        out.append(row)
    return out


def word_size(ctx, rounds=WS_ROUNDS, launches=WS_LAUNCHES):
    """Butterflies per second of each word form on primes of the chain (and a
    30-bit prime), with the modulus bits they carry per second and per byte
    moved (a word read and written once per pass)."""
    primes = [int(p) for p in ctx.primes]
    cases = [("u64", 0, max(primes)), ("u64", 0, max(p for p in primes if p.bit_length() <= 53)),
             ("binary64", 1, max(p for p in primes if p.bit_length() <= 42)),
             ("u32", 2, prime_below(30, 2 * ctx.N))]
    out = []
    for name, form, q in cases:
        rate = ctx.butterfly_rate(form, q, rounds, launches)
        bits = q.bit_length()
        word = 4 if form == 2 else 8
        out.append({"form": name, "q_bits": bits, "q": q, "butterflies_per_s": rate,
                    "modulus_bits_per_s": rate * bits, "modulus_bits_per_word_byte": bits / word})
        print(json.dumps(out[-1]), flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--limbs", default=",".join(str(s) for s in SIZES))
    ap.add_argument("--json", default=None)
    ap.add_argument("--calls", type=int, default=0, help="only issue this many calls per size (for profilers)")
    ap.add_argument("--chain", default=None,
                    help="time the benchmarked chain under schedules 'name:r4,r8,s4;...' instead of scanning")
    ap.add_argument("--word-size", action="store_true", help="butterfly rates of the word forms instead of scanning")
    ap.add_argument("--word-size-counters", default=None,
                    help="counter directory of a --word-size run: instructions per butterfly (reads --json)")
    a = ap.parse_args(argv)
    if a.word_size_counters:
        with open(a.json) as f:
            cases = json.load(f)
        for row in word_size_counters(a.word_size_counters, cases):
            print(json.dumps(row), flush=True)
        return
    import torch
    from . import ckks
    torch.cuda.set_device(0)
    if a.chain:
        sch = []
        for item in a.chain.split(";"):
            name, b = item.split(":")
            sch.append((name, tuple(int(v) for v in b.split(","))))
        res = chain_times(sch)
        if a.json:
            with open(a.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    ctx = ckks.Context.from_set("p16b", bootstrapping=False)
    if a.word_size:
        res = word_size(ctx)
        if a.json:
            with open(a.json, "w") as f:
                json.dump(res, f, indent=1)
        ctx.close()
        return
    if a.calls:
        issue(ctx, [int(s) for s in a.limbs.split(",")], ctx.np_, a.calls)
        ctx.close()
        return
    rows = scan(ctx, [int(s) for s in a.limbs.split(",")], ctx.np_)
    r4, r8, s4, best = choose(rows)
    res = {"r4_max_limbs": r4, "r8_max_limbs": r8, "s4_max_limbs": s4, "fastest_variant": best, "rows": rows}
    print(json.dumps({k: v for k, v in res.items() if k != "rows"}), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
