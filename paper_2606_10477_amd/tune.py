"""Provision the degree-versus-iterations table on this GPU (paper §4.2, Alg. 2 and 3).

Runs the encrypted inverse square root with the tuner's own keys over a grid
of Chebyshev degrees x Newton iterations at several input levels, measures the
MRE against FP64 and the time of each configuration, profiles the unit cost of
every primitive at every level, predicts each configuration's time from its
operation trace, and selects, per (level, MRE target), the pair with minimum
predicted time.  Writes a JSON report (the tuning table plus predicted versus
measured times and the speedup over a fixed configuration).

    python -m paper_2606_10477_amd.tune --out tuning.json
"""
import argparse
import json
import os
import sys
import time

import numpy as np

P16 = dict(log_n=16, max_level=27, num_special=7, digit_size=10, hamming_weight=192)


def run(levels, degrees, iters, targets, lo, hi, batch, reps, fixed, tuner_seed=777, quiet=False):
    import torch
    from . import ckks, inputs, tuner

    torch.cuda.set_device(0)
    t_start = time.perf_counter()
    ctx = ckks.Context(**P16)
    ctx.keygen(tuner_seed)              # the tuner's own keys, not a client's
    x = inputs.log_uniform(ctx.n, lo, hi, 11)
    cts = {l: ctx.encrypt(x, l, 2.0 ** 50, 12 + l) for l in levels}
    lv = sorted(set(range(0, max(levels) + 1)))
    costs = tuner.profile_unit_costs(ctx, lv, batch=batch, reps=reps)
    if not quiet:
        print(f"profiled {len(costs)} unit costs", file=sys.stderr, flush=True)
    rows = tuner.sweep(ctx, x, cts, degrees, iters, lo, hi, batch=batch, reps=reps, costs=costs)
    table = {}
    for l in levels:
        for tgt in targets:
            r = tuner.select(rows, tgt, l)
            table.setdefault(str(l), {})[f"{tgt:.3g}"] = None if r is None else \
                {"degree": r["d"], "iters": r["i"], "mre": r["m"], "t_pred": r["t_pred"], "t_meas": r["t"]}
    fixed_rows = {l: next((r for r in rows if r["level"] == l and r["d"] == fixed[0] and r["i"] == fixed[1]
                           and r.get("ok")), None) for l in levels}
    speedup = {}
    for l in levels:
        best = tuner.select(rows, targets[-1], l)
        fr = fixed_rows[l]
        if best and fr:
            speedup[str(l)] = {"fixed": [fixed[0], fixed[1]], "fixed_t": fr["t"], "fixed_mre": fr["m"],
                               "tuned": [best["d"], best["i"]], "tuned_t": best["t"], "tuned_mre": best["m"],
                               "speedup": fr["t"] / best["t"]}
    ok = [r for r in rows if r.get("ok")]
    err = [abs(r["t_pred"] - r["t"]) / r["t"] for r in ok]
    report = {
        "params": "N=2^16, q0 60-bit + 27 x 40-bit, 7 x 60-bit special, dnum 3, h 192",
        "input": f"x log-uniform in [{lo}, {hi}], encrypted at scale 2^50",
        "batch": batch, "grid": {"degrees": degrees, "iters": iters, "levels": levels},
        "targets": targets, "table": table, "speedup_vs_fixed": speedup,
        "prediction_rel_error": {"median": float(np.median(err)), "max": float(np.max(err))} if err else None,
        "rows": rows, "tuning_wall_s": time.perf_counter() - t_start,
        "unit_costs": {f"{op}@{l}": v for (op, l), v in sorted(costs.items(), key=lambda kv: (kv[0][1], kv[0][0]))},
    }
    ctx.close()
    return report


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="gpurun_out/tuning.json")
    ap.add_argument("--levels", default="13,17,21,27")
    ap.add_argument("--degrees", default="7,15,31,63,127")
    ap.add_argument("--iters", default="1,2,3,4,5,6")
    ap.add_argument("--targets", default="1e-6,1e-7,3.1e-8")
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    ints = lambda s: [int(v) for v in s.split(",")]
    rep = run(ints(args.levels), ints(args.degrees), ints(args.iters),
              [float(v) for v in args.targets.split(",")], 2.0 ** -10, 1.0, args.batch, args.reps, (31, 3))
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "w") as f:
        json.dump(rep, f, indent=1)
    summary = {"table": rep["table"], "speedup_vs_fixed": rep["speedup_vs_fixed"],
               "prediction_rel_error": rep["prediction_rel_error"], "tuning_wall_s": rep["tuning_wall_s"]}
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
