"""Serving loop for encrypted inverse square roots with continuous batching.

Requests arrive over time; each carries 1..32 ciphertexts at one input level
and an MRE target, which the tuning table maps to a (degree, Pre-BTS
indicator c, iterations) setting.  The scheduler admits arrived requests while
their estimated device working set fits the memory budget, groups the
admitted ciphertexts of all requests by (level, degree, c, iterations) and
runs the oldest group as one batched launch sequence (up to `max_batch`
ciphertexts), bootstrapping keys resident in HBM.  Requests that arrive
while a batch is on the GPU are admitted at the next scheduling round, so work
from different requests shares launches.  Every ciphertext's result is the same
alone and in the mix: batch members never interact.

The baseline ("one at a time") serves requests strictly in arrival order, each
request's ciphertexts in one batched call, with no sharing across requests.
"""
import os
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    cts: list               # single ciphertexts, one level
    level: int
    target: float
    degree: int = 0
    iters: int = 0
    c: int = 0
    outs: dict = field(default_factory=dict)
    admitted: float = None
    done: float = None


def lookup(table, level, target):
    """(degree, c, iters) for (level, target) from a tuning table
    {level: {target: {"degree": d, "c": c, "iters": i}}} (c defaults to 0);
    falls back to the closest tuned level not above `level`, then to the
    strictest target."""
    usable = {k for k, row in table.items() if any(v is not None for v in row.values())}
    lv = str(level)
    if lv not in usable:
        below = [int(k) for k in usable if int(k) <= level]
        if not below:
            raise KeyError(f"no tuned level <= {level}")
        lv = str(max(below))
    row = table[lv]
    key = f"{target:.3g}"
    ent = row.get(key)
    if ent is None:
        ent = next(v for k, v in sorted(row.items(), key=lambda kv: float(kv[0])) if v is not None)
    return ent["degree"], ent.get("c", 0), ent["iters"]


class Server:
    def __init__(self, ctx, table, max_batch=64, mem_budget=None, ct_factor=24, lo=2.0 ** -10, hi=1.0):
        self.ctx = ctx
        self.table = table
        self.max_batch = max_batch
        self.lo, self.hi = lo, hi
        self.ct_factor = ct_factor       # working-set multiple of one input ciphertext
        if mem_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            mem_budget = int(0.7 * free)
        self.mem_budget = mem_budget
        self.in_use = 0
        self.queue = []                   # arrived, not admitted
        self.active = []                  # admitted, not finished
        self.log = []

    def est_bytes(self, req):
        return len(req.cts) * 2 * (req.level + 1) * self.ctx.N * 8 * self.ct_factor

    def submit(self, req):
        req.degree, req.c, req.iters = lookup(self.table, req.level, req.target)
        self.queue.append(req)

    def _admit(self, now):
        still = []
        for r in self.queue:
            need = self.est_bytes(r)
            if self.in_use + need <= self.mem_budget or not self.active:
                self.in_use += need
                r.admitted = now
                self.active.append(r)
            else:
                still.append(r)
        self.queue = still

    def step(self, clock):
        """One scheduling round: admit, pick the oldest group, run it."""
        self._admit(clock())
        if not self.active:
            return 0
        oldest = min(self.active, key=lambda r: r.arrival)
        key = (oldest.level, oldest.degree, oldest.c, oldest.iters)
        work = []                          # (request, ct index)
        for r in sorted(self.active, key=lambda r: r.arrival):
            if (r.level, r.degree, r.c, r.iters) != key:
                continue
            for k in range(len(r.cts)):
                if k not in r.outs and len(work) < self.max_batch:
                    work.append((r, k))
        cts = [r.cts[k] for r, k in work]
        outs = self.ctx.invsqrt_batch(cts, key[1], key[3], a=self.lo, b=self.hi, pre_bts=bool(key[2]))
        self.ctx.sync()
        t = clock()
        for (r, k), y in zip(work, outs):
            r.outs[k] = y
        finished = [r for r in self.active if len(r.outs) == len(r.cts)]
        for r in finished:
            r.done = t
            self.in_use -= self.est_bytes(r)
            self.active.remove(r)
        self.log.append({"t": t, "group": key, "batch": len(cts), "finished": [r.rid for r in finished]})
        return len(cts)


def run_continuous(ctx, table, requests, max_batch=64, mem_budget=None):
    """Serve `requests` (arrival times relative to start) with continuous
    batching; returns the server (requests carry admitted/done times)."""
    srv = Server(ctx, table, max_batch=max_batch, mem_budget=mem_budget)
    pending = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    i = 0
    while i < len(pending) or srv.queue or srv.active:
        now = clock()
        while i < len(pending) and pending[i].arrival <= now:
            srv.submit(pending[i])
            i += 1
        if not srv.queue and not srv.active:
            time.sleep(max(0.0, pending[i].arrival - clock()))
            continue
        srv.step(clock)
    return srv


def run_one_at_a_time(ctx, table, requests, lo=2.0 ** -10, hi=1.0):
    """Baseline: requests in arrival order, one at a time (each request's
    ciphertexts in one batched call)."""
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    for r in sorted(requests, key=lambda r: r.arrival):
        r.degree, r.c, r.iters = lookup(table, r.level, r.target)
        wait = r.arrival - clock()
        if wait > 0:
            time.sleep(wait)
        r.admitted = clock()
        outs = ctx.invsqrt_batch(r.cts, r.degree, r.iters, a=lo, b=hi, pre_bts=bool(r.c))
        ctx.sync()
        r.outs = dict(enumerate(outs))
        r.done = clock()
    return requests


def summarize(requests):
    lat = np.array([r.done - r.arrival for r in requests])
    n_ct = sum(len(r.cts) for r in requests)
    span = max(r.done for r in requests) - min(r.arrival for r in requests)
    return {"requests": len(requests), "ciphertexts": int(n_ct),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()), "ciphertexts_per_s": n_ct / span, "span_s": span}


DEFAULT_TABLE = {"8": {"1e-06": {"degree": 31, "c": 0, "iters": 3}, "1e-07": {"degree": 31, "c": 0, "iters": 3},
                       "3.1e-08": {"degree": 31, "c": 0, "iters": 3}}}


def main(argv=None):
    """Serving sweep at N = 2^16 on the bootstrapping parameter set (relin,
    rotation and conjugation keys resident): Poisson arrivals at each rate,
    request sizes Geometric(0.25) truncated to [1, 32], levels in [5, 8] and
    MRE targets drawn per request; continuous batching versus one request at a
    time."""
    import argparse
    import json

    import torch

    from . import ckks, inputs

    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="10,40,160")
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--levels", default="5,6,7,8", help="input levels (those the tuning table can serve)")
    ap.add_argument("--table", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_mi355x_bts.json"),
                    help="tuning JSON from paper_2606_10477_amd.tune")
    ap.add_argument("--max-batch", type=int, default=16,
                    help="ciphertexts per launch sequence (bootstrapping throughput saturates near 8-16)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    table = DEFAULT_TABLE
    if args.table and os.path.exists(args.table):
        with open(args.table) as f:
            table = json.load(f)["table"]
    torch.cuda.set_device(0)
    ctx = ckks.Context.from_set("p16b")
    ctx.keygen(9, ctx.bts_galois())
    levels = [int(v) for v in args.levels.split(",")]
    out = {"workload": "CryptoInvSqrt serving at N=2^16 with bootstrapping keys resident, Poisson arrivals, "
                       f"sizes Geometric(0.25) in [1,32], levels {levels}, targets 1e-6/1e-7/3.1e-8",
           "table": args.table, "runs": []}
    for rate in [float(v) for v in args.rates.split(",")]:
        n = args.requests
        arr = inputs.poisson_arrivals(n, rate, 40)
        sizes = inputs.geometric_sizes(n, 0.25, 1, 32, 41)
        lv = inputs.choice(n, levels, 42)
        tg = inputs.choice(n, [1e-6, 1e-7, 3.1e-8], 43)
        cts = []
        for k in range(n):
            X = np.stack([inputs.log_uniform(ctx.n, 2.0 ** -10, 1.0, 7000 + 64 * k + j)
                          for j in range(int(sizes[k]))])
            cts.append(ctx.encrypt_batch(X, lv[k], 2.0 ** 50, 90000 + 64 * k))
        ctx.sync()
        res = {}
        # every mode runs twice on the same ciphertexts; the first pass warms
        # the device memory pool and is not reported
        for mode in ("continuous", "one_at_a_time"):
            for rep in range(2):
                reqs = [Request(k, float(arr[k]), cts[k], lv[k], tg[k]) for k in range(n)]
                if mode == "continuous":
                    srv = run_continuous(ctx, table, reqs, max_batch=args.max_batch)
                    s = summarize(reqs)
                    s["mean_batch"] = float(np.mean([e["batch"] for e in srv.log]))
                else:
                    run_one_at_a_time(ctx, table, reqs)
                    s = summarize(reqs)
                del reqs
            res[mode] = s
        del cts
        res["rate_per_s"] = rate
        res["throughput_gain"] = res["continuous"]["ciphertexts_per_s"] / res["one_at_a_time"]["ciphertexts_per_s"]
        out["runs"].append(res)
        print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f)
    ctx.close()


if __name__ == "__main__":
    main()
