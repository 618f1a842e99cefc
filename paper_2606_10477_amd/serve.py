"""Serving loop for encrypted inverse square roots with continuous batching.

Requests arrive over time; each carries 1..32 ciphertexts at one input level
and an MRE target, which the tuning table maps to a (degree, Pre-BTS
indicator c, iterations) setting.  The server runs on one or more lanes: a
lane is a library context (the same parameter set and keys) on a HIP stream
of its own, all streams at the default priority.  A group -- admitted
ciphertexts that share (level, degree, c, iterations), up to `max_batch`,
oldest request first -- is issued on an idle lane as one batched launch
sequence and runs on the device while the host keeps scheduling: requests
that arrive meanwhile are admitted and their groups start on another lane,
so work from different requests overlaps on the GPU.  Completion is polled
without blocking (ckks_stream_done); a request's latency runs from its
arrival to the device completion of its last group (device events on the
lane's stream).

Admission follows the library's own memory figures (ckks_mem_info): a
request is admitted while its estimated working set, together with that of
admitted requests not yet issued, fits the GPU's free memory plus the lanes'
cached pool blocks, less a reserve.  The working set per ciphertext and
level starts from a multiple of the ciphertext's size and is replaced by the
measured pool high-water mark of issued groups.

Every ciphertext's result is the same alone and in the mix: batch members
never interact and every lane computes the same words.  The baseline ("one
at a time") serves requests strictly in arrival order on one lane, each
request's ciphertexts in one batched call, synchronously.
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
    run_level: int = None   # the level the ciphertexts are dropped to before the chain (route())
    admitted: float = None
    done: float = None
    issued: int = 0         # ciphertexts handed to groups so far


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


def _entry_time(table, level, target):
    """Measured (else predicted) seconds of the table's own entry for
    (level, target), or None when the level has no such entry."""
    ent = table.get(str(level), {}).get(f"{target:.3g}")
    if not ent:
        return None
    return ent.get("t_meas", ent.get("t_pred"))


def route(table, level, target, tol=0.02):
    """(run level, degree, c, iters) of a request: its tuned setting, run at
    the lowest tuned level not above `level` whose own table entry for
    `target` is the same setting at no more than (1 + tol) times the
    measured time of the entry it came from (dropping limbs from a
    ciphertext costs no level budget the setting needs: the table says the
    lower level reaches the target as fast).  Requests that meet at one run
    level and setting share launches.  The choice depends only on the table
    and the request, so a request's result is the same alone or in a mix.
    Tables without times (no t_meas / t_pred) route nothing."""
    d, c, i = lookup(table, level, target)
    t = _entry_time(table, level, target)
    if t is None:
        return level, d, c, i
    for low in sorted(int(k) for k in table):
        if low >= level:
            break
        tl = _entry_time(table, low, target)
        if tl is not None and tl <= t * (1.0 + tol) and lookup(table, low, target) == (d, c, i):
            return low, d, c, i
    return level, d, c, i


class Lane:
    """A context on a stream of its own.  With a torch stream, device events
    time each group's completion; without one (tests), the host clock at the
    poll that sees it finished does."""

    def __init__(self, ctx, stream=None):
        self.ctx = ctx
        self.stream = stream
        self.group = None          # (key, [(request, ct index)], outs, end event, issue time)
        self.t0 = None

    def start_clock(self):
        if self.stream is not None:
            import torch
            self.t0 = torch.cuda.Event(enable_timing=True)
            self.t0.record(self.stream)

    def issue(self, key, work, lo, hi, now):
        cts = [r.cts[k] if r.cts[k].level == key[0] else self.ctx.drop_level(r.cts[k], key[0]) for r, k in work]
        outs = self.ctx.invsqrt_batch(cts, key[1], key[3], a=lo, b=hi, pre_bts=bool(key[2]))
        end = None
        if self.stream is not None:
            import torch
            end = torch.cuda.Event(enable_timing=True)
            end.record(self.stream)
        self.group = (key, work, outs, end, now)

    def finished(self):
        return self.group is not None and self.ctx.stream_done()

    def done_time(self, now):
        end = self.group[3]
        if end is None or self.t0 is None:
            return now
        return self.t0.elapsed_time(end) / 1e3


class Server:
    def __init__(self, lanes, table, max_batch=64, reserve_bytes=1 << 30, ct_factor=24, lo=2.0 ** -10, hi=1.0):
        self.lanes = [ln if isinstance(ln, Lane) else Lane(ln) for ln in (lanes if isinstance(lanes, list)
                                                                           else [lanes])]
        self.table = table
        self.max_batch = max_batch
        self.lo, self.hi = lo, hi
        self.reserve = reserve_bytes
        self.ct_factor = ct_factor       # first working-set estimate: a multiple of one input ciphertext
        self.ct_bytes = self.lanes[0].ctx.mem_info()["ct_bytes"]
        self.ws = {}                     # level -> measured working set per ciphertext (bytes)
        self.queue = []                  # arrived, not admitted
        self.active = []                 # admitted, not finished
        self.log = []
        self.max_in_flight = 0
        self.last_finished = 0

    def est_bytes(self, req, n=None):
        n = len(req.cts) if n is None else n
        lv = req.run_level if req.run_level is not None else req.level
        per = self.ws.get(lv, self.ct_factor * self.ct_bytes[lv])
        return n * per

    def available(self):
        info = [ln.ctx.mem_info() for ln in self.lanes]
        return info[0]["device_free"] + sum(i["pool_cached"] for i in info) - self.reserve

    def submit(self, req):
        req.run_level, req.degree, req.c, req.iters = route(self.table, req.level, req.target)
        self.queue.append(req)

    def _admit(self, now):
        if not self.queue:
            return
        pending = sum(self.est_bytes(r, len(r.cts) - r.issued) for r in self.active)
        room = self.available() - pending
        still = []
        for r in self.queue:
            need = self.est_bytes(r)
            if need <= room or not self.active:
                room -= need
                r.admitted = now
                self.active.append(r)
            else:
                still.append(r)
        self.queue = still

    def _next_group(self):
        """The oldest admitted request with ciphertexts not yet issued sets
        the group key; its and later requests' ciphertexts of the same key
        fill the group up to max_batch."""
        cand = [r for r in sorted(self.active, key=lambda r: r.arrival) if r.issued < len(r.cts)]
        if not cand:
            return None, []
        key = (cand[0].run_level, cand[0].degree, cand[0].c, cand[0].iters)
        work = []
        for r in cand:
            if (r.run_level, r.degree, r.c, r.iters) != key:
                continue
            while r.issued < len(r.cts) and len(work) < self.max_batch:
                work.append((r, r.issued))
                r.issued += 1
        return key, work

    def _finish(self, lane, now):
        key, work, outs, _, _ = lane.group
        t = lane.done_time(now)
        for (r, k), y in zip(work, outs):
            r.outs[k] = y
        finished = [r for r in self.active if len(r.outs) == len(r.cts)]
        for r in finished:
            r.done = t
            self.active.remove(r)
        self.log.append({"t": t, "group": key, "batch": len(work), "lane": self.lanes.index(lane),
                         "finished": [r.rid for r in finished]})
        lane.group = None

    def step(self, clock):
        """One scheduling round: collect finished groups, admit arrivals by
        memory, issue a group on every idle lane.  Returns the number of
        ciphertexts issued (last_finished: the number collected)."""
        moved = 0
        self.last_finished = 0
        for ln in self.lanes:
            if ln.finished():
                self.last_finished += len(ln.group[1])
                self._finish(ln, clock())
        self._admit(clock())
        for ln in self.lanes:
            if ln.group is not None:
                continue
            key, work = self._next_group()
            if not work:
                break
            before = ln.ctx.mem_info(reset_peak=True)["pool_in_use"]
            ln.issue(key, work, self.lo, self.hi, clock())
            peak = ln.ctx.mem_info()["pool_peak"]
            # working set of the group's temporaries per ciphertext (its outputs stay allocated too)
            per = max(0, peak - before) / len(work)
            self.ws[key[0]] = max(self.ws.get(key[0], 0), per)
            moved += len(work)
        self.max_in_flight = max(self.max_in_flight, sum(1 for ln in self.lanes if ln.group is not None))
        return moved

    def busy(self):
        return bool(self.queue or self.active or any(ln.group is not None for ln in self.lanes))


def run_continuous(lanes, table, requests, max_batch=64, reserve_bytes=1 << 30, poll_s=2e-4):
    """Serve `requests` (arrival times relative to start) with continuous
    batching on `lanes` (contexts, or Lane objects with their streams);
    returns the server (requests carry admitted/done times)."""
    srv = Server(lanes, table, max_batch=max_batch, reserve_bytes=reserve_bytes)
    pending = sorted(requests, key=lambda r: r.arrival)
    for ln in srv.lanes:
        ln.start_clock()
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    i = 0
    while i < len(pending) or srv.busy():
        now = clock()
        while i < len(pending) and pending[i].arrival <= now:
            srv.submit(pending[i])
            i += 1
        if srv.step(clock) or srv.last_finished:
            continue
        # nothing issued or finished: wait for the next arrival or poll again
        nxt = pending[i].arrival - clock() if i < len(pending) else poll_s
        time.sleep(max(0.0, min(poll_s, nxt)) if srv.busy() else max(0.0, nxt))
    return srv


def run_one_at_a_time(ctx, table, requests, lo=2.0 ** -10, hi=1.0):
    """Baseline: requests in arrival order, one at a time (each request's
    ciphertexts in one batched call)."""
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    for r in sorted(requests, key=lambda r: r.arrival):
        r.run_level, r.degree, r.c, r.iters = route(table, r.level, r.target)
        wait = r.arrival - clock()
        if wait > 0:
            time.sleep(wait)
        r.admitted = clock()
        cts = [c if c.level == r.run_level else ctx.drop_level(c, r.run_level) for c in r.cts]
        outs = ctx.invsqrt_batch(cts, r.degree, r.iters, a=lo, b=hi, pre_bts=bool(r.c))
        ctx.sync()
        r.outs = dict(enumerate(outs))
        r.done = clock()
    return requests


def run_fixed_single(ctx, requests, degree=31, iters=3, lo=2.0 ** -10, hi=1.0):
    """The plain fixed-configuration single-ciphertext form: every ciphertext
    of every request in arrival order through CryptoInvSqrt (degree, iters)
    with lazy bootstrapping, one ciphertext per call, from its own level."""
    t0 = time.perf_counter()
    clock = lambda: time.perf_counter() - t0
    for r in sorted(requests, key=lambda r: r.arrival):
        r.run_level, r.degree, r.c, r.iters = r.level, degree, 0, iters
        wait = r.arrival - clock()
        if wait > 0:
            time.sleep(wait)
        r.admitted = clock()
        r.outs = {k: ctx.invsqrt(c, degree, iters, a=lo, b=hi) for k, c in enumerate(r.cts)}
        ctx.sync()
        r.done = clock()
    return requests


def fixed_meets_target(table_rows, level, target, degree=31, iters=3):
    """Whether the tuning rows' measured MRE of (degree, 0, iters) at `level`
    meets `target` (None when the rows do not hold that setting)."""
    for row in table_rows or []:
        if row.get("ok") and row["level"] == level and row["d"] == degree and row["i"] == iters and row["c"] == 0:
            return row["m"] <= target
    return None


def summarize(requests):
    lat = np.array([r.done - r.arrival for r in requests])
    n_ct = sum(len(r.cts) for r in requests)
    span = max(r.done for r in requests) - min(r.arrival for r in requests)
    return {"requests": len(requests), "ciphertexts": int(n_ct),
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean()), "ciphertexts_per_s": n_ct / span, "span_s": span}


DEFAULT_TABLE = {"8": {"1e-06": {"degree": 31, "c": 0, "iters": 3}, "1e-07": {"degree": 31, "c": 0, "iters": 3},
                       "3.1e-08": {"degree": 31, "c": 0, "iters": 3}}}


def make_lanes(n, keys_seed=9, params="p16b"):
    """n contexts of one parameter set with the same keys (the same seed),
    each on a torch stream of its own at the default priority."""
    import torch

    from . import ckks
    lanes = []
    for _ in range(n):
        s = torch.cuda.Stream()
        ctx = ckks.Context.from_set(params, stream=s.cuda_stream)
        ctx.keygen(keys_seed, ctx.bts_galois())
        lanes.append(Lane(ctx, s))
    return lanes


def main(argv=None):
    """Serving sweep at N = 2^16 on a bootstrapping parameter set (relin,
    rotation and conjugation keys resident): Poisson arrivals at each rate,
    request sizes Geometric(0.25) truncated to [1, 32], levels in [5, 8] (in
    [5, 11] on the 11-level set) and MRE targets drawn per request; continuous batching on several lanes
    versus one request at a time (tuned settings), and versus the plain
    fixed configuration (31, 3) one ciphertext per call."""
    import argparse
    import json
    import sys

    import torch

    from . import inputs, tuner

    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="10,40,160")
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--params", choices=["p16b", "p16c"], default="p16b",
                    help="bootstrapping set: p16b (8 computation levels, dnum 3) or p16c (11, dnum 6)")
    ap.add_argument("--levels", default=None,
                    help="input levels (those the tuning table can serve; default 5-8 on p16b, 5-11 on p16c)")
    ap.add_argument("--table", default=None,
                    help="tuning JSON from paper_2606_10477_amd.tune (default: the committed table of the set)")
    ap.add_argument("--max-batch", type=int, default=16,
                    help="ciphertexts per launch sequence (bootstrapping throughput saturates near 8-16)")
    ap.add_argument("--lanes", type=int, default=2, help="contexts on streams of their own")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    here = os.path.dirname(os.path.abspath(__file__))
    if args.table is None:
        args.table = os.path.join(here, {"p16b": "tuning_mi355x_bts.json", "p16c": "tuning_mi355x_bts11.json"}[args.params])
    if args.levels is None:
        args.levels = {"p16b": "5,6,7,8", "p16c": "5,6,7,8,9,10,11"}[args.params]
    torch.cuda.set_device(0)
    table, key_note, rows = DEFAULT_TABLE, "no table: the fixed (31, 0, 3) for every request", None
    if args.table and os.path.exists(args.table):
        with open(args.table) as f:
            rep = json.load(f)
        table, rows = rep["table"], rep.get("rows")
        problem = tuner.check_table_key(rep.get("key"), tuner.table_key(args.params))
        if problem and problem[0] == "error":
            raise SystemExit(problem[1])
        key_note = problem[1] if problem else "table key matches this GPU, parameter set and library"
        if problem:
            print(key_note, file=sys.stderr, flush=True)
    lanes = make_lanes(args.lanes, params=args.params)
    ctx = lanes[0].ctx
    levels = [int(v) for v in args.levels.split(",")]
    out = {"workload": f"CryptoInvSqrt serving at N=2^16 (set {args.params}) with bootstrapping keys resident, "
                       "Poisson arrivals, "
                       f"sizes Geometric(0.25) in [1,32], levels {levels}, targets 1e-6/1e-7/3.1e-8",
           "table": args.table, "table_key": key_note, "lanes": args.lanes, "runs": []}
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
        # the device memory pools and is not reported
        for mode in ("continuous", "one_at_a_time", "fixed_single"):
            for rep in range(2):
                reqs = [Request(k, float(arr[k]), cts[k], lv[k], tg[k]) for k in range(n)]
                if mode == "continuous":
                    srv = run_continuous(lanes, table, reqs, max_batch=args.max_batch)
                    s = summarize(reqs)
                    s["mean_batch"] = float(np.mean([e["batch"] for e in srv.log]))
                    s["max_groups_in_flight"] = srv.max_in_flight
                    s["working_set_per_ct_mib"] = {str(k): round(v / 2 ** 20, 1) for k, v in sorted(srv.ws.items())}
                elif mode == "one_at_a_time":
                    run_one_at_a_time(ctx, table, reqs)
                    s = summarize(reqs)
                else:
                    run_fixed_single(ctx, reqs)
                    s = summarize(reqs)
                    meets = [fixed_meets_target(rows, r.level, r.target) for r in reqs]
                    s["requests_meeting_target"] = (sum(1 for m in meets if m) if all(m is not None for m in meets)
                                                    else None)
                del reqs
            res[mode] = s
        del cts
        res["rate_per_s"] = rate
        res["throughput_gain"] = res["continuous"]["ciphertexts_per_s"] / res["one_at_a_time"]["ciphertexts_per_s"]
        res["gain_vs_fixed_single"] = (res["continuous"]["ciphertexts_per_s"]
                                       / res["fixed_single"]["ciphertexts_per_s"])
        out["runs"].append(res)
        print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f)
    for ln in lanes:
        ln.ctx.close()


if __name__ == "__main__":
    main()
