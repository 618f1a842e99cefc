"""Benchmark: encrypted inverse square roots per second at N = 2^16.

One step = CryptoInvSqrt (paper Alg. 1: Chebyshev initial value, Newton
steps, bootstrapping whenever levels run out) of the fixed configuration
(degree 31, 3 Newton steps) on one ciphertext (--batch: several, as one
batched launch sequence) already resident in HBM, on the 128-bit parameter
set with bootstrapping "p16b" (log2 QP ~ 1544, dnum 3, h 192): from the top
computation level 8 the chain bootstraps once.  Prints one JSON line: value =
ciphertexts/s for the whole job, the roofline of the dominant kernel family
measured live with HIP events on the library's stream, the MRE of the result
against FP64, the same chain batched (ciphertexts/s at --extra-batch), the
CPU oracle timed on a bounded sample (one ciphertext on one core, then one
ciphertext per process on all cores after the GPU work), and whether the
GPU's result words equal the oracle's.  Beside it ("tuned_11_levels"): the
tuned form on the bootstrapping set with 11 computation levels ("p16c", dnum
6), the (degree, c, iterations) its committed tuning table picks for
3.1e-8 at the top level, one ciphertext per step and batched, with its MRE.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
PARAMS = "p16b"
LO, HI = 2.0 ** -10, 1.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=1, help="ciphertexts per step")
    ap.add_argument("--degree", type=int, default=31)
    ap.add_argument("--iters", type=int, default=3)
    ap.add_argument("--level", type=int, default=8, help="input level")
    ap.add_argument("--extra-batch", type=int, default=16, help="also time this many ciphertexts per step (0: skip)")
    ap.add_argument("--latency-runs", type=int, default=20, help="single-ciphertext runs timed one by one (p50/p99)")
    ap.add_argument("--graph-runs", type=int, default=10,
                    help="replays of the one-ciphertext chain captured as a HIP graph, against as many eager runs "
                         "(0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tuned-11", dest="tuned_11", action="store_false",
                    help="skip the tuned form on the 11-level set")
    ap.add_argument("--cpu-limit", type=int, default=480,
                    help="seconds after the start the CPU baseline may run until")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="processes of the all-core CPU phase (0: the CPUs this process may use, at most 16)")
    return ap.parse_args()


def start_cpu_baseline(args):
    """Start the oracle on the same chain in a child process (plain CPU; it
    never touches the GPU), before this process initialises the GPU, so that
    its set-up and its one-core run go alongside the GPU timing; its
    all-core phase waits for a line on stdin (sent when the GPU work ends)."""
    procs = args.cpu_procs or min(16, len(os.sched_getaffinity(0)))
    cmd = [sys.executable, "-m", "oracle.chain_timer", "--level", str(args.level), "--degree", str(args.degree),
           "--iters", str(args.iters), "--procs", str(procs), "--wait-go"]
    env = dict(os.environ, OMP_NUM_THREADS="1")
    return subprocess.Popen(cmd, cwd=ROOT, stdin=subprocess.PIPE, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                            text=True, env=env)


def finish_cpu_baseline(proc, args, limit_s):
    """(cpu_baseline dict, the oracle's one-core result record or None)."""
    try:
        proc.stdin.write("go\n")
        proc.stdin.flush()
    except OSError:
        pass
    try:
        out, err = proc.communicate(timeout=limit_s)
    except subprocess.TimeoutExpired:
        proc.kill()
        proc.communicate()
        return {"value": None, "unit": "ciphertexts/s", "cores": None, "kind": "oracle",
                "sample": f"oracle did not finish within the time limit ({limit_s:.0f} s left at the end of the GPU run)"}, None
    if proc.returncode != 0:
        return {"value": None, "unit": "ciphertexts/s", "cores": None, "kind": "oracle",
                "sample": "oracle failed: " + err.strip()[-200:]}, None
    r = json.loads(out.strip().splitlines()[-1])
    chain = (f"the same chain (degree {args.degree}, {args.iters} Newton steps, bootstrapping when levels run "
             f"out) at N=2^16 from level {args.level}")
    single = {"value": round(1.0 / r["seconds"], 6), "cores": 1, "seconds": round(r["seconds"], 2),
              "mre": r["mre"]}
    base = {"unit": "ciphertexts/s", "kind": "oracle", "cpu_model": r["cpu_model"], "nproc": r["nproc"],
            "affinity": r["affinity"], "setup_seconds": round(r["setup_seconds"], 1), "single_core": single}
    a = r.get("allcore")
    if a and a["completed"]:
        base.update({"value": round(a["ciphertexts_per_s"], 6), "cores": a["procs"],
                     "sample": f"{a['completed']} ciphertexts through {chain}, one per process on {a['procs']} "
                               f"processes (keys shared copy-on-write after one set-up, not timed), after the GPU "
                               f"work: {a['wall_seconds']:.1f} s wall, {a['per_ct_seconds_mean']:.1f} s per "
                               f"ciphertext; one ciphertext alone on one core: {r['seconds']:.1f} s"})
    else:
        base.update({"value": single["value"], "cores": 1,
                     "sample": f"1 ciphertext through {chain}, single-threaded: {r['seconds']:.1f} s "
                               f"(set-up {r['setup_seconds']:.0f} s not timed)"})
    return base, r


def copy_gbps(torch, mib=512, reps=5):
    """Practical HBM ceiling: a plain device-to-device copy of `mib` MiB (read
    + write bytes over the median of `reps` copies, timed with HIP events)."""
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    del src, dst
    return 2 * n / sorted(ts)[len(ts) // 2] / 1e9


def ntt_traffic(alg_bytes_per_launch):
    """Measured HBM bytes per NTT launch (FETCH_SIZE + WRITE_SIZE counter runs,
    scaled by a plain copy's counters, stored by traffic_record.py) at the
    average size of this run's launches; None when the NTT kernels changed
    since the counters were taken."""
    from paper_2606_10477_amd import traffic_record
    try:
        with open(traffic_record.RECORD) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("kernels_hip_sha256") != traffic_record.kernels_sha256():
        return None
    return round(rec["ratio_to_algorithmic"] * alg_bytes_per_launch)


def tuned_11_levels(args, ckks, inputs):
    """The tuned configuration on the 11-level set, timed like the fixed one
    (inputs resident, `steps` steps after a warm-up; then --extra-batch per
    step).  None when the tuning table is absent."""
    path = os.path.join(ROOT, "paper_2606_10477_amd", "tuning_mi355x_bts11.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rep = json.load(f)
    top = max(int(l) for l in rep["table"])
    pick = rep["table"][str(top)].get("3.1e-08")
    if pick is None:
        return None
    d, c, it = pick["degree"], pick["c"], pick["iters"]
    ctx = ckks.Context.from_set("p16c")
    try:
        ctx.keygen(9, ctx.bts_galois() if (pick["bts"] or c) else [])
        nmax = max(1, args.extra_batch)
        xs = [inputs.log_uniform(ctx.n, LO, HI, 1 + i) for i in range(nmax)]
        cts = ctx.encrypt_batch(np.stack(xs), top, 2.0 ** 50, 3)

        def step(B):
            if B == 1:
                return [ctx.invsqrt(cts[0], d, it, a=LO, b=HI, pre_bts=bool(c))]
            return ctx.invsqrt_batch(cts[:B], d, it, a=LO, b=HI, pre_bts=bool(c))

        for _ in range(max(1, args.warmup)):
            step(1)
        ctx.sync()
        ctx.trace(True)
        out = step(1)
        n_bts = sum(1 for op in ctx.trace_read() if op[0] == "bootstrap")
        ctx.trace(False)
        ctx.sync()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = step(1)
        ctx.sync()
        dt = time.perf_counter() - t0
        ref = 1 / np.sqrt(xs[0])
        mre = float(np.mean(np.abs(ctx.decrypt(out[0]).real - ref) / ref))
        lat = []
        for _ in range(args.latency_runs):
            t1 = time.perf_counter()
            o1 = step(1)
            ctx.sync()
            lat.append(1e3 * (time.perf_counter() - t1))
            del o1
        graph = None
        if args.graph_runs > 0:
            # the chain without a bootstrap is short (a few hundred launches): replayed as one HIP
            # graph, against eager runs, with the replay's words checked against eager's
            ref_words = step(1)[0].words()
            gr = ctx.invsqrt_graph(cts[0], d, it, a=LO, b=HI, pre_bts=bool(c))
            same = bool(np.array_equal(gr.run(cts[0]).words(), ref_words))
            ctx.sync()
            t1 = time.perf_counter()
            for _ in range(args.graph_runs):
                o1 = gr.run(cts[0])
                del o1
            ctx.sync()
            tg = (time.perf_counter() - t1) / args.graph_runs
            same = same and bool(np.array_equal(gr.run(cts[0]).words(), ref_words))
            gr.close()
            graph = {"runs": args.graph_runs, "replay_ms": round(tg * 1e3, 3), "replay_equals_eager": same}
        res = {"params": "p16c: " + ckks_params_about("p16c"), "input_level": top, "graph": graph,
               "degree": d, "c": c, "iters": it, "bootstraps_per_ct": n_bts, "mre": mre,
               "ciphertexts_per_s": round(args.steps / dt, 3), "ms_per_step": round(dt * 1e3 / args.steps, 3),
               "latency": {"runs": len(lat), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                           "p99_ms": round(float(np.percentile(lat, 99)), 3)} if lat else None,
               "table": os.path.basename(path)}
        if args.extra_batch > 1:
            step(args.extra_batch)
            ctx.sync()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                ob = step(args.extra_batch)
                del ob
            ctx.sync()
            dtb = time.perf_counter() - t1
            res["batched"] = {"batch": args.extra_batch,
                              "ciphertexts_per_s": round(args.extra_batch * args.steps / dtb, 3),
                              "ms_per_step": round(dtb * 1e3 / args.steps, 3)}
        return res
    finally:
        ctx.close()


def ckks_params_about(name):
    from paper_2606_10477_amd import params
    return params.load(name)["about"]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    t_start = time.perf_counter()
    cpu_proc = None if args.no_cpu_baseline else start_cpu_baseline(args)
    import torch
    from paper_2606_10477_amd import ckks, inputs

    torch.cuda.set_device(0)
    ctx = ckks.Context.from_set(PARAMS)
    ctx.keygen(9, ctx.bts_galois())
    nmax = max(args.batch, args.extra_batch)
    xs = [inputs.log_uniform(ctx.n, LO, HI, 1 + i) for i in range(nmax)]
    cts = ctx.encrypt_batch(np.stack(xs), args.level, 2.0 ** 50, 3)
    ctx.sync()

    def step(B):
        if B == 1:
            return [ctx.invsqrt(cts[0], args.degree, args.iters, a=LO, b=HI)]
        return ctx.invsqrt_batch(cts[:B], args.degree, args.iters, a=LO, b=HI)

    for _ in range(args.warmup):
        out = step(args.batch)
        del out
    ctx.sync()
    torch.cuda.synchronize()
    ctx.trace(True)
    out = step(args.batch)
    n_bts = sum(1 for op in ctx.trace_read() if op[0] == "bootstrap")
    ctx.trace(False)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step(args.batch)
    ctx.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # kernel-family timing: HIP events around every NTT / key-switch call on
    # the library's stream, over a second pass of the same steps (the events
    # add gaps between kernels, so the throughput above is taken without them)
    print(f"timed {args.steps} steps: {dt * 1e3 / args.steps:.2f} ms per step", file=sys.stderr, flush=True)
    ctx.profile(True)
    for _ in range(args.steps):
        out_p = step(args.batch)
        del out_p
    ctx.sync()
    fam = {}
    for name in ("ntt", "keyswitch"):
        n, ms, by = ctx.profile_read(name)
        fam[name] = (n, ms, by)
    ctx.profile(False)
    print("kernel-family timing done", file=sys.stderr, flush=True)
    # single-ciphertext latency: each run synchronised on its own
    lat = []
    for _ in range(args.latency_runs):
        t1 = time.perf_counter()
        o1 = step(1)
        ctx.sync()
        lat.append(1e3 * (time.perf_counter() - t1))
        del o1
    latency = None
    if lat:
        latency = {"runs": len(lat), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                   "p99_ms": round(float(np.percentile(lat, 99)), 3)}
    # the one-ciphertext chain captured as a HIP graph: replay time against
    # eager runs of the same chain, and the replay's words against eager's
    graph = None
    if args.graph_runs > 0:
        ref_words = step(1)[0].words()
        gr = ctx.invsqrt_graph(cts[0], args.degree, args.iters, a=LO, b=HI)
        same = bool(np.array_equal(gr.run(cts[0]).words(), ref_words))
        ctx.sync()
        t1 = time.perf_counter()
        for _ in range(args.graph_runs):
            o1 = step(1)
            del o1
        ctx.sync()
        te = (time.perf_counter() - t1) / args.graph_runs
        t1 = time.perf_counter()
        for _ in range(args.graph_runs):
            o1 = gr.run(cts[0])
            del o1
        ctx.sync()
        tg = (time.perf_counter() - t1) / args.graph_runs
        same = same and bool(np.array_equal(gr.run(cts[0]).words(), ref_words))
        gr.close()
        graph = {"runs": args.graph_runs, "eager_ms": round(te * 1e3, 3), "replay_ms": round(tg * 1e3, 3),
                 "replay_equals_eager": same}
    print("latency and graph runs done", file=sys.stderr, flush=True)
    batched = None
    if args.extra_batch > 1:
        out2 = step(args.extra_batch)
        del out2
        ctx.sync()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            out2 = step(args.extra_batch)
        ctx.sync()
        dtb = time.perf_counter() - t1
        batched = {"batch": args.extra_batch, "ciphertexts_per_s": round(args.extra_batch * args.steps / dtb, 3),
                   "ms_per_step": round(dtb * 1e3 / args.steps, 3)}
        del out2

    ref = 1 / np.sqrt(xs[0])
    z = ctx.decrypt(out[0]).real
    mre = float(np.mean(np.abs(z - ref) / ref))
    out_level = out[0].level
    gpu_sha = hashlib.sha256(np.ascontiguousarray(out[0].words(), dtype="<u8").tobytes()).hexdigest()
    gpu_scale = float(out[0].scale).hex()
    logqp = float(sum(np.log2(float(p)) for p in ctx.primes))

    # roofline of the NTT (the metric's kernel and the largest share of kernel
    # time: forward + inverse passes); the key switch is reported beside it
    dom = "ntt"
    n, ms, by = fam[dom]
    achieved = (by / (ms / 1e3)) / 1e9 if ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": ntt_traffic(by / max(n, 1)), "kernel": dom,
            "launches": n, "avg_launch_us": round(ms * 1e3 / max(n, 1), 2),
            "share_of_step": round(ms / 1e3 / dt, 3) if dt > 0 else None,
            "timed_by": "HIP events around each call on the library stream, second pass of the same steps"}
    cg = copy_gbps(torch)
    roof["copy_GBps"] = round(cg, 1)          # measured practical ceiling (512 MiB device copy)
    roof["frac_of_copy"] = round(achieved / cg, 4) if cg > 0 else None
    if roof["traffic"] is not None and ms > 0:
        # measured HBM bytes (counter record) at the same launch times: what the passes really move
        roof["traffic_GBps"] = round(roof["traffic"] * n / (ms / 1e3) / 1e9, 1)
    # algorithmic bytes per ciphertext of each family (the NTT's 16 N per limb;
    # the key switch's input, key once per batch and output), over the profiled pass
    others = {k: {"calls": v[0], "gpu_ms": round(v[1], 3),
                  "GB/s": round((v[2] / (v[1] / 1e3)) / 1e9, 1) if v[1] > 0 else None,
                  "algorithmic_GB_per_ct": round(v[2] / 1e9 / (args.batch * args.steps), 3)}
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
        "config": {"workload": f"CryptoInvSqrt fixed configuration: degree {args.degree}, {args.iters} Newton steps, "
                               f"bootstrapping whenever levels run out ({n_bts} per ciphertext), "
                               f"x log-uniform in [2^-10,1], input level {args.level}",
                   "ring_degree": 65536, "slots": 32768, "batch": args.batch,
                   "params": f"{PARAMS}: log2 QP {logqp:.0f}: q0 60-bit, {ctx.l_after + 3} x 40-bit, "
                             f"{ctx.L - ctx.l_after - 3} x 52-bit (EvalMod/CoeffToSlot), 7 x 60-bit special, "
                             f"dnum 3, h 192; l_afterBTS {ctx.l_after}",
                   "bootstraps_per_ct": n_bts, "output_level": out_level},
        "mre": mre,
        "latency": latency,
        "batched": batched,
        "graph": graph,
        "roofline": roof,
        "kernel_families": others,
    }
    ctx.close()
    if args.tuned_11:
        res["tuned_11_levels"] = tuned_11_levels(args, ckks, inputs)
        if res["tuned_11_levels"]:
            t = res["tuned_11_levels"]
            t["speedup_vs_fixed_c1"] = round(t["ciphertexts_per_s"] / res["value"], 3)
        print("tuned 11-level form done", file=sys.stderr, flush=True)
    if cpu_proc is not None:
        print("waiting for the CPU baseline (oracle, one ciphertext)", file=sys.stderr, flush=True)
        left = max(10.0, args.cpu_limit - (time.perf_counter() - t_start))
        res["cpu_baseline"], orc = finish_cpu_baseline(cpu_proc, args, left)
        if orc is not None and args.batch >= 1:
            res["parity_words_equal"] = bool(orc["sha256"] == gpu_sha and orc["level"] == out_level
                                             and orc["scale"] == gpu_scale)
            res["parity"] = {"what": "SHA-256 of the result words of ciphertext 0, GPU vs the oracle on the same "
                                     "seeds", "gpu": gpu_sha[:16], "oracle": orc["sha256"][:16]}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
