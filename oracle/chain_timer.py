"""Time the oracle on the benchmark's workload (test infrastructure: run only
by the CPU-baseline leg of the benchmark).

The whole CryptoInvSqrt chain (Chebyshev degree d, i Newton steps,
bootstrapping whenever levels run out) at N = 2^16 on the bootstrapping
parameter set "p16b", with the benchmark's seeds (keys 9, input i + 1,
encryption i + 3 for ciphertext i).  Set-up (keys, bootstrapping
configuration, encryption) is not timed.

Phase 1: ciphertext 0 on one core; its result words' SHA-256 ([2][level+1][N],
uint64 little endian) lets the benchmark compare the GPU's result.
Phase 2 (with --procs P > 1): P independent ciphertexts in P forked
processes (keys shared copy-on-write), for an all-core throughput; with
--wait-go it starts only after a line arrives on stdin, so that it does not
compete with GPU timing.  Prints one JSON line.

    python -m oracle.chain_timer --level 8 --degree 31 --iters 3 --procs 16

With --per-op it times the chain's single operations on one core instead
(products at three levels, a rotation, a rescale, each bootstrapping step):

    python -m oracle.chain_timer --per-op
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

LO, HI = 2.0 ** -10, 1.0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def one(o, O, inputs, args, i):
    x = inputs.log_uniform(o.n, LO, HI, 1 + i)
    ct = o.encrypt(x, args.level, 2.0 ** 50, 3 + i)
    t1 = time.perf_counter()
    y = o.invsqrt(ct, args.degree, args.iters, LO, HI)
    dt = time.perf_counter() - t1
    ref = 1 / np.sqrt(x)
    mre = float(np.mean(np.abs(o.decrypt(y).real - ref) / ref))
    sha = hashlib.sha256(np.ascontiguousarray(y.words(), dtype="<u8").tobytes()).hexdigest()
    return {"seconds": dt, "mre": mre, "level": y.level, "scale": float(y.scale).hex(), "sha256": sha}


def per_op(o, inputs):
    """Single-core seconds of the chain's operations on the same set: the
    product with relinearisation and rescale at the top, middle and bottom
    computation levels, a rotation, a rescale, and each bootstrapping step."""
    x = inputs.log_uniform(o.n, LO, HI, 1)
    out = {}

    def tm(name, f):
        t0 = time.perf_counter()
        r = f()
        out[name] = time.perf_counter() - t0
        print(f"{name}: {out[name]:.3f} s", file=sys.stderr, flush=True)
        return r
    top = o.encrypt(x, o.l_after, 2.0 ** 50, 3)
    for lv in (o.l_after, 4, 1):
        c = o.level_to(top, lv) if lv != o.l_after else top
        tm(f"mult_relin_rescale@{lv}", lambda c=c: o.mult_rs(c, c))
    tm(f"rotate@{o.l_after}", lambda: o.rotate(top, 1))
    tm(f"rescale@{o.l_after}", lambda: o.rescale(o.mul_int(top, 3)))
    y0 = o.invsqrt(top, 31, 0, LO, HI)
    r = tm("mod_raise", lambda: o.mod_raise(o.drop_level(y0, 0)))
    y = tm("coeff_to_slot", lambda: o.coeff_to_slot(r))
    e = tm("eval_mod", lambda: o.eval_mod(o.add(y, o.conjugate(y))))
    tm("slot_to_coeff", lambda: o.slot_to_coeff(e))
    tm("bootstrap", lambda: o.bootstrap(y0, 512))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--level", type=int, default=8)
    ap.add_argument("--degree", type=int, default=31)
    ap.add_argument("--iters", type=int, default=3)
    ap.add_argument("--procs", type=int, default=1, help="processes of the all-core phase (1: skip it)")
    ap.add_argument("--wait-go", action="store_true", help="start the all-core phase on a line from stdin")
    ap.add_argument("--per-op", action="store_true", help="time the chain's single operations instead")
    args = ap.parse_args()
    from oracle import oracle as O
    from paper_2606_10477_amd import inputs
    t0 = time.perf_counter()
    o = O.Context.from_set("p16b")
    o.keygen(9, o.bts_galois())
    t_setup = time.perf_counter() - t0
    if args.per_op:
        print(json.dumps({"per_op_seconds": per_op(o, inputs), "setup_seconds": t_setup, "cores": 1,
                          "cpu_model": cpu_model(), "nproc": os.cpu_count()}), flush=True)
        return
    res = one(o, O, inputs, args, 0)
    res.update({"setup_seconds": t_setup, "cores": 1, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                "affinity": len(os.sched_getaffinity(0))})
    if args.procs > 1:
        if args.wait_go:
            sys.stdin.readline()
        pipes = []
        t2 = time.perf_counter()
        for i in range(args.procs):
            r, w = os.pipe()
            pid = os.fork()
            if pid == 0:                      # child: one ciphertext, result on the pipe
                os.close(r)
                try:
                    out = json.dumps(one(o, O, inputs, args, 100 + i)).encode()
                except Exception as e:        # noqa: BLE001 - reported to the parent
                    out = json.dumps({"error": str(e)}).encode()
                os.write(w, out)
                os.close(w)
                os._exit(0)
            os.close(w)
            pipes.append((pid, r))
        done = []
        for pid, r in pipes:
            buf = b""
            while True:
                chunk = os.read(r, 65536)
                if not chunk:
                    break
                buf += chunk
            os.close(r)
            os.waitpid(pid, 0)
            done.append(json.loads(buf.decode()))
        wall = time.perf_counter() - t2
        ok = [d for d in done if "error" not in d]
        res["allcore"] = {"procs": args.procs, "completed": len(ok), "wall_seconds": wall,
                          "ciphertexts_per_s": len(ok) / wall,
                          "per_ct_seconds_mean": float(np.mean([d["seconds"] for d in ok])) if ok else None,
                          "mre_max": max(d["mre"] for d in ok) if ok else None}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
