"""Degree-versus-iterations tuner for CryptoInvSqrt (paper §4.2, Alg. 2 and 3).

Host logic of the paper's provisioning step:
  * ``get_opt_iter`` -- Alg. 2 (GetOptIter) after its loop: the threshold
    MRE_delta = (floor(alpha) + delta) 10^l from MRE_min = alpha 10^l, and the
    smallest iteration count whose MRE is within it;
  * ``optimize_params`` -- Alg. 3's final selection per level: m_theta from the
    level's smallest MRE, u1 = fastest tuple with m <= m_theta (accuracy
    first), u2 = fastest tuple overall (speed first);
  * ``level_cases`` -- Alg. 3's enumeration of input levels l_BTS+1..l_max and
    the conditions under which c = 0 (l >= l_BTS + 3) and c = 1
    (l < l_afterBTS - 1) are explored.

On top of these, the cost model used on this GPU: the library records the
operation trace of a run (op, level, batch); each primitive's unit cost is
profiled on the device; the predicted time of a configuration is the sum of
unit costs over its trace.  ``sweep`` measures MRE and time for a grid of
(degree, iterations) at given input levels and ``select`` picks the pair that
meets an MRE target at minimum predicted time.
"""
import math
import time

import numpy as np


# --------------------------------------------------------------------------
# Alg. 2 / Alg. 3 host rules
# --------------------------------------------------------------------------
def mantissa_exponent(m):
    """m = alpha * 10^l with 1 <= alpha < 10 (l = floor(log10 m))."""
    if not (m > 0 and math.isfinite(m)):
        raise ValueError("MRE must be positive and finite")
    l = math.floor(math.log10(m))
    alpha = m / 10.0 ** l
    # log10 rounding at exact powers of ten
    if alpha >= 10.0:
        alpha /= 10.0
        l += 1
    elif alpha < 1.0:
        alpha *= 10.0
        l -= 1
    return alpha, l


def threshold(m_min, delta):
    """(floor(alpha) + delta) * 10^l for m_min = alpha * 10^l."""
    alpha, l = mantissa_exponent(m_min)
    return (math.floor(alpha) + delta) * 10.0 ** l


def get_opt_iter(M, T, delta):
    """Alg. 2 lines 11-16.  M[k], T[k] are the MRE and cumulative time after
    k+1 Newton iterations.  Returns (I, M[I], T[I]) with I counted from 1.
    If no iteration is within the threshold (possible for delta < 1), the
    iteration with the smallest MRE is returned."""
    m_min = min(M)
    thr = threshold(m_min, delta)
    within = [k for k, m in enumerate(M) if m <= thr]
    k = within[0] if within else int(np.argmin(M))
    return k + 1, M[k], T[k]


def _argmin_time(rows):
    # ties: lower MRE, then smaller degree
    return min(rows, key=lambda r: (r["t"], r["m"], r["d"]))


def optimize_params(D, theta):
    """Alg. 3 lines 19-27.  D maps level -> list of dicts with keys d, c, i,
    m, t.  Returns level -> (u1, u2), each a (d, c, i) tuple."""
    R = {}
    for l, rows in D.items():
        if not rows:
            continue
        m_min = min(r["m"] for r in rows)
        m_theta = threshold(m_min, theta)
        u1 = _argmin_time([r for r in rows if r["m"] <= m_theta])
        u2 = _argmin_time(rows)
        R[l] = ((u1["d"], u1["c"], u1["i"]), (u2["d"], u2["c"], u2["i"]))
    return R


def level_cases(l_bts, l_after_bts, l_max):
    """Alg. 3 lines 6-17: for each explored input level, which Pre-BTS
    indicators are tried."""
    out = {}
    for l in range(l_bts + 1, l_max + 1):
        cs = []
        if l >= l_bts + 3:
            cs.append(0)
        if l < l_after_bts - 1:
            cs.append(1)
        out[l] = cs
    return out


def mre(values, ref):
    values = np.asarray(values)
    ref = np.asarray(ref)
    return float(np.mean(np.abs(values - ref) / np.abs(ref)))


# --------------------------------------------------------------------------
# Cost model
# --------------------------------------------------------------------------
OPS = ("hmult", "rescale", "rotate", "mul_scalar", "add", "sub", "add_const", "drop", "copy", "bootstrap",
       "lincomb", "lincomb_term")
BTS_ANY_LEVEL = -1     # a bootstrap costs the same from any input level (it starts at level 0)


def _words(ctx, level, B, seed):
    from . import inputs
    return [inputs.uniform_words((2, level + 1, ctx.N), ctx.primes[:level + 1], seed + b) for b in range(B)]


PIPELINE = 8


def profile_unit_costs(ctx, levels, batch=1, reps=5, rot_step=None, bts_bound=None):
    """Median wall time (s) of each primitive at each level, on `batch`
    ciphertexts of uniform words, per call of PIPELINE calls issued back to
    back and then synchronised.  With bts_bound, also the
    bootstrap (message bound bts_bound), stored under level BTS_ANY_LEVEL."""
    costs = {}
    if bts_bound is not None:
        lvl = min(levels)
        singles = [ctx.ct_import(w, lvl, 2.0 ** 40) for w in _words(ctx, lvl, batch, 2000)]
        a = ctx.pack(singles) if batch > 1 else singles[0]
        ctx.bootstrap(a, bts_bound)
        ctx.sync()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = ctx.bootstrap(a, bts_bound)
            ctx.sync()
            ts.append(time.perf_counter() - t0)
            del r
        costs[("bootstrap", BTS_ANY_LEVEL)] = float(np.median(ts))
    for lvl in levels:
        singles = [ctx.ct_import(w, lvl, 2.0 ** 40) for w in _words(ctx, lvl, batch, 1000 + lvl)]
        a = ctx.pack(singles) if batch > 1 else singles[0]
        fns = {
            "hmult": lambda: ctx.hmult(a, a),
            "mul_scalar": lambda: ctx.mul_int(a, 3),
            "add": lambda: ctx.add(a, a),
            "sub": lambda: ctx.sub(a, a),
            "add_const": lambda: ctx.add_const(a, 0.5),
            "copy": lambda: ctx.drop_level(a, lvl),
        }
        if lvl >= 1:
            fns["rescale"] = lambda: ctx.rescale(a)
            fns["drop"] = lambda: ctx.drop_level(a, lvl - 1)
        if rot_step is not None:
            fns["rotate"] = lambda: ctx.rotate(a, rot_step)
        # products of a Chebyshev wave share one launch sequence (2-4 of them
        # in a batch): profile hmult and rescale at 2x and 4x the batch too
        for m in BATCH_MULTIPLES:
            am = ctx.pack(singles * m)
            fns[f"hmult*{m}"] = (lambda am=am: ctx.hmult(am, am))
            if lvl >= 1:
                fns[f"rescale*{m}"] = (lambda am=am: ctx.rescale(am))
        for op, fn in fns.items():
            fn()
            ctx.sync()
            ts = []
            for _ in range(reps):
                # PIPELINE calls back to back, as ops follow each other in a
                # chain: the GPU queue then hides the host's launch overhead,
                # which a synchronised single call would count in full
                t0 = time.perf_counter()
                for _ in range(PIPELINE):
                    r = fn()
                    del r
                ctx.sync()
                ts.append((time.perf_counter() - t0) / PIPELINE)
            costs[(op, lvl)] = float(np.median(ts))
    derive_lincomb_costs(costs)
    return costs


def derive_lincomb_costs(costs):
    """A fused linear combination (one kernel) is traced as one "lincomb" line
    for its launch and one "lincomb_term" line per further term or sum: the
    launch costs what an integer multiply costs at that level and batch (one
    read, one write), each further term what an addition adds to it (one more
    read)."""
    for (op, lvl), v in list(costs.items()):
        if op == "mul_scalar" and ("add", lvl) in costs:
            costs[("lincomb", lvl)] = v
            costs[("lincomb_term", lvl)] = max(0.0, costs[("add", lvl)] - v)
    return costs


BATCH_MULTIPLES = (2, 4)


def _unit_cost(costs, op, lvl, m):
    """Cost of `op` at `lvl` on m times the profiled batch: piecewise linear
    through the profiled multiples (1, 2, 4), extended linearly; m times the
    single cost when only that was profiled."""
    c1 = costs.get((op, BTS_ANY_LEVEL if op == "bootstrap" else lvl))
    if c1 is None or m <= 1:
        return c1
    pts = [(1, c1)] + [(k, costs[(f"{op}*{k}", lvl)]) for k in BATCH_MULTIPLES if (f"{op}*{k}", lvl) in costs]
    if len(pts) == 1:
        return c1 * m
    for (m0, t0), (m1, t1) in zip(pts, pts[1:]):
        if m <= m1:
            return t0 + (t1 - t0) * (m - m0) / (m1 - m0)
    (m0, t0), (m1, t1) = pts[-2], pts[-1]
    return t1 + (t1 - t0) * (m - m1) / (m1 - m0)


def predict(trace, costs, base_batch=1):
    """Sum of unit costs over an operation trace [(op, level, B), ...] of a run
    on base_batch ciphertexts (an op on B = m base_batch ciphertexts, such as
    a Chebyshev wave's batched products, costs the profiled m-fold batch)."""
    total = 0.0
    missing = set()
    for op, lvl, B in trace:
        c = _unit_cost(costs, op, lvl, max(1, int(B) // max(1, base_batch)))
        if c is None:
            missing.add((op, lvl))
            continue
        total += c
    return total, missing


# --------------------------------------------------------------------------
# Sweep and selection (one MI355X, encrypted runs with the tuner's own keys)
# --------------------------------------------------------------------------
def sweep(ctx, x, ct_by_level, degrees, iters, lo, hi, batch=1, reps=3, costs=None, cs_by_level=None, B=0.0):
    """For each input level, Pre-BTS indicator c (cs_by_level[level], default
    [0]) and (degree, iterations): MRE of the decrypted result against FP64
    1/sqrt(x), measured time (median of `reps`, all `batch` ciphertexts), the
    operation trace (bootstraps counted) and the predicted time.  Settings
    that do not fit the levels are recorded with ok=False.  B > 1: the
    chain pre-normalises x by B homomorphically (x in [lo, hi])."""
    import sys
    ref = 1.0 / np.sqrt(x)
    rows = []
    t0 = time.perf_counter()
    for lvl, ct in ct_by_level.items():
        for c in (cs_by_level or {}).get(lvl, [0]):
            for d in degrees:
                for it in iters:
                    rows.append(_measure(ctx, ct, lvl, c, d, it, lo, hi, batch, reps, costs, ref, B))
            print(f"swept level {lvl}, c = {c}: {len(rows)} settings, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    return rows


def _measure(ctx, ct, lvl, c, d, it, lo, hi, batch, reps, costs, ref, B=0.0):
    from .ckks import CkksError
    cts = [ct] * batch

    def run():
        if batch == 1:
            return ctx.invsqrt(ct, d, it, a=lo, b=hi, pre_bts=bool(c), B=B)
        return ctx.invsqrt_batch(cts, d, it, a=lo, b=hi, pre_bts=bool(c), B=B)[0]

    row = {"level": lvl, "d": d, "i": it, "c": c}
    try:
        ctx.trace(True)
        ctx.sync()
        t0 = time.perf_counter()
        y = run()
        ctx.sync()
        row["t_first_s"] = time.perf_counter() - t0   # the traced run that also yields the MRE
        tr = ctx.trace_read()
        ctx.trace(False)
    except CkksError:
        ctx.trace(False)
        row["ok"] = False
        return row
    row["ok"] = True
    row["m"] = mre(ctx.decrypt(y).real, ref)
    row["out_level"] = y.level
    ts = []
    for _ in range(reps):
        ctx.sync()
        t0 = time.perf_counter()
        run()
        ctx.sync()
        ts.append(time.perf_counter() - t0)
    row["t"] = float(np.median(ts)) / batch
    row["t_timed_s"] = float(np.sum(ts))
    row["ops"] = len(tr)
    row["bts"] = sum(1 for op in tr if op[0] == "bootstrap")
    if costs is not None:
        row["t_pred"] = predict(tr, costs, base_batch=batch)[0]
    return row


def select(rows, target, level, key="t_pred"):
    """The (degree, c, iterations) at `level` with MRE <= target at minimum
    `key` time (ties: lower MRE, fewer bootstraps, smaller degree); None if
    none qualifies."""
    ok = [r for r in rows if r.get("ok") and r["level"] == level and r["m"] <= target and key in r]
    if not ok:
        return None
    return min(ok, key=lambda r: (r[key], r["m"], r.get("bts", 0), r["d"]))


def exploration_report(rows, levels, targets, profile_s):
    """Measured-time exhaustive exploration (every setting timed, as the
    paper's Alg. 3 does) against the cost model (every setting run once for
    its MRE and operation trace; times predicted from the profiled unit
    costs).  Per (level, target): the measured-time pick, the cost-model pick
    and the cost-model pick's regret (its measured time over the measured
    optimum, minus 1); and the GPU seconds each route spends."""
    ok = [r for r in rows if r.get("ok")]
    picks = {}
    regrets = []
    for lvl in levels:
        for tgt in targets:
            rm = select(rows, tgt, lvl, key="t")
            rp = select(rows, tgt, lvl, key="t_pred")
            if rm is None or rp is None:
                picks.setdefault(str(lvl), {})[f"{tgt:.3g}"] = None
                continue
            reg = rp["t"] / rm["t"] - 1.0
            regrets.append(reg)
            picks.setdefault(str(lvl), {})[f"{tgt:.3g}"] = {
                "measured": [rm["d"], rm["c"], rm["i"]], "predicted": [rp["d"], rp["c"], rp["i"]],
                "same": (rm["d"], rm["c"], rm["i"]) == (rp["d"], rp["c"], rp["i"]), "regret": reg}
    first = float(sum(r.get("t_first_s", 0.0) for r in rows))
    timed = float(sum(r.get("t_timed_s", 0.0) for r in ok))
    return {"settings": len(rows), "feasible": len(ok), "picks": picks,
            "max_regret": max(regrets) if regrets else None,
            "measured_exhaustive_s": first + timed, "cost_model_s": first + profile_s,
            "runs_for_mre_s": first, "timing_runs_s": timed, "unit_cost_profile_s": profile_s}


def alg3_from_rows(rows, delta=1.0, theta=1.0, key="t"):
    """Alg. 3's table from sweep rows: for each (level, d, c) the iteration
    curve M[1..i_max], T[1..i_max] (T is the time of the whole run up to that
    iteration), Alg. 2 picks the iteration count, and optimize_params the
    accuracy-first u1 and speed-first u2 per level.  Curves with a missing
    iteration (infeasible settings) are skipped."""
    by = {}
    for r in rows:
        if r.get("ok") and key in r:
            by.setdefault((r["level"], r["d"], r["c"]), {})[r["i"]] = r
    D = {}
    for (lvl, d, c), its in sorted(by.items()):
        n = max(its)
        if sorted(its) != list(range(1, n + 1)):
            continue
        M = [its[i]["m"] for i in range(1, n + 1)]
        T = [its[i][key] for i in range(1, n + 1)]
        I, m, t = get_opt_iter(M, T, delta)
        D.setdefault(lvl, []).append({"d": d, "c": c, "i": I, "m": m, "t": t})
    return D, optimize_params(D, theta)


def table_key(params_name):
    """What a tuning table is valid for: the GPU, the parameter set (name and
    hash of its definition) and the library build it was measured with."""
    import torch

    from . import ckks, params
    return {"gpu": torch.cuda.get_device_name(0), "params": params_name,
            "params_sha256": params.set_sha256(params_name), "library_sha256": ckks.library_sha256()}


def check_table_key(stored, current):
    """Problems of using a table keyed `stored` where the key is `current`:
    ("error", msg) for another parameter set (the table's levels and
    iteration counts belong to another chain), ("warn", msg) for another GPU
    or library build (the choices stay valid, their times may not), or None."""
    if stored is None:
        return ("warn", "tuning table has no key (GPU, parameter set, library)")
    for k in ("params", "params_sha256"):
        if stored.get(k) != current.get(k):
            return ("error", f"tuning table is for parameter set {stored.get('params')} "
                             f"({str(stored.get('params_sha256'))[:12]}), not {current.get('params')} "
                             f"({str(current.get('params_sha256'))[:12]})")
    diff = [k for k in ("gpu", "library_sha256") if stored.get(k) != current.get(k)]
    if diff:
        return ("warn", "tuning table was measured with another " + " and ".join(diff) + "; re-tune for its times")
    return None

