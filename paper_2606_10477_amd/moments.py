"""Skewness, kurtosis and Pearson correlation of encrypted columns: the
statistics of §5.3 whose denominators need 1/sigma, computed from the z-scores
that znorm.py produces (z = (x - mean) * CryptoInvSqrt(var / B) / sqrt(B)).

The paper evaluates these measures (following PP-STAT) but prints no formula;
the population definitions are used:
  skewness   = mean over rows of z^3,
  kurtosis   = mean over rows of z^4 - 3   (excess kurtosis, as the paper reports),
  PCC(a, b)  = mean over rows of z_a z_b.
Every column (or column pair) goes through the same launches: ciphertext j of
every column forms one batch, as in znorm.py.  Each result sits in every slot
of one ciphertext per column (pair).
"""

from .znorm import _log2_exact, mul_pow2_down, rotate_and_sum


def _stack(ctx, cts):
    return ctx.pack(cts) if len(cts) > 1 else cts[0]


def _unstack(ctx, ct, n):
    return ctx.unpack(ct) if n > 1 else [ct]


def _mean(ctx, cts, rows):
    """Mean over all slots of all ciphertexts of a column (batched over columns)."""
    s = cts[0]
    for c in cts[1:]:
        s = ctx.add(s, c)
    s = rotate_and_sum(ctx, s, ctx.n)
    return mul_pow2_down(ctx, s, -_log2_exact(rows))


def skew_kurt(ctx, z_cols, rows):
    """z_cols[c][j]: z-score ciphertext j of column c (one level and scale).
    Returns (skewness, excess kurtosis), one ciphertext per column each."""
    ncol, nct = len(z_cols), len(z_cols[0])
    Z = [_stack(ctx, [z_cols[c][j] for c in range(ncol)]) for j in range(nct)]
    Z2 = [ctx.rescale(ctx.hmult(z, z)) for z in Z]
    lv = Z2[0].level
    Z3 = [ctx.rescale(ctx.hmult(z2, ctx.level_to(z, lv))) for z2, z in zip(Z2, Z)]
    Z4 = [ctx.rescale(ctx.hmult(z2, z2)) for z2 in Z2]
    skew = _mean(ctx, Z3, rows)
    kurt = ctx.add_const(_mean(ctx, Z4, rows), -3.0)
    return _unstack(ctx, skew, ncol), _unstack(ctx, kurt, ncol)


def pcc(ctx, z_cols, rows, pairs):
    """Pearson correlation of each column pair (a, b): one ciphertext per pair."""
    nct = len(z_cols[0])
    prods = []
    for j in range(nct):
        za = _stack(ctx, [z_cols[a][j] for a, _ in pairs])
        zb = _stack(ctx, [z_cols[b][j] for _, b in pairs])
        prods.append(ctx.rescale(ctx.hmult(za, zb)))
    return _unstack(ctx, _mean(ctx, prods, rows), len(pairs))


def reference(data, pairs=()):
    """FP64 values of the same measures (population moments) for checking."""
    import numpy as np
    z = (data - data.mean(axis=1, keepdims=True)) / data.std(axis=1, keepdims=True)
    skew = (z ** 3).mean(axis=1)
    kurt = (z ** 4).mean(axis=1) - 3.0
    r = np.array([(z[a] * z[b]).mean() for a, b in pairs])
    return skew, kurt, r


def main(argv=None):
    """Skewness, kurtosis and PCC of a synthetic encrypted table on one GPU
    (after its z-score standardisation), N = 2^16."""
    import argparse
    import json
    import time

    import numpy as np
    import torch

    from . import ckks, inputs, znorm

    ap = argparse.ArgumentParser()
    ap.add_argument("--rows", type=int, default=1 << 20)
    ap.add_argument("--cols", type=int, default=64)
    ap.add_argument("--level", type=int, default=27)
    ap.add_argument("--B", type=float, default=128.0)
    ap.add_argument("--degree", type=int, default=127)
    ap.add_argument("--iters", type=int, default=3)
    ap.add_argument("--seed", type=int, default=21)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    ctx = ckks.Context.from_set("p16")
    ctx.keygen(9, [ctx.galois_rot(s) for s in znorm.rotation_steps(ctx.n)])
    per = args.rows // ctx.n
    data, _, _ = inputs.skewed_table(args.rows, args.cols, args.seed)
    cols = [ctx.encrypt_batch(data[c].reshape(per, ctx.n), args.level, 2.0 ** 40, 10000 + per * c)
            for c in range(args.cols)]
    ctx.sync()
    pairs = [(c, c + 1) for c in range(0, args.cols - 1, 2)]
    t0 = time.perf_counter()
    z, _, _ = znorm.znorm(ctx, cols, args.rows, args.B, args.degree, args.iters, 2.0 ** -14, 1.0)
    ctx.sync()
    t_z = time.perf_counter() - t0
    t0 = time.perf_counter()
    sk, ku = skew_kurt(ctx, z, args.rows)
    pc = pcc(ctx, z, args.rows, pairs)
    ctx.sync()
    t_m = time.perf_counter() - t0
    rs, rk, rp = reference(data, pairs)
    gs = np.array([ctx.decrypt(c).real[0] for c in sk])
    gk = np.array([ctx.decrypt(c).real[0] for c in ku])
    gp = np.array([ctx.decrypt(c).real[0] for c in pc])
    rep = {"workload": f"skewness, excess kurtosis of {args.cols} columns and PCC of {len(pairs)} column pairs, "
                       f"{args.rows} rows ({per} ciphertexts per column), input level {args.level}, "
                       f"z-scores by invsqrt ({args.degree}, {args.iters}) on [2^-14, 1], B={args.B}",
           "znorm_s": t_z, "moments_s": t_m, "z_level": z[0][0].level,
           "skew_max_abs_err": float(np.max(np.abs(gs - rs))),
           "kurt_max_abs_err": float(np.max(np.abs(gk - rk))),
           "pcc_max_abs_err": float(np.max(np.abs(gp - rp)))}
    print(json.dumps(rep), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rep, f)
    ctx.close()


if __name__ == "__main__":
    main()
