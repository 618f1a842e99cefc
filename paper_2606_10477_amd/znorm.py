"""Batched z-score standardisation of an encrypted table (the Z-score normalisation of paper §5.3,
invsqrt of the variance in the denominator).

Each column of R rows is packed into R / (N/2) ciphertexts.  All columns go
through the same launches: ciphertext j of every column forms one batch, so a
column-wise reduction is a batched addition and every primitive runs once over
all columns.

Per column (x_1..x_R, R = rows):
  S1 = sum of the column's ciphertexts, then rotate-and-sum over the slots
       (log2(N/2) rotations by 1, 2, 4, ...): every slot holds sum x;
  S2 = the same for the squares x^2;
  m1 = (S1 * 1/sqrt(B)) * 2^-log2(R)  -> mean / sqrt(B);
  m2 = S2 * 2^-(log2(R) + log2(B))     -> E[x^2] / B;
  v  = m2 - m1^2 = var / B     (B: pre-normalisation constant of the paper,
                                chosen so that var / B lies in the invsqrt domain);
  r  = CryptoInvSqrt(v) = sqrt(B) / sigma;
  z_j = (x_j - mean) * (r / sqrt(B)),  mean = S1 * 2^-log2(R).
Factors that are powers of two (R and B must be) are applied as exact integer
plaintexts 2^(40+e) at plaintext scale 2^40 followed by a rescale, so they
add no rounding; only 1/sqrt(B) goes through a rounded constant, and it is of
order one.  (A single Mul_P by 1/(R sqrt(B)) ~ 1e-6 would keep only ~20 bits
of the constant, which the cancellation in E[x^2] - mean^2 amplifies.)
"""
import math

import numpy as np


def rotate_and_sum(ctx, ct, n):
    """Sum over all n slots, replicated in every slot: log2(n) rotations."""
    acc = ct
    k = 1
    while k < n:
        acc = ctx.add(acc, ctx.rotate(acc, k))
        k <<= 1
    return acc


def _log2_exact(v):
    e = int(round(math.log2(v)))
    if 2.0 ** e != v:
        raise ValueError("rows and B must be powers of two")
    return e


def mul_pow2_down(ctx, ct, e):
    """Multiply by 2^e (e <= 0) exactly: the integer 2^(40+e) at plaintext
    scale 2^40, then rescale (one level, no constant rounding)."""
    return ctx.rescale(ctx.mul_const(ct, 2.0 ** e, 2.0 ** 40))


def rotation_steps(n):
    return [1 << k for k in range(int(math.log2(n)))]


def znorm(ctx, col_cts, rows, B, degree, iters, lo, hi):
    """col_cts[c][j]: ciphertext j of column c (all at one level and scale).
    Returns z_cts[c][j] and the batched variance / invsqrt ciphertexts."""
    ncol = len(col_cts)
    nct = len(col_cts[0])
    X = [ctx.pack([col_cts[c][j] for c in range(ncol)]) if ncol > 1 else col_cts[0][j] for j in range(nct)]
    s1 = X[0]
    sq = [ctx.rescale(ctx.hmult(x, x)) for x in X]
    s2 = sq[0]
    for j in range(1, nct):
        s1 = ctx.add(s1, X[j])
        s2 = ctx.add(s2, sq[j])
    del sq
    s1 = rotate_and_sum(ctx, s1, ctx.n)
    s2 = rotate_and_sum(ctx, s2, ctx.n)
    lr, lb = _log2_exact(rows), _log2_exact(B)
    m1 = mul_pow2_down(ctx, ctx.mul_const_down(s1, 1.0 / math.sqrt(B)), -lr)
    m2 = mul_pow2_down(ctx, s2, -(lr + lb))
    m1sq = ctx.rescale(ctx.hmult(m1, m1))
    # both operands carry exact non-canonical scales: retarget both one level down
    lv = min(m1sq.level, m2.level) - 1
    v = ctx.sub(ctx.level_to(m2, lv), ctx.level_to(m1sq, lv))
    r = ctx.invsqrt_batch([v], degree, iters, a=lo, b=hi)[0] if ncol == 1 else \
        _invsqrt_packed(ctx, v, degree, iters, lo, hi)
    rs = ctx.mul_const_down(r, 1.0 / math.sqrt(B))
    mean = mul_pow2_down(ctx, s1, -lr)
    z = []
    for j in range(nct):
        lvd = min(X[j].level, mean.level, rs.level + 1)
        diff = ctx.sub(ctx.level_to(X[j], lvd), ctx.level_to(mean, lvd))
        lvm = min(diff.level, rs.level)
        zz = ctx.rescale(ctx.hmult(ctx.level_to(diff, lvm), ctx.level_to(rs, lvm)))
        z.append(ctx.unpack(zz) if ncol > 1 else [zz])
    z_cols = [[z[j][c] for j in range(nct)] for c in range(ncol)]
    return z_cols, v, r


def _invsqrt_packed(ctx, v, degree, iters, lo, hi):
    # invsqrt_batch takes single ciphertexts; unpack, run as one batch, repack
    parts = ctx.unpack(v)
    outs = ctx.invsqrt_batch(parts, degree, iters, a=lo, b=hi)
    return ctx.pack(outs)


def main(argv=None):
    """Z-score standardisation of a synthetic encrypted table on one GPU:
    rows x cols values, N = 2^16 (2^15 slots per ciphertext)."""
    import argparse
    import json
    import time

    import torch

    from . import ckks, inputs

    ap = argparse.ArgumentParser()
    ap.add_argument("--rows", type=int, default=1 << 20)
    ap.add_argument("--cols", type=int, default=64)
    ap.add_argument("--level", type=int, default=22)
    ap.add_argument("--B", type=float, default=128.0)
    ap.add_argument("--degree", type=int, default=127)
    ap.add_argument("--iters", type=int, default=3)
    ap.add_argument("--check-cols", type=int, default=2)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    ctx = ckks.Context.from_set("p16")
    ctx.keygen(9, [ctx.galois_rot(s) for s in rotation_steps(ctx.n)])
    per = args.rows // ctx.n
    data, _, _ = inputs.column_table(args.rows, args.cols, 21)
    t0 = time.perf_counter()
    cols = [ctx.encrypt_batch(data[c].reshape(per, ctx.n), args.level, 2.0 ** 40, 10000 + per * c)
            for c in range(args.cols)]
    ctx.sync()
    t_enc = time.perf_counter() - t0
    t0 = time.perf_counter()
    z, v, r = znorm(ctx, cols, args.rows, args.B, args.degree, args.iters, 2.0 ** -14, 1.0)
    ctx.sync()
    t_run = time.perf_counter() - t0
    errs = []
    for c in range(min(args.check_cols, args.cols)):
        zz = np.concatenate([ctx.decrypt(z[c][j]).real for j in range(per)])
        ref = (data[c] - data[c].mean()) / data[c].std()
        errs.append(float(np.mean(np.abs(zz - ref))))
    rep = {"workload": f"z-score of {args.rows} x {args.cols} table, {per} ciphertexts per column, "
                       f"input level {args.level}, invsqrt ({args.degree}, {args.iters}) on [2^-14, 1], B={args.B}",
           "ciphertexts": per * args.cols, "encrypt_s": t_enc, "znorm_s": t_run,
           "invsqrt_ciphertexts": args.cols, "z_mean_abs_err_checked_cols": errs}
    print(json.dumps(rep), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rep, f)
    ctx.close()


if __name__ == "__main__":
    main()
