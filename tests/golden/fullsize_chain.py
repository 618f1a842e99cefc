"""The benchmarked workload's steps at full size, as one recipe of C-ABI-level
calls that runs on either side (the oracle's Context or the GPU library's):
both expose the same operations under the same names.  The recipe holds no
arithmetic; it only names the calls and their order.

Workload (the benchmark's): an N = 2^16 bootstrapping set ("p16b", the
benchmark's, or "p16c", 11 computation levels), keys from seed 9 with the
bootstrapping rotations, x = log-uniform in [2^-10, 1] from input seed 1,
encrypted at the set's top computation level (l_afterBTS: 8 or 11) with scale
2^50 and seed 3.
Steps (paper §2.1 bootstrapping, Alg. 1):
  enc      the input ciphertext
  cheb     the Chebyshev initial value y0 (degree 31; invsqrt with 0 steps)
  raise    ModRaise of y0 dropped to level 0
  cts      CoeffToSlot of the raised ciphertext
  conj     its conjugate
  re, im   y + conj(y) and X^(3N/2) (y - conj(y))   (the real/imaginary split)
  evm_re   EvalMod of re
  evm_im   EvalMod of im
  stc      SlotToCoeff of evm_re + X^(N/2) evm_im
  bts      the whole bootstrap of y0 with message bound 512
  invsqrt  CryptoInvSqrt (31, 3) of enc: the benchmark's step
  invsqrt_tuned  CryptoInvSqrt (63, 2) of enc: the tuned pick for 3.1e-8 at
           the 11-level set's top level (no bootstrap there; one on p16b)
  invsqrt_pre    CryptoInvSqrt (31, 3) of enc with Pre-BTS (the paper's c = 1:
           x bootstrapped before the Chebyshev step)
  invsqrt_paper  the paper's domain: x = linspace(0.001, 100, N/2) encrypted
           as it is at the top level (scale 2^50, seed 5), pre-normalised by
           B = 100 in the chain, CryptoInvSqrt (126, 3) on [0.001, 100]
"""
import hashlib

import numpy as np

LO, HI = 2.0 ** -10, 1.0
KEY_SEED, INPUT_SEED, ENC_SEED = 9, 1, 3
IN_SCALE = 2.0 ** 50
DEGREE, ITERS, BTS_BOUND = 31, 3, 512
TUNED_DEGREE, TUNED_ITERS = 63, 2
PAPER_LO, PAPER_HI, PAPER_B, PAPER_DEGREE, PAPER_ITERS, PAPER_SEED = 0.001, 100.0, 100.0, 126, 3, 5
STEPS = ("enc", "cheb", "raise", "cts", "conj", "re", "im", "evm_re", "evm_im", "stc", "bts", "invsqrt",
         "invsqrt_tuned", "invsqrt_pre", "invsqrt_paper")
N_SAMPLES = 48


def digest(ct):
    """level, scale (hex), SHA-256 of the words [2][level+1][N] (uint64 LE)
    and sampled words at fixed positions (for locating a difference)."""
    w = np.ascontiguousarray(ct.words(), dtype="<u8")
    rng = np.random.default_rng(1234)
    pos = [(int(rng.integers(0, 2)), int(rng.integers(0, w.shape[1])), int(rng.integers(0, w.shape[2])))
           for _ in range(N_SAMPLES)]
    return {"level": int(ct.level), "scale": float(ct.scale).hex(),
            "sha256": hashlib.sha256(w.tobytes()).hexdigest(),
            "samples": [[p, l, t, str(int(w[p, l, t]))] for p, l, t in pos]}


def run(ctx, x, only=None, on_step=None, x_paper=None):
    """Run the steps on `ctx` (keys already generated) and return
    {step: digest}.  `only` limits the run to a subset of STEPS (their
    prerequisites are computed as needed); x_paper is the paper-domain input
    (invsqrt_paper is skipped without it)."""
    want = set(STEPS if only is None else only)
    out = {}

    def rec(name, ct):
        if name in want:
            out[name] = digest(ct)
            if on_step:
                on_step(name, out[name])

    enc = ctx.encrypt(x, ctx.l_after, IN_SCALE, ENC_SEED)
    rec("enc", enc)
    if want & {"cheb", "raise", "cts", "conj", "re", "im", "evm_re", "evm_im", "stc", "bts"}:
        y0 = ctx.invsqrt(enc, DEGREE, 0, LO, HI)
        rec("cheb", y0)
        if want & {"raise", "cts", "conj", "re", "im", "evm_re", "evm_im", "stc"}:
            r = ctx.mod_raise(ctx.drop_level(y0, 0))
            rec("raise", r)
            y = ctx.coeff_to_slot(r)
            del r
            rec("cts", y)
            yc = ctx.conjugate(y)
            rec("conj", yc)
            re = ctx.add(y, yc)
            im = ctx.mul_monomial(ctx.sub(y, yc), 3 * ctx.N // 2)
            del y, yc
            rec("re", re)
            rec("im", im)
            er = ctx.eval_mod(re)
            rec("evm_re", er)
            ei = ctx.eval_mod(im)
            rec("evm_im", ei)
            del re, im
            z = ctx.slot_to_coeff(ctx.add(er, ctx.mul_monomial(ei, ctx.N // 2)))
            rec("stc", z)
            del er, ei, z
        if "bts" in want:
            rec("bts", ctx.bootstrap(y0, BTS_BOUND))
    if "invsqrt" in want:
        rec("invsqrt", ctx.invsqrt(enc, DEGREE, ITERS, LO, HI))
    if "invsqrt_tuned" in want:
        rec("invsqrt_tuned", ctx.invsqrt(enc, TUNED_DEGREE, TUNED_ITERS, LO, HI))
    if "invsqrt_pre" in want:
        rec("invsqrt_pre", ctx.invsqrt(enc, DEGREE, ITERS, LO, HI, pre_bts=True))
    if "invsqrt_paper" in want and x_paper is not None:
        xp = ctx.encrypt(x_paper, ctx.l_after, IN_SCALE, PAPER_SEED)
        rec("invsqrt_paper", ctx.invsqrt(xp, PAPER_DEGREE, PAPER_ITERS, PAPER_LO, PAPER_HI, B=PAPER_B))
    return out
