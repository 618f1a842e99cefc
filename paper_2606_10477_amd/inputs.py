"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module draws random numbers only; it holds none of the method's
arithmetic.  Recipes (all numpy PCG64, ``np.random.default_rng(seed)``):

- ``log_uniform(n, lo, hi, seed)``: x = exp(U(ln lo, ln hi)), the input of the
  inverse square root (n = N/2 slots per ciphertext).
- ``linspace_input(n, A, B)``: the evenly spaced grid the paper uses for its
  provisioning runs (Alg. 3 encrypts linspace(A, B, N/2)).
- ``uniform_words(shape, primes, seed)``: uniform residues mod each prime (used
  as generic ciphertext/polynomial words for per-operation parity tests);
  axis -2 indexes the prime.
"""
import numpy as np


def log_uniform(n, lo, hi, seed):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def linspace_input(n, A, B):
    return np.linspace(A, B, n)


def uniform_words(shape, primes, seed):
    """Uniform integers in [0, q_i) for an array of shape (..., len(primes), N)."""
    rng = np.random.default_rng(seed)
    primes = np.asarray(primes, dtype=np.uint64)
    assert shape[-2] == len(primes)
    out = np.empty(shape, dtype=np.uint64)
    for i, q in enumerate(primes):
        out[..., i, :] = rng.integers(0, int(q), size=shape[:-2] + (shape[-1],), dtype=np.uint64)
    return out


def small_ints(shape, bound, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(-bound, bound + 1, size=shape, dtype=np.int64)
