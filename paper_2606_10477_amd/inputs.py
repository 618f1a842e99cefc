"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module draws random numbers only; it holds none of the method's
arithmetic.  Recipes (all numpy PCG64, ``np.random.default_rng(seed)``):

- ``log_uniform(n, lo, hi, seed)``: x = exp(U(ln lo, ln hi)), the input of the
  inverse square root (n = N/2 slots per ciphertext).
- ``linspace_input(n, A, B)``: the evenly spaced grid the paper uses for its
  provisioning runs (Alg. 3 encrypts linspace(A, B, N/2)).
- ``column_table(rows, cols, seed)``: the synthetic statistics table: column c
  ~ N(mu_c, sigma_c^2) with mu_c ~ U[-5, 5] and sigma_c ~ log-U[0.1, 10].
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


def column_table(rows, cols, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-5, 5, cols)
    sigma = np.exp(rng.uniform(np.log(0.1), np.log(10), cols))
    data = rng.standard_normal((cols, rows)) * sigma[:, None] + mu[:, None]
    return data, mu, sigma


def skewed_table(rows, cols, seed):
    """Columns for the moment statistics: column c has mean ~ U[-5, 5] and
    std ~ logU[0.1, 10] like column_table, but a standardised gamma shape
    (shape k ~ U[1, 10]: skewness 2/sqrt(k), excess kurtosis 6/k), and each odd
    column is correlated with the even one before it (rho ~ U[-0.9, 0.9])."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-5, 5, cols)
    sigma = np.exp(rng.uniform(np.log(0.1), np.log(10), cols))
    k = rng.uniform(1, 10, cols)
    rho = rng.uniform(-0.9, 0.9, cols)
    z = np.empty((cols, rows))
    for c in range(cols):
        g = (rng.gamma(k[c], 1.0, rows) - k[c]) / np.sqrt(k[c])
        if c % 2 == 1:
            g = rho[c] * z[c - 1] + np.sqrt(1 - rho[c] ** 2) * g
        z[c] = g
    data = z * sigma[:, None] + mu[:, None]
    return data, mu, sigma


def poisson_arrivals(n, rate, seed):
    """Arrival times (s) of n requests of a Poisson process with `rate` per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def geometric_sizes(n, p, lo, hi, seed):
    """Request sizes ~ Geometric(p) truncated to [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.clip(rng.geometric(p, n), lo, hi)


def choice(n, options, seed):
    rng = np.random.default_rng(seed)
    return [options[k] for k in rng.integers(0, len(options), n)]
