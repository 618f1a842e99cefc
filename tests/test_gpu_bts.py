"""GPU parity of bootstrapping and of CryptoInvSqrt with the bootstrapping
policy (paper §2.1 BTS, Alg. 1 with BTS whenever levels run out), through the
C-ABI, against the CPU oracle on the same seeded inputs.

Small set (N = 2^10): computation levels 0..8 as in the full set, with the
bootstrapping levels above them (3 SlotToCoeff levels on 40-bit primes, 9
EvalMod and 3 CoeffToSlot levels on 52-bit primes), digits of 2 primes, 2
special primes, h = 192.  Every step must give identical ciphertext words.

Full set (N = 2^16, "p16b"): q_0 60-bit, 8 + 3 primes near 2^40, 12 primes
near 2^52, 7 special 60-bit primes, digits of 8 primes (dnum = 3), log2 QP
~ 1544, h = 192: bootstrapping accuracy and the fixed configuration (degree
31, 3 Newton steps) from level 8 with one lazy bootstrap, MRE <= 3.1e-8.
Word-for-word parity at this size is in test_gpu_fullsize_parity.py.
"""
import numpy as np
import pytest

from paper_2606_10477_amd import inputs

pytestmark = pytest.mark.gpu

BTS = (3, 9, 3, 52)
SMALL = dict(log_n=10, max_level=8, num_special=2, digit_size=2, hamming_weight=192, bts=BTS)
EVALMOD = (25.0, 4, 31)   # K, r, Chebyshev degree


def _ck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_10477_amd import ckks
    return ckks


def same(gct, oct_):
    assert gct.level == oct_.level
    assert gct.scale == oct_.scale
    gw, ow = gct.words(), oct_.words()
    if not np.array_equal(gw, ow):
        bad = np.argwhere(gw != ow)
        raise AssertionError(f"{len(bad)} words differ, first at {bad[:5].tolist()}")


@pytest.fixture(scope="module")
def pair(oracle_mod):
    ck = _ck()
    g = ck.Context(**SMALL)
    o = oracle_mod.Context(10, 8, 2, 2, h=192, bts=BTS)
    g.bts_setup(*EVALMOD)
    o.bts_config(*EVALMOD)
    gal = g.bts_galois()
    g.keygen(4, gal)
    o.keygen(4, gal)
    yield g, o
    g.close()


def test_chain_and_rotation_keys_match(pair):
    g, o = pair
    assert g.L == o.L == 23
    assert np.array_equal(g.primes, o.primes)
    assert np.array_equal(g.ladder, o.ladder)
    assert g.bts_rotations() == o.bts_rotations()


def test_mod_raise_and_monomial_bit_exact(pair):
    g, o = pair
    x = inputs.log_uniform(g.n, 1.0, 32.0, 5)
    gc, oc = g.encrypt(x, 0, g.ladder[0], 70), o.encrypt(x, 0, o.ladder[0], 70)
    same(gc, oc)
    same(g.mod_raise(gc), o.mod_raise(oc))
    for k in (g.N // 2, 3 * g.N // 2, 1, 2 * g.N - 1):
        same(g.mul_monomial(gc, k), o.mul_monomial(oc, k))


def test_hoisted_rotations_bit_exact(pair):
    g, o = pair
    x = inputs.log_uniform(g.n, 1.0, 2.0, 9)
    gc, oc = g.encrypt(x, 12, g.ladder[12], 69), o.encrypt(x, 12, o.ladder[12], 69)
    steps = [0] + g.bts_rotations()[:4]
    for gr, orr in zip(g.rotate_hoisted(gc, steps), o.rotate_hoisted(oc, steps)):
        same(gr, orr)


def test_slot_transforms_and_evalmod_bit_exact(pair):
    g, o = pair
    x = inputs.log_uniform(g.n, 1.0, 32.0, 6)
    gc, oc = g.encrypt(x, 0, g.ladder[0], 71), o.encrypt(x, 0, o.ladder[0], 71)
    gr, orr = g.mod_raise(gc), o.mod_raise(oc)
    gy, oy = g.coeff_to_slot(gr), o.coeff_to_slot(orr)
    same(gy, oy)
    gs, os_ = g.add(gy, g.conjugate(gy)), o.add(oy, o.conjugate(oy))
    same(gs, os_)
    ge, oe = g.eval_mod(gs), o.eval_mod(os_)
    same(ge, oe)
    assert ge.level == g.l_after + 3
    same(g.slot_to_coeff(ge), o.slot_to_coeff(oe))


@pytest.mark.parametrize("bound", [64, 512])
def test_bootstrap_bit_exact_and_accurate(pair, bound):
    g, o = pair
    x = inputs.log_uniform(g.n, 1.0, 32.0, 7)
    gc, oc = g.encrypt(x, 1, g.ladder[1], 72), o.encrypt(x, 1, o.ladder[1], 72)
    gb, ob = g.bootstrap(gc, bound), o.bootstrap(oc, bound)
    same(gb, ob)
    assert gb.level == g.l_after
    rel = np.abs(g.decrypt(gb).real - x) / x
    assert np.mean(rel) < 2e-3, np.mean(rel)


def test_bootstrap_batch_equals_single(pair):
    g, _ = pair
    xs = [inputs.log_uniform(g.n, 1.0, 32.0, 20 + i) for i in range(3)]
    cts = [g.encrypt(x, 0, g.ladder[0], 80 + i) for i, x in enumerate(xs)]
    outs = g.unpack(g.bootstrap(g.pack(cts), 512))
    for c, y in zip(cts, outs):
        same(y, g.bootstrap(c, 512))


@pytest.mark.parametrize("degree,iters,level,literal,pre", [(31, 3, 8, False, False), (7, 5, 8, False, False),
                                                            (15, 3, 8, True, False), (31, 2, 5, False, False),
                                                            (15, 2, 5, False, True), (63, 2, 8, False, False),
                                                            (127, 1, 8, False, False)])
def test_invsqrt_with_bootstrapping_bit_exact(pair, degree, iters, level, literal, pre):
    """Lazy BTS of y (one or two bootstraps), the Alg.-1-literal BTS after the
    Chebyshev step, the Pre-BTS of x forced by its level (level 5 < depth 5 + 1
    for degree 31) and asked for (c = 1 at level 5); degrees 63 and 127 from
    the top level 8 without Pre-BTS (depth 6 and 7, plus the affine map)."""
    g, o = pair
    lo, hi = 2.0 ** -10, 1.0
    x = inputs.log_uniform(g.n, lo, hi, 8)
    gc, oc = g.encrypt(x, level, 2.0 ** 50, 73), o.encrypt(x, level, 2.0 ** 50, 73)
    gy = g.invsqrt(gc, degree, iters, lo, hi, literal=literal, pre_bts=pre)
    oy = o.invsqrt(oc, degree, iters, lo, hi, literal=literal, pre_bts=pre)
    same(gy, oy)
    if (degree, iters, level) == (31, 3, 8):
        ref = 1 / np.sqrt(x)
        mre = np.mean(np.abs(g.decrypt(gy).real - ref) / ref)
        print(f"N=2^10 (31,3) from level 8 with BTS: MRE {mre:.3g}", flush=True)
        assert mre < 1e-7


@pytest.mark.parametrize("degree,iters,level,pre", [(14, 3, 8, False), (30, 2, 8, False), (14, 3, 8, True),
                                                    (30, 2, 4, False)])
def test_invsqrt_prenormalised_paper_domain_bit_exact(pair, degree, iters, level, pre):
    """The paper's domain and pre-normalisation (§2.3, §4.3: linspace over
    [0.001, 100], B = 100, degrees 2^d_e - 2) with lazy bootstrapping, from
    the top level, with Pre-BTS asked for, and from level 4 where degree 30
    forces it (x divided by B before the bootstrap): GPU words equal the
    oracle's; accuracy against 1/sqrt(x)."""
    g, o = pair
    A, Bv = 0.001, 100.0
    x = np.linspace(A, Bv, g.n)
    gc, oc = g.encrypt(x, level, 2.0 ** 50, 74), o.encrypt(x, level, 2.0 ** 50, 74)
    gy = g.invsqrt(gc, degree, iters, A, Bv, pre_bts=pre, B=100.0)
    oy = o.invsqrt(oc, degree, iters, A, Bv, pre_bts=pre, B=100.0)
    same(gy, oy)
    ref = 1 / np.sqrt(x)
    mre = np.mean(np.abs(g.decrypt(gy).real - ref) / ref)
    print(f"N=2^10 paper domain ({degree},{iters}) from level {level}, Pre-BTS {pre}, B=100: MRE {mre:.3g}",
          flush=True)
    assert mre < 1e-2


@pytest.fixture(scope="module")
def full():
    ck = _ck()
    g = ck.Context.from_set("p16b")
    g.keygen(11, g.bts_galois())
    yield g
    g.close()


def test_full_size_chain(full):
    g = full
    bits = [int(p).bit_length() for p in g.primes]
    assert g.L == 23 and len(bits) == 31
    assert bits[0] == 60 and all(40 <= b <= 41 for b in bits[1:12])
    assert all(52 <= b <= 53 for b in bits[12:24]) and all(b == 60 for b in bits[24:])
    digits = [sum(np.log2(float(p)) for p in g.primes[i:i + 8]) for i in range(0, 24, 8)]
    assert max(digits) < sum(np.log2(float(p)) for p in g.primes[24:])   # P exceeds every digit
    assert 1540 < sum(np.log2(float(p)) for p in g.primes) < 1560


def test_full_size_bootstrap_accuracy(full):
    """Bootstrapping error at N = 2^16 on 1/sqrt(x) values (|y| <= 32): the
    mean relative error is 3.4e-4 with message bound 64 and 2.9e-4 with 512
    (the oracle gives the same words, hence the same figures; on this set and
    on the previous one with 7 computation levels and 10 EvalMod levels
    alike); the bounds leave 1.4x."""
    g = full
    x = inputs.log_uniform(g.n, 2.0 ** -10, 1.0, 9)
    y = 1 / np.sqrt(x)
    c = g.encrypt(y, 0, g.ladder[0], 74)
    for bound, lim in ((64, 5e-4), (512, 4e-4)):
        b = g.bootstrap(c, bound)
        rel = np.abs(g.decrypt(b).real - y) / y
        print(f"N=2^16 BTS of 1/sqrt(x) values, bound {bound}: level {b.level}, "
              f"mean rel err {np.mean(rel):.3g}, max {np.max(rel):.3g}", flush=True)
        assert b.level == g.l_after == 8 and np.mean(rel) < lim


def test_full_size_invsqrt_with_one_bootstrap(full):
    g = full
    lo, hi = 2.0 ** -10, 1.0
    x = inputs.log_uniform(g.n, lo, hi, 10)
    c = g.encrypt(x, 8, 2.0 ** 50, 75)
    g.trace(True)
    y = g.invsqrt(c, 31, 3, lo, hi)
    tr = g.trace_read()
    g.trace(False)
    ref = 1 / np.sqrt(x)
    mre = np.mean(np.abs(g.decrypt(y).real - ref) / ref)
    n_bts = sum(1 for op in tr if op[0] == "bootstrap")
    print(f"N=2^16 (31,3) from level 8: {n_bts} bootstrap(s), output level {y.level}, MRE {mre:.3g}", flush=True)
    assert n_bts == 1
    assert mre <= 3.1e-8


def test_invsqrt_graph_replays_match_eager(pair):
    """The captured chain (with its bootstrap) replayed several times, on
    different inputs of the captured shape, with eager work and
    synchronisations between the replays: every replay equals the eager
    result word for word; the same for a batch of 3."""
    g, _ = pair
    lo, hi = 2.0 ** -10, 1.0
    xs = [inputs.log_uniform(g.n, lo, hi, 40 + i) for i in range(4)]
    cts = [g.encrypt(x, 8, 2.0 ** 50, 90 + i) for i, x in enumerate(xs)]
    graph = g.invsqrt_graph(cts[0], 31, 3, lo, hi)
    for rep in range(3):
        for ct in cts:
            eager = g.invsqrt(ct, 31, 3, lo, hi)
            same(graph.run(ct), eager)
            g.sync()
            g.rescale(g.hmult(ct, ct))      # eager work between replays
    graph.close()
    batch = g.pack(cts[:3])
    gb = g.invsqrt_graph(batch, 15, 3, lo, hi)
    for rep in range(2):
        outs = g.unpack(gb.run(batch))
        for ct, y in zip(cts[:3], outs):
            same(y, g.invsqrt(ct, 15, 3, lo, hi))
        g.sync()
    gb.close()
