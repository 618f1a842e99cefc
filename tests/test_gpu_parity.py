"""GPU parity: every operation of the HIP library through the C-ABI against the
CPU oracle on the same seeded inputs.  Ciphertext words must be identical
(bit-exact); decoded values within 1e-12 relative.

Sizes: the N = 2^12 parameter set (q_0 60-bit + 13 scaling primes, one
special prime, dense secret) runs the whole CryptoInvSqrt chain (Alg. 1) with
degree 15 and 2 Newton steps; the N = 2^16 set (q_0 + 27 scaling primes,
7 special primes, digits of 10 primes, h = 192 secret) checks each primitive
at full size, several levels.
"""
import numpy as np
import pytest

from paper_2606_10477_amd import inputs

pytestmark = pytest.mark.gpu


def _gpu_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_10477_amd import ckks
    return ckks


P12 = dict(log_n=12, max_level=13, num_special=1, digit_size=1, hamming_weight=0)
P16 = dict(log_n=16, max_level=27, num_special=7, digit_size=10, hamming_weight=192)


def _galois(ctx, steps, conj=True):
    g = [ctx.galois_rot(k) for k in steps]
    if conj:
        g.append(2 * ctx.N - 1)
    return g


@pytest.fixture(scope="module")
def pair12(oracle_mod):
    ck = _gpu_mod()
    g = ck.Context(**P12)
    o = oracle_mod.Context(12, 13, 1, 1, h=0)
    gal = _galois(g, [1, -3, 7])
    g.keygen(2, gal)
    o.keygen(2, gal)
    yield g, o
    g.close()


@pytest.fixture(scope="module")
def pair16(oracle_mod):
    ck = _gpu_mod()
    g = ck.Context(**P16)
    o = oracle_mod.Context(16, 27, 7, 10, h=192)
    gal = _galois(g, [1, 5])
    g.keygen(9, gal)
    o.keygen(9, gal)
    yield g, o
    g.close()


def same(gct, oct_):
    assert gct.level == oct_.level
    assert gct.scale == oct_.scale
    gw, ow = gct.words(), oct_.words()
    if not np.array_equal(gw, ow):
        bad = np.argwhere(gw != ow)
        raise AssertionError(f"{len(bad)} words differ, first at {bad[:5].tolist()}")


def test_context_primes_match(pair12, pair16):
    for g, o in (pair12, pair16):
        assert np.array_equal(g.primes, o.primes)
        assert np.array_equal(g.ladder, o.ladder)


@pytest.mark.parametrize("which", ["12", "16"])
def test_ntt_bit_exact(pair12, pair16, which):
    import torch
    g, o = pair12 if which == "12" else pair16
    rng = np.random.default_rng(40)
    idx = np.arange(g.np_, dtype=np.uint32)
    host = inputs.uniform_words((g.np_, g.N), g.primes, 41)
    dev = torch.from_numpy(host.view(np.int64)).cuda()
    g.ntt_device(dev.data_ptr(), g.np_, idx, inverse=False)
    torch.cuda.synchronize()
    got = dev.cpu().numpy().view(np.uint64)
    for i in rng.choice(g.np_, size=min(8, g.np_), replace=False):
        assert np.array_equal(got[i], o.ntt(int(i), host[i])), f"forward limb {i}"
    g.ntt_device(dev.data_ptr(), g.np_, idx, inverse=True)
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy().view(np.uint64), host)
    # inverse on fresh data against the oracle
    dev2 = torch.from_numpy(host.view(np.int64)).cuda()
    g.ntt_device(dev2.data_ptr(), g.np_, idx, inverse=True)
    torch.cuda.synchronize()
    got2 = dev2.cpu().numpy().view(np.uint64)
    for i in [0, g.np_ - 1]:
        assert np.array_equal(got2[i], o.intt(int(i), host[i])), f"inverse limb {i}"


@pytest.mark.parametrize("words_per_thread", ["4s4", 4, 8, 16])
@pytest.mark.parametrize("fp64", [True, False])
def test_ntt16_schedules_bit_exact(pair16, words_per_thread, fp64):
    """Every N = 2^16 transform variant (4 words per thread with 4 or 16
    sub-transforms per workgroup, 8 or 16 words per thread; the
    40-bit primes' butterflies in binary64 or on integers) against the
    oracle's negacyclic NTT, on single limbs, a ragged count and all limbs of
    the chain (60-bit and 40-bit primes), including all-(q-1) limbs."""
    import torch
    g, o = pair16
    big = 1 << 20
    g.ntt_schedule(*{"4s4": (big, big, big), 4: (big, big, 0), 8: (0, big, 0), 16: (0, 0, 0)}[words_per_thread])
    g.ntt_arith(-1 if fp64 else 0)
    try:
        for n in (1, 3, g.np_):
            idx = np.array([(5 * i + 1) % g.np_ for i in range(n)], dtype=np.uint32)
            host = inputs.uniform_words((g.np_, g.N), g.primes, 43 + n)[idx]
            host[0] = g.primes[idx[0]] - 1
            dev = torch.from_numpy(host.view(np.int64)).cuda()
            g.ntt_device(dev.data_ptr(), n, idx, inverse=False)
            torch.cuda.synchronize()
            got = dev.cpu().numpy().view(np.uint64)
            for i in range(n):
                assert np.array_equal(got[i], o.ntt(int(idx[i]), host[i])), f"forward {n} limbs, limb {i}"
            dev2 = torch.from_numpy(host.view(np.int64)).cuda()
            g.ntt_device(dev2.data_ptr(), n, idx, inverse=True)
            torch.cuda.synchronize()
            got2 = dev2.cpu().numpy().view(np.uint64)
            for i in range(n):
                assert np.array_equal(got2[i], o.intt(int(idx[i]), host[i])), f"inverse {n} limbs, limb {i}"
    finally:
        g.ntt_schedule(-1, -1, -1)
        g.ntt_arith(-1)


def test_encrypt_decrypt_parity(pair12):
    g, o = pair12
    x = inputs.log_uniform(g.n, 2 ** -8, 1.0, 1)
    for lvl, sc, seed in [(13, 2.0 ** 50, 3), (4, 2.0 ** 40, 5), (0, 2.0 ** 40, 6)]:
        gc, oc = g.encrypt(x, lvl, sc, seed), o.encrypt(x, lvl, sc, seed)
        same(gc, oc)
        zg, zo = g.decrypt(gc), o.decrypt(oc)
        assert np.max(np.abs(zg - zo)) <= 1e-12 * np.max(np.abs(zo))


def test_primitive_ops_parity_small(pair12):
    g, o = pair12
    x = inputs.log_uniform(g.n, 2 ** -8, 1.0, 1)
    y = inputs.log_uniform(g.n, 2 ** -8, 1.0, 2)
    ga, oa = g.encrypt(x, 13, 2.0 ** 40, 3), o.encrypt(x, 13, 2.0 ** 40, 3)
    gb, ob = g.encrypt(y, 13, 2.0 ** 40, 4), o.encrypt(y, 13, 2.0 ** 40, 4)
    same(g.add(ga, gb), o.add(oa, ob))
    same(g.sub(ga, gb), o.sub(oa, ob))
    same(g.mul_int(ga, -7), o.mul_int(oa, -7))
    same(g.mul_const(ga, 0.375, 2.0 ** 38), o.mul_const(oa, 0.375, 2.0 ** 38))
    same(g.add_const(ga, -0.8125), o.add_const(oa, -0.8125))
    same(g.drop_level(ga, 6), o.drop_level(oa, 6))
    same(g.rescale(ga), o.rescale(oa))
    same(g.level_to(ga, 9), o.level_to(oa, 9))
    same(g.mul_const_down(ga, 1.5), o.mul_const_down(oa, 1.5))
    gm, om = g.hmult(ga, gb), o.hmult(oa, ob)
    same(gm, om)
    same(g.rescale(gm), o.rescale(om))
    for k in (1, -3, 7):
        same(g.rotate(ga, k), o.rotate(oa, k))
    same(g.conjugate(ga), o.conjugate(oa))
    # lower levels, including the single-prime digits near the bottom
    gl, ol = g.level_to(ga, 2), o.level_to(oa, 2)
    same(gl, ol)
    same(g.hmult(gl, gl), o.hmult(ol, ol))
    same(g.rotate(gl, 1), o.rotate(ol, 1))


def test_uniform_word_inputs_small(pair12):
    """Operations are integer maps: check them on arbitrary words too."""
    g, o = pair12
    for lvl in (13, 5, 1):
        w = inputs.uniform_words((2, lvl + 1, g.N), g.primes[:lvl + 1], 50 + lvl)
        ga, oa = g.ct_import(w, lvl, 2.0 ** 40), o.ct_import(w, lvl, 2.0 ** 40)
        same(g.rescale(ga), o.rescale(oa))
        same(g.hmult(ga, ga), o.hmult(oa, oa))
        same(g.rotate(ga, 7), o.rotate(oa, 7))


def test_errors_small(pair12):
    ck = _gpu_mod()
    g, _ = pair12
    x = inputs.log_uniform(g.n, 2 ** -8, 1.0, 1)
    a = g.encrypt(x, 3, 2.0 ** 40, 3)
    b = g.encrypt(x, 2, 2.0 ** 40, 3)
    with pytest.raises(ck.CkksError) as e:
        g.add(a, b)
    assert e.value.status == -2
    with pytest.raises(ck.CkksError) as e:
        g.rotate(a, 2)
    assert e.value.status == -4
    c = g.encrypt(x, 3, 2.0 ** 45, 3)
    with pytest.raises(ck.CkksError) as e:
        g.add(a, c)
    assert e.value.status == -3
    z = g.encrypt(x, 0, 2.0 ** 40, 3)
    with pytest.raises(ck.CkksError) as e:
        g.rescale(z)
    assert e.value.status == -2
    with pytest.raises(ck.CkksError):
        g.encrypt(x, 14, 2.0 ** 40, 3)


def test_cheb_newton_invsqrt_chain_small(pair12, oracle_mod):
    """Alg. 1 at N = 2^12: degree 15, 2 Newton steps; every intermediate and
    the result bit-exact, MRE equal to the oracle's."""
    g, o = pair12
    x = inputs.log_uniform(g.n, 2 ** -8, 1.0, 1)
    gx, ox = g.encrypt(x, 13, 2.0 ** 50, 3), o.encrypt(x, 13, 2.0 ** 50, 3)
    cf = oracle_mod.cheb_coeffs_invsqrt(15, 2 ** -8, 1.0)
    from paper_2606_10477_amd import ckks
    assert np.array_equal(cf, ckks.cheb_coeffs_invsqrt(15, 2 ** -8, 1.0))
    gy, oy = g.cheb_eval(gx, cf, 2 ** -8, 1.0), o.cheb_eval(ox, cf, 2 ** -8, 1.0)
    same(gy, oy)
    gh, oh = g.mul_const_down(gx, 0.5), o.mul_const_down(ox, 0.5)
    same(gh, oh)
    gn, on = g.newton_step(gy, gh), o.newton_step(oy, oh)
    same(gn, on)
    gr, orr = g.newton_step(gy, gx, raw_x=True), o.newton_step(oy, ox, raw_x=True)
    same(gr, orr)
    gi = g.invsqrt(gx, 15, 2, a=2 ** -8, b=1.0)
    oi = o.invsqrt(ox, 15, 2, 2 ** -8, 1.0)
    same(gi, oi)
    ref = 1 / np.sqrt(x)
    zg = g.decrypt(gi).real
    mre = np.mean(np.abs(zg - ref) / ref)
    assert abs(mre - 2.7e-5) < 0.2e-5
    # odd degrees and a degree below the baby-step size
    for d in (7, 1, 2):
        cf = oracle_mod.cheb_coeffs_invsqrt(d, 2 ** -8, 1.0)
        same(g.cheb_eval(gx, cf, 2 ** -8, 1.0), o.cheb_eval(ox, cf, 2 ** -8, 1.0))


@pytest.mark.parametrize("log_n", [8, 9])
def test_small_ring_paths_bit_exact(oracle_mod, log_n):
    """N = 2^8 and 2^9: the launch shapes used below 2^10 (one word per thread
    in the linear combinations, ModDown finish and multiply-add passes; leaf by
    leaf baby-step sums at 2^8, the one-pass form at 2^9): a Chebyshev +
    Newton chain, products and hoisted rotations bit-exact vs the oracle."""
    ck = _gpu_mod()
    g = ck.Context(log_n=log_n, max_level=11, num_special=1, digit_size=2, hamming_weight=0)
    o = oracle_mod.Context(log_n, 11, 1, 2, h=0)
    try:
        steps = [1, -3, 7]
        gal = _galois(g, steps)
        g.keygen(5, gal)
        o.keygen(5, gal)
        x = inputs.log_uniform(g.n, 2 ** -8, 1.0, 40 + log_n)
        gx, ox = g.encrypt(x, 11, 2.0 ** 50, 7), o.encrypt(x, 11, 2.0 ** 50, 7)
        same(gx, ox)
        cf = oracle_mod.cheb_coeffs_invsqrt(15, 2 ** -8, 1.0)
        same(g.cheb_eval(gx, cf, 2 ** -8, 1.0), o.cheb_eval(ox, cf, 2 ** -8, 1.0))
        same(g.invsqrt(gx, 15, 2, a=2 ** -8, b=1.0), o.invsqrt(ox, 15, 2, 2 ** -8, 1.0))
        same(g.hmult(gx, gx), o.hmult(ox, ox))
        for gr, orr in zip(g.rotate_hoisted(gx, steps), o.rotate_hoisted(ox, steps)):
            same(gr, orr)
    finally:
        g.close()


def _batched_ops_match(g, lvl, seed0):
    xs = [g.encrypt(inputs.log_uniform(g.n, 2 ** -8, 1.0, seed0 + i), lvl, 2.0 ** 40, seed0 + 10 + i)
          for i in range(3)]
    ys = [g.encrypt(inputs.log_uniform(g.n, 2 ** -8, 1.0, seed0 + 20 + i), lvl, 2.0 ** 40, seed0 + 30 + i)
          for i in range(3)]
    bx, by = g.pack(xs), g.pack(ys)
    assert bx.count == 3

    failures = []

    def check(name, batched, singles):
        parts = g.unpack(batched)
        for i, (p, s1) in enumerate(zip(parts, singles)):
            if p.level != s1.level or p.scale != s1.scale:
                failures.append(f"{name}: member {i} level/scale")
            elif not np.array_equal(p.words(), s1.words()):
                failures.append(f"{name}: member {i} differs")

    check("add", g.add(bx, by), [g.add(a, b) for a, b in zip(xs, ys)])
    check("mul_int", g.mul_int(bx, -5), [g.mul_int(a, -5) for a in xs])
    check("add_const", g.add_const(bx, 0.25), [g.add_const(a, 0.25) for a in xs])
    check("drop", g.drop_level(bx, lvl - 2), [g.drop_level(a, lvl - 2) for a in xs])
    check("rescale", g.rescale(bx), [g.rescale(a) for a in xs])
    check("level_to", g.level_to(bx, lvl - 3), [g.level_to(a, lvl - 3) for a in xs])
    check("rotate", g.rotate(bx, 1), [g.rotate(a, 1) for a in xs])
    check("conjugate", g.conjugate(bx), [g.conjugate(a) for a in xs])
    check("hmult", g.hmult(bx, by), [g.hmult(a, b) for a, b in zip(xs, ys)])
    check("hmult_same", g.hmult(bx, bx), [g.hmult(a, a) for a in xs])
    assert not failures, failures


def test_batched_primitives_small(pair12):
    g, _ = pair12
    _batched_ops_match(g, 13, 100)
    _batched_ops_match(g, 3, 200)


def test_batched_primitives_full_size(pair16):
    g, _ = pair16
    _batched_ops_match(g, 13, 300)


def test_batch_equals_single_small(pair12):
    g, o = pair12
    xs = [g.encrypt(inputs.log_uniform(g.n, 2 ** -8, 1.0, 10 + i), 13, 2.0 ** 50, 20 + i) for i in range(3)]
    outs = g.invsqrt_batch(xs, 15, 2, a=2 ** -8, b=1.0)
    for x, y in zip(xs, outs):
        single = g.invsqrt(x, 15, 2, a=2 ** -8, b=1.0)
        assert np.array_equal(single.words(), y.words())


# ---------------------------------------------------------------------------
# N = 2^16 (full size): primitives bit-exact at several levels
# ---------------------------------------------------------------------------
def test_full_size_encrypt_and_ops(pair16):
    g, o = pair16
    x = inputs.log_uniform(g.n, 2 ** -10, 1.0, 1)
    gx, ox = g.encrypt(x, 11, 2.0 ** 50, 3), o.encrypt(x, 11, 2.0 ** 50, 3)
    same(gx, ox)
    zg, zo = g.decrypt(gx), o.decrypt(ox)
    assert np.max(np.abs(zg - zo)) <= 1e-12 * np.max(np.abs(zo))
    gh, oh = g.mul_const_down(gx, 0.5), o.mul_const_down(ox, 0.5)
    same(gh, oh)
    gm, om = g.hmult(gh, gh), o.hmult(oh, oh)
    same(gm, om)
    same(g.rescale(gm), o.rescale(om))
    same(g.rotate(gh, 5), o.rotate(oh, 5))
    same(g.conjugate(gh), o.conjugate(oh))


@pytest.mark.parametrize("lvl", [27, 19, 9, 1])
def test_full_size_keyswitch_levels(pair16, lvl):
    """hmult (tensor + hybrid key switch with 3/2/1 digits) and rescale on
    uniform words at levels spanning every digit count."""
    g, o = pair16
    w = inputs.uniform_words((2, lvl + 1, g.N), g.primes[:lvl + 1], 70 + lvl)
    ga, oa = g.ct_import(w, lvl, 2.0 ** 40), o.ct_import(w, lvl, 2.0 ** 40)
    same(g.hmult(ga, ga), o.hmult(oa, oa))
    same(g.rescale(ga), o.rescale(oa))


def test_full_size_invsqrt_bit_exact_and_mre(pair16):
    """CryptoInvSqrt at N = 2^16, degree 31, 3 Newton steps, x log-uniform in
    [2^-10, 1] encrypted at level 13 with scale 2^50 (enough levels that no
    bootstrapping is needed): result bit-exact, MRE <= 3.1e-8."""
    g, o = pair16
    x = inputs.log_uniform(g.n, 2 ** -10, 1.0, 1)
    gx, ox = g.encrypt(x, 13, 2.0 ** 50, 3), o.encrypt(x, 13, 2.0 ** 50, 3)
    gy = g.invsqrt(gx, 31, 3)
    oy = o.invsqrt(ox, 31, 3, 2 ** -10, 1.0)
    same(gy, oy)
    ref = 1 / np.sqrt(x)
    mre = np.mean(np.abs(g.decrypt(gy).real - ref) / ref)
    assert mre <= 3.1e-8, mre


def test_full_size_batch_equals_single(pair16):
    """A batch of 3 ciphertexts through one launch sequence gives the same
    words as three single calls (N = 2^16, degree 31, 3 Newton steps)."""
    g, _ = pair16
    xs = [g.encrypt(inputs.log_uniform(g.n, 2 ** -10, 1.0, 30 + i), 13, 2.0 ** 50, 40 + i) for i in range(3)]
    outs = g.invsqrt_batch(xs, 31, 3)
    for x, y in zip(xs, outs):
        assert np.array_equal(g.invsqrt(x, 31, 3).words(), y.words())
