"""Pins of the oracle's bootstrapping (paper §2.1 BTS) against facts that do
not come from the oracle itself:

* ModRaise: the raised ciphertext decrypts, exactly (big-integer CRT of the
  residues, secret key from the oracle), to m + q_0 I with I an integer
  polynomial of small norm, and to m again modulo q_0;
* CoeffToSlot: slots of the output hold (p_k + i p_{k+n}) / (2 q_0 K) in
  bit-reversed order, p the exact raised plaintext (numpy, from the
  definition of the canonical embedding's coefficient packing);
* EvalMod: the output equals sin(2 pi K u) for the decrypted input u
  (closed form of cos(2^r theta) composed with the shift by a quarter turn);
* monomials: X^(N/2) multiplies every slot by i, X^N is negation (compared
  with the integer multiply by -1), X^(2N) is the identity;
* bootstrap and CryptoInvSqrt with bootstrapping: decrypted values against
  FP64 (values / 1/sqrt(x)).
"""
import numpy as np
import pytest

from paper_2606_10477_amd import inputs

BTS = (3, 9, 3, 52)


@pytest.fixture(scope="module")
def o8(oracle_mod):
    o = oracle_mod.Context(8, 3, 2, 2, h=16, bts=BTS)
    o.bts_config(25.0, 4, 31)
    o.keygen(3, o.bts_galois())
    return o


@pytest.fixture(scope="module")
def o10(oracle_mod):
    o = oracle_mod.Context(10, 8, 2, 2, h=192, bts=BTS)
    o.bts_config(25.0, 4, 31)
    o.keygen(4, o.bts_galois())
    return o


def test_bootstrapping_chain_shape(o10):
    o = o10
    bits = [int(p).bit_length() for p in o.primes]
    N = o.N
    assert o.L == 8 + 15
    assert bits[0] == 60
    assert all(40 <= b <= 41 for b in bits[1:12])          # computation + SlotToCoeff
    assert all(52 <= b <= 53 for b in bits[12:24])         # EvalMod + CoeffToSlot
    assert len(set(int(p) for p in o.primes)) == len(o.primes)
    assert all(int(p) % (2 * N) == 1 for p in o.primes)
    # canonical scales: ~2^40 on the computation levels, ~2^52 on EvalMod
    assert np.all(np.abs(np.log2(o.ladder[:9]) - 40) < 1e-3)
    assert np.all(np.abs(np.log2(o.ladder[11:21]) - 52) < 1e-3)
    with pytest.raises(Exception):
        o.bts_config(25.0, 3, 31)                           # depth 5 + 3 != 9 EvalMod levels


def _exact_plain(o, ct):
    """Exact centred plaintext c0 + c1 s of a ciphertext (Python big ints)."""
    w = ct.words()
    s = o.secret().astype(int)
    nz = np.nonzero(s)[0]
    L = ct.level
    N = o.N
    qs = [int(q) for q in o.primes[:L + 1]]
    res = []
    for i, q in enumerate(qs):
        c0 = [int(v) for v in o.intt(i, w[0, i])]
        c1 = [int(v) for v in o.intt(i, w[1, i])]
        m = list(c0)
        for j in nz:
            sj = int(s[j])
            for k in range(N):
                t = k + j
                if t < N:
                    m[t] = (m[t] + sj * c1[k]) % q
                else:
                    m[t - N] = (m[t - N] - sj * c1[k]) % q
        res.append(m)
    Q = 1
    for q in qs:
        Q *= q
    out = []
    for k in range(N):
        x = 0
        for i, q in enumerate(qs):
            Qi = Q // q
            x += res[i][k] * Qi * pow(Qi, -1, q)
        x %= Q
        out.append(x - Q if x > Q // 2 else x)
    return out


def _bitrev(n):
    b = n.bit_length() - 1
    return np.array([int(format(i, '0%db' % b)[::-1], 2) for i in range(n)])


def test_mod_raise_invariant_and_coeff_to_slot(o8):
    o = o8
    q0 = int(o.primes[0])
    x = inputs.log_uniform(o.n, 1.0, 32.0, 1)
    ct = o.encrypt(x, 0, o.ladder[0], 5)
    m0 = _exact_plain(o, ct)                     # centred mod q_0
    raised = o.mod_raise(ct)
    assert raised.level == o.L
    p = _exact_plain(o, raised)
    I = [(pk - mk) // q0 for pk, mk in zip(p, m0)]
    assert all((pk - mk) % q0 == 0 for pk, mk in zip(p, m0))
    assert max(abs(i) for i in I) <= 12            # h = 16: |I| well below K = 25
    assert max(abs(i) for i in I) >= 1
    # CoeffToSlot: slot k holds (p_br(k) + i p_{br(k)+n}) / (2 q_0 K)
    y = o.coeff_to_slot(raised)
    assert y.level == o.L - 3
    z = o.decrypt(y)
    n = o.n
    br = _bitrev(n)
    K = 25.0
    want = (np.array([p[k] for k in br], dtype=float) + 1j * np.array([p[k + n] for k in br], dtype=float)) / (2 * q0 * K)
    assert np.max(np.abs(z - want)) < 1e-9


def test_eval_mod_is_the_shifted_cosine_composition(o8):
    o = o8
    K = 25.0
    rng = np.random.default_rng(3)
    t = rng.integers(-10, 11, o.n) + rng.uniform(-0.01, 0.01, o.n)
    u = t / K
    ct = o.encrypt(u, o.L - 3, o.ladder[o.L - 3], 6)
    e = o.eval_mod(ct)
    assert e.level == o.l_after + 3
    got = o.decrypt(e).real
    assert np.max(np.abs(got - np.sin(2 * np.pi * K * u))) < 1e-7


def test_monomials(o8):
    o = o8
    x = inputs.log_uniform(o.n, 1.0, 2.0, 2)
    ct = o.encrypt(x, 2, o.ladder[2], 7)
    N = o.N
    z = o.decrypt(ct)
    zi = o.decrypt(o.mul_monomial(ct, N // 2))
    assert np.max(np.abs(zi - 1j * z)) < 1e-9
    assert np.array_equal(o.mul_monomial(ct, N).words(), o.mul_int(ct, -1).words())
    assert np.array_equal(o.mul_monomial(o.mul_monomial(ct, N // 2), 3 * N // 2).words(), ct.words())


def test_bootstrap_accuracy(o10):
    o = o10
    x = inputs.log_uniform(o.n, 1.0, 32.0, 3)
    ct = o.encrypt(x, 1, o.ladder[1], 8)
    b = o.bootstrap(ct, 512)
    assert b.level == o.l_after
    assert abs(np.log2(b.scale) - 40) < 1e-3
    rel = np.abs(o.decrypt(b).real - x) / x
    assert np.mean(rel) < 1e-4 and np.max(rel) < 1e-3


def test_invsqrt_with_lazy_bootstrap(o10):
    o = o10
    lo, hi = 2.0 ** -10, 1.0
    x = inputs.log_uniform(o.n, lo, hi, 4)
    ct = o.encrypt(x, 8, 2.0 ** 50, 9)
    y = o.invsqrt(ct, 31, 3, lo, hi)
    ref = 1 / np.sqrt(x)
    # 8 -> affine 7 -> Chebyshev (5 levels) 2 -> Newton 0 -> BTS 8 -> Newton
    # (x/2 at 7) 5 -> last Newton (x at 8) 3
    assert y.level == 3
    assert np.mean(np.abs(o.decrypt(y).real - ref) / ref) < 1e-7


def test_hoisted_rotations_roll_the_slots(o8):
    """Hoisted rotations (one ModUp for several automorphisms) decrypt to the
    rolled slot vector, as the plain rotation does; their words differ from
    the plain rotation's only by key-switching noise."""
    o = o8
    x = inputs.log_uniform(o.n, 1.0, 2.0, 11)
    ct = o.encrypt(x, 5, o.ladder[5], 12)
    steps = o.bts_rotations()[:3]
    outs = o.rotate_hoisted(ct, [0] + steps)
    assert np.array_equal(outs[0].words(), ct.words())
    for k, r in zip(steps, outs[1:]):
        assert np.max(np.abs(o.decrypt(r).real - np.roll(x, -k))) < 1e-6
        plain = o.decrypt(o.rotate(ct, k)).real
        assert np.max(np.abs(o.decrypt(r).real - plain)) < 1e-6


def _plain_chain(x, cf, lo, hi, iters):
    """FP64 CryptoInvSqrt: Chebyshev value of the same coefficients, then the
    Newton iteration of §2.2 (no encryption)."""
    t = (2 * x - lo - hi) / (hi - lo)
    y = np.polynomial.chebyshev.chebval(t, cf)
    for _ in range(iters):
        y = 0.5 * y * (3 - x * y * y)
    return y


def test_invsqrt_literal_branch(oracle_mod, o10):
    """Alg. 1 as printed bootstraps y0 right after the Chebyshev step (its
    line 4).  From level 8 with degree 15: y0 at 8 - 1 - 4 = 3 is
    bootstrapped to 8, then the three Newton steps run at 7, 5 and 3 (the
    last one on x itself at 8), ending at 1 -- two levels lower than the lazy
    schedule (no bootstrap until a step lacks levels, ending at 3).  The
    result follows the FP64 chain: the bootstrap's error in y0 (~1e-4 at
    message bound 512) is squared away by the Newton steps."""
    o = o10
    lo, hi = 2.0 ** -10, 1.0
    x = inputs.log_uniform(o.n, lo, hi, 21)
    ct = o.encrypt(x, 8, 2.0 ** 50, 22)
    cf = oracle_mod.cheb_coeffs_invsqrt(15, lo, hi)
    lit = o.invsqrt(ct, 15, 3, lo, hi, literal=True)
    lazy = o.invsqrt(ct, 15, 3, lo, hi)
    assert lit.level == 1 and lazy.level == 3
    plain = _plain_chain(x, cf, lo, hi, 3)
    ref = 1 / np.sqrt(x)
    mre_plain = np.mean(np.abs(plain - ref) / ref)     # degree 15, 3 steps: ~1.4e-4 in FP64
    for y in (lit, lazy):
        z = o.decrypt(y).real
        assert np.max(np.abs(z - plain) / ref) < 1e-5
        assert abs(np.mean(np.abs(z - ref) / ref) - mre_plain) < 0.01 * mre_plain


def test_invsqrt_pre_bts_branch(oracle_mod, o10):
    """Pre-BTS (§4.2's c = 1): x is bootstrapped first (message bound
    16 ceil(b)) and the whole chain -- the Chebyshev step, ct_x and the last
    step's x -- then runs on the bootstrapped x~.  So the result is the FP64
    chain applied to x~ (the decrypted bootstrap of x, computed separately),
    up to the chain's own noise, while against 1/sqrt(x) it carries x~'s error
    (the Pre-BTS floor).  Forced by the level (5 < depth 5 + 1 for degree 31)
    and asked for at level 8; the bootstrapped x sits at l_afterBTS = 8."""
    o = o10
    lo, hi = 2.0 ** -10, 1.0
    x = inputs.log_uniform(o.n, lo, hi, 23)
    for level, ask, d, it in ((5, False, 31, 2), (8, True, 15, 3)):
        ct = o.encrypt(x, level, 2.0 ** 50, 24 + level)
        y = o.invsqrt(ct, d, it, lo, hi, pre_bts=ask)
        xb = o.decrypt(o.bootstrap(ct, 16)).real
        cf = oracle_mod.cheb_coeffs_invsqrt(d, lo, hi)
        want = _plain_chain(xb, cf, lo, hi, it)
        z = o.decrypt(y).real
        ref = 1 / np.sqrt(x)
        assert np.max(np.abs(z - want) / ref) < 1e-5
        # the floor: x~'s relative error passes to 1/sqrt as half of it
        floor = np.mean(np.abs(xb - x) / x) / 2
        assert np.mean(np.abs(z - ref) / ref) < 4 * floor + 1e-6
        assert np.mean(np.abs(z - ref) / ref) > floor / 4


def test_invsqrt_pre_bts_prenormalised(oracle_mod, o10):
    """Pre-BTS in the paper's domain (x in [0.001, 100], B = 100): x itself
    cannot be bootstrapped at scale 2^50 (its bound exceeds the room the
    60-bit q0 leaves above the scale), so the chain first divides by B (one
    level) and bootstraps u = x/B with bound 16; the Chebyshev step then runs
    on [a/B, b/B] directly and the Newton steps on u~, scaled back by
    1/sqrt(B).  The result is the FP64 chain on u~ (the decrypted bootstrap of
    u, computed separately through the same public operations) times
    1/sqrt(B), up to the chain's noise; against 1/sqrt(x) it carries the
    approximation's own error plus u~'s relative error halved.  Asked for at level 8 and forced at level 4
    (degree 30 needs 5 + 1 levels)."""
    o = o10
    A, Bv, Bn = 0.001, 100.0, 100.0
    x = np.linspace(A, Bv, o.n)
    ref = 1 / np.sqrt(x)
    for level, ask, d, it in ((8, True, 14, 3), (4, False, 30, 2)):
        ct = o.encrypt(x, level, 2.0 ** 50, 60 + level)
        y = o.invsqrt(ct, d, it, A, Bv, pre_bts=ask, B=Bn)
        ut = o.decrypt(o.bootstrap(o.mul_const_down(ct, 1.0 / Bn), 16)).real
        cf = oracle_mod.cheb_coeffs_invsqrt(d, A / Bn, Bv / Bn)
        want = _plain_chain(ut, cf, A / Bn, Bv / Bn, it) / np.sqrt(Bn)
        z = o.decrypt(y).real
        assert np.max(np.abs(z - want) / ref) < 1e-5
        floor = np.mean(np.abs(ut - x / Bn) / (x / Bn)) / 2
        plain = _plain_chain(x / Bn, cf, A / Bn, Bv / Bn, it) / np.sqrt(Bn)   # the approximation's own error
        m, m_plain = np.mean(np.abs(z - ref) / ref), np.mean(np.abs(plain - ref) / ref)
        assert floor / 4 < m < m_plain + 4 * floor + 1e-5
    # without B the input's bound (100) does not fit the bootstrap at this scale
    with pytest.raises(oracle_mod.OracleError):
        o.invsqrt(o.encrypt(x, 8, 2.0 ** 50, 68), 14, 3, A, Bv, pre_bts=True)


def _bitrev_idx(n):
    b = n.bit_length() - 1
    return np.array([int(format(i, '0%db' % b)[::-1], 2) for i in range(n)])


def test_slot_to_coeff_is_the_packing(o8):
    """SlotToCoeff of a fresh ciphertext with slots w (at the EvalMod output
    level l_afterBTS + 3) yields the polynomial whose coefficients k' = br(k)
    and br(k) + n hold Re(w_k) and Im(w_k) (the inverse of CoeffToSlot's
    packing, pinned in test_mod_raise_invariant_and_coeff_to_slot) times the
    constant q_0 / (2 pi s_0) = 2^5 / (2 pi) that SlotToCoeff absorbs (the
    sine's 1/(2 pi) and the content scale s_0 = q_0 2^-5 of a unit message).
    Checked on the decrypted coefficients (numpy, no transform)."""
    o = o8
    rng = np.random.default_rng(8)
    n, N = o.n, o.N
    wr, wi = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    lv = o.l_after + 3
    cr = o.encrypt(wr, lv, o.ladder[lv], 31)
    ci = o.encrypt(wi, lv, o.ladder[lv], 32)
    w = o.add(cr, o.mul_monomial(ci, N // 2))
    z = o.slot_to_coeff(w)
    assert z.level == o.l_after
    m = o.decrypt_coeffs(z) / z.scale
    br = _bitrev_idx(n)
    want = np.zeros(N)
    want[br] = wr
    want[br + n] = wi
    want *= 2.0 ** 5 / (2 * np.pi)
    assert np.max(np.abs(m - want)) < 1e-6


@pytest.mark.parametrize("name,l_after,digit,K", [("p16b", 8, 8, 7), ("p16c", 11, 5, 5)])
def test_full_size_bootstrapping_sets_budget(oracle_mod, name, l_after, digit, K):
    """The N = 2^16 bootstrapping sets (§2.1: log2 QP ~ 1555 for 128-bit
    security, l_afterBTS 11 to 12 in the paper's HEaaN set): prime sizes by
    role, every prime = 1 mod 2N and distinct, the special modulus above every
    digit of hybrid key switching, and the total modulus within 1540..1560 bits."""
    o = oracle_mod.Context.from_set(name, bootstrapping=False)
    ps = [int(p) for p in o.primes]
    L = l_after + 15
    assert o.l_after == l_after and o.L == L and len(ps) == L + 1 + K
    bits = [p.bit_length() for p in ps]
    assert bits[0] == 60 and all(40 <= b <= 41 for b in bits[1:l_after + 4])
    assert all(52 <= b <= 53 for b in bits[l_after + 4:L + 1]) and all(b == 60 for b in bits[L + 1:])
    assert len(set(ps)) == len(ps) and all(p % (2 * o.N) == 1 for p in ps)
    logp = [np.log2(float(p)) for p in ps]
    digits = [sum(logp[i:min(i + digit, L + 1)]) for i in range(0, L + 1, digit)]
    assert o.dnum == len(digits) and max(digits) < sum(logp[L + 1:])
    assert 1540 < sum(logp) < 1560
