"""GPU tests of the batched workloads: batch encryption, batched z-score
standardisation (bit-exact against the oracle run column by column), and the
serving loop (each result identical alone and in the mix)."""
import math

import numpy as np
import pytest

from paper_2606_10477_amd import inputs

pytestmark = pytest.mark.gpu

# N = 2^12 with 24 scaling primes (insecure, test only): enough levels for
# squares, the two means, CryptoInvSqrt (degree 127, 3 steps) and the final product
SMALL = dict(log_n=12, max_level=24, num_special=1, digit_size=1, hamming_weight=0)


def _ck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_10477_amd import ckks
    return ckks


@pytest.fixture(scope="module")
def small(oracle_mod):
    ck = _ck()
    g = ck.Context(**SMALL)
    o = oracle_mod.Context(12, 24, 1, 1, h=0)
    gal = [g.galois_rot(1 << k) for k in range(11)]
    g.keygen(5, gal)
    o.keygen(5, gal)
    yield g, o
    g.close()


def test_encrypt_batch_equals_single(small):
    g, _ = small
    X = np.stack([inputs.log_uniform(g.n, 2 ** -8, 1.0, 60 + i) for i in range(5)])
    outs = g.encrypt_batch(X, 20, 2.0 ** 45, 900)
    for i in range(5):
        assert np.array_equal(outs[i].words(), g.encrypt(X[i], 20, 2.0 ** 45, 900 + i).words())


def _oracle_znorm(o, cts, rows, B, d, it, lo, hi):
    s1 = cts[0]
    sq = [o.rescale(o.hmult(x, x)) for x in cts]
    s2 = sq[0]
    for j in range(1, len(cts)):
        s1 = o.add(s1, cts[j])
        s2 = o.add(s2, sq[j])
    for acc_name in ("s1", "s2"):
        acc = s1 if acc_name == "s1" else s2
        k = 1
        while k < o.n:
            acc = o.add(acc, o.rotate(acc, k))
            k <<= 1
        if acc_name == "s1":
            s1 = acc
        else:
            s2 = acc
    lr, lb = int(math.log2(rows)), int(math.log2(B))
    m1 = o.rescale(o.mul_const(o.mul_const_down(s1, 1.0 / math.sqrt(B)), 2.0 ** -lr, 2.0 ** 40))
    m2 = o.rescale(o.mul_const(s2, 2.0 ** -(lr + lb), 2.0 ** 40))
    m1sq = o.rescale(o.hmult(m1, m1))
    lv = min(m1sq.level, m2.level) - 1
    v = o.sub(o.level_to(m2, lv), o.level_to(m1sq, lv))
    r = o.invsqrt(v, d, it, lo, hi)
    rs = o.mul_const_down(r, 1.0 / math.sqrt(B))
    mean = o.rescale(o.mul_const(s1, 2.0 ** -lr, 2.0 ** 40))
    z = []
    for x in cts:
        lvd = min(x.level, mean.level, rs.level + 1)
        diff = o.sub(o.level_to(x, lvd), o.level_to(mean, lvd))
        lvm = min(diff.level, rs.level)
        z.append(o.rescale(o.hmult(o.level_to(diff, lvm), o.level_to(rs, lvm))))
    return z, v, r


def test_znorm_batched_bit_exact_vs_oracle(small):
    from paper_2606_10477_amd import znorm
    g, o = small
    cols, per = 3, 2
    rows = per * g.n
    data, mu, sigma = inputs.column_table(rows, cols, 7)
    B, lo, hi, d, it = 128.0, 2.0 ** -14, 1.0, 127, 3
    gcols, ocols = [], []
    for c in range(cols):
        chunks = data[c].reshape(per, g.n)
        gcols.append([g.encrypt(chunks[j], 24, 2.0 ** 40, 100 * c + j) for j in range(per)])
        ocols.append([o.encrypt(chunks[j], 24, 2.0 ** 40, 100 * c + j) for j in range(per)])
    z, v, r = znorm.znorm(g, gcols, rows, B, d, it, lo, hi)
    vparts = g.unpack(v)
    for c in range(cols):
        oz, ov, orr = _oracle_znorm(o, ocols[c], rows, B, d, it, lo, hi)
        assert np.array_equal(vparts[c].words(), ov.words())
        for j in range(per):
            assert z[c][j].level == oz[j].level and z[c][j].scale == oz[j].scale
            assert np.array_equal(z[c][j].words(), oz[j].words())
    # accuracy against FP64 z-scores
    c = 0
    zz = np.concatenate([g.decrypt(z[c][j]).real for j in range(per)])
    ref = (data[c] - data[c].mean()) / data[c].std()
    assert np.max(np.abs(zz - ref)) < 1e-4


def _oracle_mean(o, cts, rows):
    """mean over all slots of a column's ciphertexts: sum the ciphertexts,
    rotate-and-sum over the slots, times 2^-log2(rows) as an exact integer
    plaintext at scale 2^40 and one rescale."""
    s = cts[0]
    for c in cts[1:]:
        s = o.add(s, c)
    k = 1
    while k < o.n:
        s = o.add(s, o.rotate(s, k))
        k <<= 1
    return o.rescale(o.mul_const(s, 2.0 ** -int(math.log2(rows)), 2.0 ** 40))


def _oracle_skew_kurt(o, z, rows):
    """Population skewness mean(z^3) and excess kurtosis mean(z^4) - 3 of one
    column's z-scores, on the oracle, written here from the definitions."""
    z2 = [o.rescale(o.hmult(v, v)) for v in z]
    z3 = [o.rescale(o.hmult(a, o.level_to(v, a.level))) for a, v in zip(z2, z)]
    z4 = [o.rescale(o.hmult(a, a)) for a in z2]
    return _oracle_mean(o, z3, rows), o.add_const(_oracle_mean(o, z4, rows), -3.0)


def _oracle_pcc(o, za, zb, rows):
    """Pearson correlation mean(z_a z_b) of two columns' z-scores."""
    return _oracle_mean(o, [o.rescale(o.hmult(a, b)) for a, b in zip(za, zb)], rows)


def test_moments_batched_bit_exact_vs_oracle(small):
    """Skewness, excess kurtosis and PCC (from the z-scores) of 3 skewed,
    pairwise-correlated columns, batched on the GPU (moments.py), against the
    oracle run column by column (pair by pair) through the composition
    written in this file from the definitions, word for word; values
    against FP64."""
    from paper_2606_10477_amd import moments, znorm
    g, o = small
    cols, per = 3, 2
    rows = per * g.n
    data, _, _ = inputs.skewed_table(rows, cols, 11)
    # degree 127: var / B reaches 1e-4 here, where degree 31 + 3 steps has not converged
    B, lo, hi, d, it = 128.0, 2.0 ** -14, 1.0, 127, 3
    gcols, ocols = [], []
    for c in range(cols):
        chunks = data[c].reshape(per, g.n)
        gcols.append([g.encrypt(chunks[j], 24, 2.0 ** 40, 200 * c + j) for j in range(per)])
        ocols.append([o.encrypt(chunks[j], 24, 2.0 ** 40, 200 * c + j) for j in range(per)])
    gz, _, _ = znorm.znorm(g, gcols, rows, B, d, it, lo, hi)
    oz = [_oracle_znorm(o, ocols[c], rows, B, d, it, lo, hi)[0] for c in range(cols)]
    pairs = [(0, 1), (1, 2)]
    gs, gk = moments.skew_kurt(g, gz, rows)
    gp = moments.pcc(g, gz, rows, pairs)
    for c in range(cols):
        os_, ok = _oracle_skew_kurt(o, oz[c], rows)
        assert np.array_equal(gs[c].words(), os_.words()), f"skewness column {c}"
        assert np.array_equal(gk[c].words(), ok.words()), f"kurtosis column {c}"
    for k, (a, b) in enumerate(pairs):
        op = _oracle_pcc(o, oz[a], oz[b], rows)
        assert np.array_equal(gp[k].words(), op.words()), f"pcc pair {a, b}"
    rs, rk, rp = moments.reference(data, pairs)
    for c in range(cols):
        assert abs(g.decrypt(gs[c]).real[0] - rs[c]) < 1e-4
        assert abs(g.decrypt(gk[c]).real[0] - rk[c]) < 1e-3
    for k in range(len(pairs)):
        assert abs(g.decrypt(gp[k]).real[0] - rp[k]) < 1e-4


def test_serving_alone_equals_in_the_mix(small):
    """Continuous batching on two lanes (contexts with the same keys, each on
    a stream of its own): groups of different requests run on the device at
    the same time, and every result equals the request run alone.  The table
    gives the level-16 3.1e-8 entry the level-12 setting at the same time,
    so that request is routed to level 12 (its inputs dropped) and shares a
    launch with the level-12 ones; alone it runs the same routed chain."""
    import torch
    from paper_2606_10477_amd import ckks, serve
    g, _ = small
    gal = [g.galois_rot(1 << k) for k in range(11)]
    lanes = []
    for _ in range(2):
        st = torch.cuda.Stream()
        lc = ckks.Context(**SMALL, stream=st.cuda_stream)
        lc.keygen(5, gal)
        lanes.append(serve.Lane(lc, st))
    table = {"12": {"1e-06": {"degree": 15, "iters": 2, "t_meas": 0.004},
                    "3.1e-08": {"degree": 15, "iters": 3, "t_meas": 0.005}},
             "16": {"1e-06": {"degree": 7, "iters": 3, "t_meas": 0.004},
                    "3.1e-08": {"degree": 15, "iters": 3, "t_meas": 0.005}}}
    sizes = [3, 1, 4, 2, 2]
    levels = [12, 16, 12, 16, 12]
    targets = [1e-6, 3.1e-8, 1e-6, 1e-6, 3.1e-8]
    reqs = []
    for k in range(5):
        X = np.stack([inputs.log_uniform(g.n, 2 ** -10, 1.0, 300 + 10 * k + j) for j in range(sizes[k])])
        cts = g.encrypt_batch(X, levels[k], 2.0 ** 45, 500 + 10 * k)
        reqs.append(serve.Request(k, 0.0, cts, levels[k], targets[k]))
    g.sync()
    srv = serve.run_continuous(lanes, table, reqs, max_batch=16, reserve_bytes=0)
    assert any(e["batch"] > max(sizes) for e in srv.log)   # requests shared a launch sequence
    assert srv.max_in_flight == 2                          # two groups on the device at once
    assert {e["lane"] for e in srv.log} == {0, 1}
    for ln in lanes:
        ln.ctx.sync()
    assert [r.run_level for r in reqs] == [12, 12, 12, 16, 12]
    for r in reqs:
        assert r.done is not None and r.done >= r.arrival
        cts = [c if c.level == r.run_level else g.drop_level(c, r.run_level) for c in r.cts]
        alone = g.invsqrt_batch(cts, r.degree, r.iters)
        for k, y in enumerate(alone):
            assert np.array_equal(r.outs[k].words(), y.words())
    for r in reqs:
        r.outs = {}
    for ln in lanes:
        ln.ctx.close()


def test_znorm_full_size_accuracy():
    """N = 2^16 parameters, 4 columns of 2^17 rows (4 ciphertexts each),
    invsqrt (127, 3) on the variance domain [2^-14, 1]: z-scores against FP64."""
    ck = _ck()
    from paper_2606_10477_amd import znorm
    g = ck.Context.from_set("p16")
    g.keygen(9, [g.galois_rot(s) for s in znorm.rotation_steps(g.n)])
    cols, per = 4, 4
    rows = per * g.n
    data, _, _ = inputs.column_table(rows, cols, 8)
    gcols = []
    for c in range(cols):
        gcols.append(g.encrypt_batch(data[c].reshape(per, g.n), 22, 2.0 ** 40, 1000 + 10 * c))
    z, v, r = znorm.znorm(g, gcols, rows, 128.0, 127, 3, 2.0 ** -14, 1.0)
    errs = []
    for c in range(cols):
        zz = np.concatenate([g.decrypt(z[c][j]).real for j in range(per)])
        ref = (data[c] - data[c].mean()) / data[c].std()
        errs.append(float(np.mean(np.abs(zz - ref))))
    print("znorm full size: mean absolute z error per column", errs, flush=True)
    assert max(errs) < 1e-5
    g.close()
