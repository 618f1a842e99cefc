"""The entry point that allocates nothing (ckks_hmult_relin_noalloc): through
the C-ABI, its words equal ckks_hmult_relin's on two calls in a row, the
second with a smaller input (a lower level), on the N = 2^12 set and on the
N = 2^16 plain set; a product needing more than the scratch array holds is
refused before anything runs."""
import numpy as np
import pytest

from paper_2606_10477_amd import inputs

pytestmark = pytest.mark.gpu


def _ck():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_10477_amd import ckks
    return ckks


def _check(g, level, seed):
    import torch
    x = inputs.log_uniform(g.n, 2.0 ** -8, 1.0, seed)
    y = inputs.log_uniform(g.n, 2.0 ** -8, 1.0, seed + 1)
    a = g.encrypt(x, level, g.ladder[level], seed + 2)
    b = g.encrypt(y, level, g.ladder[level], seed + 3)
    want = g.hmult(a, b)
    out = torch.zeros(2 * (level + 1) * g.N, dtype=torch.int64, device="cuda")
    sc = g.hmult_noalloc(a, b, out.data_ptr())
    g.sync()
    got = out.cpu().numpy().view(np.uint64).reshape(2, level + 1, g.N)
    print(f"N={g.N} level {level}: noalloc product vs hmult_relin", flush=True)
    assert sc == want.scale
    assert np.array_equal(got, want.words())


def test_noalloc_product_equals_hmult_small():
    ck = _ck()
    g = ck.Context.from_set("p12")
    try:
        g.keygen(5)
        _check(g, 13, 10)
        _check(g, 4, 20)
    finally:
        g.close()


def test_noalloc_product_equals_hmult_full_size():
    ck = _ck()
    g = ck.Context.from_set("p16")
    try:
        g.keygen(6)
        _check(g, 20, 30)
        _check(g, 6, 40)
        # level 27 needs 259 limbs of 512 KiB, more than the array's 128 MiB
        import torch
        x = inputs.log_uniform(g.n, 2.0 ** -8, 1.0, 50)
        a = g.encrypt(x, 27, g.ladder[27], 51)
        out = torch.zeros(2 * 28 * g.N, dtype=torch.int64, device="cuda")
        with pytest.raises(ck.CkksError) as e:
            g.hmult_noalloc(a, a, out.data_ptr())
        assert "scratch" in str(e.value)
    finally:
        g.close()
