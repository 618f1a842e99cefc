"""Word-for-word parity of the benchmarked workload at full size (N = 2^16,
the benchmark's bootstrapping set "p16b" and the set with 11 computation
levels "p16c"; paper §2.1 bootstrapping and Alg. 1), through the C-ABI,
against digests the oracle wrote (tests/golden/fullsize_chain_<set>.json, by
make_fullsize_golden.py, which calls only the oracle): after the
encryption, the Chebyshev step, ModRaise, CoeffToSlot, the conjugation and
the real/imaginary split, both EvalMods, SlotToCoeff, the whole bootstrap,
the whole CryptoInvSqrt (31, 3) chain, the tuned (63, 2) chain (no
bootstrap from p16c's top level), the (31, 3) chain with Pre-BTS (c = 1) and
the paper's domain (linspace(0.001, 100), B = 100, degree 126, 3 steps), the
GPU's level, scale and SHA-256 of all words must equal the oracle's.  The GPU runs
in the benchmark's launch configuration (one ciphertext, the library's
default schedules).
"""
import json
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import fullsize_chain as F  # noqa: E402

from paper_2606_10477_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["p16b", "p16c"])
def test_fullsize_chain_words_equal_the_oracle(name):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_10477_amd import ckks
    with open(os.path.join(HERE, "golden", f"fullsize_chain_{name}.json")) as f:
        want = json.load(f)["steps"]
    g = ckks.Context.from_set(name)
    try:
        g.keygen(F.KEY_SEED, g.bts_galois())
        x = inputs.log_uniform(g.n, F.LO, F.HI, F.INPUT_SEED)
        bad = []

        def check(step, d):
            w = want[step]
            ok = (d["level"], d["scale"], d["sha256"]) == (w["level"], w["scale"], w["sha256"])
            diff = [s for s, t in zip(d["samples"], w["samples"]) if s != t]
            print(f"{step}: level {d['level']} {'equal' if ok else 'DIFFERENT'}"
                  + ("" if ok else f" (level {w['level']}, scale {w['scale']} vs {d['scale']}, "
                                   f"{len(diff)} of {len(d['samples'])} sampled words differ, e.g. {diff[:3]})"),
                  flush=True)
            if not ok:
                bad.append(step)

        got = F.run(g, x, on_step=check, x_paper=inputs.linspace_input(g.n, F.PAPER_LO, F.PAPER_HI))
        assert set(got) == set(want)
        assert not bad, f"steps whose words differ from the oracle's: {bad}"
    finally:
        g.close()
