"""The stored oracle digests are current and describe the level schedule the
paper fixes (CPU only).

fullsize_chain_<set>.json must have been written from the present oracle,
recipe and parameter set (else regenerate it with
tests/golden/make_fullsize_golden.py <set>).  Its levels follow from the
method.  On p16b: input at the top level 8; the affine map (one level) and a
degree-31 Chebyshev evaluation (5 levels, §4.3's d_e) leave y0 at 2;
ModRaise to the top of the chain (23); CoeffToSlot three levels; EvalMod 5 +
4 double angles; SlotToCoeff three more, ending on l_afterBTS = 8;
CryptoInvSqrt (31, 3) ends at 3 (one Newton step at 2, bootstrap to 8, steps
at 7 and 5).  On p16c (11 computation levels, the same bootstrap): y0 at 5,
ModRaise to 26, CoeffToSlot to 23, EvalMod to 14, SlotToCoeff to 11;
CryptoInvSqrt (31, 3) ends at 9 (Newton steps at 5 and 3 down to 1, bootstrap
to 11, the last step at 11).  The tuned step (63, 2): on p16c y0 at 4 and
two Newton steps down to 0, no bootstrap; on p16b y0 at 1, bootstrap to 8,
steps at 7 and 5, ending at 3.  With Pre-BTS x is bootstrapped to the top
level first, and the levels are those of the plain (31, 3) chain (3 / 9).
The paper's domain (126, 3) with B = 100: the affine map and degree 126 take
8 levels, so on p16b y0 is at 0, bootstrapped to 8, steps at 7, 5 and 3 end
at 1; on p16c y0 at 3, one step to 1, bootstrap to 11, steps at 10 and 8 end
at 6.
"""
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_fullsize_golden as M  # noqa: E402

LEVELS = {
    "p16b": {"enc": 8, "cheb": 2, "raise": 23, "cts": 20, "conj": 20, "re": 20, "im": 20,
             "evm_re": 11, "evm_im": 11, "stc": 8, "bts": 8, "invsqrt": 3, "invsqrt_tuned": 3,
             "invsqrt_pre": 3, "invsqrt_paper": 1},
    "p16c": {"enc": 11, "cheb": 5, "raise": 26, "cts": 23, "conj": 23, "re": 23, "im": 23,
             "evm_re": 14, "evm_im": 14, "stc": 11, "bts": 11, "invsqrt": 9, "invsqrt_tuned": 0,
             "invsqrt_pre": 9, "invsqrt_paper": 6},
}


@pytest.mark.parametrize("name", M.SETS)
def test_fullsize_golden_is_current(name):
    with open(M.out_path(name)) as f:
        rec = json.load(f)
    assert rec["sources_sha256"] == M.source_digest(name), \
        f"oracle, parameter set or recipe changed: rerun tests/golden/make_fullsize_golden.py {name}"


@pytest.mark.parametrize("name", M.SETS)
def test_fullsize_golden_levels(name):
    with open(M.out_path(name)) as f:
        st = json.load(f)["steps"]
    lv = {k: v["level"] for k, v in st.items()}
    assert lv == LEVELS[name]
    assert all(len(v["sha256"]) == 64 for v in st.values())
