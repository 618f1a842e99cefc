"""The stored oracle digests are current and describe the level schedule the
paper fixes (CPU only).

fullsize_chain_p16b.json must have been written from the present oracle,
parameter sets and recipe (else regenerate it with
tests/golden/make_fullsize_golden.py).  Its levels follow from the method:
input at the top level 8; the affine map (one level) and a degree-31
Chebyshev evaluation (5 levels, §4.3's d_e) leave y0 at 2; ModRaise to the
top of the chain (23); CoeffToSlot three levels; EvalMod 5 + 4 double angles;
SlotToCoeff three more, ending on l_afterBTS = 8; CryptoInvSqrt (31, 3) ends
at 3 (one Newton step at 2, bootstrap to 8, steps at 7 and 5).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_fullsize_golden as M  # noqa: E402


def test_fullsize_golden_is_current():
    with open(M.OUT) as f:
        rec = json.load(f)
    assert rec["sources_sha256"] == M.source_digest(), \
        "oracle, parameter sets or recipe changed: rerun tests/golden/make_fullsize_golden.py"


def test_fullsize_golden_levels():
    with open(M.OUT) as f:
        st = json.load(f)["steps"]
    lv = {k: v["level"] for k, v in st.items()}
    assert lv == {"enc": 8, "cheb": 2, "raise": 23, "cts": 20, "conj": 20, "re": 20, "im": 20,
                  "evm_re": 11, "evm_im": 11, "stc": 8, "bts": 8, "invsqrt": 3}
    assert all(len(v["sha256"]) == 64 for v in st.values())
