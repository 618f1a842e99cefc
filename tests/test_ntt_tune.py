"""Host logic of the NTT schedule tuner: the limb-count bounds it derives
from timed rows."""
from paper_2606_10477_amd import ntt_tune


def _row(n, t4, t8, t16, t4s4=None):
    t4s4 = 2 * t4 if t4s4 is None else t4s4
    return {"limbs": n, "fwd_R4s4_us": t4s4, "inv_R4s4_us": t4s4, "fwd_R4_us": t4, "inv_R4_us": t4,
            "fwd_R8_us": t8, "inv_R8_us": t8, "fwd_R16_us": t16, "inv_R16_us": t16}


def test_choose_bounds():
    rows = [_row(1, 5, 6, 7), _row(4, 6, 7, 8), _row(16, 9, 8, 10), _row(32, 12, 11, 11.5), _row(64, 20, 19, 18)]
    r4, r8, s4, best = ntt_tune.choose(rows)
    assert (r4, r8, s4) == (4, 32, 0)
    assert [b for _, b in best] == [4, 4, 8, 8, 16]


def test_choose_never_small():
    rows = [_row(1, 9, 8, 7), _row(8, 9, 8, 7)]
    assert ntt_tune.choose(rows)[:2] == (0, 0)


def test_choose_stops_at_first_loss():
    # a later win of the 4-word variant after a loss does not extend the bound
    rows = [_row(1, 5, 6, 7), _row(2, 8, 6, 7), _row(3, 5, 6, 7)]
    assert ntt_tune.choose(rows)[:2] == (1, 2)


def test_choose_tolerates_near_ties():
    # 24 limbs: the 4-word variant is 0.5 % slower than the 16-word one
    rows = [_row(16, 10, 11, 11), _row(24, 27.25, 28, 27.1), _row(32, 28, 29, 29), _row(40, 36, 36, 33)]
    assert ntt_tune.choose(rows)[:2] == (32, 32)
    assert ntt_tune.choose(rows, tol=0.0)[:2] == (16, 16)


def test_choose_small_workgroups():
    # 4 sub-transforms per workgroup win up to 2 limbs, 16 per workgroup up to 8
    rows = [_row(1, 5, 6, 7, 4), _row(2, 6, 7, 8, 5.9), _row(4, 6, 7, 8, 6.5), _row(8, 7, 8, 9, 8),
            _row(16, 9, 8, 10, 12)]
    r4, r8, s4, best = ntt_tune.choose(rows)
    assert (r4, r8, s4) == (8, 16, 2)
    assert [b for _, b in best] == ["4s4", "4s4", 4, 4, 8]
