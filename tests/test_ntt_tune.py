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


def test_word_size_prime_helpers():
    # primality against trial division on small numbers and known large primes / composites
    def trial(n):
        return n > 1 and all(n % d for d in range(2, int(n ** 0.5) + 1))
    assert [n for n in range(2000) if ntt_tune._is_prime(n)] == [n for n in range(2000) if trial(n)]
    assert ntt_tune._is_prime(998244353) and ntt_tune._is_prime(2 ** 61 - 1)
    assert not ntt_tune._is_prime(3215031751)          # strong pseudoprime to bases 2, 3, 5, 7
    assert not ntt_tune._is_prime((2 ** 31 - 1) * (2 ** 19 - 1))
    q = ntt_tune.prime_below(30, 1 << 17)
    assert q < 2 ** 30 and q % (1 << 17) == 1 and trial(q)
    assert all(not trial(p) for p in range(q + (1 << 17), 2 ** 30, 1 << 17))


def test_word_size_counters(tmp_path):
    # two cases, one warm-up + 20 timed dispatches each, in case order; the warm-up's
    # counters (here 10x larger) must not enter the averages
    per = ntt_tune.WS_THREADS * ntt_tune.WS_ROUNDS * 12
    lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    did = 0
    for ipb in (24.0, 6.0):
        for k in range(21):
            did += 1
            v = ipb * per / 64 * (10 if k == 0 else 1)
            lines.append(f"{did},void gpu::k_butterfly_rate<0>(),SQ_INSTS_VALU,{v / 2}")
            lines.append(f"{did},void gpu::k_butterfly_rate<0>(),SQ_INSTS_VALU,{v / 2}")   # two instances summed
            lines.append(f"{did},other(),SQ_INSTS_VALU,1")
    (tmp_path / "run_counter_collection.csv").write_text("\n".join(lines) + "\n")
    cases = [{"form": "u64", "butterflies_per_s": 1e12}, {"form": "u32", "butterflies_per_s": 3e12}]
    rows = ntt_tune.word_size_counters(str(tmp_path), cases)
    assert [round(r["SQ_INSTS_VALU_per_butterfly"], 6) for r in rows] == [24.0, 6.0]
    peak = 256 * 2.4e9 * 64
    assert abs(rows[0]["valu_bound_butterflies_per_s"] - peak / 24) < 1
    assert abs(rows[1]["valu_issue_pct"] - 100 * 3e12 / (peak / 6)) < 1e-9
