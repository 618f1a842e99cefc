"""Host logic of the paper's provisioning algorithms (Alg. 2, Alg. 3) and of
the cost model; no GPU."""
import math

import pytest

from paper_2606_10477_amd import tuner


def test_threshold_worked_example():
    # MRE_min = 2.94e-8 -> l = -8, alpha = 2.94; with delta = 1 the threshold is 3e-8
    alpha, l = tuner.mantissa_exponent(2.94e-8)
    assert l == -8 and abs(alpha - 2.94) < 1e-12
    assert abs(tuner.threshold(2.94e-8, 1) - 3e-8) < 1e-20
    assert abs(tuner.threshold(2.94e-8, 0.5) - 2.5e-8) < 1e-20


@pytest.mark.parametrize("m", [1e-8, 1e-3, 1.0, 100.0, 7.0e-9, 9.999999e-5])
def test_mantissa_in_range(m):
    alpha, l = tuner.mantissa_exponent(m)
    assert 1.0 <= alpha < 10.0
    assert math.isclose(alpha * 10.0 ** l, m, rel_tol=1e-12)


def test_mantissa_rejects_nonpositive():
    with pytest.raises(ValueError):
        tuner.mantissa_exponent(0.0)


def test_get_opt_iter_smallest_within_threshold():
    # Newton MRE curve that falls then floors at noise: the first iteration
    # within (floor(alpha)+delta)*10^l of the minimum is chosen, not the argmin
    M = [2e-3, 2e-5, 3.4e-8, 3.1e-8, 3.05e-8, 3.2e-8]
    T = [1, 2, 3, 4, 5, 6]
    I, m, t = tuner.get_opt_iter(M, T, delta=1)
    assert (I, m, t) == (3, 3.4e-8, 3)          # threshold 4e-8
    I, m, t = tuner.get_opt_iter(M, T, delta=0.1)
    assert (I, m, t) == (4, 3.1e-8, 4)          # threshold 3.1e-8
    # delta below the mantissa fraction empties the set -> argmin fallback
    I, m, t = tuner.get_opt_iter(M, T, delta=0.0)
    assert (I, m) == (5, 3.05e-8)


def test_optimize_params_u1_u2():
    D = {7: [dict(d=126, c=0, i=5, m=3.06e-8, t=0.68), dict(d=126, c=1, i=4, m=9.25e-7, t=0.35),
             dict(d=14, c=0, i=12, m=3.2e-8, t=0.90), dict(d=62, c=0, i=6, m=5.0e-8, t=0.50)]}
    R = tuner.optimize_params(D, theta=1)
    # m_theta = (3 + 1) e-8: accuracy-first picks the fastest tuple within it
    assert R[7] == ((126, 0, 5), (126, 1, 4))
    R = tuner.optimize_params(D, theta=3)       # m_theta = 6e-8 admits (62, 0, 6)
    assert R[7][0] == (62, 0, 6)


def test_level_cases_lattigo_and_heaan_sets():
    # Lattigo: l_BTS = 0, l_afterBTS = l_max = 11 -> 11 levels; c = 0 only
    # possible from level 3, c = 1 only below level 10
    cases = tuner.level_cases(0, 11, 11)
    assert sorted(cases) == list(range(1, 12))
    assert [l for l, cs in cases.items() if cs == [0]] == [10, 11]
    assert [l for l, cs in cases.items() if cs == [1]] == [1, 2]
    assert all(cs == [0, 1] for l, cs in cases.items() if 3 <= l <= 9)
    # HEaaN FGb: (l_max, l_BTS, l_afterBTS) = (12, 3, 12) -> levels 4..12 (9 levels)
    cases = tuner.level_cases(3, 12, 12)
    assert sorted(cases) == list(range(4, 13))
    assert [l for l, cs in cases.items() if cs == [0]] == [11, 12]
    assert [l for l, cs in cases.items() if cs == [1]] == [4, 5]


def test_predict_sums_unit_costs():
    costs = {("hmult", 5): 2.0, ("rescale", 5): 0.5, ("add", 4): 0.1}
    trace = [("hmult", 5, 1), ("rescale", 5, 1), ("add", 4, 1), ("add", 4, 1)]
    total, missing = tuner.predict(trace, costs)
    assert total == pytest.approx(2.7) and not missing
    total, missing = tuner.predict(trace + [("rotate", 3, 1)], costs)
    assert missing == {("rotate", 3)}


def test_predict_fused_linear_combination():
    """A fused linear combination of T terms is one launch: it costs one
    integer multiply plus (T - 1) times what an addition adds to it, not T
    multiplies and T - 1 additions."""
    costs = tuner.derive_lincomb_costs({("mul_scalar", 4): 8.0, ("add", 4): 9.0, ("mul_scalar", 5): 8.5})
    assert costs[("lincomb", 4)] == 8.0 and costs[("lincomb_term", 4)] == 1.0
    assert ("lincomb", 5) not in costs                  # no addition profiled at that level
    trace = [("lincomb", 4, 1)] + [("lincomb_term", 4, 1)] * 7
    assert tuner.predict(trace, costs)[0] == pytest.approx(8.0 + 7 * 1.0)
    # an addition profiled faster than the multiply: further terms cost nothing, never less
    assert tuner.derive_lincomb_costs({("mul_scalar", 2): 8.0, ("add", 2): 7.0})[("lincomb_term", 2)] == 0.0


def test_predict_batched_products():
    """An op on m x the base batch costs the profiled m-fold batch
    (interpolated between the profiled multiples, extended past the last)."""
    costs = {("hmult", 5): 2.0, ("hmult*2", 5): 2.5, ("hmult*4", 5): 3.5, ("add", 5): 0.1}
    assert tuner.predict([("hmult", 5, 2)], costs)[0] == pytest.approx(2.5)
    assert tuner.predict([("hmult", 5, 3)], costs)[0] == pytest.approx(3.0)
    assert tuner.predict([("hmult", 5, 6)], costs)[0] == pytest.approx(4.5)
    # relative to the run's own batch: B = 8 on a batch-4 run is the 2-fold cost
    assert tuner.predict([("hmult", 5, 8)], costs, base_batch=4)[0] == pytest.approx(2.5)
    # no multiples profiled: linear in m
    assert tuner.predict([("add", 5, 3)], costs)[0] == pytest.approx(0.3)


def test_select_meets_target_at_min_time():
    rows = [dict(level=11, d=31, i=3, c=0, ok=True, m=1.1e-8, t_pred=5.0),
            dict(level=11, d=63, i=2, c=0, ok=True, m=6.7e-9, t_pred=4.5),
            dict(level=11, d=15, i=4, c=0, ok=True, m=4.0e-8, t_pred=3.0),
            dict(level=11, d=127, i=1, c=0, ok=False)]
    r = tuner.select(rows, 3.1e-8, 11)
    assert (r["d"], r["i"]) == (63, 2)
    assert tuner.select(rows, 1e-9, 11) is None


def test_alg3_from_measured_rows():
    """Alg. 2 on each (level, degree, c) curve, then Alg. 3's u1 / u2."""
    rows = []
    for i, (m, t) in enumerate([(2e-3, 1.0), (2e-5, 2.0), (3.0e-8, 3.0), (2.9e-8, 4.0)], 1):
        rows.append({"level": 5, "d": 7, "c": 0, "i": i, "m": m, "t": t, "ok": True})
    for i, (m, t) in enumerate([(1e-4, 2.5), (2.5e-6, 3.5)], 1):
        rows.append({"level": 5, "d": 31, "c": 1, "i": i, "m": m, "t": t, "ok": True})
    rows.append({"level": 5, "d": 63, "c": 0, "i": 1, "ok": False})
    D, R = tuner.alg3_from_rows(rows, delta=1.0, theta=1.0)
    # (7, 0): threshold from 2.9e-8 -> 3e-8, first within is i = 3 (t = 3.0)
    # (31, 1): threshold from 2.5e-6 -> 3e-6, i = 2 (t = 3.5)
    assert {(e["d"], e["c"], e["i"]) for e in D[5]} == {(7, 0, 3), (31, 1, 2)}
    # accuracy-first: m_theta from 3.0e-8 -> 4e-8 keeps only (7, 0, 3); speed-first: fastest
    assert R[5] == ((7, 0, 3), (7, 0, 3))


def test_exploration_report_regret_and_cost():
    """Measured-time picks against cost-model picks: where the prediction
    ranks two settings the wrong way round, the regret is the measured time
    of its pick over the measured optimum; the cost model's GPU seconds leave
    out the timing runs."""
    rows = [dict(level=7, d=31, i=3, c=0, ok=True, m=1e-8, t=2.0, t_pred=2.2, t_first_s=2.5, t_timed_s=6.0),
            dict(level=7, d=15, i=4, c=0, ok=True, m=2e-8, t=2.1, t_pred=2.0, t_first_s=2.6, t_timed_s=6.3),
            dict(level=7, d=7, i=6, c=0, ok=True, m=2e-6, t=3.0, t_pred=3.0, t_first_s=3.5, t_timed_s=9.0),
            dict(level=7, d=63, i=1, c=0, ok=False, t_first_s=0.1)]
    rep = tuner.exploration_report(rows, [7], [1e-5, 3.1e-8, 1e-9], profile_s=4.0)
    p = rep["picks"]["7"]
    assert p["3.1e-08"]["measured"] == [31, 0, 3] and p["3.1e-08"]["predicted"] == [15, 0, 4]
    assert not p["3.1e-08"]["same"] and p["3.1e-08"]["regret"] == pytest.approx(0.05)
    assert p["1e-09"] is None
    assert rep["max_regret"] == pytest.approx(0.05)
    assert rep["measured_exhaustive_s"] == pytest.approx(8.7 + 21.3)
    assert rep["cost_model_s"] == pytest.approx(8.7 + 4.0)
    assert (rep["settings"], rep["feasible"]) == (4, 3)


def test_moment_reference_matches_scipy():
    """The FP64 reference of the moment statistics (population skewness,
    excess kurtosis, Pearson correlation) against scipy's definitions."""
    import numpy as np
    from scipy import stats
    from paper_2606_10477_amd import inputs, moments
    data, _, _ = inputs.skewed_table(4096, 4, 5)
    sk, ku, r = moments.reference(data, [(0, 1), (2, 3)])
    assert np.allclose(sk, stats.skew(data, axis=1, bias=True), rtol=1e-10, atol=1e-12)
    assert np.allclose(ku, stats.kurtosis(data, axis=1, fisher=True, bias=True), rtol=1e-10, atol=1e-12)
    assert np.allclose(r, [stats.pearsonr(data[0], data[1])[0], stats.pearsonr(data[2], data[3])[0]], rtol=1e-10)
    # the generator's shapes: skewness 2/sqrt(k) > 0.6, correlated odd columns
    assert sk[0] > 0.5 and sk[2] > 0.5 and abs(r[0]) > 0.05


def test_table_key_check():
    """A table is refused for another parameter set and only flagged for
    another GPU or library build."""
    from paper_2606_10477_amd import params
    cur = {"gpu": "g", "params": "p16b", "params_sha256": params.set_sha256("p16b"), "library_sha256": "L"}
    assert tuner.check_table_key(dict(cur), cur) is None
    assert tuner.check_table_key(None, cur)[0] == "warn"
    assert tuner.check_table_key(dict(cur, gpu="h"), cur)[0] == "warn"
    assert tuner.check_table_key(dict(cur, library_sha256="M"), cur)[0] == "warn"
    other = dict(cur, params="p16", params_sha256=params.set_sha256("p16"))
    assert tuner.check_table_key(other, cur)[0] == "error"
    assert params.set_sha256("p16b") != params.set_sha256("p16")
    assert tuner.check_table_key(dict(cur, params_sha256="x"), cur)[0] == "error"
