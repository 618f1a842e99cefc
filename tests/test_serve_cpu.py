"""Scheduler logic of the serving loop, with a fake context (no GPU)."""
import pytest

from paper_2606_10477_amd import serve


class FakeCt:
    def __init__(self, tag, level=None):
        self.tag = tag
        self.level = level


class FakeCtx:
    """Stands in for a library context: records launches, finishes them at
    once (or when told), reports memory figures."""
    N = 1 << 12

    def __init__(self, free=1 << 40, immediate=True):
        self.calls = []
        self.drops = []
        self.levels = []
        self.free = free
        self.immediate = immediate
        self.pending = False
        self.in_use = 0

    def drop_level(self, ct, level):
        self.drops.append((ct.tag, ct.level, level))
        return FakeCt(ct.tag, level)

    def invsqrt_batch(self, cts, degree, iters, a=None, b=None, pre_bts=False):
        self.calls.append((len(cts), degree, iters) + ((1,) if pre_bts else ()))
        self.levels.append(sorted({c.level for c in cts}))
        self.pending = not self.immediate
        return [FakeCt(("y", c.tag, degree, iters)) for c in cts]

    def stream_done(self):
        return not self.pending

    def mem_info(self, reset_peak=False):
        return {"device_free": self.free, "pool_cached": 0, "pool_in_use": self.in_use, "pool_peak": self.in_use,
                "ct_bytes": [2 * (l + 1) * self.N * 8 for l in range(32)]}

    def sync(self):
        self.pending = False


TABLE = {"13": {"1e-06": {"degree": 15, "iters": 2}, "1e-07": {"degree": 31, "iters": 2},
                "3.1e-08": {"degree": 31, "iters": 3}},
         "17": {"1e-06": {"degree": 7, "iters": 3}, "1e-07": {"degree": 31, "iters": 2},
                "3.1e-08": {"degree": 63, "iters": 2}},
         "20": {"1e-06": {"degree": 15, "c": 1, "iters": 3}}}


def mk(rid, t, n, level, target):
    return serve.Request(rid, t, [FakeCt((rid, k), level) for k in range(n)], level, target)


def test_lookup_exact_and_fallback():
    assert serve.lookup(TABLE, 13, 3.1e-8) == (31, 0, 3)
    assert serve.lookup(TABLE, 19, 1e-6) == (7, 0, 3)    # closest tuned level below
    assert serve.lookup(TABLE, 20, 1e-6) == (15, 1, 3)   # Pre-BTS setting
    nulls = {"3": {"1e-06": None}, "5": {"1e-06": {"degree": 7, "c": 0, "iters": 6}}}
    assert serve.lookup(nulls, 5, 1e-6) == (7, 0, 6)
    with pytest.raises(KeyError):
        serve.lookup(nulls, 4, 1e-6)                     # level 3 has no feasible setting
    with pytest.raises(KeyError):
        serve.lookup(TABLE, 5, 1e-6)


def test_groups_share_one_batch_and_results_are_attributed():
    ctx = FakeCtx()
    srv = serve.Server(ctx, TABLE, max_batch=64, reserve_bytes=0)
    for r in [mk(0, 0.0, 3, 13, 3.1e-8), mk(1, 0.0, 5, 13, 3.1e-8), mk(2, 0.0, 2, 17, 1e-6)]:
        srv.submit(r)
    reqs = list(srv.queue)
    clock = lambda: 1.0
    assert srv.step(clock) == 8              # both (13, 31, 3) requests in one launch sequence
    assert ctx.calls[-1] == (8, 31, 3)
    assert srv.step(clock) == 2
    assert ctx.calls[-1] == (2, 7, 3)
    assert srv.step(clock) == 0 and not srv.busy()   # the last group collected
    for r in reqs:
        assert r.done == 1.0 and len(r.outs) == len(r.cts)
        for k, y in r.outs.items():
            assert y.tag == ("y", (r.rid, k), r.degree, r.iters)


def test_pre_bts_setting_is_its_own_group():
    ctx = FakeCtx()
    srv = serve.Server(ctx, TABLE, max_batch=64, reserve_bytes=0)
    for r in [mk(0, 0.0, 2, 20, 1e-6), mk(1, 0.5, 3, 13, 1e-6)]:
        srv.submit(r)
    clock = lambda: 1.0
    assert srv.step(clock) == 2
    assert ctx.calls[-1] == (2, 15, 3, 1)      # bootstraps x first
    assert srv.step(clock) == 3
    assert ctx.calls[-1] == (3, 15, 2)
    srv.step(clock)
    assert not srv.busy()


def test_max_batch_splits_and_request_completes_when_all_parts_done():
    ctx = FakeCtx()
    srv = serve.Server(ctx, TABLE, max_batch=4, reserve_bytes=0)
    r = mk(0, 0.0, 10, 13, 1e-6)
    srv.submit(r)
    sizes = []
    t = [0.0]

    def clock():
        t[0] += 1
        return t[0]
    while srv.busy():
        sizes.append(srv.step(clock))
    # each round collects the finished group and issues the next one
    assert sizes == [4, 4, 2, 0]
    assert [e["batch"] for e in srv.log] == [4, 4, 2]
    assert r.done is not None and sorted(r.outs) == list(range(10))


def test_admission_by_the_librarys_free_memory():
    one = 2 * 14 * FakeCtx.N * 8 * 24       # first estimate for one ciphertext at level 13
    ctx = FakeCtx(free=3 * one, immediate=False)
    srv = serve.Server(ctx, TABLE, max_batch=64, reserve_bytes=0)
    a, b = mk(0, 0.0, 2, 13, 3.1e-8), mk(1, 0.1, 2, 13, 3.1e-8)
    srv.submit(a)
    srv.submit(b)
    srv._admit(0.0)
    assert srv.active == [a] and srv.queue == [b]   # b must wait for memory
    assert srv.step(lambda: 1.0) == 2               # a issued, still running
    assert a.done is None and srv.queue == [b]
    ctx.sync()                                      # a's group completes ...
    ctx.free = 10 * one                             # ... and its memory is free again
    srv.step(lambda: 2.0)
    assert a.done == 2.0 and b.admitted == 2.0      # b admitted once the memory is there
    ctx.sync()
    srv.step(lambda: 3.0)
    assert b.done == 3.0


def test_two_lanes_overlap_groups():
    """A request arriving while another's group runs on lane 0 starts on
    lane 1 before lane 0 finishes; each lane's results go to its requests."""
    l0, l1 = FakeCtx(immediate=False), FakeCtx(immediate=False)
    srv = serve.Server([l0, l1], TABLE, max_batch=64, reserve_bytes=0)
    a, b = mk(0, 0.0, 3, 13, 3.1e-8), mk(1, 0.1, 2, 17, 1e-6)
    srv.submit(a)
    assert srv.step(lambda: 0.0) == 3 and l0.calls == [(3, 31, 3)]
    srv.submit(b)
    assert srv.step(lambda: 0.2) == 2 and l1.calls == [(2, 7, 3)]   # lane 0 is still busy
    assert srv.max_in_flight == 2 and a.done is None and b.done is None
    l1.sync()
    srv.step(lambda: 0.3)
    assert b.done == 0.3 and a.done is None
    l0.sync()
    srv.step(lambda: 0.5)
    assert a.done == 0.5 and not srv.busy()
    assert {k: y.tag for k, y in a.outs.items()} == {k: ("y", (0, k), 31, 3) for k in range(3)}


def test_summary():
    rs = [mk(i, 0.1 * i, 2, 13, 1e-6) for i in range(4)]
    for i, r in enumerate(rs):
        r.done = r.arrival + 0.5 + 0.1 * i
    s = serve.summarize(rs)
    assert s["ciphertexts"] == 8 and s["p50_latency_s"] == pytest.approx(0.65)


TIMED = {"6": {"3.1e-08": {"degree": 31, "c": 0, "iters": 4, "t_meas": 0.034}},
         "7": {"1e-06": {"degree": 15, "c": 0, "iters": 4, "t_meas": 0.0177},
               "3.1e-08": {"degree": 31, "c": 0, "iters": 3, "t_meas": 0.0183}},
         "8": {"1e-06": {"degree": 15, "c": 0, "iters": 4, "t_meas": 0.0176},
               "3.1e-08": {"degree": 31, "c": 0, "iters": 3, "t_meas": 0.0183}}}


def test_route_to_the_lowest_level_with_the_same_setting_and_time():
    assert serve.route(TIMED, 8, 3.1e-8) == (7, 31, 0, 3)      # same setting, same measured time at 7
    assert serve.route(TIMED, 8, 1e-6) == (7, 15, 0, 4)        # 17.7 ms within 2 % of 17.6 ms
    assert serve.route(TIMED, 8, 1e-6, tol=0.0) == (8, 15, 0, 4)
    assert serve.route(TIMED, 7, 3.1e-8) == (7, 31, 0, 3)      # level 6 has another setting
    assert serve.route(TIMED, 6, 3.1e-8) == (6, 31, 0, 4)
    assert serve.route(TABLE, 17, 1e-6) == (17, 7, 0, 3)       # no times: nothing routed


def test_routed_requests_share_a_group_at_the_run_level():
    ctx = FakeCtx()
    srv = serve.Server(ctx, TIMED, max_batch=64, reserve_bytes=0)
    a, b = mk(0, 0.0, 2, 8, 3.1e-8), mk(1, 0.0, 3, 7, 3.1e-8)
    srv.submit(a)
    srv.submit(b)
    assert (a.run_level, b.run_level) == (7, 7)
    assert srv.step(lambda: 1.0) == 5                           # one launch sequence for both
    assert ctx.calls == [(5, 31, 3)] and ctx.levels == [[7]]
    assert sorted(d[0] for d in ctx.drops) == [(0, 0), (0, 1)]  # only the level-8 inputs were dropped
    srv.step(lambda: 2.0)
    assert a.done and b.done and not srv.busy()


def test_one_at_a_time_routes_like_the_server():
    ctx = FakeCtx()
    r = mk(0, 0.0, 2, 8, 3.1e-8)
    serve.run_one_at_a_time(ctx, TIMED, [r])
    assert r.run_level == 7 and ctx.levels == [[7]] and len(r.outs) == 2


class FakeSingleCtx(FakeCtx):
    def invsqrt(self, ct, degree, iters, a=None, b=None):
        self.calls.append((1, degree, iters))
        return FakeCt(("y", ct.tag, degree, iters), ct.level)


def test_fixed_single_baseline_and_target_check():
    ctx = FakeSingleCtx()
    rs = [mk(0, 0.0, 2, 8, 3.1e-8), mk(1, 0.0, 1, 5, 1e-6)]
    serve.run_fixed_single(ctx, rs)
    assert ctx.calls == [(1, 31, 3)] * 3 and all(len(r.outs) == len(r.cts) for r in rs)
    rows = [{"ok": True, "level": 8, "d": 31, "i": 3, "c": 0, "m": 1.1e-8},
            {"ok": True, "level": 5, "d": 31, "i": 3, "c": 0, "m": 4.9e-3}]
    assert serve.fixed_meets_target(rows, 8, 3.1e-8) is True
    assert serve.fixed_meets_target(rows, 5, 1e-6) is False
    assert serve.fixed_meets_target(rows, 6, 1e-6) is None
