"""Serving scheduler on the CPU: admission by footprint, continuous batching,
coverage of every particle exactly once, latency bookkeeping.  A stand-in
executor completes a step after a simulated time proportional to its rows."""

import math

import pytest

from paper_2011_05755_amd import serve


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExecutor:
    def __init__(self, clock, sec_per_row=1e-6):
        self.clock = clock
        self.sec_per_row = sec_per_row
        self.busy_until = 0.0
        self.log = []           # (launch time, [(rid, n0, n)])
        self.admitted = []
        self.released = []

    def admit(self, r):
        self.admitted.append(r.rid)

    def release(self, r):
        self.released.append(r.rid)

    def launch(self, pieces):
        rows = sum(p.n * p.req.S for p in pieces)
        start = max(self.clock.t, self.busy_until)        # steps run one after another
        self.busy_until = start + rows * self.sec_per_row
        self.log.append((self.clock.t, [(p.req.rid, p.n0, p.n) for p in pieces]))
        return self.busy_until

    def done(self, h):
        return self.clock.t >= h

    def wait(self, h):
        self.clock.t = max(self.clock.t, h)


def req(N, L=64, T=2, rid_hint=0):
    return serve.Request(refset_id=rid_hint, N=N, L=L, shift_max=T)


def test_percentile_nearest_rank():
    xs = [5.0, 1.0, 3.0, 2.0, 4.0]
    assert serve.percentile(xs, 50) == 3.0
    assert serve.percentile(xs, 99) == 5.0
    assert serve.percentile(xs, 0) == 1.0
    assert math.isnan(serve.percentile([], 50))


def test_every_particle_is_scheduled_once_in_contiguous_pieces():
    clk = SimClock()
    ex = FakeExecutor(clk)
    srv = serve.Server(ex, hbm_budget=1 << 40, step_rows=5000)
    arrivals = [(0.0, req(1000)), (0.001, req(37, T=1)), (0.5, req(333, T=3))]
    stats = serve.run_trace(srv, arrivals, clock=clk, sleep=clk.sleep)
    assert stats["requests"] == 3 and stats["particles"] == 1370
    for _, r in arrivals:
        spans = sorted((n0, n) for _, ps in ex.log for rid, n0, n in ps if rid == r.rid)
        pos = 0
        for n0, n in spans:
            assert n0 == pos and n >= 1
            pos += n
        assert pos == r.N
        assert r.t_done is not None and r.latency >= 0
    assert sorted(ex.admitted) == sorted(ex.released) == [0, 1, 2]


def test_a_request_arriving_during_a_long_one_joins_the_next_step():
    clk = SimClock()
    ex = FakeExecutor(clk, sec_per_row=1e-6)
    srv = serve.Server(ex, hbm_budget=1 << 40, step_rows=25 * 200)     # 200 particles of S=25 per step
    long, short = req(20000), req(50)
    stats = serve.run_trace(srv, [(0.0, long), (0.02, short)], clock=clk, sleep=clk.sleep)
    assert stats["requests"] == 2
    first_short = min(t for t, ps in ex.log if any(rid == short.rid for rid, _, _ in ps))
    # a FIFO queue would start it only after the long request (0.5 s of work)
    assert first_short < 0.02 + 3 * 0.005 + 1e-9
    assert short.t_done < long.t_done
    assert short.latency < 0.05


def test_admission_respects_the_hbm_budget_in_arrival_order():
    clk = SimClock()
    ex = FakeExecutor(clk)
    r1, r2, r3 = req(100), req(100), req(10)
    fp = r1.footprint()
    srv = serve.Server(ex, hbm_budget=fp + fp // 2 + 1000, workspace_bytes=1000, step_rows=1000)
    stats = serve.run_trace(srv, [(0.0, r1), (0.0001, r2), (0.0002, r3)], clock=clk, sleep=clk.sleep)
    assert stats["requests"] == 3
    # r2 does not fit next to r1; r3 would, but admission is first come, first admitted
    assert r2.t_admit >= r1.t_done
    assert r3.t_admit >= r2.t_admit
    assert srv.peak_used <= srv.budget
    assert ex.admitted == [0, 1, 2]


def test_requests_larger_than_the_budget_and_budgets_below_the_workspace_are_rejected():
    clk = SimClock()
    srv = serve.Server(FakeExecutor(clk), hbm_budget=10_000, workspace_bytes=0)
    with pytest.raises(ValueError):
        srv.submit(req(1000), 0.0)
    with pytest.raises(ValueError):
        serve.Server(FakeExecutor(clk), hbm_budget=100, workspace_bytes=100)


def test_steps_stay_within_the_row_budget_and_share_it():
    clk = SimClock()
    ex = FakeExecutor(clk)
    srv = serve.Server(ex, hbm_budget=1 << 40, step_rows=10_000)
    rs = [req(3000, T=t) for t in (1, 2, 3, 4)]
    serve.run_trace(srv, [(0.0, r) for r in rs], clock=clk, sleep=clk.sleep)
    S = {r.rid: r.S for r in rs}
    for _, ps in ex.log:
        rows = sum(n * S[rid] for rid, _, n in ps)
        assert rows <= 10_000 + max(S.values())
    first = ex.log[0][1]
    assert [rid for rid, _, _ in first] == [r.rid for r in rs]     # every active request in the first step


class RefusingExecutor(FakeExecutor):
    """Refuses requests on refset 99 at launch and on refset 98 at admission
    (as the library refuses a refset that is not loaded)."""

    def admit(self, r):
        if r.refset_id == 98:
            raise RuntimeError("refset 98 is not loaded")
        super().admit(r)

    def launch(self, pieces):
        if any(p.req.refset_id == 99 for p in pieces):
            raise RuntimeError("refset 99 is not loaded")
        return super().launch(pieces)


def test_a_failing_request_fails_alone_and_the_others_complete():
    clk = SimClock()
    ex = RefusingExecutor(clk)
    srv = serve.Server(ex, hbm_budget=1 << 40, step_rows=4000)
    good = [req(500), req(120, T=1), req(700, T=3)]
    bad_launch, bad_admit = req(300, rid_hint=99), req(50, rid_hint=98)
    arrivals = [(0.0, good[0]), (0.0, bad_launch), (0.001, good[1]), (0.002, bad_admit), (0.003, good[2])]
    stats = serve.run_trace(srv, arrivals, clock=clk, sleep=clk.sleep)
    assert stats["requests"] == 3 and stats["failed_requests"] == 2
    assert stats["particles"] == sum(r.N for r in good)
    for r in good:                                   # every good particle scheduled exactly once
        assert r.error is None and r.t_done is not None
        spans = sorted((n0, n) for _, ps in ex.log for rid, n0, n in ps if rid == r.rid)
        assert sum(n for _, n in spans) == r.N and spans[0][0] == 0
    assert "refset 99" in bad_launch.error and "refset 98" in bad_admit.error
    assert bad_launch.t_done is not None and bad_admit.t_done is not None
    assert not any(rid == bad_launch.rid for _, ps in ex.log for rid, _, _ in ps)
    assert bad_launch in srv.failed and bad_admit in srv.failed and bad_launch not in srv.finished
    assert srv.used == 0 and not srv.active               # budgets released
    assert sorted(ex.released) == sorted(r.rid for r in good + [bad_launch, bad_admit])
    # a step that held the bad request's piece was launched again without it
    assert any(len(ps) >= 2 for _, ps in ex.log)
