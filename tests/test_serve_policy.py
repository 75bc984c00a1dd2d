"""Serving scheduler policy (host logic only, a simulated backend; no GPU)."""
import math

import pytest

from paper_1812_01307_amd.serve import Request, Server, percentile


class FakeBackend:
    """Residual norms follow ||r_e|| = 1 + exp(-e / tau) after e epochs in a
    slot (tau per request), so the stop epoch of every request is known."""

    def __init__(self, state_bytes=100, geom_bytes=1000):
        self.sb, self.gb = state_bytes, geom_bytes
        self.states = []
        self.dropped = 0
        self.launches = []

    def geometry_bytes(self, g):
        return self.gb

    def state_bytes(self, g, slots):
        return self.sb * slots

    def new_state(self, g, slots):
        h = {"slots": [None] * slots, "e": [0] * slots, "lam": [0.0] * slots, "g": g}
        self.states.append(h)
        return h

    def drop_state(self, h):
        self.dropped += 1
        h["dead"] = True

    def admit(self, h, g, k, req):
        assert not h.get("dead")
        assert h["slots"][k] is None
        h["slots"][k] = req
        h["e"][k] = 0

    def set_lambdas(self, h, lams):
        h["lam"] = list(lams)

    def launch(self, h, g, epochs):
        for k, req in enumerate(h["slots"]):
            if req is not None:
                assert h["lam"][k] == req.lam
                h["e"][k] += epochs
        self.launches.append((h["g"], epochs))

    @staticmethod
    def norm(e, tau):
        return 1.0 + math.exp(-e / tau)

    def res_change(self, h):
        now, prev = [], []
        for k, req in enumerate(h["slots"]):
            if req is None:
                now.append(0.0)
                prev.append(0.0)
            else:
                tau = req.y
                now.append(self.norm(h["e"][k], tau) ** 2)
                prev.append(self.norm(h["e"][k] - 1, tau) ** 2)
        return now, prev

    def take_result(self, h, k):
        return ("x", h["slots"][k].rid, h["e"][k])

    def release(self, h, k):
        h["slots"][k] = None


def expected_epochs(tau, chunk, tol, max_epochs):
    e = chunk
    while e < max_epochs:
        a, b = FakeBackend.norm(e, tau), FakeBackend.norm(e - 1, tau)
        if abs(a - b) / b < tol:
            return e
        e += chunk
    return max_epochs


def _requests(n, geoms=("g0", "g1", "g2")):
    return [Request(rid=i, geometry=geoms[i % len(geoms)], y=3.0 + 2.0 * i, lam=0.01 * (i + 1),
                    arrival=0.0) for i in range(n)]


def _server(fb, **kw):
    srv = Server(fb, clock=lambda: 0.0, **kw)
    for g in ("g0", "g1", "g2"):
        srv.add_geometry(g, g)
    return srv


def test_every_request_stops_by_the_rule_at_chunk_boundaries():
    fb = FakeBackend()
    srv = _server(fb, slots=4, chunk=10, tol=1e-4, max_epochs=300)
    reqs = _requests(11)
    for r in reqs:
        srv.submit(r)
    while srv.busy:
        srv.step()
    assert len(srv.done) == 11
    for r in reqs:
        assert r.x == ("x", r.rid, r.epochs)
        assert r.epochs == expected_epochs(r.y, 10, 1e-4, 300)
        assert r.stop == ("converged" if r.epochs < 300 else "max_epochs")


def test_result_is_the_same_alone_and_in_the_mix():
    mix = _requests(9)
    fb = FakeBackend()
    srv = _server(fb, slots=2, chunk=10)
    # staggered admissions: one new request before each round
    pending = list(mix)
    while pending or srv.busy:
        if pending:
            srv.submit(pending.pop(0))
        srv.step()
    for r in mix:
        alone = _requests(9)[r.rid]
        fb2 = FakeBackend()
        s2 = _server(fb2, slots=2, chunk=10)
        s2.submit(alone)
        while s2.busy:
            s2.step()
        assert alone.epochs == r.epochs and alone.x == r.x


def test_hbm_budget_bounds_admission_and_other_geometries_proceed():
    # budget: 3 geometries (3000) + 2 states of 4 slots (800)
    fb = FakeBackend(state_bytes=100, geom_bytes=1000)
    srv = _server(fb, slots=4, chunk=10, hbm_bytes=3800)
    reqs = [Request(rid=i, geometry="g0", y=50.0, lam=0.01, arrival=0.0) for i in range(9)]
    reqs.append(Request(rid=9, geometry="g1", y=5.0, lam=0.01, arrival=0.0))
    for r in reqs:
        srv.submit(r)
    srv.step()
    # g0 got two states (8 slots), its ninth request and g1's request wait for memory
    assert srv.resident_bytes() <= 3800
    assert sum(b.active for b in srv.batches) == 8
    assert len(srv.queue) == 2
    while srv.busy:
        srv.step()
        assert srv.resident_bytes() <= 3800
    assert len(srv.done) == 10
    # g1's request was served once a state became idle and was released
    assert fb.dropped >= 1


def test_idle_states_are_reused_and_lambdas_follow_slots():
    fb = FakeBackend()
    srv = _server(fb, slots=4, chunk=10)
    a = Request(rid=0, geometry="g0", y=3.0, lam=0.5)
    srv.submit(a)
    while srv.busy:
        srv.step()
    b = Request(rid=1, geometry="g0", y=3.0, lam=0.25)
    srv.submit(b)
    srv.step()
    assert len(fb.states) == 1          # the idle state took the new request
    assert fb.states[0]["lam"][0] == 0.25
    while srv.busy:
        srv.step()
    assert b.epochs == a.epochs


def test_run_follows_arrival_times():
    t = [0.0]
    fb = FakeBackend()
    srv = Server(fb, slots=2, chunk=10, clock=lambda: t[0])
    srv.add_geometry("g0", "g0")
    reqs = [Request(rid=i, geometry="g0", y=3.0, lam=0.1, arrival=float(i)) for i in range(3)]

    def sleep(dt):
        t[0] += dt

    orig_step = srv.step

    def step():
        t[0] += 0.25  # each round takes a quarter second
        return orig_step()

    srv.step = step
    done = srv.run(reqs, sleep=sleep)
    assert [r.rid for r in done] == [0, 1, 2]
    for r in done:
        assert r.admitted >= r.arrival and r.finished > r.admitted and r.latency > 0


def test_cancel_queued_and_running_requests_leaves_the_others_unchanged():
    def serve(cancel_at):
        fb = FakeBackend()
        srv = _server(fb, slots=2, chunk=10, tol=1e-4, max_epochs=300)
        reqs = _requests(7)
        for r in reqs:
            srv.submit(r)
        rounds = 0
        while srv.busy:
            for rnd, rid in cancel_at:
                if rnd == rounds:
                    assert srv.cancel(rid)
            srv.step()
            rounds += 1
        return srv, {r.rid: r for r in reqs}

    base_srv, base = serve([])
    # before the first scheduling step request 6 is still queued (2 slots per
    # geometry, 3 geometries); before the third, request 1 is running
    srv, got = serve([(0, 6), (2, 1)])
    assert not srv.cancel(6) and not srv.cancel(99)
    assert {r.rid for r in srv.cancelled} == {1, 6}
    assert got[1].stop == got[6].stop == "cancelled" and got[6].epochs == 0
    assert got[1].epochs == 20 and got[1].x is None
    for rid in (0, 2, 3, 4, 5):
        assert got[rid].epochs == base[rid].epochs and got[rid].x == base[rid].x
    assert {r.rid for r in srv.done} == {0, 2, 3, 4, 5}


def test_invalid_requests_and_settings_are_rejected():
    fb = FakeBackend()
    srv = _server(fb)
    with pytest.raises(KeyError):
        srv.submit(Request(rid=0, geometry="nope", y=1.0, lam=0.1))
    with pytest.raises(ValueError):
        srv.submit(Request(rid=0, geometry="g0", y=1.0, lam=-1.0))
    with pytest.raises(ValueError):
        Server(fb, chunk=7, max_epochs=300)
    with pytest.raises(ValueError):
        srv.add_geometry("g0", "g0")
    small = Server(fb, hbm_bytes=500)
    with pytest.raises(MemoryError):
        small.add_geometry("g", "g")


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50 and percentile(v, 99) == 99 and percentile(v, 100) == 100
    assert percentile([7.0], 99) == 7.0


def test_state_width_follows_demand():
    """A lone request of a geometry gets a one-slot state; requests that share a
    geometry (waiting together, or arriving while one runs) get full-width
    states; the widths are 1 or powers of two from 4 up to the server's."""
    be = FakeBackend()
    srv = Server(be, slots=8, chunk=10, tol=1e-4, max_epochs=300)
    for g in ("a", "b", "c"):
        srv.add_geometry(g, g)
    srv.submit(Request(rid=0, geometry="a", y=50.0, lam=1.0))
    srv.submit(Request(rid=1, geometry="b", y=50.0, lam=1.0))
    srv.submit(Request(rid=2, geometry="b", y=50.0, lam=1.0))
    srv.step()
    widths = {b.geometry: len(b.slots) for b in srv.batches}
    assert widths == {"a": 1, "b": 4}  # two of "b": room for four
    assert sum(b.active for b in srv.batches) == 3
    # a second request of "a" while the first runs: a new state of 4 slots
    srv.submit(Request(rid=3, geometry="a", y=50.0, lam=2.0))
    srv.submit(Request(rid=4, geometry="c", y=50.0, lam=1.0))
    srv.step()
    assert sorted(len(b.slots) for b in srv.batches if b.geometry == "a") == [1, 4]
    assert [len(b.slots) for b in srv.batches if b.geometry == "c"] == [1]
    # six more of "c" at once (one running): the new state holds 8
    for i in range(6):
        srv.submit(Request(rid=10 + i, geometry="c", y=50.0, lam=1.0))
    srv.step()
    assert sorted(len(b.slots) for b in srv.batches if b.geometry == "c") == [1, 8]
    while srv.busy:
        srv.step()
    assert sorted(r.rid for r in srv.done) == [0, 1, 2, 3, 4] + list(range(10, 16))
    for r in srv.done:
        assert r.epochs == expected_epochs(50.0, 10, 1e-4, 300)
    # a narrow server: 4 slots; slot counts below 4 other than 1 do not exist
    assert Server(be, slots=4)._width(3) == 4 and Server(be, slots=2)._width(2) == 1
    assert Server(be, slots=16)._width(2) == 4 and Server(be, slots=16)._width(3) == 8
    assert Server(be, slots=16)._width(5) == 16 and Server(be, slots=12)._width(30) == 8


def test_idle_narrow_state_gives_way_to_a_wider_one():
    be = FakeBackend()
    srv = Server(be, slots=8, chunk=10, tol=1e-4, max_epochs=20)
    srv.add_geometry("a", "a")
    srv.submit(Request(rid=0, geometry="a", y=50.0, lam=1.0))
    while srv.busy:
        srv.step()
    assert [len(b.slots) for b in srv.batches] == [1] and be.dropped == 0
    # the one-slot state is idle: a lone request reuses it ...
    srv.submit(Request(rid=1, geometry="a", y=50.0, lam=1.0))
    srv.step()
    assert [len(b.slots) for b in srv.batches] == [1] and be.dropped == 0
    while srv.busy:
        srv.step()
    # ... three at once replace it with a state of 8 (room for twice the load)
    for i in range(3):
        srv.submit(Request(rid=2 + i, geometry="a", y=50.0, lam=1.0))
    srv.step()
    assert [len(b.slots) for b in srv.batches] == [8] and be.dropped == 1
    assert srv.batches[0].active == 3
