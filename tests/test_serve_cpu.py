"""The continuous-batching loop on the CPU: an oracle-backed fake backend with
a service-time model stands in for the GPU, so admission, batching, ordering
and latency accounting are tested without a device."""
import time

import numpy as np
import pytest

from oracle import pyoracle as O
from paper_2503_13092_amd import serve, synth

G = synth.default_geometry()
W = synth.mlp_weights()


class FakeBackend:
    def __init__(self, pool, n_slots=2, max_events=16, max_seeds=10 ** 6, max_hits=10 ** 7,
                 service=lambda n: 1e-3 + 1e-5 * n):
        self.pool, self.n_slots, self.max_events = pool, n_slots, max_events
        self.max_seeds, self.max_hits = max_seeds, max_hits
        self.service = service
        self.state = {}
        self.submitted = []

    def submit(self, slot, e0, e1):
        assert slot not in self.state, "slot reused while busy"
        n = e1 - e0
        assert n <= self.max_events
        sub = self.pool.batch.subset(np.arange(e0, e1))
        assert sub.n_seeds <= self.max_seeds and sub.n_hits <= self.max_hits
        r = O.run_path(sub, G, W, cap=8)
        st = r["stored"]
        verts = np.zeros((n, 8, 6))
        v = r["vertices"]
        for k in range(n):
            for m in range(v["count"][k]):
                q = k * 8 + m
                verts[k, m] = [v["i"][q], v["j"][q], v["x"][q], v["y"][q], v["z"][q], v["doca"][q]]
        res = serve.BatchResult(e0, n, sub.seed_off.copy(), st["nhits"], st["hits"], r["score"],
                                np.stack([st[k] for k in ("x", "y", "tx", "ty", "qop", "chi2")], 1),
                                v["count"].copy(), verts)
        self.state[slot] = (time.perf_counter() + self.service(n), res)
        self.submitted.append((e0, e1))

    def done(self, slot):
        return time.perf_counter() >= self.state[slot][0]

    def fetch(self, slot):
        return self.state.pop(slot)[1]


@pytest.fixture(scope="module")
def pool():
    return serve.EventPool(synth.generate(2, n_events=60, seed=5))


def test_every_event_served_once_in_order(pool):
    be = FakeBackend(pool)
    srv = serve.Server(be, pool)
    arr = serve.poisson_arrivals(3000.0, 150, seed=1)
    seen = []
    lat, st = srv.run(arr, on_result=lambda a0, a1, res: seen.append((a0, a1)))
    assert st.rejected == 0 and np.all(np.isfinite(lat)) and np.all(lat > 0)
    flat = [k for a0, a1 in seen for k in range(a0, a1)]
    assert sorted(flat) == list(range(150))
    assert st.max_in_flight <= be.n_slots
    # events are admitted in arrival order and never wrap the pool inside a batch
    for e0, e1 in be.submitted:
        assert 0 <= e0 < e1 <= pool.size


def test_results_same_alone_and_in_the_mix(pool):
    be = FakeBackend(pool)
    srv = serve.Server(be, pool)
    got = {}

    def keep(a0, a1, res):
        for k in range(a1 - a0):
            got[a0 + k] = res.event(k)

    srv.run(serve.poisson_arrivals(5000.0, 60, seed=2), on_result=keep)
    for e in (0, 7, 31, 59):
        alone = FakeBackend(pool)
        alone.submit(0, e, e + 1)
        r = alone.fetch(0).event(0)
        for k in ("nhits", "hits", "score", "state", "vertices"):
            assert np.array_equal(r[k], got[e][k]), (e, k)


def test_continuous_batching_under_load(pool):
    # arrivals faster than one slot can serve: batches grow, all slots stay busy
    be = FakeBackend(pool, n_slots=2, max_events=16, service=lambda n: 2e-3 + 5e-5 * n)
    srv = serve.Server(be, pool)
    lat, st = srv.run(serve.poisson_arrivals(20000.0, 200, seed=3))
    assert st.mean_batch > 2.0 and st.max_in_flight == 2
    assert all(e1 - e0 <= 16 for e0, e1 in be.submitted)


def test_memory_admission(pool):
    cap_seeds = int(pool.seeds_per_event[:10].max()) + 1
    be = FakeBackend(pool, max_seeds=cap_seeds)
    srv = serve.Server(be, pool)
    lat, st = srv.run(serve.poisson_arrivals(2000.0, 40, seed=4))
    for e0, e1 in be.submitted:
        assert pool.seeds_per_event[e0:e1].sum() <= cap_seeds
    too_big = int(np.sum(pool.seeds_per_event[:40] > cap_seeds))
    assert st.rejected == too_big
    assert np.sum(np.isnan(lat)) == too_big


def test_latency_is_from_scheduled_arrival(pool):
    be = FakeBackend(pool, service=lambda n: 5e-3)
    srv = serve.Server(be, pool)
    arr = np.arange(1, 21) * 0.02    # far apart: every event waits only for its own service
    lat, st = srv.run(arr, warmup_frac=0.0)
    # at least the service time; well under the 20 ms spacing (host scheduling noise allowed)
    assert np.all(lat >= 5e-3) and np.median(lat) < 5e-3 + 12e-3


def test_saturated_server_reports_censored_lower_bounds(pool):
    """A server slower than the arrivals, stopped by its time limit: events
    still queued count with (end - arrival) as a lower bound on their latency,
    'sustained' counts completed events only, and the run says it is censored."""
    be = FakeBackend(pool, n_slots=1, max_events=2, service=lambda n: 20e-3)
    srv = serve.Server(be, pool)
    arr = serve.poisson_arrivals(2000.0, 400, seed=6)
    lat, st = srv.run(arr, warmup_frac=0.0, time_limit_s=0.15)
    assert st.saturated and st.censored > 0
    assert st.completed == int(np.sum(np.isfinite(lat)))
    assert st.completed + st.censored + st.rejected == st.offered
    assert st.sustained == pytest.approx(st.completed / st.duration_s)
    # the median over all offered events is at least what the queue already waited
    waited = np.sort(st.duration_s - arr[(arr <= st.duration_s) & ~np.isfinite(lat)])
    assert st.p50_ms >= 1e3 * np.median(np.concatenate([waited, lat[np.isfinite(lat)]])) - 1e-6


def test_rejected_events_are_not_counted_as_served(pool):
    cap_seeds = int(pool.seeds_per_event[:10].max()) + 1
    be = FakeBackend(pool, max_seeds=cap_seeds)
    srv = serve.Server(be, pool)
    lat, st = srv.run(serve.poisson_arrivals(2000.0, 40, seed=4))
    assert st.rejected > 0 and not st.saturated
    assert st.completed == 40 - st.rejected
    assert st.sustained == pytest.approx(st.completed / st.duration_s)
