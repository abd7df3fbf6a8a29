"""Serving logic on the CPU: admission by HBM budget, per-instance order, eviction, failure
handling and continuous batching, with an oracle-backed fake executor."""
import time

import numpy as np
import pytest

from gen import configs as G
from gen import screens as S
from oracle import wfs as OW
from paper_1408_0698_amd.serve import Instance, Request, Server, latency_report


class FakeExecutor:
    """Each batch 'runs' for `duration` seconds; results are the oracle's slopes of the 8 m sensor."""

    def __init__(self, duration=0.002, inst_bytes=1000, slot=100, shared=0, fail_on=()):
        self.duration = duration
        self.inst_bytes = inst_bytes
        self.slot = slot
        self.shared = shared
        self.fail_on = set(fail_on)
        self.created, self.destroyed = [], []
        self.launched = []
        self.sensor = OW.Sensor(G.CFG0)

    def shared_bytes(self):
        return self.shared

    def instance_bytes(self, cls):
        return self.inst_bytes

    def slot_bytes(self, cls):
        return self.slot

    def create_instance(self, inst):
        self.created.append(inst.iid)

    def destroy_instance(self, inst):
        self.destroyed.append(inst.iid)

    def launch(self, batch):
        if any(r.rid in self.fail_on for r in batch):
            raise RuntimeError("injected launch failure")
        self.launched.append([r.rid for r in batch])
        return {"t": time.perf_counter() + self.duration, "reqs": list(batch)}

    def poll(self, h):
        return time.perf_counter() >= h["t"]

    def collect(self, h):
        out = {}
        for r in h["reqs"]:
            opd = S.ngs8m_opd(1, frame0=r.frame, seed=100 + r.instance)[:, None]
            out[r.rid] = self.sensor.measure(opd)["slopes"][0]
        return out


def _stream(n, n_inst, rate=5000.0, seed=1):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1 / rate, n))
    frames = [0] * n_inst
    reqs = []
    for k in range(n):
        i = int(rng.integers(0, n_inst))
        reqs.append(Request(k, i, frames[i], float(t[k])))
        frames[i] += 1
    return reqs


def test_all_complete_in_order_and_within_budget():
    ex = FakeExecutor(inst_bytes=1000, slot=100)
    inst = [Instance(i, "8m", 100 + i) for i in range(3)]
    srv = Server(ex, inst, budget_bytes=3000 + 300)       # three instances + three slots
    reqs = _stream(60, 3)
    out = srv.run(reqs)
    assert all(r.status == "done" for r in out) and len(out) == 60
    assert srv.max_used <= srv.adm.budget
    for i in range(3):
        mine = sorted((r for r in out if r.instance == i), key=lambda r: r.frame)
        adm = [r.admitted for r in mine]
        assert adm == sorted(adm), "requests of one instance admitted out of order"
    rep = latency_report(out)
    assert rep["completed"] == 60 and rep["p99_ms"] >= rep["p50_ms"] > 0


def test_budget_below_one_instance_rejects():
    ex = FakeExecutor(inst_bytes=1000, slot=100)
    srv = Server(ex, [Instance(0, "8m", 1)], budget_bytes=1050)
    out = srv.run(_stream(5, 1))
    assert all(r.status == "rejected" for r in out)


def test_budget_below_shared_state_raises():
    with pytest.raises(MemoryError):
        Server(FakeExecutor(shared=10_000), [Instance(0, "8m", 1)], budget_bytes=5000)


def test_single_slot_serialises_but_completes():
    ex = FakeExecutor(inst_bytes=1000, slot=100, duration=0.001)
    srv = Server(ex, [Instance(0, "8m", 1)], budget_bytes=1100)      # the instance and one slot
    out = srv.run(_stream(20, 1))
    assert all(r.status == "done" for r in out)
    assert max(len(b) for b in ex.launched) == 1


def test_eviction_when_instances_do_not_fit_together():
    ex = FakeExecutor(inst_bytes=1000, slot=100, duration=0.0005)
    srv = Server(ex, [Instance(0, "8m", 1), Instance(1, "8m", 2)], budget_bytes=1200)
    out = srv.run(_stream(30, 2, rate=500.0))
    assert all(r.status == "done" for r in out)
    assert len(ex.destroyed) >= 1 and srv.max_used <= 1200


def test_failed_launch_fails_its_requests_and_the_server_goes_on():
    ex = FakeExecutor(fail_on={3})
    srv = Server(ex, [Instance(0, "8m", 1)], budget_bytes=10_000, max_batch=1)
    out = srv.run(_stream(10, 1, rate=1000.0))
    st = {r.rid: r.status for r in out}
    assert st[3] == "failed" and sum(v == "done" for v in st.values()) == 9


def test_cancel_queued_request():
    ex = FakeExecutor()
    srv = Server(ex, [Instance(0, "8m", 1)], budget_bytes=10_000)
    r = Request(0, 0, 0, 0.0)
    srv.submit(r)
    assert srv.cancel(0) and r.status == "cancelled" and not srv.queue


def test_continuous_batching_launches_while_earlier_batches_run():
    ex = FakeExecutor(duration=0.02, inst_bytes=10, slot=1)
    inst = [Instance(i, "8m", 100 + i) for i in range(4)]
    srv = Server(ex, inst, budget_bytes=10_000)
    out = srv.run(_stream(200, 4, rate=20000.0))
    assert all(r.status == "done" for r in out)
    # several batches were launched, and some began before the first one finished
    assert srv.launches > 1
    first_done = min(r.done for r in out)
    assert sum(1 for r in out if r.admitted < first_done) > len(ex.launched[0])


def test_results_do_not_depend_on_the_mix():
    ex = FakeExecutor(inst_bytes=10, slot=1)
    inst = [Instance(i, "8m", 100 + i) for i in range(2)]
    srv = Server(ex, inst, budget_bytes=10_000)
    reqs = _stream(12, 2)
    srv.run(reqs)
    for r in reqs[:4]:
        alone = Server(FakeExecutor(inst_bytes=10, slot=1), inst, budget_bytes=10_000)
        rr = Request(r.rid, r.instance, r.frame, 0.0)
        alone.run([rr])
        assert np.array_equal(alone.results[r.rid], srv.results[r.rid])


def test_binding_budget_evicts_holds_and_reports():
    """A budget for one resident instance at a time: requests alternating between two instances
    force evictions, are held for HBM, still finish in per-instance order, and the report counts
    the holds and queue waits."""
    ex = FakeExecutor(duration=0.001, inst_bytes=1000, slot=100)
    inst = [Instance(0, "39m", 1), Instance(1, "39m", 2)]
    srv = Server(ex, inst, budget_bytes=1000 + 2 * 100)    # one instance, two slots
    reqs = [Request(k, k % 2, k // 2, 0.0005 * k) for k in range(20)]
    out = srv.run(reqs, timeout=30)
    assert all(r.status == "done" for r in out)
    assert srv.evictions >= 5 and len(ex.destroyed) == srv.evictions
    assert srv.max_used <= srv.adm.budget
    rep = latency_report(out)
    assert rep["held_for_hbm"] > 0 and rep["queue_wait_p99_ms"] > 0.0
    for i in range(2):
        mine = [r for r in sorted(out, key=lambda r: r.admitted) if r.instance == i]
        assert [r.frame for r in mine] == sorted(r.frame for r in mine)


def test_slot_that_does_not_fit_evicts_idle_instances():
    """Every instance resident and idle, and the budget too small for one more staging slot: the
    request evicts an idle instance for its slot instead of waiting for ever."""
    ex = FakeExecutor(duration=0.001, inst_bytes=1000, slot=500)
    inst = [Instance(i, "39m", i) for i in range(4)]
    srv = Server(ex, inst, budget_bytes=4 * 1000 + 300)   # all four fit, a slot does not
    for i in inst:                                         # make all four resident
        assert srv._make_resident(srv.instances[i.iid])
    assert srv.adm.used == 4000
    out = srv.run([Request(0, 2, 0, 0.0), Request(1, 0, 0, 0.0), Request(2, 3, 0, 0.0)], timeout=10)
    assert all(r.status == "done" for r in out)
    assert srv.evictions >= 1 and srv.max_used <= srv.adm.budget
