"""Served mix on the GPU: each request's slopes are the same alone and in the mix."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_mix_invariance_and_latency(torch_dev):
    from paper_1408_0698_amd.serve import GpuExecutor, Request, Server, latency_report, make_mix
    instances, reqs = make_mix(n_small=4, n_large=2, rate_hz=2000.0, duration_s=0.15, seed=7)
    ex = GpuExecutor(keep_results=True)
    srv = Server(ex, instances, budget_bytes=6 << 30)
    assert srv.warm() == len(instances)
    out = srv.run(reqs, timeout=120)
    rep = latency_report(out)
    assert rep["completed"] == len(reqs), rep
    assert srv.launches > 1 and srv.max_used <= srv.adm.budget
    rng = np.random.default_rng(3)
    big = [r for r in reqs if instances[r.instance].cls == "39m"]
    small = [r for r in reqs if instances[r.instance].cls == "8m"]
    sample = list(rng.choice(big, 3, replace=False)) + list(rng.choice(small, 3, replace=False))
    for r in sample:
        alone_ex = GpuExecutor(keep_results=True)
        alone = Server(alone_ex, instances, budget_bytes=6 << 30)
        alone.run([Request(r.rid, r.instance, r.frame, 0.0)], timeout=60)
        a, b = alone.results[r.rid], srv.results[r.rid]
        assert np.array_equal(a[0], b[0]), f"request {r.rid} differs alone and in the mix"
        if a[1] is not None:
            assert np.array_equal(a[1], b[1])


def test_small_instance_matches_oracle(torch_dev):
    """An 8 m request through the server equals the oracle on the same screen window."""
    from gen import configs as G
    from gen import screens as S
    from oracle import wfs as OW
    from paper_1408_0698_amd.serve import GpuExecutor, Instance, Request, Server
    inst = [Instance(0, "8m", seed=123)]
    ex = GpuExecutor(keep_results=True)
    srv = Server(ex, inst, budget_bytes=2 << 30)
    srv.run([Request(0, 0, 517, 0.0)], timeout=60)
    got = srv.results[0][0]
    opd = S.ngs8m_opd(1, frame0=517, seed=123)[:, None]
    want = OW.Sensor(G.CFG0).measure(opd)["slopes"][0]
    assert np.abs(got - want).max() < 1e-3


def test_budget_too_small_for_large_instance_rejects(torch_dev):
    from paper_1408_0698_amd.serve import GpuExecutor, Instance, Request, Server
    ex = GpuExecutor()
    inst = [Instance(0, "39m", 1), Instance(1, "8m", 2)]
    budget = ex.shared_bytes() + ex.instance_bytes("8m") + ex.slot_bytes("8m") + (1 << 20)
    assert budget < ex.shared_bytes() + ex.instance_bytes("39m") + ex.slot_bytes("39m")
    srv = Server(ex, inst, budget_bytes=budget)
    out = srv.run([Request(0, 0, 0, 0.0), Request(1, 1, 0, 0.0)], timeout=60)
    st = {r.rid: r.status for r in out}
    assert st[0] == "rejected" and st[1] == "done"
