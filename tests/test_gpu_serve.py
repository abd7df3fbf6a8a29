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
    # continuous batching: a batch is launched while an earlier one is still on the device
    assert srv.max_inflight >= 2, srv.max_inflight
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


def _served_39m_want(frame, inst_seed, noise_seed, sub_lgs, sub_ngs):
    """The oracle's measurement of one 39 m request: 9 residual wavefronts (screen window minus the
    three DM surfaces shifted for each guide star's direction), then the 6 LGS and 3 NGS sensors
    on the sampled sub-apertures, noise keyed by (noise_seed, frame)."""
    import math

    from gen import configs as G
    from gen import screens as S
    from oracle import dm as OD
    from oracle import wfs as OW
    screen = S.screen_opd_m(2048, 4.875e-2, seed=inst_seed).astype(np.float32).astype(np.float64)
    surfaces, sizes = [], []
    for d, (alt, pitch) in enumerate(G.DMS):
        act = OD.actuators(800, 4.875e-2, alt, pitch, G.DM_FIELD_RADIUS_ARCSEC)
        size = OD.surface_size(800, 4.875e-2, alt, G.DM_FIELD_RADIUS_ARCSEC)
        c = S.dm_coefficients(len(act), inst_seed * 10 + d).astype(np.float32).astype(np.float64)
        surfaces.append(OD.dm_surface(size, act, c, pitch, G.DM_COUPLING, G.DM_PATCH))
        sizes.append(size)
    # guide stars: 6 LGS at 45 arcsec, 3 NGS at 60 arcsec; screen window (50 k, 50 k + t)
    dirs = ([(45 * math.cos(math.radians(60 * w)), 45 * math.sin(math.radians(60 * w))) for w in range(6)]
            + [(60 * math.cos(math.radians(120 * j)), 60 * math.sin(math.radians(120 * j))) for j in range(3)])
    t = frame % (2048 - 800 - 400 + 1)
    opd = np.empty((9, 800, 800))
    for k, (tx, ty) in enumerate(dirs):
        org = [(sz // 2 - 400 + OD.footprint_shift_px(alt, ty, 4.875e-2),
                sz // 2 - 400 + OD.footprint_shift_px(alt, tx, 4.875e-2)) for sz, (alt, _) in zip(sizes, G.DMS)]
        opd[k] = OD.residual_opd(screen, (50 * k, 50 * k + t), surfaces, org, 800)
    lgs = OW.Sensor(G.CFG1, 6, G.launch_positions(G.CFG1, 6))
    ngs = OW.Sensor(G.CFG4_NGS, 3)
    want_l = lgs.measure(opd[None, :6], seed=noise_seed, frame0=frame, subset=sub_lgs)
    want_n = ngs.measure(opd[None, 6:], seed=noise_seed, frame0=frame, subset=sub_ngs)
    return want_l, want_n, lgs.n_valid, ngs.n_valid


def test_large_instance_requests_match_oracle(torch_dev):
    """Three 39 m requests served together with 8 m traffic (noise on): on sampled sub-apertures of
    all 9 sensors, counts equal the oracle's except explained ties, read noise and slopes within
    the tolerances."""
    from gen import configs as G
    from paper_1408_0698_amd.serve import GpuExecutor, Instance, Request, Server
    from tests.test_gpu_wfs import check_noisy
    inst = [Instance(0, "39m", seed=201), Instance(1, "8m", seed=101)]
    ex = GpuExecutor(keep_images=True)
    srv = Server(ex, inst, budget_bytes=4 << 30)
    frames = (3, 4, 517)
    reqs = [Request(k, 0, f, 1e-4 * k) for k, f in enumerate(frames)]
    reqs += [Request(10 + k, 1, k, 5e-5 * k) for k in range(6)]
    out = srv.run(reqs, timeout=120)
    assert all(r.status == "done" for r in out)
    rng = np.random.default_rng(5)
    sub_lgs = np.sort(rng.choice(4928, 24, replace=False))
    sub_ngs = np.array([0, 3])
    for k, f in enumerate(frames):
        print(f"served 39 m request, frame {f}", flush=True)
        sl_l, sl_n, im_l, im_n = srv.results[k]
        seed = ex._seed(reqs[k])
        want_l, want_n, nv_l, nv_n = _served_39m_want(f, 201, seed, sub_lgs, sub_ngs)
        got_l = {"images": im_l[None][:, :, sub_lgs].astype(np.float64), "slopes": sl_l[None][..., sub_lgs].astype(np.float64)}
        got_n = {"images": im_n[None][:, :, sub_ngs].astype(np.float64), "slopes": sl_n[None][..., sub_ngs].astype(np.float64)}
        check_noisy(G.CFG1, 6, None, got_l, want_l, seed, f, lambda w: w * nv_l + sub_lgs)
        check_noisy(G.CFG4_NGS, 3, None, got_n, want_n, seed, f, lambda w: w * nv_n + sub_ngs)
