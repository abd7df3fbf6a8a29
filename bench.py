"""Benchmark: Shack-Hartmann frames/s for 6 LGS sensors of 80x80 sub-apertures on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--frames-per-step B]

A step is one sh_wfs_measure launch over B frames of the 39 m workload
(6 LGS x 4928 valid 10x10-px sub-apertures, FFT 40, sodium kernel,
16x16 detector, 500 photons + 3 e- read noise, thresholded centroid).
OPD frames are resident in HBM before timing starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# nominal FFT flops of one 40x40 complex 2-D transform: 5 N^2 log2(N^2); three per sub-aperture
# (the convention's count; the band-limited kernels execute fewer operations, see COUNTERS)
FLOP_PER_SUBAP_NOMINAL = 3 * 5 * 40 * 40 * math.log2(40 * 40)
PEAK_FP32_TFLOPS = 157.3
# VALU issue slots: 256 CUs x 4 SIMDs, one wave64 slot per SIMD every 4 cycles at 2.4 GHz; two FP32
# instructions of different wavefronts can share a slot (dual issue, counted by SQ_ACTIVE_INST_VALU2),
# which is how the FP32 vector peak (157.3 TFLOP/s = 2 FMA slots' worth) is reached
PEAK_VALU_SLOTS = 256 * 4 * 2.4e9 / 4
# launch variants of the 40-point shapes whose measurement is two kernels (fused stages up to the
# detector, then noise and centroid); the roofline time covers both
DETECTOR_SPLIT_VARIANTS = (6, 7, 8, 9, 10, 11, 12)
CSRC = os.path.join(ROOT, "paper_1408_0698_amd", "csrc")
# executed FLOPs (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_{F32,F64}), VALU instructions and HBM bytes
# (FETCH_SIZE, WRITE_SIZE) per frame of the default launch variant, from rocprofv3 runs of this bench
COUNTERS = os.path.join(ROOT, "profiles", "wfs_measure_lgs39m_counters.json")
LATENCY_LAUNCHES = 200


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("wfs_kernels.hip", "regfft.h", "noise.h", "internal.h", "band_rebin.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(variant, noise_head):
    """Per-frame counter totals of the committed summary for this launch variant and noise-kernel
    head, or None if the kernel sources changed since the counters were taken or that
    configuration was not profiled."""
    try:
        with open(COUNTERS) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("configs", {}).get(f"{variant}/{noise_head}")


def cpu_baseline(cfg, launch, opd, min_seconds=10.0):
    """The FP64 oracle on a bounded sample: every 4th valid sub-aperture of each sensor, repeated
    until min_seconds of CPU time have been spent; scaled to whole frames/s."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import wfs as OW

    sens = OW.Sensor(cfg, 6, launch)
    sub = np.arange(0, sens.n_valid, 4)
    for w in range(6):
        sens.khat(w, sub)               # plan setup, outside the timed region
    reps = 0
    t0 = time.perf_counter()
    while True:
        sens.measure(opd[:1], seed=698, frame0=0, subset=sub)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    per_frame = el / reps * (sens.n_valid / len(sub))
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    return {"value": 1.0 / per_frame, "unit": "frames/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{len(sub)} of {sens.n_valid} sub-apertures of each of the 6 sensors (every 4th), "
                      f"noise on, {reps} repetitions in {el:.1f} s, scaled to whole frames; kernel spectra "
                      f"computed before timing"}


def _time(fn, n, stream):
    """Milliseconds per call of fn() over n calls, HIP events on `stream`."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(n):
        fn(k)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / n


def ex_ngs8m(stream):
    """8 m NGS frame: eager launch, captured graph replay, and 4096 frames per launch."""
    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import shwfs
    out = {}
    # 8 m NGS (80 sub-apertures): launch-bound.  Graphs: one loop step per graph (measure with the
    # device frame counter, counter += 1), and K = 32 steps per graph (offsets 0..31, one counter += 32)
    plan0 = shwfs.WfsPlan(G.CFG0)
    K = 32
    opd0 = torch.from_numpy(S.ngs8m_opd(K)[:, None].copy()).cuda()
    sl0 = torch.zeros((K, 1, 2, plan0.n_valid), device="cuda")
    ctr = torch.zeros(1, dtype=torch.int64, device="cuda")
    gstream = torch.cuda.Stream()      # graph capture needs a stream other than the NULL stream
    with torch.cuda.stream(gstream):
        with shwfs.Graph.capture(gstream) as cap:
            plan0.measure_devframe(opd0[:1], sl0[:1], ctr, stream=gstream)
            shwfs.counter_add(ctr, 1, stream=gstream)
        g1 = cap.graph
        with shwfs.Graph.capture(gstream) as cap:
            for k in range(K):
                plan0.measure_devframe(opd0[k:k + 1], sl0[k:k + 1], ctr, stream=gstream, frame_offset=k)
            shwfs.counter_add(ctr, K, stream=gstream)
        gk = cap.graph
        for _ in range(20):
            g1.launch(gstream)
            gk.launch(gstream)
        ms_graph = _time(lambda k: g1.launch(gstream), 500, gstream)
        ms_graph_k = _time(lambda k: gk.launch(gstream), 100, gstream) / K
        # the frames' views made once, so that the loop times the library call, not tensor slicing
        ov = [opd0[k:k + 1] for k in range(K)]
        sv = [sl0[k:k + 1] for k in range(K)]
        ms_eager = _time(lambda k: plan0.measure(ov[k % K], sv[k % K], frame0=k, stream=gstream), 500, gstream)
    torch.cuda.synchronize()
    out["ngs8m_graph_frames_per_s"] = 1e3 / ms_graph
    out["ngs8m_graph32_frames_per_s"] = 1e3 / ms_graph_k
    out["ngs8m_eager_frames_per_s"] = 1e3 / ms_eager
    # 8 m NGS, 4096 frames per launch (batch of loop steps)
    opd0b = torch.from_numpy(S.ngs8m_opd(4096)[:, None].copy()).cuda()
    sl0b = torch.zeros((4096, 1, 2, plan0.n_valid), device="cuda")
    with torch.cuda.stream(stream):
        plan0.measure(opd0b, sl0b, stream=stream)
        ms_b = _time(lambda k: plan0.measure(opd0b, sl0b, frame0=4096 * k, stream=stream), 10, stream)
    out["ngs8m_b4096_frames_per_s"] = 4096e3 / ms_b
    out["ngs8m_b4096_tflops_nominal"] = 4096 * plan0.n_valid * 5 * 256 * math.log2(256) / (ms_b * 1e-3) / 1e12
    del opd0b, sl0b
    return out


def ex_precision(stream):
    """The 6-LGS frame with the sub-aperture DFTs as MFMA GEMMs (bf16, bf16 and fp16 hi+lo)."""
    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import shwfs
    out = {}
    # precision form: the 6-LGS frame with MFMA DFT GEMMs (noise on)
    launch = G.launch_positions(G.CFG1, 6)
    opd1 = torch.from_numpy(S.lgs39m_opd(2, 6)).cuda()
    mm = {}
    for name, prec, mult in (("bf16", G.PREC_BF16, 1), ("bf16x3", G.PREC_BF16X3, 3), ("fp16x3", G.PREC_FP16X3, 3)):
        pl = shwfs.WfsPlan(G.CFG1.replace(flags=G.CFG1.flags | (prec << 4)), 6, launch)
        sl = torch.zeros((1, 6, 2, pl.n_valid), device="cuda")
        with torch.cuda.stream(stream):
            for k in range(3):
                pl.measure(opd1[k % 2:k % 2 + 1], sl, seed=1, frame0=k, stream=stream)
            ms = _time(lambda k: pl.measure(opd1[k % 2:k % 2 + 1], sl, seed=1, frame0=k, stream=stream), 20, stream)
        # 102 16x16x16 products per sub-aperture, each one (bf16) or three (split) MFMA instructions
        flops = 6 * pl.n_valid * 102 * mult * 2 * 16 * 16 * 16
        mm[name] = {"frames_per_s": 1e3 / ms, "ms_per_frame": ms, "mfma_tflops": flops / (ms * 1e-3) / 1e12,
                    "mfma_frac_of_2500": flops / (ms * 1e-3) / 2.5e15}
        pl.close()
    out["precision_mfma"] = mm
    del opd1
    return out


def ex_sodium(stream):
    """The 6-LGS frame in the sodium sub-layer form (3 sub-layers)."""
    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import shwfs
    out = {}
    launch = G.launch_positions(G.CFG1, 6)
    opd1 = torch.from_numpy(S.lgs39m_opd(2, 6)).cuda()
    # sodium sub-layer form (3 sub-layers, shared wavefront, noise on): the form of the paper's
    # 4.5 s per-sensor step; per-sensor ms is the time of the 6-sensor frame / 6
    pls = shwfs.WfsPlan(G.CFG1, 6, launch, sodium=G.SODIUM)
    sls = torch.zeros((1, 6, 2, pls.n_valid), device="cuda")
    opds = opd1.unsqueeze(2).expand(-1, -1, G.SODIUM_NSUB, -1, -1)
    with torch.cuda.stream(stream):
        pls.autotune(opd1[:1], sls, reps=10, stream=stream)
        for k in range(3):
            pls.measure_sodium(opds[k % 2:k % 2 + 1], sls, seed=1, frame0=k, stream=stream)
        ms = _time(lambda k: pls.measure_sodium(opds[k % 2:k % 2 + 1], sls, seed=1, frame0=k, stream=stream),
                   20, stream)
    out["sodium3_frames_per_s"] = 1e3 / ms
    out["sodium3_ms_per_sensor_step"] = ms / 6
    pls.close()
    return out


def ex_ngs512(stream):
    """3 NGS sensors of 2x2 sub-apertures of 400 px (FFT 512)."""
    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import shwfs
    out = {}
    # 3 NGS, 2x2 sub-apertures of 400 px padded to 512, noise on
    plan4 = shwfs.WfsPlan(G.CFG4_NGS, 3)
    opd4 = torch.from_numpy(S.lgs39m_opd(4, 3)).cuda()
    sl4 = torch.zeros((4, 3, 2, plan4.n_valid), device="cuda")
    with torch.cuda.stream(stream):
        for _ in range(3):
            plan4.measure(opd4, sl4, seed=1, stream=stream)
        ms4 = _time(lambda k: plan4.measure(opd4, sl4, seed=1, frame0=4 * k, stream=stream), 20, stream)
    out["ngs512_3x2x2_frames_per_s"] = 4e3 / ms4
    return out


def ex_psf(stream):
    """Science PSF of 9 stars x 20 frames: DM surfaces, residuals and PSF accumulation."""
    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import shwfs
    out = {}
    # science PSF: DM surfaces from commands, residuals for 9 stars x 20 frames, PSF accumulation
    scr = torch.from_numpy(S.screen_opd_m(2048, 4.875e-2).astype(np.float32)).cuda()
    dms, coefs, surfs = [], [], []
    for d, (alt, pitch) in enumerate(G.DMS):
        dm = shwfs.DmPlan(800, 4.875e-2, alt, pitch, G.DM_FIELD_RADIUS_ARCSEC, G.DM_COUPLING, G.DM_PATCH)
        dms.append(dm)
        coefs.append(torch.from_numpy(S.dm_coefficients(dm.n_act, 100 + d).astype(np.float32)).cuda())
        surfs.append(torch.zeros((dm.size, dm.size), device="cuda"))
    arcsec = np.pi / 180 / 3600
    nfr = G.CFG3_FRAMES
    scr_o, dm_o = [], []
    for (tx, ty) in G.CFG3_STARS:
        for t in range(nfr):
            scr_o.append((0, t))
            dm_o.append([(sf.shape[0] // 2 - 400 + int(np.floor(alt * ty * arcsec / 4.875e-2 + 0.5)),
                          sf.shape[0] // 2 - 400 + int(np.floor(alt * tx * arcsec / 4.875e-2 + 0.5)))
                         for sf, (alt, _) in zip(surfs, G.DMS)])
    res = torch.zeros((len(scr_o), 800, 800), device="cuda")
    psf = shwfs.PsfPlan(800, 4.875e-2, 0.14, 1600, G.CFG3.wavelength_m)
    acc = torch.zeros((9, 1600, 1600), device="cuda")
    sr = torch.zeros((9, nfr), device="cuda")

    def psf_step(k):
        for dm, c, sf in zip(dms, coefs, surfs):
            dm.surface(c, sf, stream=stream)
        shwfs.residual_opd(scr, surfs, 800, scr_o, dm_o, res, stream=stream)
        psf.accumulate_stars(res.view(9, nfr, 800, 800), acc, sr, stream=stream)

    with torch.cuda.stream(stream):
        psf_step(0)
        ms3 = _time(psf_step, 3, stream)
        ms_acc = _time(lambda k: psf.accumulate_stars(res.view(9, nfr, 800, 800), acc, sr, stream=stream), 3, stream)
    out["psf_9stars_x20_star_frames_per_s"] = 9 * nfr * 1e3 / ms3
    out["psf_step_ms"] = ms3
    out["psf_accumulate_ms"] = ms_acc
    # algorithmic HBM bytes per star-frame of the PSF kernels: OPD 2.56 MB + intermediate written and
    # read 2 x 10.24 MB, plus the accumulator read and written once per star per call (2 x 10.24 MB / 20)
    per_sf = 800 * 800 * 4 + 2 * 800 * 1600 * 8 + 2 * 1600 * 1600 * 4 / nfr
    out["psf_accumulate_GBps"] = per_sf * 9 * nfr / (ms_acc * 1e-3) / 1e9
    out["psf_accumulate_frac_of_8TBps"] = per_sf * 9 * nfr / (ms_acc * 1e-3) / 8e12
    out["psf_mean_strehl_last_frame"] = float(sr[:, -1].mean().item())
    del res, acc
    torch.cuda.synchronize()
    return out


def ex_openloop(stream):
    """LGS wavefronts from the atmosphere: 6 LGS x 3 sodium sub-layers projected through three 2048^2
    layers with the cone effect, plus each laser's uplink tilt, then the sodium-layer measurement."""
    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import shwfs
    cfg = G.CFG1
    out = {}
    layers = [(torch.from_numpy(S.screen_opd_m(2048, cfg.pupil_dx_m, G.SCREEN_SEED + k).astype(np.float32)).cuda(),
               cfg.pupil_dx_m, h, 1023.5, 1023.5) for k, h in enumerate((0.0, 4000.0, 12700.0))]
    launch = G.launch_positions(cfg, 6)
    ang = np.arange(6) * np.pi / 3
    dirs = [(45.0 * G.ARCSEC * np.cos(a), 45.0 * G.ARCSEC * np.sin(a)) for a in ang]
    lgs = [(lx, ly, tx, ty, cfg.na_height_m) for (lx, ly), (tx, ty) in zip(launch, dirs)]
    targets = [(tx, ty, cfg.na_height_m + dh) for tx, ty in dirs for dh in G.SODIUM[0]]
    tilt = torch.zeros((6, 2), dtype=torch.float64, device="cuda")
    tilt18 = torch.zeros((18, 2), dtype=torch.float64, device="cuda")
    opd = torch.zeros((1, 6, 3, cfg.pupil_n, cfg.pupil_n), device="cuda")
    plan = shwfs.WfsPlan(cfg, 6, launch, sodium=G.SODIUM)
    sl = torch.zeros((1, 6, 2, plan.n_valid), device="cuda")

    def project(k):
        shwfs.project_layers(layers, cfg.pupil_n, cfg.pupil_dx_m, targets, opd.view(18, cfg.pupil_n, cfg.pupil_n),
                             tilt=tilt18, stream=stream)

    def uplink(k):
        shwfs.uplink_tilt(layers, lgs, 0.4, 64, tilt, stream=stream)
        tilt18.copy_(tilt.repeat_interleave(3, dim=0))

    def frame(k):
        uplink(k)
        project(k)
        plan.measure_sodium(opd, sl, seed=1, frame0=k, stream=stream)

    with torch.cuda.stream(stream):
        frame(0)
        ms_proj = _time(project, 10, stream)
        ms_up = _time(uplink, 10, stream)
        ms_frame = _time(frame, 10, stream)
    out["openloop_project_18x800x800_ms"] = ms_proj
    # gathered bytes per output sample: 3 layers x 4 taps (mostly L2 hits); written 4 B
    out["openloop_project_Gsamples_per_s"] = 18 * cfg.pupil_n ** 2 / (ms_proj * 1e-3) / 1e9
    out["openloop_uplink_6lgs_ms"] = ms_up
    out["openloop_lgs_frame_ms"] = ms_frame
    out["openloop_uplink_tilt_mas_lgs0"] = [float(v) / G.ARCSEC * 1e3 for v in tilt[0].cpu()]
    return out


def ex_psf_extras(stream):
    """Encircled energy of 9 integrated 1600^2 PSFs at 20 radii, and a 3-wavelength colour-weighted PSF
    of 20 frames of one star."""
    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import shwfs
    out = {}
    cfg = G.CFG3
    plans = [shwfs.PsfPlan(cfg.pupil_n, cfg.pupil_dx_m, cfg.obstruction, cfg.fft_m, l)
             for l in (1.65e-6, 1.5e-6, 1.8e-6)]
    scr = S.screen_opd_m(2048, cfg.pupil_dx_m)
    opd = torch.from_numpy(np.stack([scr[:800, t:t + 800] * 0.1 for t in range(G.CFG3_FRAMES)])
                           .astype(np.float32)).cuda()
    poly = torch.zeros((1600, 1600), device="cuda")
    acc = torch.zeros((9, 1600, 1600), device="cuda")
    with torch.cuda.stream(stream):
        plans[0].accumulate(opd, acc[0], stream=stream)
        for s_ in range(1, 9):
            acc[s_].copy_(acc[0])
        radii = [2.0 * (k + 1) for k in range(20)]
        # the first call grows the plan's workspaces: outside the timed calls
        ee = plans[0].encircled_energy(acc, radii, stream=stream)
        ms_ee = _time(lambda k: plans[0].encircled_energy(acc, radii, out=ee, stream=stream), 20, stream)

        def poly_step(k):
            poly.zero_()
            shwfs.polychromatic_psf(plans, (0.5, 0.2, 0.3), opd, poly, stream=stream)

        poly_step(0)
        ms_poly = _time(poly_step, 2, stream)
    out["ee_9psf_20radii_ms"] = ms_ee
    out["ee_GBps"] = 9 * 1600 * 1600 * 4 / (ms_ee * 1e-3) / 1e9
    out["ee_r2px_r10px_r40px"] = [float(ee[0, 0]), float(ee[0, 4]), float(ee[0, 19])]
    out["poly_psf_3lambda_20frames_ms"] = ms_poly
    return out


EXTRAS = ("ngs8m", "precision", "sodium", "ngs512", "psf", "calibration", "loop", "openloop", "psf_extras",
          "served")
EXTRAS_DEFAULT = EXTRAS


def extras(stream, which=EXTRAS):
    """Secondary workloads, each timed with HIP events on its stream."""
    import torch
    fns = {"ngs8m": ex_ngs8m, "precision": ex_precision, "sodium": ex_sodium, "ngs512": ex_ngs512, "psf": ex_psf,
           "calibration": calibration, "loop": closed_loop, "openloop": ex_openloop, "psf_extras": ex_psf_extras}
    out = {}
    for name in which:
        if name == "served":
            out["served"], out["served_load_sweep"], out["served_knee_req_per_s"] = served()
        else:
            out.update(fns[name](stream))
        torch.cuda.synchronize()
    return out


def calibration(stream):
    """Push-pull interaction matrix of one LGS sensor (launcher 0, noise off) over every actuator of the
    ground DM (pitch 10 px): 2 frames per mode, influence frames, measurement and combination on the GPU."""
    import time

    import numpy as np
    import torch

    from gen import configs as G
    from paper_1408_0698_amd import calib, shwfs
    cfg = G.CFG1.replace(flags=0)
    plan = shwfs.WfsPlan(cfg, 1, G.launch_positions(G.CFG1, 6)[:1])
    alt, pitch = G.DMS[0]
    dm = shwfs.DmPlan(800, 4.875e-2, alt, pitch, G.DM_FIELD_RADIUS_ARCSEC, G.DM_COUPLING, G.DM_PATCH)
    r0 = (dm.size - 800) // 2
    acts = np.arange(dm.n_act, dtype=np.int32)
    with torch.cuda.stream(stream):
        calib.interaction_matrix(plan, dm, acts[:512], 50e-9, r0, r0, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        im = calib.interaction_matrix(plan, dm, acts, 50e-9, r0, r0, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    ok = bool(torch.isfinite(im).all().item())
    del im
    return {"calibration_modes": int(dm.n_act), "calibration_s": dt, "calibration_frames_per_s": 2 * dm.n_act / dt,
            "calibration_finite": ok}


def closed_loop(stream):
    """Closed-loop step of the 39 m system on the device: 3 DM surfaces from 8219 commands, residuals of the
    6 LGS directions, the 6-LGS measurement, the 8219 x 59,136 control-matrix product (1.94 GB, synthetic)
    and the integrator.  Also the product alone against the HBM roofline."""
    import math

    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import loop, shwfs
    launch = G.launch_positions(G.CFG1, 6)
    plan = shwfs.WfsPlan(G.CFG1, 6, launch)
    dms = [(shwfs.DmPlan(800, 4.875e-2, alt, pitch, G.DM_FIELD_RADIUS_ARCSEC, G.DM_COUPLING, G.DM_PATCH), alt)
           for alt, pitch in G.DMS]
    n_modes = sum(d.n_act for d, _ in dms)
    n_slopes = 6 * 2 * plan.n_valid
    gen = torch.Generator(device="cuda")
    gen.manual_seed(G.SCREEN_SEED)
    cm = torch.randn((n_modes, n_slopes), device="cuda", generator=gen) * (1e-9 / math.sqrt(n_slopes))
    scr = torch.from_numpy(S.screen_opd_m(2048, 4.875e-2).astype(np.float32)).cuda()
    dirs = [(45 * math.cos(math.radians(60 * w)), 45 * math.sin(math.radians(60 * w))) for w in range(6)]
    lp = loop.ClosedLoop(plan, dms, dirs, scr, cm, 0.5, seed=G.NOISE_SEED)
    origins = lambda t: [(50 * w, 50 * w + t % 800) for w in range(6)]
    with torch.cuda.stream(stream):
        for t in range(3):
            lp.step(origins(t), t, stream=stream)
        ms = _time(lambda k: lp.step(origins(k), 3 + k, stream=stream), 20, stream)
        sl = lp.slopes.view(-1)
        ms_r = _time(lambda k: lp.recon.step(cm, sl, 0.5, lp.coefs, stream=stream), 20, stream)
    ok = bool(torch.isfinite(lp.coefs).all().item())
    nbytes = n_modes * n_slopes * 4 + n_slopes * 4 + 2 * n_modes * 4
    out = {"loop_step_ms": ms, "loop_steps_per_s": 1e3 / ms, "loop_modes": n_modes, "loop_slopes": n_slopes,
           "recon_ms": ms_r, "recon_GBps": nbytes / (ms_r * 1e-3) / 1e9, "recon_frac_of_8TBps": nbytes / (ms_r * 1e-3) / 8e12,
           "loop_finite": ok}
    del cm, lp
    torch.cuda.synchronize()
    return out


def _binding_budget(ex):
    """HBM budget of the served runs: the shared plans, 3 of the 4 large instances and all 8 small
    ones resident, 3 large and 16 small staging slots.  A request for the large instance that is
    not resident waits for HBM and evicts an idle one."""
    return (ex.shared_bytes() + 3 * ex.instance_bytes("39m") + 8 * ex.instance_bytes("8m")
            + 3 * ex.slot_bytes("39m") + 16 * ex.slot_bytes("8m"))


def _served_run(ex, budget, rate_hz, duration_s, warm_s, seed):
    from paper_1408_0698_amd.serve import Server, latency_report, make_mix
    instances, reqs = make_mix(rate_hz=rate_hz, duration_s=warm_s + duration_s, seed=seed)
    srv = Server(ex, instances, budget)
    srv.warm()
    ev0 = dict(ex.stats)
    out = srv.run(reqs, timeout=600)
    rep = latency_report([r for r in out if r.arrival >= warm_s])
    print(f"served: {rate_hz:.0f} req/s for {warm_s + duration_s:.2f} s: {rep.get('completed')} completed, "
          f"p99 {rep.get('p99_ms', float('nan')):.3f} ms, {srv.evictions} evictions", file=sys.stderr, flush=True)
    rep.update({"offered_req_per_s": rate_hz, "duration_s": duration_s, "warmup_s": warm_s,
                "requests": sum(r.arrival >= warm_s for r in reqs), "launches": srv.launches,
                "max_inflight_batches": srv.max_inflight, "evictions": srv.evictions,
                "restores": ex.stats["restored"] - ev0["restored"], "max_hbm_used_bytes": srv.max_used,
                "budget_bytes": budget})
    return rep


def served(duration_s=30.0, warm_s=2.0):
    """Served mix: Poisson arrivals at 2000 req/s, 70% 8 m frames and 30% 39 m frames (6 LGS + 3 NGS)
    over 12 instances (8 small, 4 large), continuous batching under a binding HBM budget; 30 s
    measured after 2 s of warm-up, p50/p99 arrival -> slopes-ready latency; then a load sweep (1 s
    per rate after 0.25 s of warm-up) up to saturation."""
    from paper_1408_0698_amd.serve import GpuExecutor
    ex = GpuExecutor()
    budget = _binding_budget(ex)
    main = _served_run(ex, budget, 2000.0, duration_s, warm_s, seed=2000)
    sweep, knee = [], None
    for rate in (2000.0, 4000.0, 8000.0, 16000.0, 24000.0, 32000.0, 48000.0, 64000.0):
        rep = _served_run(ex, budget, rate, 1.0, 0.25, seed=int(rate) + 1)
        sweep.append(rep)
        if rep["frames_per_s"] >= 0.95 * rate:
            knee = rate
        else:
            break              # saturated: completed rate below the offered rate
    return main, sweep, knee


# (name, VALU instructions per iteration of the probe's loop)
VALU_PROBE_KINDS = (("fp32 fma", 16), ("fp32 add", 16), ("dpp move", 16), ("sine", 16), ("fp64 fma", 16),
                    ("64-bit integer multiply-add + xor", 32))


def valu_probe(blocks=2048, iters=2048, reps=5):
    """Issue cost of VALU instruction kinds (lib/libshw_probe.so): 8 independent chains per lane,
    blocks of 256 lanes (2048 blocks: 8 wavefronts on every SIMD of 256 CUs; the FMA probe also at
    2 and 1 wavefronts per SIMD).  Cycles per wave64 instruction per SIMD at 2.4 GHz from the launch
    time (HIP events, mean of `reps` launches)."""
    import ctypes

    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1408_0698_amd", "lib", "libshw_probe.so"))
    lib.shw_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.shw_probe_valu.restype = ctypes.c_int
    torch.cuda.set_device(0)
    out = torch.zeros(blocks * 256, device="cuda")
    st = torch.cuda.current_stream()
    runs = [(kind, name, per_iter, blocks) for kind, (name, per_iter) in enumerate(VALU_PROBE_KINDS)]
    runs += [(0, VALU_PROBE_KINDS[0][0], VALU_PROBE_KINDS[0][1], b) for b in (blocks // 4, blocks // 8)]
    res = []
    def launch(kind, nb):
        rc = lib.shw_probe_valu(kind, nb, iters, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"shw_probe_valu({kind}) returned {rc}")

    for kind, name, per_iter, nb in runs:
        launch(kind, nb)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            launch(kind, nb)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        waves_per_simd = nb * 4 / (256 * 4)
        res.append({"probe": name, "blocks": nb, "waves_per_simd": waves_per_simd, "ms": ms,
                    "wave_instructions": nb * 4 * iters * per_iter,
                    "cycles_per_wave_instruction_per_simd_at_2.4GHz":
                        ms * 1e-3 * 2.4e9 / (waves_per_simd * iters * per_iter)})
    return {"valu_probe": res, "lanes_per_block": 256, "iters": iters}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--frames-per-step", type=int, default=1)
    ap.add_argument("--resident-frames", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--extras", default=",".join(EXTRAS_DEFAULT),
                    help="comma-separated secondary workloads to run after the headline")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--noise-head", type=int, default=0, choices=(0, 2, 4, 6),
                    help="with --no-autotune: the noise kernel's inversion head (default: the plan's, 4)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="with --no-autotune: the launch variant (default: the plan's)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="before timing, run 5 plain device copies of this many MB (profiler counter scale)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only time the VALU issue probes (calibration of the roofline's issue model) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a design note",
              file=sys.stderr)
        sys.exit(2)
    if args.valu_probe:
        print(json.dumps(valu_probe()))
        return

    import numpy as np
    import torch

    from gen import configs as G
    from gen import screens as S
    from paper_1408_0698_amd import shwfs

    torch.cuda.set_device(0)
    cfg = G.CFG1
    launch = G.launch_positions(cfg, 6)
    plan = shwfs.WfsPlan(cfg, 6, launch)
    B = args.frames_per_step
    nres = max(args.resident_frames, B)
    opd_host = S.lgs39m_opd(nres, 6)
    opd = torch.from_numpy(opd_host).cuda()
    slopes = torch.zeros((B, 6, 2, plan.n_valid), device="cuda")
    stream = torch.cuda.current_stream()

    if args.calibrate_copy_mb > 0:
        n = args.calibrate_copy_mb * (1 << 20) // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.variant >= 0:
        plan.set_variant(args.variant)
    variant = plan.variant
    if args.noise_head:
        plan.set_noise_head(args.noise_head)
    tuned = None
    if not args.no_autotune:
        import tempfile

        from paper_1408_0698_amd import autotune
        os.environ.setdefault("SHW_AUTOTUNE_CACHE", os.path.join(tempfile.gettempdir(), "shwfs_autotune.json"))
        tuned = autotune.tuned_variant(plan, opd[:B], slopes, "gfx950", reps=20, stream=stream, retune=True)
        variant = tuned["variant"]

    def step(k):
        f0 = (k * B) % (nres - B + 1)
        plan.measure(opd[f0:f0 + B], slopes, seed=G.NOISE_SEED, frame0=k * B, stream=stream)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    # timed region: K steps back to back, HIP events on the launch stream around the whole region
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for k in range(args.steps):
        step(args.warmup + k)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    frames = args.steps * B
    value = frames / wall
    avg_launch_ms = e0.elapsed_time(e1) / args.steps
    # per-launch latency percentiles, from a separate run of LATENCY_LAUNCHES launches with events
    # around every launch
    n_lat = LATENCY_LAUNCHES
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_lat)]
    for k in range(n_lat):
        ev[k][0].record(stream)
        step(args.warmup + args.steps + k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])      # ms per launch (B frames)
    subaps = 6 * plan.n_valid * B
    launch_s = avg_launch_ms * 1e-3
    nominal = FLOP_PER_SUBAP_NOMINAL * subaps / launch_s / 1e12
    kernels = ("wfs_fused_kernel<10,40,40,16,lgs>"
               + (" + det_noise_kernel<16>" if variant in DETECTOR_SPLIT_VARIANTS else ""))
    ctr = measured_counters(variant, plan.noise_head)
    if ctr is not None:
        # executed FP32 FLOPs of both kernels (FMA = 2) per frame, from the committed counters
        fp32 = ctr["fp32_flop_per_frame"] * B / launch_s / 1e12
        roof = {"bound": "alu", "achieved": fp32, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": fp32 / PEAK_FP32_TFLOPS,
                "traffic": ctr["hbm_bytes_per_frame"] * B,
                "flops": "executed FP32 (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F32, FMA = 2) per frame, "
                         "counters in profiles/wfs_measure_lgs39m_valu.md",
                "fp64_tflops": ctr["fp64_flop_per_frame"] * B / launch_s / 1e12,
                "valu_slot_frac": (ctr["valu_issue_slots_per_frame"] * B / launch_s / PEAK_VALU_SLOTS
                                   if "valu_issue_slots_per_frame" in ctr else None),
                "valu_slot_note": "VALU issue slots per frame (wave instructions less the dual-issued ones, "
                                  "SQ_INSTS_VALU - SQ_ACTIVE_INST_VALU2, from the committed counters of another "
                                  "run) over this run's launch time, against 256 CU x 4 SIMD x 2.4 GHz / 4 cycles; "
                                  "a stream of independent FP32 FMAs at full occupancy reaches about 0.75 by this "
                                  "measure (bench.py --valu-probe, profiles/valu_issue_probe.md)",
                "nominal_tflops": nominal,
                "nominal_note": "3 x 5 N^2 log2 N^2 per sub-aperture (three full 40x40 transforms); the "
                                "band-limited kernels execute fewer operations",
                "kernel": f"sh_wfs_measure launch variant {variant}, noise head {plan.noise_head}: {kernels}",
                "avg_launch_ms": avg_launch_ms}
    else:
        # kernels changed since the counters were taken: no executed count, nominal reported alone
        roof = {"bound": "alu", "achieved": None, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": None, "nominal_tflops": nominal,
                "kernel": f"sh_wfs_measure launch variant {variant}: {kernels}",
                "avg_launch_ms": avg_launch_ms}
    out = {
        "metric": "SH-WFS frames/s (6 LGS, 80x80 subaps) + p50/p99 latency; % FP32/HBM roofline",
        "value": value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lgs39m: 6 LGS SH-WFS, 800x800 pupil at 4.875e-2 m, 80x80 subaps of 10x10 px, "
                               "FFT 40, sodium kernel, 16x16 det px, 500 ph + 3 e- RON, threshold 3 e-",
                   "frames_per_step": B, "subaps_per_frame": 6 * plan.n_valid},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "per": f"launch of {B} frame(s), HIP events on the launch stream, {n_lat} launches "
                              f"after the timed region"},
        "roofline": roof,
        "launch_variant": variant,
        "autotune_ms_per_variant": tuned["ms_per_launch"] if tuned else None,
        "autotune": ({"variant": tuned["variant"], "noise_head": tuned["noise_head"], "params": tuned["params"],
                      "ms_per_noise_head": tuned["ms_per_noise_head"]} if tuned else None),
    }
    if not args.no_extras:
        out["extras"] = extras(stream, [w for w in args.extras.split(",") if w])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, launch, opd_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
