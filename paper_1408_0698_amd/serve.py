"""Served simulation: continuous batching of wavefront-sensor frame requests.

Several simulated telescopes ("instances") keep their phase screen and DM
state resident on the GPU.  A request asks for the slopes of one loop
step (frame) of one instance.  The server admits requests while HBM
allows (instance state + per-request staging buffers against a budget),
keeps requests of one instance in arrival order, and launches every
admitted request at once, also while earlier batches are still running:
one residual-OPD launch per instance and one work-list measurement launch
per sensor geometry.  Each class of instance has its own stream, so the
8 m and 39 m work overlaps on the device.  Noise is keyed by (instance
seed, frame), so a request's result does not depend on what it was
batched with.

Instance classes (the served mix):
  "8m"  : one NGS sensor, 80x80 pupil, 10x10 sub-apertures (FFT 16);
          a 512^2 screen at 0.1 m, frame t = window (t div 432, t mod 432).
  "39m" : 6 LGS sensors of 80x80 sub-apertures (FFT 40, sodium kernel) and
          3 NGS sensors of 2x2 sub-apertures of 400 px (FFT 512); a 2048^2
          screen and three DMs; sensor k looks through screen window
          (50k, 50k + t) minus the DM surfaces shifted for its direction.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Dict, List, Optional

ARCSEC = math.pi / (180.0 * 3600.0)


@dataclasses.dataclass
class Request:
    rid: int
    instance: int
    frame: int
    arrival: float                 # seconds on the server clock
    admitted: Optional[float] = None
    done: Optional[float] = None
    status: str = "waiting"        # waiting | running | done | failed | rejected | cancelled
    error: Optional[str] = None
    held: bool = False             # had to wait for HBM (instance residency or a staging slot)

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


@dataclasses.dataclass
class Instance:
    iid: int
    cls: str
    seed: int
    resident: bool = False
    inflight: int = 0
    last_used: float = 0.0


class Admission:
    """HBM accounting: resident instance state plus staging bytes of running requests."""

    def __init__(self, budget_bytes: int, shared_bytes: int = 0):
        self.budget = int(budget_bytes)
        self.used = int(shared_bytes)

    def fits(self, nbytes: int) -> bool:
        return self.used + nbytes <= self.budget

    def take(self, nbytes: int):
        assert self.fits(nbytes)
        self.used += nbytes

    def give(self, nbytes: int):
        self.used -= nbytes
        assert self.used >= 0


class Server:
    """Continuous-batching scheduler.  `executor` does the device work (see GpuExecutor)."""

    def __init__(self, executor, instances: List[Instance], budget_bytes: int, max_batch: int = 256):
        self.ex = executor
        if hasattr(executor, "bind"):
            executor.bind(instances)
        # the server owns its own records of residency and load
        self.instances = {i.iid: dataclasses.replace(i, resident=False, inflight=0, last_used=0.0) for i in instances}
        self.adm = Admission(budget_bytes, executor.shared_bytes())
        if self.adm.used > self.adm.budget:
            raise MemoryError(f"budget {budget_bytes} B below the shared plan state {self.adm.used} B")
        self.max_batch = max_batch
        self.queue: "collections.deque[Request]" = collections.deque()
        self.inflight = []          # (handle, [requests])
        self.finished: List[Request] = []
        self.results: Dict[int, object] = {}
        self.max_used = self.adm.used
        self.launches = 0
        self.evictions = 0             # idle resident instances evicted to admit another
        self.max_inflight = 0          # most batches on the device at once
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ------------------------------------------------------------ admission
    def _make_room(self, need: int, keep: Instance) -> bool:
        """Evict idle resident instances other than `keep` until `need` bytes fit.  True if they fit."""
        if not self.adm.fits(need):
            # victims: idle instances whose eviction alone makes room first (least recently used
            # first among them), then the others least recently used first, so that small
            # instances are not evicted one by one for a large request
            deficit = self.adm.used + need - self.adm.budget
            idle = sorted((i for i in self.instances.values() if i.resident and i.inflight == 0 and i is not keep),
                          key=lambda i: (self.ex.instance_bytes(i.cls) < deficit, i.last_used))
            if sum(self.ex.instance_bytes(i.cls) for i in idle) < deficit:
                return False       # evicting every idle instance would not make room: evict none
            for victim in idle:
                self.ex.destroy_instance(victim)
                victim.resident = False
                self.evictions += 1
                self.adm.give(self.ex.instance_bytes(victim.cls))
                if self.adm.fits(need):
                    break
        return self.adm.fits(need)

    def _make_resident(self, inst: Instance) -> bool:
        need = self.ex.instance_bytes(inst.cls)
        if not self._make_room(need, inst):
            return False
        self.ex.create_instance(inst)
        self.adm.take(need)
        inst.resident = True
        return True

    def warm(self) -> int:
        """Make instances resident ahead of traffic, in id order, while the budget allows
        (one staging slot per class is kept free).  Returns the number made resident."""
        n = 0
        for inst in sorted(self.instances.values(), key=lambda i: i.iid):
            need = self.ex.instance_bytes(inst.cls) + self.ex.slot_bytes(inst.cls)
            if not inst.resident and self.adm.fits(need):
                self.ex.create_instance(inst)
                self.adm.take(self.ex.instance_bytes(inst.cls))
                inst.resident = True
                n += 1
        return n

    def submit(self, req: Request):
        inst = self.instances[req.instance]
        floor = self.ex.instance_bytes(inst.cls) + self.ex.slot_bytes(inst.cls) + self.ex.shared_bytes()
        if floor > self.adm.budget:
            req.status = "rejected"
            req.error = f"instance needs {floor} B, budget {self.adm.budget} B"
            self.finished.append(req)
            return
        self.queue.append(req)

    def cancel(self, rid: int) -> bool:
        for r in self.queue:
            if r.rid == rid:
                self.queue.remove(r)
                r.status = "cancelled"
                self.finished.append(r)
                return True
        return False

    def _admit(self) -> List[Request]:
        batch, blocked = [], set()
        keep = collections.deque()
        while self.queue and len(batch) < self.max_batch:
            r = self.queue.popleft()
            inst = self.instances[r.instance]
            if r.instance in blocked:           # an earlier request of this instance is waiting
                keep.append(r)
                continue
            ok = inst.resident or self._make_resident(inst)
            slot = self.ex.slot_bytes(inst.cls)
            # a resident instance whose staging slot does not fit may evict idle others for it
            if ok and self._make_room(slot, inst):
                self.adm.take(slot)
                inst.inflight += 1
                inst.last_used = self.now()
                r.admitted = self.now()
                r.status = "running"
                batch.append(r)
            else:
                blocked.add(r.instance)
                r.held = True
                keep.append(r)
        keep.extend(self.queue)
        self.queue = keep
        return batch

    # ------------------------------------------------------------ progress
    def _retire(self, reqs, failed: Optional[str] = None):
        t = self.now()
        for r in reqs:
            inst = self.instances[r.instance]
            inst.inflight -= 1
            self.adm.give(self.ex.slot_bytes(inst.cls))
            r.done = t
            r.status = "failed" if failed else "done"
            r.error = failed
            self.finished.append(r)

    def step(self) -> bool:
        """Poll running batches, admit and launch what fits.  Returns True if anything happened."""
        busy = False
        still = []
        for h, reqs in self.inflight:
            try:
                fin = self.ex.poll(h)
            except Exception as e:  # a failed batch fails its requests; the server goes on
                self._retire(reqs, failed=f"{type(e).__name__}: {e}")
                busy = True
                continue
            if fin:
                res = self.ex.collect(h)
                if res:
                    self.results.update(res)
                self._retire(reqs)
                busy = True
            else:
                still.append((h, reqs))
        self.inflight = still
        batch = self._admit()
        if batch:
            self.max_used = max(self.max_used, self.adm.used)
            try:
                h = self.ex.launch(batch)
                self.launches += 1
                self.inflight.append((h, batch))
                self.max_inflight = max(self.max_inflight, len(self.inflight))
            except Exception as e:
                self._retire(batch, failed=f"{type(e).__name__}: {e}")
            busy = True
        return busy

    def run(self, arrivals: List[Request], idle_sleep: float = 20e-6, timeout: float = 600.0) -> List[Request]:
        """Feed requests at their arrival times (server clock starts now) until all are finished."""
        self.t0 = time.perf_counter()
        pending = collections.deque(sorted(arrivals, key=lambda r: r.arrival))
        n = len(pending)
        while len(self.finished) < n:
            t = self.now()
            if t > timeout:
                raise TimeoutError(f"served stream not finished after {timeout} s")
            while pending and pending[0].arrival <= t:
                self.submit(pending.popleft())
            busy = self.step()
            if not busy:
                nxt = pending[0].arrival - self.now() if pending else idle_sleep
                time.sleep(max(0.0, min(idle_sleep, nxt)))
        return self.finished


def latency_report(reqs: List[Request]) -> dict:
    import numpy as np
    done = [r for r in reqs if r.status == "done"]
    lat = np.array([r.latency for r in done]) * 1e3
    if len(done) == 0:
        return {"completed": 0}
    span = max(r.done for r in done) - min(r.arrival for r in done)
    wait = np.array([r.admitted - r.arrival for r in done]) * 1e3
    return {"completed": len(done), "failed": sum(r.status == "failed" for r in reqs),
            "rejected": sum(r.status == "rejected" for r in reqs),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "frames_per_s": len(done) / span if span > 0 else float("nan"),
            "queue_wait_p50_ms": float(np.percentile(wait, 50)), "queue_wait_p99_ms": float(np.percentile(wait, 99)),
            "held_for_hbm": sum(r.held for r in done)}


# ---------------------------------------------------------------- GPU executor

class GpuExecutor:
    """Device state and launches through libshwfs; torch provides memory and streams only."""

    def __init__(self, keep_results: bool = False, keep_images: bool = False):
        import torch

        from gen import configs as G
        from . import shwfs
        self.torch, self.G, self.s = torch, G, shwfs
        self.keep = keep_results or keep_images
        self.keep_images = keep_images
        # instance state lives in pinned host memory once created; making an instance resident again
        # after an eviction is an asynchronous copy, not a regeneration
        self.host = {}
        self.stats = {"created": 0, "restored": 0, "evicted": 0}
        self.streams = {"8m": torch.cuda.Stream(), "39m": torch.cuda.Stream()}
        self.plan8 = shwfs.WfsPlan(G.CFG0)
        self.plan_lgs = shwfs.WfsPlan(G.CFG1, 6, G.launch_positions(G.CFG1, 6))
        self.plan_ngs = shwfs.WfsPlan(G.CFG4_NGS, 3)
        self.dm_plans = [shwfs.DmPlan(800, 4.875e-2, alt, pitch, G.DM_FIELD_RADIUS_ARCSEC, G.DM_COUPLING, G.DM_PATCH)
                         for alt, pitch in G.DMS]
        self.state = {}
        self.n_valid = {"8m": self.plan8.n_valid, "lgs": self.plan_lgs.n_valid, "ngs": self.plan_ngs.n_valid}
        # guide-star directions (arcsec): 6 LGS at 45", 3 NGS at 60"
        self.dirs = ([(45 * math.cos(math.radians(60 * w)), 45 * math.sin(math.radians(60 * w))) for w in range(6)]
                     + [(60 * math.cos(math.radians(120 * j)), 60 * math.sin(math.radians(120 * j)))
                        for j in range(3)])

    def shared_bytes(self) -> int:
        return self.plan8.device_bytes + self.plan_lgs.device_bytes + self.plan_ngs.device_bytes

    def instance_bytes(self, cls: str) -> int:
        if cls == "8m":
            return 512 * 512 * 4
        dm = sum(p.size * p.size * 4 + p.n_act * 4 for p in self.dm_plans)
        return 2048 * 2048 * 4 + dm

    def slot_bytes(self, cls: str) -> int:
        if cls == "8m":
            return 80 * 80 * 4 + 2 * self.n_valid["8m"] * 4
        return 9 * 800 * 800 * 4 + (6 * 2 * self.n_valid["lgs"] + 3 * 2 * self.n_valid["ngs"]) * 4

    def create_instance(self, inst: Instance):
        import numpy as np

        from gen import screens as S
        torch = self.torch
        st = self.streams[inst.cls]
        if inst.iid in self.host:
            # resident again after an eviction: copy the saved state on the class stream (ordered
            # before the work that uses it)
            with torch.cuda.stream(st):
                self.state[inst.iid] = {k: ([h.to("cuda", non_blocking=True) for h in v] if isinstance(v, list)
                                            else v.to("cuda", non_blocking=True))
                                        for k, v in self.host[inst.iid].items()}
            self.stats["restored"] += 1
            return
        if inst.cls == "8m":
            scr = torch.from_numpy(S.screen_opd_m(512, 0.1, seed=inst.seed).astype(np.float32)).pin_memory()
            host = {"screen": scr}
        else:
            scr = torch.from_numpy(S.screen_opd_m(2048, 4.875e-2, seed=inst.seed).astype(np.float32)).pin_memory()
            surfs = []
            with torch.cuda.stream(st):
                for d, p in enumerate(self.dm_plans):
                    c = torch.from_numpy(S.dm_coefficients(p.n_act, inst.seed * 10 + d).astype(np.float32)).cuda()
                    sf = torch.empty((p.size, p.size), device="cuda")
                    p.surface(c, sf, stream=st)
                    surfs.append(sf)
            st.synchronize()
            host = {"screen": scr, "surfaces": [sf.cpu().pin_memory() for sf in surfs]}
        self.host[inst.iid] = host
        with torch.cuda.stream(st):
            self.state[inst.iid] = {k: ([h.to("cuda", non_blocking=True) for h in v] if isinstance(v, list)
                                        else v.to("cuda", non_blocking=True)) for k, v in host.items()}
        self.stats["created"] += 1

    def destroy_instance(self, inst: Instance):
        # only idle instances are evicted: no queued work reads this state any more
        if self.state.pop(inst.iid, None) is not None:
            self.stats["evicted"] += 1

    def _origins_39m(self, frame: int):
        t = frame % (2048 - 800 - 400 + 1)
        scr_o, dm_o = [], []
        for k, (tx, ty) in enumerate(self.dirs):
            scr_o.append((50 * k, 50 * k + t))
            row = []
            for p, (alt, _) in zip(self.dm_plans, self.G.DMS):
                sy = int(math.floor(alt * ty * ARCSEC / 4.875e-2 + 0.5))
                sx = int(math.floor(alt * tx * ARCSEC / 4.875e-2 + 0.5))
                row.append((p.size // 2 - 400 + sy, p.size // 2 - 400 + sx))
            dm_o.append(row)
        return scr_o, dm_o

    def launch(self, batch: List[Request]):
        torch, s = self.torch, self.s
        by_cls = collections.defaultdict(list)
        for r in batch:
            by_cls[self._cls(r)].append(r)
        handle = {"events": [], "slots": {}, "reqs": batch}
        for cls, reqs in by_cls.items():
            # requests of one instance take contiguous staging slots: one residual launch per instance
            reqs = sorted(reqs, key=lambda r: (r.instance, r.frame))
            groups = collections.OrderedDict()
            for k, r in enumerate(reqs):
                groups.setdefault(r.instance, []).append(k)
            st = self.streams[cls]
            with torch.cuda.stream(st):
                if cls == "8m":
                    opd = torch.empty((len(reqs), 1, 80, 80), device="cuda")
                    sl = torch.empty((len(reqs), 1, 2, self.n_valid["8m"]), device="cuda")
                    im = (torch.empty((len(reqs), 1, self.n_valid["8m"], 8, 8), device="cuda")
                          if self.keep_images else None)
                    for iid, ks in groups.items():
                        org = [((reqs[k].frame % (432 * 432)) // 432, reqs[k].frame % 432) for k in ks]
                        s.residual_opd(self.state[iid]["screen"], [], 80, org, [[] for _ in ks],
                                       opd[ks[0]:ks[-1] + 1].view(-1, 80, 80), stream=st)
                    s.measure_batch([(self.plan8, opd[k], sl[k], None if im is None else im[k], self._seed(r), r.frame)
                                     for k, r in enumerate(reqs)], stream=st)
                    handle["slots"][cls] = (reqs, opd, sl, None, im, None)
                else:
                    opd = torch.empty((len(reqs), 9, 800, 800), device="cuda")
                    sl_l = torch.empty((len(reqs), 6, 2, self.n_valid["lgs"]), device="cuda")
                    sl_n = torch.empty((len(reqs), 3, 2, self.n_valid["ngs"]), device="cuda")
                    im_l = im_n = None
                    if self.keep_images:
                        im_l = torch.empty((len(reqs), 6, self.n_valid["lgs"], 16, 16), device="cuda")
                        im_n = torch.empty((len(reqs), 3, self.n_valid["ngs"], 16, 16), device="cuda")
                    for iid, ks in groups.items():
                        stt = self.state[iid]
                        scr_o, dm_o = [], []
                        for k in ks:
                            a_, b_ = self._origins_39m(reqs[k].frame)
                            scr_o += a_
                            dm_o += b_
                        s.residual_opd(stt["screen"], stt["surfaces"], 800, scr_o, dm_o,
                                       opd[ks[0]:ks[-1] + 1].view(-1, 800, 800), stream=st)
                    s.measure_batch([(self.plan_lgs, opd[k, :6], sl_l[k], None if im_l is None else im_l[k],
                                      self._seed(r), r.frame) for k, r in enumerate(reqs)], stream=st)
                    s.measure_batch([(self.plan_ngs, opd[k, 6:], sl_n[k], None if im_n is None else im_n[k],
                                      self._seed(r), r.frame) for k, r in enumerate(reqs)], stream=st)
                    handle["slots"][cls] = (reqs, opd, sl_l, sl_n, im_l, im_n)
                ev = torch.cuda.Event()
                ev.record(st)
                handle["events"].append(ev)
        return handle

    def _cls(self, r):
        return self.cls_of[r.instance]

    def _seed(self, r):
        return 0x5EED0000 + r.instance

    def bind(self, instances: List[Instance]):
        self.cls_of = {i.iid: i.cls for i in instances}

    def poll(self, h) -> bool:
        return all(e.query() for e in h["events"])

    def collect(self, h):
        if not self.keep:
            return None
        out = {}
        for cls, (reqs, _opd, a, b, ia, ib) in h["slots"].items():
            a_h = a.cpu().numpy()
            b_h = b.cpu().numpy() if b is not None else None
            ia_h = ia.cpu().numpy() if ia is not None else None
            ib_h = ib.cpu().numpy() if ib is not None else None
            for k, r in enumerate(reqs):
                res = (a_h[k].copy(), None if b_h is None else b_h[k].copy())
                if self.keep_images:
                    res += (ia_h[k].copy(), None if ib_h is None else ib_h[k].copy())
                out[r.rid] = res
        return out


def make_mix(n_small=8, n_large=4, rate_hz=2000.0, duration_s=1.0, frac_large=0.3, seed=2000):
    """Poisson request stream over the served mix: instances and requests (frames in per-instance order)."""
    import numpy as np

    from gen import screens as S
    instances = [Instance(i, "8m", seed=100 + i) for i in range(n_small)] + \
                [Instance(n_small + j, "39m", seed=200 + j) for j in range(n_large)]
    t = S.poisson_arrivals(rate_hz, duration_s, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    big = rng.uniform(size=len(t)) < frac_large
    which_s = rng.integers(0, n_small, len(t))
    which_l = rng.integers(0, n_large, len(t))
    frames = collections.Counter()
    reqs = []
    for k, (tk, bk) in enumerate(zip(t, big)):
        iid = n_small + int(which_l[k]) if bk else int(which_s[k])
        reqs.append(Request(k, iid, frames[iid], float(tk)))
        frames[iid] += 1
    return instances, reqs
