"""Continuous-batching serving of PM simulation and gradient requests.

A request asks for the binned P(k) of one simulated universe ("pk") or for
the gradient of an L2 density loss with respect to its white noise and sigma8
("grad"), with its own particle count, sigma8, number of BullFrog steps and
seed.  The loop keeps one context per (shape, kind) bucket with B slots
(sized by the HBM budget), each on its own HIP stream:

* forward buckets batch continuously on device-indexed steps: a request that
  arrives while others run is admitted into a free slot (ICs for that slot
  only, its device step index set to 0), and one replay of the bucket's
  captured step graph advances every busy slot by one BullFrog step whatever
  its step index (up to three steps queued ahead of the host loop); a slot
  that finishes is read out and refilled at once;
* gradient buckets run cohorts: the requests waiting at launch time take the
  free slots and run forward, loss cotangent and adjoint together (the
  adjoint integrates its slots backwards as one), and a new cohort is queued
  on the remaining free slots without waiting for earlier cohorts to finish.

Device work is enqueued asynchronously and completion is observed with
events, so buckets overlap on the GPU.  The sequential baseline runs the
same requests one at a time on one-slot contexts.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from .sim import Config, PMSim

MIX_N = (32, 64, 128, 256)
MIX_W = (0.4, 0.3, 0.2, 0.1)


@dataclass
class Request:
    rid: int
    n_p: int
    sigma8: float
    n_steps: int
    seed: int
    kind: str            # "pk" | "grad"
    arrival: float = 0.0


@dataclass
class Result:
    rid: int
    kind: str
    arrival: float
    finished: float
    pk: np.ndarray | None = None
    dsigma8: float | None = None
    dw_norm: float | None = None
    dw_bits: int | None = None       # sum of the FP32 bit patterns of dL/dw (order-free, exact)
    batch: int = 1
    dw: np.ndarray | None = None     # dL/dw itself (kept on request, for tests)

    @property
    def latency(self):
        return self.finished - self.arrival


def shape_config(n_p, batch, max_steps=12):
    """Mass resolution of the 256^3 / 500 Mpc/h workload at every size; CIC,
    mesh 2x the particle grid per dimension."""
    return Config(n_p=n_p, n_g=2 * n_p, box=500.0 * n_p / 256, omega_m=0.31, h=0.68, n_s=0.965,
                  sigma8=0.81, spectrum="bbks", a_start=0.02, a_end=1.0, n_steps=max_steps, mak=2,
                  deconvolve=False, grad_order=4, lap_order=0, batch=batch)


def make_trace(n_requests, rate, seed=2000, grad_frac=0.3):
    """Poisson arrivals at `rate` per second; N from {32,64,128,256}^3 with
    weights .4/.3/.2/.1, sigma8 ~ U[0.6, 1.0], steps ~ U{4..12}, 30% gradients,
    request r seeded 10^6 + r."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        n_p = int(rng.choice(MIX_N, p=MIX_W))
        reqs.append(Request(r, n_p, float(rng.uniform(0.6, 1.0)), int(rng.integers(4, 13)), 10 ** 6 + r,
                            "grad" if rng.uniform() < grad_frac else "pk", t))
    return reqs


class Targets:
    """Observed density per shape for the gradient loss: the forward of a
    fixed seed plus 10% Gaussian noise (computed once, not timed)."""

    def __init__(self):
        self.cache = {}

    def get(self, n_p):
        if n_p not in self.cache:
            sim = PMSim(shape_config(n_p, 1), with_adjoint=False)
            sim.set_slot_params(n_steps=[10], sigma8=[0.81])
            sim.init_ics([54322])
            sim.run()
            d = sim.density()[0]
            gen = torch.Generator(device="cpu").manual_seed(54323 + n_p)
            noise = torch.randn(d.shape, generator=gen).to(d.device)
            self.cache[n_p] = (d + 0.1 * d.std() * noise).contiguous()
            torch.cuda.synchronize()
        return self.cache[n_p]


# ------------------------------------------------------------ batched loop

def _to_host(t):
    """Copy to pinned host memory on the current stream without waiting: the
    copy completes with the next event recorded on that stream (a blocking
    .cpu() would also wait for every other bucket's stream)."""
    h = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    h.copy_(t, non_blocking=True)
    return h


class _PkBucket:
    AHEAD = 3  # steps queued ahead of the host loop

    def __init__(self, n_p, B, stream):
        self.n_p, self.B = n_p, B
        self.stream = stream
        with torch.cuda.stream(self.stream):
            self.sim = PMSim(shape_config(n_p, B), with_adjoint=False)
        self.req = [None] * B
        self.k = [-1] * B          # host mirror of the device step index
        self.steps = [12] * B
        self.sig = [0.81] * B
        self.queue = deque()
        self.pending = []          # (event, finished slots and their requests, pk tensors)
        self.occupancy = []

    def busy(self):
        return any(r is not None for r in self.req)

    def admit(self):
        free = [b for b in range(self.B) if self.req[b] is None]
        new = []
        while free and self.queue:
            b = free.pop(0)
            r = self.queue.popleft()
            self.req[b] = r
            self.steps[b], self.sig[b] = r.n_steps, r.sigma8
            new.append(b)
        if not new:
            return
        with torch.cuda.stream(self.stream):
            self.sim.set_slot_params(n_steps=self.steps, sigma8=self.sig)
            self.sim.set_active(new)
            self.sim.init_ics([self.req[b].seed if b in new else 0 for b in range(self.B)])
            self.sim.set_active(None)
            self.sim.set_step_index([0 if b in new else -2 for b in range(self.B)])
        for b in new:
            self.k[b] = 0

    def advance(self):
        """Enqueue one device step (every slot with steps left), then the
        read-out of the slots that just finished."""
        if sum(1 for p in self.pending if not p[0].query()) >= self.AHEAD:
            return  # at most AHEAD steps in flight per bucket
        running = [b for b in range(self.B) if self.k[b] >= 0]
        if not running:
            return
        with torch.cuda.stream(self.stream):
            self.sim.step_device()
            self.occupancy.append(len(running) / self.B)
            done = []
            for b in running:
                self.k[b] = self.k[b] + 1 if self.k[b] + 1 < self.steps[b] else -1
                if self.k[b] < 0:
                    done.append(b)
            pk = None
            if done:
                self.sim.set_active(done)
                pk = _to_host(self.sim.power_spectrum(self.n_p)[1])
                self.sim.set_active(None)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        # the slots are handed back once their P(k) has been read
        self.pending.append((ev, [(b, self.req[b]) for b in done], pk))
        for b in done:
            self.req[b] = _Reserved

    def collect(self, now_fn, results):
        keep = []
        for ev, done, pk in self.pending:
            if not ev.query():
                keep.append((ev, done, pk))
                continue
            if done:
                p = pk.numpy()         # pinned copy, complete with the event
                t = now_fn()
                for b, r in done:
                    results.append(Result(r.rid, "pk", r.arrival, t, pk=p[b].copy(), batch=self.B))
                    self.req[b] = None
        self.pending = keep


class _ReservedSlot:
    """Marks a slot whose request finished but whose read-out is in flight."""


_Reserved = _ReservedSlot()


class _GradBucket:
    def __init__(self, n_p, B, targets, stream, keep_arrays=False):
        self.n_p, self.B = n_p, B
        self.stream = stream
        with torch.cuda.stream(self.stream):
            self.sim = PMSim(shape_config(n_p, B), with_adjoint=True)
        self.queue = deque()
        self.cohorts = []          # (event, requests, slots, ds, dw norms, dw bit sums, dw)
        self.free = list(range(B))
        self.steps = [12] * B
        self.sig = [0.81] * B
        self.target = targets.get(n_p)
        self.keep_arrays = keep_arrays
        self.occupancy = []

    def busy(self):
        return bool(self.cohorts)

    def launch(self):
        """Queue a cohort of waiting requests on the free slots (behind any
        cohort still in flight on this bucket's stream)."""
        if not self.free or not self.queue:
            return
        n = min(len(self.free), len(self.queue))
        reqs = [self.queue.popleft() for _ in range(n)]
        slots = [self.free.pop(0) for _ in range(n)]
        seeds = [0] * self.B
        for b, r in zip(slots, reqs):
            self.steps[b], self.sig[b], seeds[b] = r.n_steps, r.sigma8, r.seed
        with torch.cuda.stream(self.stream):
            self.sim.set_slot_params(n_steps=self.steps, sigma8=self.sig)
            self.sim.set_active(slots)
            self.sim.init_ics(seeds)
            # the forward on device-indexed steps: one graph replay per step
            # for the whole cohort (earlier cohorts' indices are back at -1)
            self.sim.set_step_index([0 if b in slots else -2 for b in range(self.B)])
            for _ in range(max(r.n_steps for r in reqs)):
                self.sim.step_device()
            delta = self.sim.density()
            g = 2.0 * (delta - self.target.unsqueeze(0))
            dw, ds = self.sim.adjoint(g)
            # the slot index goes up asynchronously from pinned memory (a
            # pageable copy would wait for everything queued on this stream)
            idx_h = torch.tensor(slots, dtype=torch.long).pin_memory()
            idx = idx_h.to(dw.device, non_blocking=True)
            dws = dw.index_select(0, idx)
            dwn = dws.double().norm(dim=1)
            dwb = dws.view(torch.int32).long().sum(dim=1)
            dss = ds.index_select(0, idx)
            self.sim.set_active(None)
            dss, dwn, dwb = _to_host(dss), _to_host(dwn), _to_host(dwb)
            dws = _to_host(dws) if self.keep_arrays else None
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.occupancy.append(n / self.B)
        self.cohorts.append((ev, reqs, slots, dss, dwn, dwb, dws, idx_h))

    def collect(self, now_fn, results):
        keep = []
        for co in self.cohorts:
            ev, reqs, slots, ds, dwn, dwb, dws, _ = co
            if not ev.query():
                keep.append(co)
                continue
            ds, dwn, dwb = ds.numpy(), dwn.numpy(), dwb.numpy()   # pinned copies, complete with the event
            dw = dws.numpy() if dws is not None else None
            t = now_fn()
            for q, r in enumerate(reqs):
                res = Result(r.rid, "grad", r.arrival, t, dsigma8=float(ds[q]), dw_norm=float(dwn[q]),
                             dw_bits=int(dwb[q]), batch=self.B)
                if dw is not None:
                    res.dw = dw[q].copy()
                results.append(res)
            self.free.extend(slots)
        self.cohorts = keep


def workspace_bytes(cfg, with_adjoint):
    """Device bytes of one context (the admission figure of the C ABI)."""
    import ctypes as C

    from . import _lib
    lib = _lib.load()
    ctx = C.c_void_p()
    ccfg = cfg.to_c()
    _lib.check(lib.pm_create(C.byref(ccfg), C.byref(ctx)), None, "pm_create")
    try:
        return int(lib.pm_workspace_bytes(ctx, int(bool(with_adjoint))))
    finally:
        lib.pm_destroy(ctx)


def plan_batches(hbm_budget_bytes, max_batch=16, sizes=MIX_N, weights=MIX_W):
    """Slots per bucket so that all buckets together fit the HBM budget
    (admission by footprint): each shape gets a share of the budget in
    proportion to its weight in the mix, 70% for P(k) and 30% for gradient
    buckets."""
    out = {}
    for kind, adj, frac in (("pk", False, 0.7), ("grad", True, 0.3)):
        for n, wgt in zip(sizes, weights):
            per_slot = workspace_bytes(shape_config(n, 1), adj)
            budget = hbm_budget_bytes * wgt * frac
            out[(kind, n)] = int(max(1, min(max_batch, budget // per_slot)))
    return out


def serve_batched(requests, hbm_budget_gb=160.0, max_batch=16, targets=None, keep_arrays=False):
    """Run the trace with continuous batching; returns results and stats."""
    targets = targets or Targets()
    sizes = sorted({r.n_p for r in requests})
    plan = plan_batches(hbm_budget_gb * 1e9, max_batch, MIX_N, MIX_W)
    pk_b = {n: _PkBucket(n, plan[("pk", n)], torch.cuda.Stream()) for n in sizes}
    gr_b = {n: _GradBucket(n, plan[("grad", n)], targets, torch.cuda.Stream(), keep_arrays) for n in sizes}
    torch.cuda.synchronize()
    reqs = deque(sorted(requests, key=lambda r: r.arrival))
    results = []
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    total = len(reqs)
    host = {}          # host seconds spent per bucket and phase (enqueueing, not GPU time)

    def timed(key, fn, *a):
        s0 = time.perf_counter()
        fn(*a)
        host[key] = host.get(key, 0.0) + time.perf_counter() - s0

    while len(results) < total:
        t = now()
        while reqs and reqs[0].arrival <= t:
            r = reqs.popleft()
            (pk_b if r.kind == "pk" else gr_b)[r.n_p].queue.append(r)
        for n, b in pk_b.items():
            timed(f"pk_{n}_collect", b.collect, now, results)
            timed(f"pk_{n}_admit", b.admit)
            timed(f"pk_{n}_advance", b.advance)
        for n, b in gr_b.items():
            timed(f"grad_{n}_collect", b.collect, now, results)
            timed(f"grad_{n}_launch", b.launch)
        if reqs and not any(b.busy() or b.queue for b in list(pk_b.values()) + list(gr_b.values())):
            time.sleep(max(0.0, min(0.002, reqs[0].arrival - now())))
    makespan = now()
    occ = [o for b in pk_b.values() for o in b.occupancy] + [o for b in gr_b.values() for o in b.occupancy]
    stats = {"makespan_s": makespan, "plan": {f"{k}_{n}": v for (k, n), v in plan.items()},
             "mean_occupancy": float(np.mean(occ)) if occ else 0.0,
             "host_s": {k: round(v, 4) for k, v in sorted(host.items(), key=lambda kv: -kv[1]) if v > 1e-3}}
    return results, stats


def serve_sequential(requests, targets=None, keep_arrays=False):
    """The plain method: one request at a time, in arrival order, one-slot
    contexts (built once per shape and kind, not timed)."""
    targets = targets or Targets()
    sims = {}
    for n in sorted({r.n_p for r in requests}):
        sims[("pk", n)] = PMSim(shape_config(n, 1), with_adjoint=False)
        sims[("grad", n)] = PMSim(shape_config(n, 1), with_adjoint=True)
        targets.get(n)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    service = []
    for r in sorted(requests, key=lambda q: q.arrival):
        while now() < r.arrival:
            time.sleep(min(0.002, r.arrival - now()))
        s = now()
        sim = sims[(r.kind, r.n_p)]
        sim.set_slot_params(n_steps=[r.n_steps], sigma8=[r.sigma8])
        sim.init_ics([r.seed])
        sim.run()
        if r.kind == "pk":
            p = sim.power_spectrum(r.n_p)[1].cpu().numpy()[0]
            results.append(Result(r.rid, "pk", r.arrival, now(), pk=p.copy()))
        else:
            delta = sim.density()
            dw, ds = sim.adjoint(2.0 * (delta - targets.get(r.n_p).unsqueeze(0)))
            dwn = float(dw.double().norm())
            dwb = int(dw.view(torch.int32).long().sum())
            res = Result(r.rid, "grad", r.arrival, now(), dsigma8=float(ds.cpu()[0]), dw_norm=dwn, dw_bits=dwb)
            if keep_arrays:
                res.dw = dw[0].cpu().numpy().copy()
            results.append(res)
        service.append(now() - s)
    return results, {"makespan_s": now(), "mean_service_s": float(np.mean(service))}


def latency_stats(results, makespan, requests=None):
    lat = np.array([r.latency for r in results])
    out = {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
           "mean_ms": float(lat.mean() * 1e3), "throughput_rps": len(results) / makespan,
           "completed": len(results)}
    if requests is not None:  # per (kind, size) class
        size = {q.rid: q.n_p for q in requests}
        by = {}
        for r in results:
            by.setdefault(f"{r.kind}_{size[r.rid]}", []).append(r.latency)
        out["by_class"] = {k: {"n": len(v), "p50_ms": float(np.percentile(v, 50) * 1e3),
                               "p99_ms": float(np.percentile(v, 99) * 1e3)} for k, v in sorted(by.items())}
    return out
