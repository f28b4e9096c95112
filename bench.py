#!/usr/bin/env python3
"""Benchmark of the PM hot path on one MI355X.

One bench step = one whole pass of the path over one synthetic universe:
Zel'dovich ICs from seeded white noise, n_steps BullFrog PM steps, the final
CIC density and its binned P(k), the loss cotangent (L2 distance to a fixed
observed density), and the adjoint back to dL/dw and dL/dsigma8.
value = particle-steps/s of forward + adjoint = N n_steps K / t(K steps).

Default workload: 512^3 particles, L = 1000 Mpc/h, flat LCDM with BBKS, the
NUFFT force (exponential-of-semicircle width 6 on the 2x upsampled 1024^3
grid, exact i k), 6 BullFrog steps (FP32 bulk, int64 fixed-point spreading).
The PM workloads (TSC/CIC with finite differences) are selectable.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BASE = dict(omega_m=0.31, h=0.68, n_s=0.965, sigma8=0.81, spectrum="bbks", a_start=0.02,
            a_end=1.0, grad_order=4, lap_order=0)
WORKLOADS = {
    "pm_256_512_tsc": dict(BASE, n_p=256, n_g=512, box=500.0, n_steps=10, mak=3, deconvolve=True),
    "pm_128_256_cic": dict(BASE, n_p=128, n_g=256, box=250.0, n_steps=10, mak=2, deconvolve=False),
    "pm_512_1024_tsc": dict(BASE, n_p=512, n_g=1024, box=1000.0, n_steps=6, mak=3, deconvolve=True),
    # NUFFT force: ES width 6 at 2x upsampling (fine grid 1024^3), exact i k
    "nufft_512_1024_es6": dict(BASE, n_p=512, n_g=1024, box=1000.0, n_steps=6, force="nufft", es_width=6,
                               es_beta=13.8, grad_order=0, mak=2, deconvolve=False),
    "nufft_128_256_es6": dict(BASE, n_p=128, n_g=256, box=250.0, n_steps=6, force="nufft", es_width=6,
                              es_beta=13.8, grad_order=0, mak=2, deconvolve=False),
}
HBM_PEAK_GBS = 8000.0


def launch_model(cfg, int64_mass=True):
    """Algorithmic HBM bytes of every timed launch of one bench step (ICs, the
    forward run, density, P(k) and the adjoint of one slot, PM force), per
    kernel class: a list of (launches, bytes per launch).  Minimum traffic:
    every input read once and every output written once; particle arrays FP32
    SoA [3][N] (12 B per particle each), the other meshes FP32 [M], half
    spectra complex64 of n^2 (n/2+1) modes (unpadded).  With int64_mass (the
    path's stated model) every deposit writes the int64 fixed-point mesh
    [M] and the forward R2C reads it; without it (this design) the deposits
    of a force evaluation write the FP32 contrast instead and the R2C reads
    that.  The lattice index of a particle and the tile binning tables are
    the design's overhead, not algorithmic bytes."""
    n, p, K = cfg.n_g, cfg.n_p, cfg.n_steps
    M, N = n ** 3, p ** 3
    mb = 8 if int64_mass else 4        # bytes per cell of the force chain's mass mesh
    Sn, Sp = 8 * n * n * (n // 2 + 1), 8 * p * p * (p // 2 + 1)   # bytes of one half spectrum
    ic_rows = [(4, 4 * N + Sp), (3, Sp + 8 * N), (1, Sp + 4 * N)]
    ic_cols = [(15, 2 * Sp), (1, 4 * Sp)]
    if cfg.force == "nufft":
        # pruned passes: only the modes |m| < n_p/2 per axis survive the
        # truncation, so the rows keep k_z < n_p/2 (Sz), the y passes touch
        # those columns and the kept k_y (Sy, all x), the x passes only the
        # kept (k_y, k_z) lines
        Sz = 8 * n * n * (p // 2)
        Sy = 8 * n * (p - 1) * (p // 2)
        return {
            # force spreads write the FP32 density; the observed field and the
            # P(k) mesh are the int64 fixed-point mesh
            "deposit": [(2 * K, 12 * N + mb * M), (2, 12 * N + 8 * M)],
            "bin": [(K, 40 * N), (K + 3, 16 * N)],
            # R2C of the mass (run, adjoint recompute; P(k) unpruned from the
            # int64 mesh), 3 force C2R per force evaluation plus the adjoint's
            # b_bar, the R2C of the adjoint's spread kernel gradient
            "fft_rows": [(2 * K, mb * M + Sz), (1, 8 * M + Sn), (7 * K, Sz + 4 * M), (K, 4 * M + Sz)] + ic_rows,
            # y forward (mass and the adjoint's gradient spread), x passes
            # (multiplier between forward and inverse x), inverse y
            "fft_cols": [(3 * K, Sz + Sy), (7 * K, 2 * Sy), (7 * K, Sy + Sz), (2, 2 * Sn)] + ic_cols,
            # read X, V and 3 force meshes, write X, V
            "gather_kick": [(K, 48 * N + 12 * M)],
            "adj_kick": [(K, 96 * N + 12 * M)],
            # spread of u . grad phi: read u and X, write the mesh (int64)
            "dipole": [(K, 24 * N + 8 * M)],
            "adj_drift": [(K + 1, 84 * N + 4 * M)],
        }
    return {
        # fixed-point mass assignment: read the positions, write the int64 mesh
        "deposit": [(2 * K, 12 * N + mb * M), (2, 12 * N + 8 * M)],
        # counting sort: read positions, write the sorted index (in the run
        # it also applies the first drift: read V, write the positions)
        "bin": [(K, 40 * N), (K + 3, 16 * N)],
        # z rows: int64 or FP32 mesh -> half spectrum, and back to FP32
        "fft_rows": [(2 * K, mb * M + Sn), (1, 8 * M + Sn), (K, 4 * M + Sn), (3 * K, Sn + 4 * M)] + ic_rows,
        # y / x passes (one with the fused multiplier): read + write the spectrum
        "fft_cols": [(9 * K + 2, 2 * Sn)] + ic_cols,
        # read X, V and phi, write X, V
        "gather_kick": [(K, 48 * N + 4 * M)],
        # read X, V, X_bar, V_bar and phi; write V, X_bar, V_bar and u
        "adj_kick": [(K, 96 * N + 4 * M)],
        # read u and X, write the FP32 mesh cotangent
        "dipole": [(K, 24 * N + 4 * M)],
        # read X, V, X_bar, V_bar and the mesh cotangent; write X, X_bar, V_bar
        "adj_drift": [(K + 1, 84 * N + 4 * M)],
    }


LDS_PEAK_GBS = 256 * 128 * 2.4  # 256 CUs x 128 B/clk x 2.4 GHz (GB/s)


def lds_model(cfg):
    """LDS bytes of the stencil accesses per launch of the ES tile kernels
    (their binding roof): 216 nodes per particle, an int64 add per node in a
    spread, an FP32 read per node and component in a gather.  The window
    fills and write-backs are design overhead.  PM workloads: {}."""
    if cfg.force != "nufft":
        return {}
    N, K = cfg.n_p ** 3, cfg.n_steps
    return {
        "deposit": [(2 * K, 216 * 8 * N), (2, 8 * 8 * N)],
        "gather_kick": [(K, 3 * 216 * 4 * N)],
        "adj_kick": [(K, 3 * 216 * 4 * N)],
        "dipole": [(K, 216 * 8 * N)],
        "adj_drift": [(K, 216 * 4 * N), (1, 8 * 4 * N)],
    }


def source_digest():
    """sha256 over the HIP/C++ sources of the library: HBM counter readings are
    valid only for the kernels they were taken on."""
    import hashlib
    d = os.path.join(ROOT, "paper_2510_05206_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per class and bench step from the committed FETCH_SIZE /
    WRITE_SIZE counter summary of this workload (scaled by a plain copy of
    known size), or None when the summary is missing or the kernels changed
    since it was taken."""
    f = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(f):
        return None
    for line in open(f):
        if line.startswith("<!-- traffic-json:"):
            rec = json.loads(line[len("<!-- traffic-json:"):].rsplit("-->", 1)[0])
            return rec["bytes_per_step"] if rec.get("sources_sha256") == source_digest() else None
    return None


def rooflines(cfg, kt, steps):
    """Per-class HBM roofline: the model's bytes over the class's measured
    time, after checking the model's launch count against the measured one.
    frac uses the stated model (int64 mass meshes); "design" gives the same
    time against this design's own minimum bytes (FP32 contrast)."""
    out = {}
    lmodel = lds_model(cfg)
    dmodel = launch_model(cfg, int64_mass=False)
    for cls, parts in launch_model(cfg).items():
        ms, nl = kt.get(cls, (0.0, 0))
        count = sum(c for c, _ in parts) * steps
        total = sum(c * b for c, b in parts) * steps
        if nl != count or ms <= 0:
            out[cls] = {"error": f"launch count {nl} != model {count}"}
            continue
        gbs = total / (ms * 1e-3) / 1e9
        out[cls] = {"achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "ms_per_step": round(ms / steps, 3), "launches_per_step": count // steps,
                    "avg_launch_us": round(ms / nl * 1e3, 2), "bytes_per_launch": round(total / count)}
        dtot = sum(c * b for c, b in dmodel[cls]) * steps
        if dtot != total:
            dgbs = dtot / (ms * 1e-3) / 1e9
            out[cls]["design"] = {"bytes_per_launch": round(dtot / count), "achieved": round(dgbs, 1),
                                  "frac": round(dgbs / HBM_PEAK_GBS, 4)}
        lparts = lmodel.get(cls)
        if lparts:
            ltot = sum(c * b for c, b in lparts) * steps
            lgbs = ltot / (ms * 1e-3) / 1e9
            out[cls]["lds"] = {"bytes_per_launch": round(ltot / count), "achieved": round(lgbs, 1),
                               "peak": round(LDS_PEAK_GBS, 1), "unit": "GB/s", "frac": round(lgbs / LDS_PEAK_GBS, 4)}
    return out


def stream_copy_gbs(gib=1.0, reps=5):
    """Measured HBM bandwidth of a plain device-to-device copy of `gib` GiB
    (read + write bytes over the median HIP-event time of `reps` copies)."""
    import torch
    src = torch.ones(int(gib * 2 ** 28), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    nbytes = 2 * src.numel() * 4
    del src, dst
    return round(nbytes / (sorted(times)[reps // 2] * 1e-3) / 1e9, 1)


def _oracle_worker(spec, seconds):
    """One worker of the oracle baseline: single-threaded FP64 gradients (one
    forward run plus the store-all reverse pass) of the bounded sample for
    about `seconds`; returns (repetitions, seconds taken)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import adjoint, philox
    from oracle.force import PMConfig
    from oracle.nbody import Problem

    prob = Problem(PMConfig(**spec["pm"]), **spec["prob"])
    w = philox.white_noise(54321, spec["pm"]["n_p"]).astype(np.float64)
    prob.spectrum_fn(), prob.steps()
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        reps = 0
        while reps == 0 or time.perf_counter() - t < seconds:
            adjoint.gradient(prob, w, lambda d: 2.0 * d)
            reps += 1
        return reps, time.perf_counter() - t


def cpu_baseline(cfg, workers=None):
    """The FP64 oracle (untuned) on the same physics at a bounded size, on the
    host's cores: one single-threaded worker process per core (at most 16,
    the CPU share of one GPU), all running at once for ~8 s; the value is the
    sum of the workers' rates."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    if cfg.force == "nufft":
        n_p, n_g, steps = 32, 64, cfg.n_steps
        kw = dict(force="nufft", es_width=cfg.es_width, es_beta=cfg.es_beta)
        what = f"NUFFT ES width {cfg.es_width}, fine grid {n_g}^3"
    else:
        n_p, n_g, steps = 64, 128, 4
        kw = {}
        what = f"{'TSC' if cfg.mak == 3 else 'CIC'} on {n_g}^3, FD{cfg.grad_order}"
    box = cfg.box * n_p / cfg.n_p          # same mass resolution
    spec = {"pm": dict(n_p=n_p, n_g=n_g, box=box, order=cfg.mak, deconvolve=cfg.deconvolve,
                       grad_order=max(cfg.grad_order, 2), lap_order=cfg.lap_order),
            "prob": dict(omega_m=cfg.omega_m, h=cfg.h, n_s=cfg.n_s, sigma8=cfg.sigma8, spectrum=cfg.spectrum,
                         a_start=cfg.a_start, a_end=cfg.a_end, n_steps=steps, **kw)}
    P = workers or max(1, min(16, os.cpu_count() or 1))
    # spawned workers: fresh interpreters that import only numpy and the oracle
    with ProcessPoolExecutor(P, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_worker, [spec] * P, [8.0] * P))
    rate = sum(r * n_p ** 3 * steps / dt for r, dt in res)
    reps = sum(r for r, _ in res)
    return {"value": rate, "unit": "particle-steps/s", "cores": P, "kind": "oracle",
            "sample": f"FP64 numpy oracle, same physics at {n_p}^3 particles ({what}, L={box:g} Mpc/h, BBKS), "
                      f"{steps} BullFrog steps forward + store-all reverse; {P} single-threaded worker processes "
                      f"at once for ~8 s each ({reps} repetitions in all) on a host with {os.cpu_count()} cores; "
                      f"the value is the sum of their rates"}


def serve_bench(n_requests, budget_gb):
    """Mixed-size serving trace.  Capacities first: the whole trace at once
    (saturation) through the sequential method and through continuous
    batching.  Then the same Poisson trace at lambda_1 = 0.7 x the sequential
    capacity (both stable) and at lambda_2 = 0.7 x the batched capacity
    (beyond what the sequential method can serve), each through both."""
    import numpy as np
    import torch

    from paper_2510_05206_amd import serve

    targets = serve.Targets()
    burst = serve.make_trace(n_requests, rate=0.0, seed=2001)
    sb, st_sb = serve.serve_sequential(burst, targets)
    mu_seq = len(sb) / st_sb["makespan_s"]
    bb, st_b = serve.serve_batched(burst, hbm_budget_gb=budget_gb, targets=targets)
    mu_bat = len(bb) / st_b["makespan_s"]
    runs = {}
    same = True
    for name, rate in (("lambda1", 0.7 * mu_seq), ("lambda2", 0.7 * mu_bat)):
        trace = serve.make_trace(n_requests, rate=rate, seed=2000)
        seq, st_seq = serve.serve_sequential(trace, targets)
        bat, st_bat = serve.serve_batched(trace, hbm_budget_gb=budget_gb, targets=targets)
        a = {r.rid: r for r in seq}
        # the same request alone and in the mix gives the same bits
        same &= all((np.array_equal(r.pk, a[r.rid].pk) if r.kind == "pk"
                     else (r.dsigma8 == a[r.rid].dsigma8 and r.dw_bits == a[r.rid].dw_bits)) for r in bat)
        runs[name] = {"rate_rps": round(rate, 3),
                      "sequential": serve.latency_stats(seq, st_seq["makespan_s"], trace),
                      "batched": serve.latency_stats(bat, st_bat["makespan_s"], trace),
                      "mean_occupancy": round(st_bat["mean_occupancy"], 3)}
    torch.cuda.synchronize()
    l1 = runs["lambda1"]
    return {
        "metric": "served requests/s, mixed 32^3-256^3 PM P(k)/gradient trace",
        "value": round(l1["batched"]["throughput_rps"], 3), "unit": "requests/s", "n_gpus": 1,
        "higher_is_better": True, "data": "synthetic Poisson trace (seeded)",
        "config": {"workload": "serving_mix", "requests": n_requests, "rate_rps": l1["rate_rps"],
                   "mix": "N in {32,64,128,256}^3 w .4/.3/.2/.1, sigma8 U[0.6,1], steps U{4..12}, 30% grad",
                   "hbm_budget_gb": budget_gb},
        "serving": {"capacity_sequential_rps": round(mu_seq, 3), "capacity_batched_rps": round(mu_bat, 3),
                    "identical_results": bool(same), "slots": st_b["plan"], **runs,
                    "saturation_host_s": st_b.get("host_s"), "saturation_makespan_s": round(st_b["makespan_s"], 3)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="nufft_512_1024_es6", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="one plain device copy of this size right before the timed steps "
                         "(reference dispatch for HBM byte counters)")
    ap.add_argument("--serve", action="store_true", help="run the mixed-size serving trace instead")
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--hbm-budget-gb", type=float, default=160.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              f"(one process per GPU, each on its own slots, is how it would shard)", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(serve_bench(args.requests, args.hbm_budget_gb)), flush=True)
        return

    import torch

    import paper_2510_05206_amd as P

    torch.cuda.set_device(0)
    d = WORKLOADS[args.workload]
    cfg = P.Config(**d)
    N, M, n_steps = cfg.N, cfg.M, cfg.n_steps
    sim = P.PMSim(cfg, with_adjoint=True)
    # observed density (untimed): the forward of another seed plus 10% noise
    sim.init_ics([54322])
    sim.run()
    dt = sim.density()
    gen = torch.Generator(device="cpu").manual_seed(54323)
    dobs = dt + 0.1 * dt.std() * torch.randn(dt.shape, generator=gen).to(dt.device)
    n_bins = cfg.n_g // 2
    out = {}

    def one_step(i):
        sim.init_ics([54321 + i])
        sim.run()
        delta = sim.density()
        out["pk"] = sim.power_spectrum(n_bins)
        dw, ds = sim.adjoint(2.0 * (delta - dobs))
        out["dw"], out["ds"] = dw, ds

    for i in range(args.warmup):
        one_step(i)
    torch.cuda.synchronize()
    if args.calibrate_copy_gib > 0:
        src = torch.ones(int(args.calibrate_copy_gib * 2 ** 28), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)          # one elementwise read + write of known size
        torch.cuda.synchronize()
        del src, dst
    copy_gbs = stream_copy_gbs()
    if not args.no_kernel_timing:
        sim.profile(True)
        sim.kernel_times()
    t0 = time.perf_counter()
    for i in range(args.steps):
        one_step(args.warmup + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = N * n_steps * args.steps / elapsed

    roof = None
    kt = {}
    if not args.no_kernel_timing:
        kt = sim.kernel_times()
        sim.profile(False)
        if True:
            by_class = rooflines(cfg, kt, args.steps)
            ok = {k: v for k, v in by_class.items() if "achieved" in v}
            dom = max(ok, key=lambda k: ok[k]["ms_per_step"])
            r = ok[dom]
            traffic = measured_traffic(args.workload)
            if traffic is not None:
                traffic = round(traffic[dom] / r["launches_per_step"])
            roof = {"bound": "hbm", "achieved": r["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": r["frac"], "traffic": traffic, "kernel": dom,
                    "stream_copy_gbs": copy_gbs, "frac_of_stream_copy": round(r["achieved"] / copy_gbs, 4),
                    "avg_launch_us": r["avg_launch_us"], "bytes_per_launch": r["bytes_per_launch"],
                    "by_class": by_class}
    assert math.isfinite(float(out["ds"][0]))

    line = {
        "metric": "particle-steps/s fwd+adjoint",
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Philox white noise, BBKS LCDM)",
        "config": {"workload": args.workload, "n_p": cfg.n_p, "n_g": cfg.n_g, "box": cfg.box,
                   "n_steps": n_steps, "mak": cfg.mak, "deconvolve": cfg.deconvolve,
                   "particles": N, "parallelism": "single GPU"},
        "roofline": roof,
        "kernel_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in kt.items()},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
