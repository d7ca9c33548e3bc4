"""Throughput benchmark of the EC-PIC step on one MI355X.

Workload: the large argon discharge (0.3 m gap, 2048-cell refined grid with
max/min cell ratio 8, 32 M electrons + 32 M Ar+, 400 V at 13.56 MHz, 20 mTorr,
dt = T_RF/1000, FP32 particle state with FP64 Poisson and diagnostics, cell
sort every 20 steps), synthetic Maxwellian load from seed 3.

One "step" is one pass of the whole hot path: field solve, gather + push +
absorption + secondary emission + collisions + deposit of x^{k+1} for every
particle, and the periodic cell sort.  Throughput = sum over the timed steps
of the live particles at step start / wall time, with the state resident in
HBM.  Prints one JSON line.

Beside it: the FP64-form GPU path on the same workload and number of steps, the
roofline of the dominant kernel (fused particle pass) from HIP-event
durations over the timed region, and the plain FP64 CPU oracle timed on a
bounded sample of the same workload on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published peak
B_ALG = {1: 32.0, 0: 48.0}     # algorithmic bytes per particle-step (FP32 state, FP64)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_particle_kernel_large_traffic.txt")
KERNEL_SOURCES = ["paper_2308_13092_amd/csrc/kernels_particles.hip",
                  "paper_2308_13092_amd/csrc/device.h"]


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source has changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t


def run_gpu(cfg, steps, warmup, autotune=False):
    import torch
    from paper_2308_13092_amd import Context
    ctx = Context([cfg])
    if autotune:
        from paper_2308_13092_amd.autotune import autotune as tune
        chosen, table = tune(ctx)
        for setting, sec in table:
            print(f"[autotune] {setting}: {sec * 1e3:.4f} ms/step", file=sys.stderr, flush=True)
        print(f"[autotune] chosen {chosen}", file=sys.stderr, flush=True)
    ctx.step(warmup)
    torch.cuda.synchronize()
    d0 = ctx.diagnostics()
    ctx.kernel_times(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = ctx.kernel_times(False)
    d1 = ctx.diagnostics()
    ps = int(d1["particle_steps"] - d0["particle_steps"])
    el = t1 - t0
    out = dict(value=ps / el, ms_per_step=1e3 * el / steps, particle_steps=ps, kt=kt,
               live=[int(v) for v in d1["n_live"]], status=int(d1["status"]),
               tuning=ctx.tuning(), sorts_in_window=int(kt["sort_launches"]),
               nu_max=[float(v) for v in d1["nu_max"]])
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


def run_rebalanced(n_per_species, steps, warmup, every=1000, settle=3):
    """The large discharge with particle rebalancing: a few passes at the start
    bring the cell counts near the target (the narrowest cells' initial
    count), then the run rebalances every ``every`` steps inside the timed
    window as well."""
    import torch
    from paper_2308_13092_amd import Context, configs
    cfg = configs.large_rebalanced(n_per_species=n_per_species, every=every)
    ctx = Context([cfg])
    live0 = int(sum(ctx.diagnostics()["n_live"]))
    pass_ms = []
    for _ in range(settle):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.rebalance()
        torch.cuda.synchronize()
        pass_ms.append(1e3 * (time.perf_counter() - t0))
    live1 = int(sum(ctx.diagnostics()["n_live"]))
    ctx.step(warmup)
    torch.cuda.synchronize()
    d0 = ctx.diagnostics()
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d1 = ctx.diagnostics()
    ps = int(d1["particle_steps"] - d0["particle_steps"])
    out = dict(value=ps / el, unit="particle-steps/s", ms_per_step=1e3 * el / steps, steps=steps,
               target_ppc=int(cfg["rebalance_ppc"]), every=every,
               passes_in_window=(int(d0["step"]) + steps) // every - int(d0["step"]) // every,
               live_initial=live0, live_after_settling=live1, live_end=int(sum(d1["n_live"])),
               pass_ms=[round(v, 2) for v in pass_ms],
               merges=[int(v) for v in d1["merges"]], splits=[int(v) for v in d1["splits"]],
               status=int(d1["status"]))
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return out


def run_sweep(steps, warmup, n_inst=256):
    """Workload 4: the batched sweep of independent discharges, all advanced by
    the same graph-replayed steps."""
    import torch
    from paper_2308_13092_amd import Context, configs
    cfgs = configs.sweep(n_inst)
    t0 = time.perf_counter()
    ctx = Context(cfgs)
    init_s = time.perf_counter() - t0
    ctx.step(warmup)
    torch.cuda.synchronize()
    ps0 = sum(int(ctx.diagnostics(i)["particle_steps"]) for i in range(n_inst))
    t0 = time.perf_counter()
    ctx.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ps1 = sum(int(ctx.diagnostics(i)["particle_steps"]) for i in range(n_inst))
    live = sum(int(sum(ctx.diagnostics(i)["n_live"])) for i in range(n_inst))
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    return dict(value=(ps1 - ps0) / el, unit="particle-steps/s", instances=n_inst, steps=steps,
                ms_per_step=1e3 * el / steps, live_particles=live, init_s=round(init_s, 2),
                config="256 discharges from seed 13092: 64-1024 uniform cells, 5e4-2e6 particles "
                       "(log-uniform), 100-500 V, 10-100 mTorr, dt = T_RF/(400-1000), FP32 state")


def run_serving(n_req, scale, cycles, rate, slots):
    """Workload 5 on a shortened trace: Poisson arrivals served with continuous
    batching; p50 / p99 latency beside throughput."""
    import torch
    from paper_2308_13092_amd import configs
    from paper_2308_13092_amd.serve import GpuBackend, Server, summarise
    trace = configs.stream(n=n_req, rate=rate, scale=scale, cycles=cycles)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    be = GpuBackend(n_slots=slots, pool_bytes=budget, precision=1)
    srv = Server(be, n_slots=slots)
    t0 = time.perf_counter()
    reqs = srv.run(trace)
    wall = time.perf_counter() - t0
    be.close()
    del be
    torch.cuda.empty_cache()
    out = summarise(reqs, wall)
    out.update(unit_latency="s", slots=slots, pool_bytes=budget, device_steps=srv.device_steps,
               trace=(f"{n_req} requests, Poisson arrivals at {rate}/s (seed 13093), 64-2048 cells, "
                      f"{scale:g} x (1e5-8e6) particles, {cycles[0]}-{cycles[1]} RF cycles each, "
                      f"FP32 state; shortened from the 256-request, 50-500-cycle stream"))
    return out


def run_serving_matched(n_req, rho, capacity, slots=256, seed=13093):
    """Workload 5 at its stated request sizes (64-2048 cells, 1e5-8e6
    particles, 50-500 RF cycles, dt = T_RF/(400-1000)) with the Poisson
    arrival rate scaled from the stated 20/s down to a load-matched one: the
    offered particle-steps per second are rho x the capacity measured for the
    batched sweep in the same run.  Only the first n_req requests of the
    seeded trace are served (the trace's length bounds the run, not its
    request sizes)."""
    import torch
    from paper_2308_13092_amd import configs
    from paper_2308_13092_amd.serve import GpuBackend, Server, summarise
    unit = configs.stream(n=n_req, rate=1.0, master_seed=seed)
    work = [2 * c["n_per_species"] * steps for _, c, steps in unit]
    mean_work = sum(work) / len(work)
    rate = rho * capacity / mean_work
    trace = configs.stream(n=n_req, rate=rate, master_seed=seed)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    be = GpuBackend(n_slots=slots, pool_bytes=budget, precision=1)
    srv = Server(be, n_slots=slots)
    t0 = time.perf_counter()
    reqs = srv.run(trace)
    wall = time.perf_counter() - t0
    be.close()
    del be
    torch.cuda.empty_cache()
    out = summarise(reqs, wall)
    out.update(unit_latency="s", slots=slots, pool_bytes=budget, device_steps=srv.device_steps,
               rate_per_s=rate, offered_load=rho, capacity_used=capacity,
               mean_request_particle_steps=mean_work,
               trace=(f"first {n_req} requests of the seeded stream (seed {seed}): 64-2048 cells, "
                      f"1e5-8e6 particles (log-uniform), 100-500 V, 10-100 mTorr, 50-500 RF cycles, "
                      f"dt = T_RF/(400-1000), FP32 state, capacity 8x the initial particles; "
                      f"arrivals Poisson at {rate:.4g}/s instead of "
                      f"20/s, so that the offered load is {rho} x the measured sweep capacity "
                      f"({capacity:.4g} particle-steps/s); request sizes as stated"))
    return out


def run_small_workloads():
    """Workloads 1 and 2 (cache-resident sizes; the HBM roofline does not apply):
    wall-clock particle-steps/s of their full runs, graph-replayed."""
    import torch
    from paper_2308_13092_amd import Context, configs
    out = {}

    def timed(cfg, steps):
        ctx = Context([cfg])
        ctx.step(20)
        torch.cuda.synchronize()
        d0 = ctx.diagnostics(0)["particle_steps"]
        t0 = time.perf_counter()
        ctx.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ps = ctx.diagnostics(0)["particle_steps"] - d0
        ctx.close()
        return dict(value=ps / el, ms_per_step=1e3 * el / steps, steps=steps)

    for g, name in ((0, "ec"), (1, "mc")):
        out[f"small_fp64_{name}"] = timed(configs.small(gather=g, precision=0), configs.SMALL_STEPS)
    for prec, name in ((0, "fp64"), (1, "fp32")):
        out[f"resolved_512_{name}"] = timed(configs.resolved(precision=prec), configs.RESOLVED_STEPS)
    out["resolved_64_ec_fp32"] = timed(configs.resolved(precision=1, n_cells=64), configs.RESOLVED_STEPS)
    out["note"] = ("small: 128 cells, 12800 + 12800 particles, dt = T_RF/400, 2000 steps; resolved: 512 "
                   "(or 64) cells, 262144 + 262144 particles, dt = T_RF/800, 16000 steps")
    return out


def cpu_baseline(n_per_species=2_000_000, seconds=12.0, min_steps=3):
    """The oracle as it stands, on one host core, stepped until ``seconds``
    of CPU work have elapsed (at least ``min_steps`` steps)."""
    from oracle.sim import Sim
    from paper_2308_13092_amd import configs
    cfg = configs.large(n_per_species=n_per_species)
    sim = Sim(cfg)
    t0 = time.perf_counter()
    ps = 0
    steps = 0
    while steps < min_steps or time.perf_counter() - t0 < seconds:
        ps += sim.sp[0].n + sim.sp[1].n
        sim.step()
        steps += 1
    el = time.perf_counter() - t0
    return dict(value=ps / el, unit="particle-steps/s", cores=1, kind="oracle",
                sample=(f"NumPy oracle (FP64 arithmetic, FP32-state contract), single thread: the large "
                        f"workload's grid, drive and density with {n_per_species} e- + {n_per_species} Ar+ "
                        f"(weights scaled), {steps} steps after the initial load ({el:.1f} s)"))


def _oracle_rate(cfg, max_steps, seconds):
    """Particle-steps/s of the oracle on one discharge, stepped up to
    max_steps or until `seconds` have elapsed (at least 3 steps)."""
    os.environ["OMP_NUM_THREADS"] = "1"
    from oracle.sim import Sim
    sim = Sim(cfg)
    t0 = time.perf_counter()
    ps = 0
    steps = 0
    while steps < max_steps and (steps < 3 or time.perf_counter() - t0 < seconds):
        ps += sum(sp.n for sp in sim.sp)
        sim.step()
        steps += 1
    el = time.perf_counter() - t0
    return dict(value=ps / el, steps=steps, seconds=round(el, 2))


def _sweep_member(i, seconds):
    from paper_2308_13092_amd import configs
    return _oracle_rate(configs.sweep(256)[i], 2000, seconds)


def cpu_baseline_workloads(seconds=5.0, workers=8, members=8):
    """The oracle on the other workloads (host cores of this machine): the
    small discharge (EC and MC, FP64) and the resolved one (FP32 state) on
    one core each, and the batched sweep as a pool of `workers` processes
    over its first `members` discharges (its aggregate is the sum of the
    concurrent members' rates)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    from paper_2308_13092_amd import configs
    out = {}
    for g, name in ((0, "ec"), (1, "mc")):
        r = _oracle_rate(configs.small(gather=g, precision=0), configs.SMALL_STEPS, seconds)
        out[f"small_fp64_{name}"] = dict(r, unit="particle-steps/s", cores=1, kind="oracle")
    r = _oracle_rate(configs.resolved(precision=1), configs.RESOLVED_STEPS, seconds)
    out["resolved_512_fp32"] = dict(r, unit="particle-steps/s", cores=1, kind="oracle")
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        rs = list(ex.map(_sweep_member, range(members), [seconds] * members))
    out["sweep"] = dict(value=sum(r["value"] for r in rs), unit="particle-steps/s", cores=workers,
                        kind="oracle", members=members,
                        sample=f"the first {members} discharges of the sweep, one process each, "
                               f"each stepped for about {seconds:g} s")
    out["note"] = ("steps run up to the workload's own count or about %g s each; rates are per "
                   "wall second on the stated cores" % seconds)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--fp64-steps", type=int, default=0, help="0: as many as --steps")
    ap.add_argument("--particles", type=int, default=32_000_000, help="per species")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-rebalance", action="store_true")
    ap.add_argument("--sweep-steps", type=int, default=2000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests of the load-matched served stream")
    ap.add_argument("--no-small", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}). Across GPUs the "
              f"discharge instances would be split between processes, one per GPU, with no "
              f"exchange between them; the benchmark measures one GPU.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2308_13092_amd import configs
    torch.cuda.set_device(0)

    cfg32 = configs.large(n_per_species=a.particles, precision=1)
    r32 = run_gpu(cfg32, a.steps, a.warmup, autotune=a.autotune)
    print(f"[bench] fp32-state: {r32['value']:.4g} p-s/s, {r32['ms_per_step']:.3f} ms/step, "
          f"live {r32['live']}", file=sys.stderr, flush=True)
    kt = r32["kt"]
    # The streaming kernel runs once per step; its HIP events bracket a sample
    # of those launches (every 4th step).
    avg_ms = kt["particle_ms"] / max(kt["particle_launches"], 1)
    per_launch = r32["particle_steps"] / a.steps
    achieved = B_ALG[1] * per_launch / (avg_ms * 1e-3) / 1e9
    # The whole step (field, streaming pass, drain, the share of the sort) at
    # the same algorithmic bytes per particle-step.
    step_achieved = B_ALG[1] * r32["value"] / 1e9
    tr = measured_traffic()
    traffic = None if tr is None else tr["bytes_per_launch"]
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic,
                    kernel=f"k_particles<F32, M_FUSED, {r32['tuning']['block']}>", avg_launch_ms=round(avg_ms, 4),
                    particles_per_launch=round(per_launch, 1), bytes_per_particle_step=B_ALG[1],
                    step_achieved=round(step_achieved, 1), step_frac=round(step_achieved / HBM_PEAK_GBS, 4),
                    kernel_frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic_gbs=(None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9, 1)),
                    traffic_frac=(None if traffic is None else round(traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)),
                    field_ms_per_launch=round(kt["field_ms"] / max(kt["field_launches"], 1), 4),
                    drain_ms_per_launch=round(kt["drain_ms"] / max(kt["drain_launches"], 1), 4),
                    sort_ms_per_launch=round(kt["sort_ms"] / max(kt["sort_launches"], 1), 4),
                    sorts_in_window=r32["sorts_in_window"])

    fp64 = None
    if not a.no_fp64:
        cfg64 = configs.large(n_per_species=a.particles, precision=0)
        steps64 = a.fp64_steps if a.fp64_steps > 0 else a.steps
        r64 = run_gpu(cfg64, steps64, a.warmup)
        kt64 = r64["kt"]
        avg64 = kt64["particle_ms"] / max(kt64["particle_launches"], 1)
        k64 = B_ALG[0] * (r64["particle_steps"] / steps64) / (avg64 * 1e-3) / 1e9
        s64 = B_ALG[0] * r64["value"] / 1e9
        fp64 = dict(value=r64["value"], ms_per_step=r64["ms_per_step"], steps=steps64,
                    sorts_in_window=r64["sorts_in_window"], fp32_speedup=r32["value"] / r64["value"],
                    roofline=dict(bound="hbm", bytes_per_particle_step=B_ALG[0],
                                  kernel="k_particles<F64, M_FUSED, 1024>", avg_launch_ms=round(avg64, 4),
                                  achieved=round(k64, 1), frac=round(k64 / HBM_PEAK_GBS, 4),
                                  step_achieved=round(s64, 1), step_frac=round(s64 / HBM_PEAK_GBS, 4),
                                  drain_ms_per_launch=round(kt64["drain_ms"] / max(kt64["drain_launches"], 1), 4),
                                  sort_ms_per_launch=round(kt64["sort_ms"] / max(kt64["sort_launches"], 1), 4)))
        print(f"[bench] fp64: {r64['value']:.4g} p-s/s, kernel {avg64:.4f} ms", file=sys.stderr, flush=True)

    rebal = None
    if not a.no_rebalance:
        rebal = run_rebalanced(a.particles, a.steps, a.warmup)
        rebal["step_speedup_vs_off"] = round(r32["ms_per_step"] / rebal["ms_per_step"], 3)
        print(f"[bench] rebalanced: {rebal['ms_per_step']:.3f} ms/step ({rebal['step_speedup_vs_off']}x "
              f"faster per step), live {rebal['live_initial']} -> {rebal['live_end']}, "
              f"passes {rebal['pass_ms']} ms", file=sys.stderr, flush=True)

    sweep = None
    if not a.no_sweep:
        sweep = run_sweep(a.sweep_steps, 100)
        print(f"[bench] sweep: {sweep['value']:.4g} p-s/s", file=sys.stderr, flush=True)
    serving = None
    if not a.no_serve:
        capacity = sweep["value"] if sweep else 1.0e11
        serving = run_serving_matched(a.serve_requests, 0.7, capacity)
        print(f"[bench] serving (load-matched, {a.serve_requests} requests at {serving['rate_per_s']:.3g}/s): "
              f"p50 {serving['p50_s']:.3f} s, p99 {serving['p99_s']:.3f} s, "
              f"{serving['throughput']:.4g} p-s/s", file=sys.stderr, flush=True)
        smoke = run_serving(64, 0.1, (5, 20), 20.0, 256)
        serving["smoke"] = dict(p50_s=smoke["p50_s"], p99_s=smoke["p99_s"], throughput=smoke["throughput"],
                                trace="smoke only: " + smoke["trace"])

    small = None
    if not a.no_small:
        small = run_small_workloads()
        print("[bench] small/resolved: " + ", ".join(f"{k} {v['value']:.3g}" for k, v in small.items()
                                                    if isinstance(v, dict)), file=sys.stderr, flush=True)

    cpu = None if a.no_cpu else cpu_baseline()
    cpu_more = None if a.no_cpu else cpu_baseline_workloads()
    line = {
        "metric": "particle-steps/sec at 1 MI355X, FP32-state vs FP64 plain; p50/p99 sweep latency",
        "value": r32["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"large argon RF-CCP: 0.3 m gap, 2048-cell refined grid (ratio 8), "
                                f"{a.particles} e- + {a.particles} Ar+, 400 V 13.56 MHz, 20 mTorr, "
                                f"dt=T_RF/1000, FP32 state, sort every 20"),
                   "particles": 2 * a.particles, "cells": 2048, "state": "fp32",
                   "tuning": r32["tuning"], "nu_max": r32["nu_max"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_workloads": cpu_more,
        "fp64_plain": fp64,
        "rebalanced": rebal,
        "batched_sweep": sweep,
        "serving": serving,
        "small_workloads": small,
        "status": r32["status"],
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
