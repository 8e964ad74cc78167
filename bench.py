#!/usr/bin/env python3
"""Benchmark of the MXE hot path on one MI355X.

A step is one diffusion step of the staggered scheme on the 256,000-site FCC
vacancy system (40^3 periodic cells, 1% vacancies, T = 1000 K, 27-node
quadrature, <= 30 FIRE updates per relaxation): neighbour-list maintenance,
relaxation (pair quadrature, density pass, force/mu pass, FIRE), master-
equation flux, time step and Euler update, all on the GPU.

Prints ONE JSON line. `value` = site-quadrature evaluations per second over the
timed steps (sites x evaluations / wall time), with every input resident in HBM.
The roofline entry reports the dominant kernel against MI355X peak, from HIP
events bracketing its launches on the launch stream during the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "site-quadrature evals/s + master-eq site-steps/s; mixed/batched vs FP64 plain"
PEAK_HBM_GBS = 8000.0
# FP64 vector: 256 CUs x 64 FP64 lanes/clock x 2.4 GHz = 39.3e12 lane-operations/s
# (78.6 TFLOP/s counting a fused multiply-add as two flops).
PEAK_FP64_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic work of one pair quadrature: 27 nodes x 90 FP64 operations (two
# exponentials, square root, reciprocal, taper and ~30 multiply-adds for the
# values, gradients and width derivatives of both radial shapes).
OPS_PER_PAIR = 27 * 90
# Algorithmic HBM bytes of the force/mu gather: each pair's 14 FP64 moments and
# its row entry (neighbour index, pair id) are read from both ends; per site the
# state, embedding terms, FIRE velocity and the six outputs.
BYTES_FORCE_PER_PAIR = 2 * (14 * 8 + 8)
BYTES_FORCE_PER_SITE = 8 + 8 + 1 + 8 * 3 + 8 * 4 + 8 * 6
# The timed runs bracket only the pair kernel with HIP events (every event
# drains the queue); the per-family breakdown comes from this many further
# steps with every family bracketed.
BREAKDOWN_STEPS = 2

# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of
# this bench (--steps 2 --warmup 1 --no-extras --no-cpu-baseline --calib-copy),
# KiB per dispatch averaged over the run's dispatches, scaled by what the same
# counters read for a 1 GiB device copy (FETCH x 2, WRITE x 1). Valid only for
# the kernel sources they were taken on: a different source hash reports null.
COUNTER_SCALE = dict(fetch=2.000, write=1.000)
COUNTERS = dict(
    sources_sha256_16="75dd4a5669ce5013",
    pair=dict(fetch_kib=159583.6, write_kib=1019787.0),
    force=dict(fetch_kib=900776.3, write_kib=13650.1),
    density=dict(fetch_kib=172829.2, write_kib=26951.2),
)
COUNTER_SOURCES = ("paper_1910_01235_amd/csrc/eam.hip", "paper_1910_01235_amd/csrc/mxe_internal.h")


def counter_traffic(family: str):
    """Scaled HBM bytes per launch of a kernel family, or None if the sources changed."""
    import hashlib
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != COUNTERS["sources_sha256_16"] or family not in COUNTERS:
        return None
    c = COUNTERS[family]
    return (COUNTER_SCALE["fetch"] * c["fetch_kib"] + COUNTER_SCALE["write"] * c["write_kib"]) * 1024.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(workload, n_sample: int):
    """The CPU oracle timed on a bounded sample of the same state."""
    import numpy as np

    import oracle as O
    s = workload.systems[0]
    n_sample = min(n_sample, s.n)
    sel = np.arange(n_sample, dtype=np.int32)
    O.lib()
    t0 = time.perf_counter()
    O.evaluate_sites(workload.eam, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, sel)
    dt = time.perf_counter() - t0
    return dict(value=n_sample / dt, unit="site-evals/s", cores=O.num_threads(), kind="oracle",
                sample=f"one evaluation (density pass over the sample and its neighbours, force/mu "
                       f"pass over the sample) of the first {n_sample} of {s.n} sites of the "
                       f"initial state; {dt:.2f} s wall")


def batched_legs(n_requests: int, n_steps: int, seed: int = 4):
    """Many independent systems: one batched plan, one at a time, and served.

    Requests: cubic vacancy or alloy systems, sizes log-uniform in [500, 50,000]
    sites, T in [600, 1200] K. Rates count site-evaluations (sites x
    evaluations) and systems completed per second of wall time."""
    import numpy as np
    import torch

    from paper_1910_01235_amd import lattice as L
    from paper_1910_01235_amd import mxe
    from paper_1910_01235_amd import serve

    systems = L.config4_requests(seed=seed, n_requests=n_requests)
    params = dict(L.DEFAULT_PARAMS)
    n_tot = sum(s.n for s in systems)
    reqs = serve.poisson_requests(systems, n_steps=n_steps, rate=0.0)

    # one at a time: a plan per request, in order (the plain path)
    torch.cuda.synchronize()
    _, one = serve.serve_one_at_a_time(L.DEFAULT_EAM, params, reqs, realtime=False)

    # all requests in one batched plan
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = mxe.Plan(systems, L.DEFAULT_EAM, params)
    st, out, ws = plan.state(systems), plan.out(), plan.workspace()
    plan.run(st, out, ws, n_steps, use_graph=True)
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - t0
    sc = plan.scalars(out)
    evals_b = sc[:, mxe.S_TOTAL_EVALS]
    site_evals = float(sum(s.n * e for s, e in zip(systems, evals_b)))
    status_b = int(np.bitwise_or.reduce(sc[:, mxe.S_STATUS].astype(np.int64)))
    del plan, st, out, ws
    torch.cuda.empty_cache()
    batched = dict(systems_per_s=len(systems) / wall_b, site_evals_per_s=site_evals / wall_b,
                   wall_s=wall_b, status=status_b)

    # served: Poisson arrivals at 0.8 x the batched capacity, continuous batching
    per_site = serve.bytes_per_site(L.DEFAULT_EAM, params)
    caps = serve.pool_capacities(24e9, per_site)
    srv = serve.Server(L.DEFAULT_EAM, params, caps)
    warm = serve.poisson_requests([L.vacancy_bulk(5, 1, 800.0, 0)], n_steps=1, rate=0.0)
    srv.serve(warm, realtime=False)  # records the step graph
    rate = 0.8 * batched["systems_per_s"]
    reqs_p = serve.poisson_requests(systems, n_steps=n_steps, rate=rate, seed=seed)
    res, rejected, st_s = srv.serve(reqs_p, realtime=True)
    served = dict(arrival_rate_per_s=rate, systems_per_s=st_s["systems_per_s"],
                  site_steps_per_s=st_s["site_steps_per_s"], p50_s=st_s["p50_s"], p99_s=st_s["p99_s"],
                  rejected=len(rejected), slots=st_s["slots"], footprint_gb=st_s["footprint_bytes"] / 1e9,
                  status=int(np.bitwise_or.reduce([r.status for r in res])) if res else 0)
    del srv
    torch.cuda.empty_cache()
    return dict(requests=len(systems), sites=n_tot, steps_per_request=n_steps,
                max_relax=params["max_relax"], batched=batched,
                one_at_a_time=dict(systems_per_s=one["systems_per_s"], makespan_s=one["makespan_s"],
                                   p50_s=one["p50_s"], p99_s=one["p99_s"]),
                batched_vs_one_at_a_time=batched["systems_per_s"] / one["systems_per_s"],
                served=served)


def timed_run(plan, st, out, ws, steps, use_graph, profile):
    """profile: False, "pair" (events around the pair kernel only: the timed
    runs) or True (every kernel family: the breakdown runs)."""
    import torch
    plan.profile(profile)
    if profile:
        plan.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(st, out, ws, steps, use_graph=use_graph)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = plan.profile_read() if profile else None
    plan.profile(False)
    sc = plan.scalars(out)[0]
    return wall, sc, prof


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=256000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the graph, FP32 and batched legs")
    ap.add_argument("--batch-requests", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with a 1 GiB device copy (reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1910_01235_amd import lattice as L
    from paper_1910_01235_amd import mxe

    torch.cuda.set_device(0)
    w = L.config1(1)
    s = w.systems[0]
    n = s.n
    n_mobile = int((s.type != L.HOST_FIXED).sum())
    log(f"workload {w.name}: {n} sites, warmup {args.warmup}, steps {args.steps}")

    plan = mxe.Plan([s], w.eam, w.params, precision="fp64")
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, args.warmup, use_graph=True)
    torch.cuda.synchronize()
    log(f"warmup done: status {int(plan.scalars(out)[0, mxe.S_STATUS])}")

    # the timed region brackets only the pair kernel (the roofline's) with events
    wall, sc, prof = timed_run(plan, st, out, ws, args.steps, use_graph=False, profile="pair")
    evals = int(sc[mxe.S_TOTAL_EVALS])
    pair_evals = float(sc[mxe.S_PAIR_EVALS])
    status = int(sc[mxe.S_STATUS])
    value = n * evals / wall
    site_steps = n_mobile * args.steps / wall
    log(f"timed: {wall:.3f} s, {evals} evaluations, status {status}")
    pair_ms, pair_launches = prof["pair"]
    # every family from BREAKDOWN_STEPS more steps with all families bracketed
    _, sc_b, prof_b = timed_run(plan, st, out, ws, BREAKDOWN_STEPS, use_graph=False, profile=True)
    evals_b, pair_evals_b = int(sc_b[mxe.S_TOTAL_EVALS]), float(sc_b[mxe.S_PAIR_EVALS])
    log(f"breakdown: {BREAKDOWN_STEPS} steps, {evals_b} evaluations")

    # roofline of each hot kernel family
    fam = {}
    for k, (ms, cnt) in prof_b.items():
        fam[k] = dict(ms_total=ms, launches=cnt, ms_avg=(ms / cnt if cnt else 0.0))
    pairs_per_launch = pair_evals / max(pair_launches, 1)
    ops = OPS_PER_PAIR * pairs_per_launch
    pair_avg_s = pair_ms / max(pair_launches, 1) / 1e3
    roof_pair = dict(bound="alu", achieved=ops / pair_avg_s / 1e12 if pair_avg_s > 0 else 0.0,
                     peak=PEAK_FP64_TOPS, unit="Tops/s", kernel="k_pair<double>",
                     traffic=counter_traffic("pair"), traffic_unit="B/launch")
    roof_pair["frac"] = roof_pair["achieved"] / roof_pair["peak"]
    evals_per_launch = evals_b / max(fam["force"]["launches"], 1)
    bytes_force = (BYTES_FORCE_PER_PAIR * pair_evals_b / max(evals_b, 1) + BYTES_FORCE_PER_SITE * n) \
        * evals_per_launch
    force_avg_s = fam["force"]["ms_avg"] / 1e3
    roof_force = dict(bound="hbm", achieved=bytes_force / force_avg_s / 1e9 if force_avg_s > 0 else 0.0,
                      peak=PEAK_HBM_GBS, unit="GB/s", kernel="k_force<double> + k_force_fold",
                      traffic=counter_traffic("force"), traffic_unit="B/launch",
                      algorithmic_bytes=bytes_force)
    roof_force["frac"] = roof_force["achieved"] / roof_force["peak"]
    dominant = max(fam, key=lambda k: fam[k]["ms_total"])
    roofline = roof_pair if dominant != "force" else roof_force

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "site-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "sites": n, "vacancies": int((s.x == 0).sum()),
                   "T_K": s.T, "quadrature_nodes": 27, "max_relax": w.params["max_relax"],
                   "precision": "fp64", "launch": "eager; HIP events around the pair kernel"},
        "site_steps_per_s": site_steps,
        "evals_in_timed_steps": evals,
        "list_builds_in_timed_steps": int(sc[mxe.S_REBUILDS]),
        "pairs_per_eval": pair_evals / max(evals, 1),
        "status": status,
        "roofline": roofline,
        "roofline_all": {"pair": roof_pair, "force": roof_force},
        "pair_ms_avg_timed": pair_ms / max(pair_launches, 1),
        "kernel_ms": fam,
        "kernel_ms_from": f"{BREAKDOWN_STEPS} steps after the timed region, every family bracketed",
        "dominant_kernel": dominant,
    }

    if not args.no_extras:
        wall_g, sc_g, _ = timed_run(plan, st, out, ws, args.steps, use_graph=True, profile=False)
        result["graph"] = dict(value=n * int(sc_g[mxe.S_TOTAL_EVALS]) / wall_g,
                               ms_per_step=wall_g / args.steps * 1e3,
                               evals=int(sc_g[mxe.S_TOTAL_EVALS]))
        log(f"graph leg: {wall_g:.3f} s")
        del st, out, ws, plan
        torch.cuda.empty_cache()
        p32 = mxe.Plan([s], w.eam, w.params, precision="fp32")
        st32, out32, ws32 = p32.state([s]), p32.out(), p32.workspace()
        p32.run(st32, out32, ws32, args.warmup, use_graph=True)
        wall_32, sc_32, _ = timed_run(p32, st32, out32, ws32, args.steps, use_graph=False,
                                      profile="pair")
        ev32 = int(sc_32[mxe.S_TOTAL_EVALS])
        _, _, prof32 = timed_run(p32, st32, out32, ws32, BREAKDOWN_STEPS, use_graph=False, profile=True)
        result["fp32_mixed"] = dict(value=n * ev32 / wall_32, ms_per_step=wall_32 / args.steps * 1e3,
                                    evals=ev32, status=int(sc_32[mxe.S_STATUS]),
                                    kernel_ms={k: v[0] for k, v in prof32.items()})
        log(f"fp32 leg: {wall_32:.3f} s")
        del st32, out32, ws32, p32
        torch.cuda.empty_cache()
        # the paper's own degree-3 rule (12 nodes in the pair's 6-D space)
        result["degree3"] = {}
        for prec in ("fp64", "fp32"):
            eam3 = dict(w.eam, quad_rule=1)
            p3 = mxe.Plan([s], eam3, w.params, precision=prec)
            st3, out3, ws3 = p3.state([s]), p3.out(), p3.workspace()
            p3.run(st3, out3, ws3, args.warmup, use_graph=True)
            wall3, sc3, _ = timed_run(p3, st3, out3, ws3, args.steps, use_graph=False, profile="pair")
            ev3 = int(sc3[mxe.S_TOTAL_EVALS])
            _, _, prof3 = timed_run(p3, st3, out3, ws3, BREAKDOWN_STEPS, use_graph=False, profile=True)
            result["degree3"][prec] = dict(
                value=n * ev3 / wall3, ms_per_step=wall3 / args.steps * 1e3, evals=ev3,
                status=int(sc3[mxe.S_STATUS]),
                kernel_ms_avg={k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof3.items()})
            log(f"degree-3 {prec} leg: {wall3:.3f} s")
            del st3, out3, ws3, p3
            torch.cuda.empty_cache()
        # state variants on the same workload: site temperatures, reservoir sites
        result["variants"] = {}
        rng = np.random.default_rng(3)
        for name in ("site_temperature", "reservoirs"):
            pv = mxe.Plan([s], w.eam, w.params, precision="fp64")
            stv, outv, wsv = pv.state([s]), pv.out(), pv.workspace()
            if name == "site_temperature":
                stv.T_site = torch.as_tensor(900.0 + 200.0 * s.q[:, 0] / s.box[0], device="cuda")
            else:
                held = rng.choice(n, n // 100, replace=False)
                res = np.zeros(n, np.int8)
                res[held[: len(held) // 2]] = mxe.RES_FIX_X
                res[held[len(held) // 2:]] = mxe.RES_FIX_MU
                val = np.where(res == mxe.RES_FIX_X, 1.0, -0.85)
                stv.reservoir = torch.as_tensor(res, device="cuda")
                stv.res_value = torch.as_tensor(val, device="cuda")
            pv.run(stv, outv, wsv, args.warmup, use_graph=True)
            wall_v, sc_v, _ = timed_run(pv, stv, outv, wsv, args.steps, use_graph=False, profile="pair")
            evv = int(sc_v[mxe.S_TOTAL_EVALS])
            _, _, prof_v = timed_run(pv, stv, outv, wsv, BREAKDOWN_STEPS, use_graph=False, profile=True)
            result["variants"][name] = dict(
                value=n * evv / wall_v, ms_per_step=wall_v / args.steps * 1e3, evals=evv,
                status=int(sc_v[mxe.S_STATUS]),
                kernel_ms_avg={k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof_v.items()})
            log(f"{name} leg: {wall_v:.3f} s")
            del stv, outv, wsv, pv
            torch.cuda.empty_cache()
        t0 = time.perf_counter()
        result["many_systems"] = batched_legs(args.batch_requests, args.batch_steps)
        log(f"batched/served legs: {time.perf_counter() - t0:.1f} s")

    if args.calib_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        result["calib_copy_bytes"] = a.numel() * 8
    if not args.no_cpu_baseline:
        log("cpu baseline")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
