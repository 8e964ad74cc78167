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
# Algorithmic work of one pair quadrature: 27 nodes x 77 FP64 operations (one
# exponential u and three multiplies for the two shapes' exponentials u^4 and
# u^3, which the synthetic potential's exponent ratios allow; square root,
# reciprocal, taper and ~30 multiply-adds for the values, gradients and width
# derivatives of both radial shapes). Two exponentials would make it 90.
OPS_PER_PAIR = 27 * 77
# Algorithmic HBM bytes of the force/mu gather: each pair's 14 FP64 moments and
# its row entry (neighbour index, pair id) are read from both ends; per site the
# state, embedding terms, FIRE velocity and the six outputs.
BYTES_FORCE_PER_PAIR = 2 * (14 * 8 + 8)
BYTES_FORCE_PER_SITE = 8 + 8 + 1 + 8 * 3 + 8 * 4 + 8 * 6
# The same gather priced with each unordered pair's 14 FP64 moments read once
# (the moment stream's own size): the gather reads each block from both ends,
# so against this count it can reach at most about half of HBM peak.
BYTES_FORCE_ONCE_PER_PAIR = 14 * 8
# Algorithmic HBM bytes of the density gather: each pair's (<f>, f0) and row entry
# read from both ends and the neighbour's emission; per site its row count, x,
# type and the five outputs (rho_bar, rho0, G, A~, B~) plus the packed record.
BYTES_DENSITY_PER_PAIR = 2 * (16 + 8 + 8)
BYTES_DENSITY_PER_SITE = 4 + 1 + 8 + 8 + 8 * 5 + 64
# The timed runs bracket only the pair kernel with HIP events (every event
# drains the queue); the per-family breakdown comes from this many further
# steps with every family bracketed.
BREAKDOWN_STEPS = 2

# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of
# this bench (--steps 2 --warmup 1 --no-extras --no-cpu-baseline --calib-copy
# --shapes gather_lanes=8,force_lanes=16,pair_block=256,pair_split=2,gather_stride=26),
# KiB per dispatch averaged over the run's dispatches, scaled by what the same
# counters read for a 1 GiB device copy (FETCH x 2, WRITE x 1). Valid only for
# the kernel sources they were taken on: a different source hash reports null.
COUNTER_SCALE = dict(fetch=2.000, write=1.000)
COUNTERS = dict(
    sources_sha256_16="2ff4811c22563528",
    pair=dict(fetch_kib=130086.8, write_kib=1019787.0),
    force=dict(fetch_kib=903744.1, write_kib=14186.7),
    density=dict(fetch_kib=137313.9, write_kib=27112.3),
)
COUNTER_SOURCES = ("paper_1910_01235_amd/csrc/eam.hip", "paper_1910_01235_amd/csrc/mxe_internal.h")


def counter_traffic(family: str):
    """Scaled HBM bytes per launch of a kernel family, or None if the sources changed."""
    if _sources_hash() != COUNTERS["sources_sha256_16"] or family not in COUNTERS:
        return None
    c = COUNTERS[family]
    return (COUNTER_SCALE["fetch"] * c["fetch_kib"] + COUNTER_SCALE["write"] * c["write_kib"]) * 1024.0


# VALU counters of the pair kernel per dispatch (summed over every shader
# engine), from two rocprofv3 --pmc runs of this bench (the HBM counters'
# options without --calib-copy). SQ_INSTS_* count wave instructions;
# VALUBusy and VALUUtilization are rocprofv3's derived metrics (percent).
# Valid only for the sources they were taken on.
VALU_COUNTERS = dict(
    sources_sha256_16="2ff4811c22563528",
    pair=dict(SQ_INSTS_VALU=209732141.5, SQ_INSTS_VALU_FMA_F64=90076895.5,
              SQ_INSTS_VALU_MUL_F64=39560002.8, SQ_INSTS_VALU_ADD_F64=9895188.5,
              SQ_INSTS_VALU_TRANS_F64=3241630.5, SQ_INSTS_VALU_FLOPS_FP64=232852358.8,
              VALUBusy=85.53, VALUUtilization=85.24),
)


def _sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def valu_counters(pair_avg_s: float):
    """Measured VALU use of the pair kernel (counters) against this run's kernel
    time, or None if the counters were taken on other sources."""
    c = VALU_COUNTERS["pair"]
    if not c or VALU_COUNTERS["sources_sha256_16"] != _sources_hash() or pair_avg_s <= 0:
        return None
    lane_ops = c["SQ_INSTS_VALU"] * 64.0
    f64 = (c["SQ_INSTS_VALU_FMA_F64"] + c["SQ_INSTS_VALU_MUL_F64"] + c["SQ_INSTS_VALU_ADD_F64"] +
           c["SQ_INSTS_VALU_TRANS_F64"]) * 64.0
    flops = c["SQ_INSTS_VALU_FLOPS_FP64"] * 64.0
    return dict(VALUBusy_pct=c["VALUBusy"], VALUUtilization_pct=c.get("VALUUtilization"),
                fp64_tflops=flops / pair_avg_s / 1e12, fp64_flops_frac=flops / pair_avg_s / 78.6e12,
                valu_lane_ops_per_s=lane_ops / pair_avg_s,
                valu_issue_frac=lane_ops / pair_avg_s / (PEAK_FP64_TOPS * 1e12),
                fp64_lane_ops_per_s=f64 / pair_avg_s,
                fp64_issue_frac=f64 / pair_avg_s / (PEAK_FP64_TOPS * 1e12),
                fp64_share_of_valu=f64 / lane_ops, source="rocprofv3 --pmc, per dispatch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload, n_sample: int, n_single: int, c0_oracle_s=None, gpu=None):
    """The CPU oracle timed on bounded samples of the same states (about 15 s of
    CPU work on a 16-thread host). A sampled evaluation still searches the
    neighbours of the whole system, so samples are whole systems where the
    rate is the point:
    * `value`: one evaluation of the first n_sample sites of the 256k-site
      workload with OpenMP on every host thread (median of 3 repeats);
    * `single_thread`: the first n_single sites on one thread;
    * `per_eval`: one evaluation of every site of the slab and nanowire
      workloads on every host thread;
    * `master_step`: the kinetic law's rates over all 256k sites (bonds built
      beforehand, untimed), median of 3;
    * `extrapolated`: full-run times from these rates and the GPU runs'
      evaluation counts (labelled as extrapolated: not run)."""
    import numpy as np

    import oracle as O
    from paper_1910_01235_amd import lattice as L
    O.lib()
    cores = O.num_threads()

    def eval_rate(w, n, repeats=3):
        s = w.systems[0]
        sel = np.arange(min(n, s.n), dtype=np.int32)
        dts = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            O.evaluate_sites(w.eam, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, sel)
            dts.append(time.perf_counter() - t0)
        return len(sel), float(np.median(dts))

    s = workload.systems[0]
    n_all, dt_all = eval_rate(workload, n_sample)
    O.set_num_threads(1)
    try:
        n_one, dt_one = eval_rate(workload, n_single, repeats=1)
    finally:
        O.set_num_threads(cores)
    out = dict(value=n_all / dt_all, unit="site-evals/s", cores=cores, kind="oracle",
               sample=f"one evaluation (density pass over the sample and its neighbours, force/mu "
                      f"pass over the sample) of the first {n_all} of {s.n} sites of the "
                      f"initial state; median {dt_all:.2f} s wall of 3 repeats on {cores} threads",
               cpu_model=cpu_model(), nproc=os.cpu_count(),
               single_thread=dict(value=n_one / dt_one, unit="site-evals/s", cores=1,
                                  sample=f"first {n_one} sites, {dt_one:.2f} s wall"))
    per_eval = {workload.name: dict(value=n_all / dt_all, unit="site-evals/s", sites=n_all)}
    for w2 in (L.config2(2), L.config3(3)):
        n2, dt2 = eval_rate(w2, w2.systems[0].n, repeats=1)
        per_eval[w2.name] = dict(value=n2 / dt2, unit="site-evals/s", sites=n2)
    out["per_eval"] = per_eval
    # the kinetic law over every site of the 256k-site state (mu = 0: the same work)
    p = workload.params
    nb, bl = O.bonds(s.box, s.periodic, s.q, s.type, p["r_bond"])
    mu = np.zeros(s.n)
    dts = []
    for _ in range(3):
        t0 = time.perf_counter()
        O.master_rates(p, s.box, s.periodic, s.T, s.x, s.type, mu, nb, bl)
        dts.append(time.perf_counter() - t0)
    n_mob = int((s.type != L.HOST_FIXED).sum())
    out["master_step"] = dict(value=n_mob / float(np.median(dts)), unit="site-steps/s",
                              sample=f"rates and time step of all {n_mob} mobile sites, median of 3")
    # full runs, extrapolated: evaluations per step as the GPU runs measured them
    ext = {}
    gpu = gpu or {}
    full = gpu.get("full_runs", {})
    for name, n_sites, n_steps, leg in ((workload.name, s.n, workload.n_steps, gpu),
                                        ("c2_alloy_slab_131k", 131072, 500, gpu.get("c2_alloy_slab_131k")),
                                        ("c3_nanowire_256k", 256410, 300, gpu.get("c3_nanowire_256k"))):
        leg = full.get(name, leg)  # the whole run's evaluation count where it was run
        if not leg or name not in per_eval:
            continue
        ev = leg.get("evals", leg.get("evals_in_timed_steps"))
        ev_per_step = ev / leg["steps"] if ev and leg.get("steps") else None
        if ev_per_step is None:
            continue
        t = n_steps * ev_per_step * n_sites / per_eval[name]["value"]
        ext[name] = dict(seconds=t, steps=n_steps, evals_per_step=ev_per_step,
                         note="extrapolated: steps x evaluations per step (GPU run, the whole run "
                              "where it was timed) x sites / the oracle's all-thread rate; not run")
    srv = gpu.get("serving")
    if srv:
        site_evals = srv["batched"]["site_evals_per_s"] * srv["batched"]["wall_s"]
        ext["serving_256_requests"] = dict(
            seconds=site_evals / per_eval[workload.name]["value"],
            note="extrapolated: the batched run's site-evaluations / the oracle's all-thread rate "
                 "on the 256k-site state; not run")
    out["extrapolated"] = ext
    if c0_oracle_s is not None:
        out["c0_full_run_s"] = c0_oracle_s
        out["c0_full_run_cores"] = cores
    return out


def sampled_errors(workload, plan, st, out, ws, precision, n_sample=64, seed=0):
    """One evaluation at the current GPU state, compared with the oracle on
    sampled sites (normwise relative errors, the tests' floors)."""
    import numpy as np
    import torch

    import oracle as O
    s = workload.systems[0]
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    q = torch.stack([st.qx, st.qy, st.qz], 1).cpu().numpy()
    sg, x = st.sigma.cpu().numpy(), st.x.cpu().numpy()
    rng = np.random.default_rng(seed)
    sel = np.sort(rng.choice(s.n, min(n_sample, s.n), replace=False)).astype(np.int32)
    eam = dict(workload.eam, quad_rule=int(plan.params.quad_rule))
    o = O.evaluate_sites(eam, s.box, s.periodic, s.T, q, sg, x, s.type, sel)
    f = torch.stack([out.fx, out.fy, out.fz, out.fsigma], 1).cpu().numpy()[sel]

    def rel(a, b, floor):
        return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))
    # FP32 moments round each pair's force terms (about 1 eV/A in the first
    # shell) to 6e-8 relative; a relaxed site's net force is what is left after
    # they cancel, so the FP32 force error is measured against that scale
    f_floor = 1e-2 if precision == "fp64" else 1.0
    return dict(sites=len(sel), force=rel(f, o["force"], f_floor), force_floor_eV_A=f_floor,
                force_floor_1e_2=rel(f, o["force"], 1e-2), force_max=float(np.abs(o["force"]).max()),
                mu=rel(out.mu.cpu().numpy()[sel], o["mu"], 1e-2),
                rho_bar=rel(out.rho_bar.cpu().numpy()[sel], o["rho_bar"], 1.0),
                e_site=rel(out.e_site.cpu().numpy()[sel], o["e_site"], 1e-2),
                bar=1e-10 if precision == "fp64" else 1e-5)


RELAX_CHUNK_BATCHED = 4   # relaxation chunk of the batched plan and the server pool
RELAX_CHUNK_SINGLE = 2    # and of single-system plans (one-at-a-time requests, full runs)
ADVANCE_ITERS = 8         # iterations per call of the iteration-level server


def serving_sweep(n_requests: int, n_steps: int, rate_factors, seed: int = 4,
                  budget_gb: float = 24.0, before_rates=(0.25, 1.0)):
    """The serving workload: independent systems run as one batched plan, one at
    a time, and served with continuous batching at Poisson arrival rates given as
    multiples of the batched capacity.

    Requests: cubic vacancy or alloy systems, sizes log-uniform in [500, 50,000]
    sites, T in [600, 1200] K, each for n_steps diffusion steps of <= 50 FIRE
    updates. Latency = completion - arrival. The one-at-a-time path is measured
    once (every request alone, back to back); its latencies under each arrival
    stream follow from the measured service times of a first-come-first-served
    single server.

    Two schedules: relaxations that end once every system of the plan has
    converged (relax_chunk > 0), and the fixed sequence of max_relax + 1
    iterations per relaxation (`fixed_sequence`, at the same absolute arrival
    rates for before_rates). Both schedules use the same launch shapes: tuned
    on the batch for the batched runs, per size octave for the one-at-a-time
    runs, and on eight requests over the size range for the server. The server runs at the
    iteration level (free-running steps, `served`) and, for before_rates, at
    the step level (`served_step_level`: one diffusion step of every resident
    system per call)."""
    import numpy as np
    import torch

    from paper_1910_01235_amd import autotune
    from paper_1910_01235_amd import lattice as L
    from paper_1910_01235_amd import mxe
    from paper_1910_01235_amd import serve

    systems = L.config4_requests(seed=seed, n_requests=n_requests)
    n_tot = sum(s.n for s in systems)
    base = dict(L.DEFAULT_PARAMS)
    # launch shapes from the project's autotuner, on this batch, and per size octave
    params, tuned = autotune.tuned_params(systems, L.DEFAULT_EAM, base, cache=None, reps=2)
    shapes = {k: tuned[k] for k in autotune.SHAPES}
    log(f"serving: {len(systems)} requests, {n_tot} sites, tuned shapes {shapes}")
    cache = autotune.Cache(path="")
    single = {}
    for s in systems:
        p1, _ = autotune.tuned_params([s], L.DEFAULT_EAM, dict(base, relax_chunk=RELAX_CHUNK_SINGLE),
                                      cache=cache, reps=3)
        single[id(s)] = p1
    octaves = {k: {kk: v[kk] for kk in autotune.SHAPES} for k, v in sorted(cache.data.items())}
    log(f"serving: shapes per size octave {octaves}")
    # the server's pool mostly holds a few systems at a time: its shapes are
    # tuned on eight requests spread over the size range
    sample = sorted(systems, key=lambda t: t.n)[::len(systems) // 8][:8]
    params_pool, tuned_pool = autotune.tuned_params(sample, L.DEFAULT_EAM, base, cache=None, reps=2)
    shapes_pool = {k: tuned_pool[k] for k in autotune.SHAPES}
    log(f"serving: pool shapes {shapes_pool}")

    def batched(p, free=False, runs=2):
        """All requests in one plan: lockstep steps (mxe_run) or free-running
        steps (mxe_advance, each system stepping as soon as it has relaxed).
        Each run times the whole job from plan creation on; the faster of
        `runs` runs is reported (an occasional free-running run has taken
        about a second longer than the same job run again), with every
        run's wall time."""
        walls, xs = [], []
        for _ in range(runs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = mxe.Plan(systems, L.DEFAULT_EAM, p)
            st, out, ws = plan.state(systems), plan.out(), plan.workspace()
            if free:
                plan.set_resume(True)
                for k in range(len(systems)):
                    plan.set_steps(k, n_steps)
                plan.advance(st, out, ws, 1 << 30, use_graph=True)
            else:
                plan.run(st, out, ws, n_steps, use_graph=True)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            sc = plan.scalars(out)
            ev = sc[:, mxe.S_TOTAL_EVALS]
            status = int(np.bitwise_or.reduce(sc[:, mxe.S_STATUS].astype(np.int64)))
            xs.append([st.x[plan.offsets[k]:plan.offsets[k + 1]].cpu().numpy() for k in range(len(systems))])
            del plan, st, out, ws
            torch.cuda.empty_cache()
        # the runs are deterministic: each should give the same x
        same = all(all(np.array_equal(a, b) for a, b in zip(xs[0], xr)) for xr in xs[1:])
        wall = min(walls)
        return dict(systems_per_s=len(systems) / wall,
                    site_evals_per_s=float(sum(s.n * e for s, e in zip(systems, ev))) / wall,
                    site_steps_per_s=n_tot * n_steps / wall, wall_s=wall, wall_s_runs=walls,
                    runs_x_bitwise_equal=bool(same),
                    evals_per_system_step=float(ev.mean() / n_steps), status=status), xs[0]

    def one_at_a_time(p, params_for, tag):
        reqs0 = serve.poisson_requests(systems, n_steps=n_steps, rate=0.0)
        res, st1 = serve.serve_one_at_a_time(
            L.DEFAULT_EAM, p, reqs0, realtime=False, params_for=params_for,
            progress=lambda k: log(f"serving: one at a time ({tag}), {k} done") if k % 128 == 0 else None)
        log(f"serving: one at a time ({tag}) {st1['makespan_s']:.1f} s")
        service = {r.rid: r.completed - r.admitted for r in res}
        return dict(systems_per_s=st1["systems_per_s"], makespan_s=st1["makespan_s"],
                    p50_s=st1["p50_s"], p99_s=st1["p99_s"], arrivals="all at t = 0"), service, res

    def fcfs(reqs, service):
        """Latencies of a first-come-first-served single server with these service times."""
        c, lat = 0.0, []
        for r in sorted(reqs, key=lambda r: (r.arrival, r.rid)):
            c = max(c, r.arrival) + service[r.rid]
            lat.append(c - r.arrival)
        lat = np.array(lat)
        return dict(p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    systems_per_s=len(lat) / c)

    def served(p, rates, service, tag, iteration_level=False):
        per_site = serve.bytes_per_site(L.DEFAULT_EAM, p)
        caps = serve.pool_capacities(budget_gb * 1e9, per_site)
        srv = serve.Server(L.DEFAULT_EAM, p, caps, iteration_level=iteration_level,
                           advance_iters=ADVANCE_ITERS)
        warm = serve.poisson_requests([L.vacancy_bulk(5, 1, 800.0, 0)], n_steps=1, rate=0.0)
        srv.serve(warm, realtime=False)  # records the step graphs
        rows = []
        for f, rate in rates:
            reqs = serve.poisson_requests(systems, n_steps=n_steps, rate=rate, seed=seed)
            res, rejected, st_s = srv.serve(
                reqs, realtime=True,
                progress=lambda k: log(f"serving ({tag}): rate {f}, {k} done") if k % 128 == 0 else None)
            rows.append(dict(
                rate_factor=f, arrival_rate_per_s=rate, systems_per_s=st_s["systems_per_s"],
                site_steps_per_s=st_s["site_steps_per_s"], p50_s=st_s["p50_s"], p99_s=st_s["p99_s"],
                makespan_s=st_s["makespan_s"], gpu_steps=st_s["gpu_steps"], rejected=len(rejected),
                status=int(np.bitwise_or.reduce([r.status for r in res])) if res else 0,
                one_at_a_time=fcfs(reqs, service)))
            log(f"serving ({tag}): rate {f} x capacity: {st_s['systems_per_s']:.1f} systems/s, "
                f"p50 {st_s['p50_s']:.2f} s, p99 {st_s['p99_s']:.2f} s")
        fp = srv.footprint_bytes / 1e9
        del srv
        torch.cuda.empty_cache()
        return rows, len(caps), fp

    # early exit (the product's schedule)
    p_b = dict(params, relax_chunk=RELAX_CHUNK_BATCHED)
    bat, x_b = batched(p_b, free=True)
    cap = bat["systems_per_s"]
    log(f"serving: batched (free-running steps) {bat['wall_s']:.1f} s, {cap:.1f} systems/s "
        f"(runs: {', '.join(f'{w:.2f}' for w in bat['wall_s_runs'])} s)")
    bat_l, x_l = batched(p_b)
    log(f"serving: batched (lockstep) {bat_l['wall_s']:.1f} s "
        f"(runs: {', '.join(f'{w:.2f}' for w in bat_l['wall_s_runs'])} s)")
    one, service, res1 = one_at_a_time(params, lambda s: single[id(s)], "early exit")
    p_pool = dict(params_pool, relax_chunk=RELAX_CHUNK_BATCHED)
    srv_rows, n_slots, fp = served(p_pool, [(f, f * cap) for f in rate_factors], service,
                                   "iteration level", iteration_level=True)
    srv_step, _, _ = served(p_pool, [(f, f * cap) for f in before_rates], service, "step level")
    # fixed sequence, same absolute arrival rates
    bat0, x_b0 = batched(params)
    log(f"serving: batched, fixed sequence {bat0['wall_s']:.1f} s "
        f"(runs: {', '.join(f'{w:.2f}' for w in bat0['wall_s_runs'])} s)")
    one0, service0, res0 = one_at_a_time(params, lambda s: dict(single[id(s)], relax_chunk=0),
                                         "fixed sequence")
    srv0, _, _ = served(dict(params_pool, relax_chunk=0), [(f, f * cap) for f in before_rates],
                        service0, "fixed sequence")
    # each pair of runs (batched free-running, lockstep and fixed sequence; one
    # at a time early exit and fixed sequence) has the same launch shapes and
    # differs only in the schedule
    same = all(np.array_equal(a, b) and np.array_equal(a, c) for a, b, c in zip(x_b, x_b0, x_l))
    dx = max(float(np.abs(a.x - b.x).max()) for a, b in zip(sorted(res1, key=lambda r: r.rid),
                                                            sorted(res0, key=lambda r: r.rid)))
    return dict(requests=len(systems), sites=n_tot, steps_per_request=n_steps,
                max_relax=params["max_relax"], shapes=shapes, shapes_one_at_a_time=octaves,
                shapes_server=shapes_pool,
                relax_chunk=dict(batched=RELAX_CHUNK_BATCHED, served=RELAX_CHUNK_BATCHED,
                                 one_at_a_time=RELAX_CHUNK_SINGLE),
                batched=bat, batched_lockstep=bat_l, one_at_a_time=one,
                batched_vs_one_at_a_time=cap / one["systems_per_s"],
                served=srv_rows, server="iteration level: free-running steps, "
                f"calls of {ADVANCE_ITERS} iterations", served_step_level=srv_step,
                slots=n_slots, footprint_gb=fp,
                fixed_sequence=dict(batched=bat0, one_at_a_time=one0, served=srv0,
                                    batched_x_bitwise_equal_all_schedules=bool(same),
                                    one_at_a_time_max_abs_dx=dx))


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


def tuned(w, precision, params=None, quad_rule=0):
    """The workload's parameters with the autotuner's launch shapes (tuned on this
    GPU for this precision and rule, or read from the tuner's cache) and the
    shapes chosen."""
    from paper_1910_01235_amd import autotune
    p, hit = autotune.tuned_params(w.systems, dict(w.eam, quad_rule=quad_rule), params or w.params,
                                   precision=precision, cache=autotune.Cache(), reps=3)
    return p, {k: hit[k] for k in autotune.SHAPES}


def fullsize_leg(w, precision, steps, warmup, quad_rule=0, params=None, late=0):
    """A large workload at its full size: `warmup` untimed and `steps` timed
    diffusion steps (eager, HIP events around the pair kernel), a breakdown of
    every kernel family over one more step, and errors against the oracle on
    sampled sites of an evaluation at the final state. params: the workload's
    parameters with launch shapes (default: tuned here). late > 0: after `late`
    more untimed steps, `steps` are timed again (`late_window`: the rate once
    the first steps' relaxation, which moves sites most, is over)."""
    import torch

    from paper_1910_01235_amd import mxe
    s = w.systems[0]
    eam = dict(w.eam, quad_rule=quad_rule)
    if params is None:
        params, shapes = tuned(w, precision, quad_rule=quad_rule)
    else:
        from paper_1910_01235_amd import autotune
        shapes = {k: params.get(k) for k in autotune.SHAPES}
    plan = mxe.Plan([s], eam, params, precision=precision)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, warmup, use_graph=True)
    wall, sc, prof = timed_run(plan, st, out, ws, steps, use_graph=False, profile="pair")
    ev = int(sc[mxe.S_TOTAL_EVALS])
    _, _, prof_b = timed_run(plan, st, out, ws, 1, use_graph=False, profile=True)
    n_mobile = int((s.type != 3).sum())
    res = dict(workload=w.name, sites=s.n, precision=precision, launch_shapes=shapes,
               value=s.n * ev / wall,
               unit="site-evals/s", site_steps_per_s=n_mobile * steps / wall,
               ms_per_step=wall / steps * 1e3, steps=steps, evals=ev,
               pairs_per_eval=float(sc[mxe.S_PAIR_EVALS]) / max(ev, 1),
               list_builds=int(sc[mxe.S_REBUILDS]), status=int(sc[mxe.S_STATUS]),
               pair_ms_avg=prof["pair"][0] / max(prof["pair"][1], 1),
               kernel_ms_avg={k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof_b.items()})
    if late > 0:
        plan.run(st, out, ws, late, use_graph=True)
        wall_l, sc_l, _ = timed_run(plan, st, out, ws, steps, use_graph=False, profile="pair")
        ev_l = int(sc_l[mxe.S_TOTAL_EVALS])
        res["late_window"] = dict(after_steps=warmup + steps + 1 + late, steps=steps,
                                  value=s.n * ev_l / wall_l, ms_per_step=wall_l / steps * 1e3,
                                  evals=ev_l, list_builds=int(sc_l[mxe.S_REBUILDS]),
                                  status=int(sc_l[mxe.S_STATUS]))
    res["error_vs_oracle"] = sampled_errors(w, plan, st, out, ws, precision)
    del st, out, ws, plan
    torch.cuda.empty_cache()
    return res


def full_run_leg(w, precision, params=None):
    """A workload's whole configured run (all its diffusion steps) as one call
    of graph replays: the end-to-end wall time, with the state uploaded first
    (not timed). Relaxations run in chunks of RELAX_CHUNK_SINGLE lean
    iterations and end once the system has converged (bitwise the fixed
    sequence's results; the alloy slab's relaxations converge within 30
    updates from about step 200)."""
    import torch

    from paper_1910_01235_amd import mxe
    s = w.systems[0]
    if params is None:
        params, shapes = tuned(w, precision)
    else:
        from paper_1910_01235_amd import autotune
        shapes = {k: params.get(k) for k in autotune.SHAPES}
    params = dict(params, relax_chunk=RELAX_CHUNK_SINGLE)
    plan = mxe.Plan([s], w.eam, params, precision=precision)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    wall, sc, _ = timed_run(plan, st, out, ws, w.n_steps, use_graph=True, profile=False)
    ev = int(sc[mxe.S_TOTAL_EVALS])
    n_mobile = int((s.type != 3).sum())
    res = dict(workload=w.name, sites=s.n, precision=precision, steps=w.n_steps, launch_shapes=shapes,
               wall_s=wall, evals=ev, value=s.n * ev / wall, unit="site-evals/s",
               site_steps_per_s=n_mobile * w.n_steps / wall, list_builds=int(sc[mxe.S_REBUILDS]),
               simulated_time_s=float(sc[mxe.S_TIME]), status=int(sc[mxe.S_STATUS]),
               launch=f"one call, graph replays; relaxations in chunks of {RELAX_CHUNK_SINGLE} "
                      "iterations ending once converged")
    del st, out, ws, plan
    torch.cuda.empty_cache()
    return res


def c0_leg():
    """The plain-method workload end to end: 256 sites, 20 diffusion steps of up
    to 50 FIRE updates, graph replays, against the oracle's run. Relaxations end
    once the system has converged (chunks of RELAX_CHUNK_SINGLE iterations, launch
    shapes tuned on the workload); the fixed sequence of 51 iterations per
    relaxation is timed beside it."""
    import numpy as np
    import torch

    import oracle as O
    from paper_1910_01235_amd import lattice as L
    from paper_1910_01235_amd import mxe
    w = L.config0(0)
    s = w.systems[0]
    p_fast, shapes = tuned(w, "fp64", dict(w.params, relax_chunk=RELAX_CHUNK_SINGLE))

    def one(params):
        plan = mxe.Plan([s], w.eam, params)
        st, out, ws = plan.state([s]), plan.out(), plan.workspace()
        plan.run(st, out, ws, 1, use_graph=True)  # records the graphs on these buffers
        torch.cuda.synchronize()
        st0 = plan.state([s])  # back to the initial state, same buffers
        for name in ("qx", "qy", "qz", "sigma", "x"):
            getattr(st, name).copy_(getattr(st0, name))
        out.scalars.zero_()
        wall, sc, _ = timed_run(plan, st, out, ws, w.n_steps, use_graph=True, profile=False)
        return plan, st, out, wall, sc

    wall_fixed = one(w.params)[3]
    plan, st, out, wall, sc = one(p_fast)
    ev = int(sc[mxe.S_TOTAL_EVALS])
    t0 = time.perf_counter()
    r = O.run(w.eam, w.params, s.box, s.periodic, s.T, w.n_steps, s.q, s.sigma, s.x, s.type)
    t_or = time.perf_counter() - t0
    x = st.x.cpu().numpy()
    q = torch.stack([st.qx, st.qy, st.qz], 1).cpu().numpy()
    dq = q - r["q"]
    dq -= np.array(s.box) * np.round(dq / np.array(s.box))
    err = dict(dx=float(np.abs((x - s.x) - (r["x"] - s.x)).max() / np.abs(r["x"] - s.x).max()),
               q_abs=float(np.abs(dq).max()),
               mu=float(np.abs(out.mu.cpu().numpy() - r["mu"]).max() / np.abs(r["mu"]).max()),
               time=abs(float(sc[mxe.S_TIME]) - r["t"]) / r["t"],
               updates_last_step=[int(sc[mxe.S_UPDATES]), int(r["updates"][-1])], bar=1e-10)
    return dict(workload=w.name, sites=s.n, steps=w.n_steps, max_relax=w.params["max_relax"],
                wall_s=wall, value=s.n * ev / wall, unit="site-evals/s", evals=ev,
                site_steps_per_s=s.n * w.n_steps / wall, ms_per_step=wall / w.n_steps * 1e3,
                launch=f"graph replays, relaxations in chunks of {RELAX_CHUNK_SINGLE} iterations ending "
                       "once converged", launch_shapes=shapes, wall_s_fixed_sequence=wall_fixed,
                status=int(sc[mxe.S_STATUS]),
                oracle_wall_s=t_or, oracle_threads=O.num_threads(), error_vs_oracle=err)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-sample", type=int, default=256000)
    ap.add_argument("--cpu-single-sample", type=int, default=16000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline leg (no other legs, no oracle errors)")
    ap.add_argument("--legs", default="graph,fp32,degree3,variants,c0,c2,c3,full,serving",
                    help="comma-separated extra legs")
    ap.add_argument("--fullsize-steps", type=int, default=3,
                    help="timed diffusion steps of the slab and nanowire legs")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-steps", type=int, default=50)
    ap.add_argument("--serve-rates", default="0.25,0.5,0.8,1.0,2.0",
                    help="arrival rates as multiples of the batched capacity")
    ap.add_argument("--shapes", default="",
                    help="launch shapes of the 256k-site legs as k=v,... (default: the autotuner's)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with a 1 GiB device copy (reference for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    legs = set() if args.no_extras else set(x for x in args.legs.split(",") if x)

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

    t0 = time.perf_counter()
    if args.shapes:
        shapes = {k: int(v) for k, v in (kv.split("=") for kv in args.shapes.split(","))}
        params = dict(w.params, **shapes)
    else:
        params, shapes = tuned(w, "fp64")
    log(f"launch shapes {shapes} ({time.perf_counter() - t0:.1f} s)")
    plan = mxe.Plan([s], w.eam, params, precision="fp64")
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
    wall_b, sc_b, prof_b = timed_run(plan, st, out, ws, BREAKDOWN_STEPS, use_graph=False, profile=True)
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
                     traffic=counter_traffic("pair"), traffic_unit="B/launch",
                     work="algorithmic: 27 nodes x 77 FP64 operations per listed pair "
                          "(nominal count, not the executed instructions)")
    roof_pair["frac"] = roof_pair["achieved"] / roof_pair["peak"]
    valu = valu_counters(pair_avg_s)
    if valu is not None:
        roof_pair["valu_counters"] = valu
    evals_per_launch = evals_b / max(fam["force"]["launches"], 1)
    bytes_force = (BYTES_FORCE_PER_PAIR * pair_evals_b / max(evals_b, 1) + BYTES_FORCE_PER_SITE * n) \
        * evals_per_launch
    force_avg_s = fam["force"]["ms_avg"] / 1e3
    roof_force = dict(bound="hbm", achieved=bytes_force / force_avg_s / 1e9 if force_avg_s > 0 else 0.0,
                      peak=PEAK_HBM_GBS, unit="GB/s", kernel="k_force<double> + k_force_fold",
                      traffic=counter_traffic("force"), traffic_unit="B/launch",
                      algorithmic_bytes=bytes_force,
                      work="each pair's 14 moments and row entry read from both ends, plus "
                           "per-site state, embedding terms and outputs")
    roof_force["frac"] = roof_force["achieved"] / roof_force["peak"]
    bytes_once = (BYTES_FORCE_ONCE_PER_PAIR * pair_evals_b / max(evals_b, 1) + BYTES_FORCE_PER_SITE * n) \
        * evals_per_launch
    roof_force["once_per_pair"] = dict(
        algorithmic_bytes=bytes_once,
        achieved=bytes_once / force_avg_s / 1e9 if force_avg_s > 0 else 0.0,
        frac=bytes_once / force_avg_s / 1e9 / PEAK_HBM_GBS if force_avg_s > 0 else 0.0,
        work="each unordered pair's 14 moments counted once (112 B), plus the per-site bytes")
    bytes_dens = (BYTES_DENSITY_PER_PAIR * pair_evals_b / max(evals_b, 1) + BYTES_DENSITY_PER_SITE * n) \
        * evals_b / max(fam["density"]["launches"], 1)
    dens_avg_s = fam["density"]["ms_avg"] / 1e3
    roof_dens = dict(bound="hbm", achieved=bytes_dens / dens_avg_s / 1e9 if dens_avg_s > 0 else 0.0,
                     peak=PEAK_HBM_GBS, unit="GB/s", kernel="k_density<double>",
                     traffic=counter_traffic("density"), traffic_unit="B/launch",
                     algorithmic_bytes=bytes_dens)
    roof_dens["frac"] = roof_dens["achieved"] / roof_dens["peak"]
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
                   "precision": "fp64", "launch": "eager; HIP events around the pair kernel",
                   "launch_shapes": shapes},
        "site_steps_per_s": site_steps,
        "evals_in_timed_steps": evals,
        "list_builds_in_timed_steps": int(sc[mxe.S_REBUILDS]),
        "pairs_per_eval": pair_evals / max(evals, 1),
        "status": status,
        "roofline": roofline,
        "roofline_all": {"pair": roof_pair, "force": roof_force, "density": roof_dens},
        "pair_ms_avg_timed": pair_ms / max(pair_launches, 1),
        "kernel_ms": fam,
        "kernel_ms_from": f"{BREAKDOWN_STEPS} steps after the timed region, every family bracketed",
        # kernel-only rate: the sites over the summed kernel-family time per
        # evaluation (every family's event time in the breakdown steps), beside
        # the wall-clock rate of the same steps
        "kernel_only": dict(
            site_evals_per_s=n * evals_b / max(sum(v["ms_total"] for v in fam.values()) / 1e3, 1e-30),
            wall_site_evals_per_s=n * evals_b / max(wall_b, 1e-30),
            steps=BREAKDOWN_STEPS, evals=evals_b,
            note="breakdown steps after the timed region, every kernel family bracketed by events"),
        "dominant_kernel": dominant,
        # the Euler step of the kinetic law on its own (event time per step)
        "master_step_site_steps_per_s": (int((s.type != 3).sum()) / (fam["master"]["ms_avg"] / 1e3)
                                         if fam["master"]["ms_avg"] > 0 else None),
    }
    if legs:
        result["error_vs_oracle"] = sampled_errors(w, plan, st, out, ws, "fp64")

    if "graph" in legs:
        wall_g, sc_g, _ = timed_run(plan, st, out, ws, args.steps, use_graph=True, profile=False)
        result["graph"] = dict(value=n * int(sc_g[mxe.S_TOTAL_EVALS]) / wall_g,
                               ms_per_step=wall_g / args.steps * 1e3,
                               evals=int(sc_g[mxe.S_TOTAL_EVALS]))
        log(f"graph leg: {wall_g:.3f} s")
    del st, out, ws, plan
    torch.cuda.empty_cache()
    # the other legs on this workload: tuned for their own precision and rule,
    # unless --shapes fixes the shapes for every leg
    leg_params = params if args.shapes else None
    if "fp32" in legs:
        result["fp32_mixed"] = fullsize_leg(w, "fp32", args.steps, args.warmup, params=leg_params)
        log(f"fp32 leg: {result['fp32_mixed']['value']:.4g} site-evals/s")
    if "degree3" in legs:
        # the paper's own degree-3 rule (12 nodes in the pair's 6-D space)
        result["degree3"] = {}
        for prec in ("fp64", "fp32"):
            result["degree3"][prec] = fullsize_leg(w, prec, args.steps, args.warmup, quad_rule=1,
                                                   params=leg_params)
            log(f"degree-3 {prec} leg: {result['degree3'][prec]['value']:.4g} site-evals/s")
    if "variants" in legs:
        # state variants on the same workload: site temperatures, reservoir sites
        result["variants"] = {}
        rng = np.random.default_rng(3)
        for name in ("site_temperature", "reservoirs"):
            pv = mxe.Plan([s], w.eam, params, precision="fp64")
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
    c0_oracle_s = None
    if "c0" in legs:
        result["c0_full_run"] = c0_leg()
        c0_oracle_s = result["c0_full_run"]["oracle_wall_s"]
        log(f"plain-method full run: {result['c0_full_run']['wall_s']:.3f} s on the GPU, "
            f"{c0_oracle_s:.1f} s for the oracle")
    if "c2" in legs:
        result["c2_alloy_slab_131k"] = fullsize_leg(L.config2(2), "fp32", args.fullsize_steps, 1, late=10)
        log(f"alloy slab leg: {result['c2_alloy_slab_131k']['value']:.4g} site-evals/s")
    if "c3" in legs:
        result["c3_nanowire_256k"] = fullsize_leg(L.config3(3), "fp32", args.fullsize_steps, 1, late=10)
        log(f"nanowire leg: {result['c3_nanowire_256k']['value']:.4g} site-evals/s")
    if "full" in legs:
        # whole configured runs, end to end (the 256k-site workload in FP64, the
        # slab and the nanowire in their FP32-mixed precision)
        result["full_runs"] = {}
        for wf, prec, pf in ((w, "fp64", params), (L.config2(2), "fp32", None), (L.config3(3), "fp32", None)):
            r = full_run_leg(wf, prec, pf)
            result["full_runs"][wf.name] = r
            log(f"full run {wf.name}: {r['steps']} steps in {r['wall_s']:.2f} s, "
                f"{r['value']:.4g} site-evals/s, status {r['status']}")
    if "serving" in legs:
        t0 = time.perf_counter()
        rates = [float(x) for x in args.serve_rates.split(",") if x]
        result["serving"] = serving_sweep(args.serve_requests, args.serve_steps, rates)
        log(f"serving legs: {time.perf_counter() - t0:.1f} s")

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
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_sample, args.cpu_single_sample, c0_oracle_s,
                                              gpu=result)
    # every run's device status: a bit that marks results invalid anywhere is listed,
    # and so is any schedule comparison that found different results
    bad = []

    def walk(o, path):
        if isinstance(o, dict):
            for k, v in o.items():
                if k == "status" and isinstance(v, int) and v & mxe.FATAL_STATUS:
                    bad.append(f"{path}/{k}={v}")
                if k.endswith("bitwise_equal") or k.endswith("bitwise_equal_all_schedules"):
                    if v is False:
                        bad.append(f"{path}/{k}=false")
                walk(v, f"{path}/{k}")
        elif isinstance(o, list):
            for i, v in enumerate(o):
                walk(v, f"{path}[{i}]")
    walk(result, "")
    result["invalid_results"] = bad
    if bad:
        log(f"results flagged invalid: {bad}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
