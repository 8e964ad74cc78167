"""Continuous batching of many independent systems on one GPU.

Requests (a system, a number of diffusion steps, an arrival time) are served
from a pool of plan slots sized to an HBM budget. Between calls the server
admits the requests that have arrived into free slots (the smallest free slot
that holds the system) and retires the systems that have finished. A call
either advances every resident system by one diffusion step of the staggered
scheme (step level), or runs a few free-running iterations in which each
system takes its Euler step as soon as its own relaxation ends (iteration
level), so no system waits for a slower one at step boundaries. Requests
that arrive while others run join as slots free up; their work shares every
launch with the resident systems. A system's results do not depend on its
slot, its batch-mates or the level.

The one-at-a-time path serves the same stream with a single-slot plan per
request, in arrival order, for comparison on the same GPU.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import lattice as L
from . import mxe

STATE_BYTES_PER_SITE = 14 * 8 + 1  # q(3), sigma, x, 9 outputs (FP64), type (int8)


@dataclass
class Request:
    rid: int
    system: L.System
    n_steps: int
    arrival: float = 0.0  # seconds after the start of serving


@dataclass
class Result:
    rid: int
    n_sites: int
    slot: int
    arrival: float
    admitted: float
    completed: float
    x: np.ndarray
    q: np.ndarray
    sigma: np.ndarray
    time_simulated: float
    status: int

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


def bytes_per_site(eam: dict, params: dict, precision: str = "fp64", probe_sites: int = 4096) -> float:
    """Device bytes per site of a slot: workspace plus state and outputs (host-side probe)."""
    n_cells = max(6, int(round((probe_sites / 4) ** (1 / 3))))
    s = L.vacancy_bulk(n_cells, 0, 300.0, 0)
    plan = mxe.Plan([s], eam, params, precision=precision)
    return plan.ws_bytes / s.n + STATE_BYTES_PER_SITE


def pool_capacities(budget_bytes: float, per_site: float, classes=(1024, 2048, 4096, 8192, 16384,
                                                                     32768, 65536)) -> list:
    """Equal numbers of slots per capacity class, as many as the budget holds.

    Request sizes drawn log-uniformly fall equally often in each octave, so each
    class gets the same number of slots. Returns the slot capacities (sites)."""
    per_round = sum(classes) * per_site
    m = int(budget_bytes // per_round)
    if m < 1:
        raise ValueError(f"budget {budget_bytes:.3g} B holds no slot of every class "
                         f"({per_round:.3g} B needed)")
    return [c for c in classes for _ in range(m)]


def pick_slot(capacities: list, free, n: int):
    """Smallest free slot that holds n sites (lowest index among equals), or None."""
    best = None
    for k in sorted(free):
        c = capacities[k]
        if c >= n and (best is None or c < capacities[best]):
            best = k
    return best


# volume per site of the FCC lattice, with a margin: a slot's cell capacity is
# sized from a cube of this volume per site
VOLUME_PER_SITE = 1.05 * L.A0_CU ** 3 / 4.0


def _template(capacity: int, r_min_box: float) -> L.System:
    """Placeholder system that defines a slot's capacity (slots start empty)."""
    side = max(r_min_box, (capacity * VOLUME_PER_SITE) ** (1.0 / 3.0))
    n = capacity
    return L.System(np.zeros((n, 3)), np.full(n, 0.1), np.ones(n), np.zeros(n, np.int8),
                    (side, side, side), (True, True, True), 300.0, f"slot{capacity}")


class Server:
    """A pool of slots on one GPU, with continuous batching over diffusion steps."""

    def __init__(self, eam: dict, params: dict, capacities: list, precision: str = "fp64",
                 device: str = "cuda", iteration_level: bool = False, advance_iters: int = 8):
        """iteration_level: systems advance with free-running steps (mxe_advance),
        each taking its Euler step as soon as its own relaxation ends; requests
        are admitted and retired between calls of advance_iters iterations.
        Otherwise every resident system takes one diffusion step per call, the
        call lasting as long as the slowest relaxation. Needs relax_chunk > 0."""
        import torch
        self.torch = torch
        self.iteration_level = iteration_level
        self.advance_iters = advance_iters
        if iteration_level and int(params.get("relax_chunk", 0)) <= 0:
            raise ValueError("iteration-level serving needs params['relax_chunk'] > 0")
        self.capacities = list(capacities)
        r_cap = eam["r_c"] + 3 * math.sqrt(2) * params.get("sigma_cap", 0.3) + params.get("skin", 0.15)
        templates = [_template(c, 2 * r_cap + 1.0) for c in self.capacities]
        self.plan = mxe.Plan(templates, eam, params, precision=precision)
        for k in range(len(templates)):
            self.plan.set_system(k, None)
        self.plan.set_resume(True)
        N = self.plan.n_sites
        z = lambda: torch.zeros(N, dtype=torch.float64, device=device)
        self.st = mxe.DeviceState(z(), z(), z(), torch.full((N,), 0.1, dtype=torch.float64, device=device),
                                  z(), torch.zeros(N, dtype=torch.int8, device=device))
        self.out = self.plan.out(device)
        self.ws = self.plan.workspace(device)
        self.free = set(range(len(templates)))
        self.device = device

    @property
    def footprint_bytes(self) -> int:
        return self.ws.numel() + self.plan.n_sites * STATE_BYTES_PER_SITE

    def fits(self, s: L.System) -> bool:
        """Does some slot (free or not) accept this system (sites and cells)?"""
        seen = set()
        for k, c in enumerate(self.capacities):
            if c >= s.n and c not in seen:  # slots of one capacity accept the same systems
                seen.add(c)
                if self.plan.check_system(k, s):
                    return True
        return False

    def pick_slot(self, s: L.System):
        """Smallest free slot that accepts the system (by sites, then by cells), or None."""
        free = set(self.free)
        while True:
            k = pick_slot(self.capacities, free, s.n)
            if k is None or self.plan.check_system(k, s):
                return k
            free.discard(k)

    def admit(self, slot: int, s: L.System, n_steps: int = 0):
        torch = self.torch
        off = int(self.plan.offsets[slot])
        n = s.n
        self.plan.set_system(slot, s)
        if self.iteration_level:
            self.plan.set_steps(slot, n_steps)
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)
        self.st.qx[off:off + n] = f(s.q[:, 0])
        self.st.qy[off:off + n] = f(s.q[:, 1])
        self.st.qz[off:off + n] = f(s.q[:, 2])
        self.st.sigma[off:off + n] = f(s.sigma)
        self.st.x[off:off + n] = f(s.x)
        self.st.type[off:off + n] = torch.as_tensor(s.type.astype(np.int8), device=self.device)
        self.out.scalars[slot * mxe.NSCALARS + mxe.S_TIME] = 0.0
        self.free.discard(slot)

    def collect(self, slot: int, n: int):
        off = int(self.plan.offsets[slot])
        g = lambda t: t[off:off + n].cpu().numpy()
        q = np.stack([g(self.st.qx), g(self.st.qy), g(self.st.qz)], axis=1)
        sc = self.out.scalars[slot * mxe.NSCALARS:(slot + 1) * mxe.NSCALARS].cpu().numpy()
        return g(self.st.x), q, g(self.st.sigma), float(sc[mxe.S_TIME]), int(sc[mxe.S_STATUS])

    def retire(self, slot: int):
        self.plan.set_system(slot, None)
        self.free.add(slot)

    def step(self):
        """One call: a diffusion step of every resident system, or (iteration
        level) up to advance_iters free-running iterations."""
        if self.iteration_level:
            self.plan.advance(self.st, self.out, self.ws, self.advance_iters, use_graph=True)
        else:
            self.plan.run(self.st, self.out, self.ws, 1, use_graph=True)

    def serve(self, requests: list, realtime: bool = True, progress=None):
        """Serve a request stream; returns (results, rejected ids, stats).
        progress: optional callable, given the number of results after each completion."""
        torch = self.torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        n_steps_of = {r.rid: r.n_steps for r in pending}
        fit = {r.rid: self.fits(r.system) for r in pending}
        rejected = [r.rid for r in pending if not fit[r.rid]]
        pending = [r for r in pending if fit[r.rid]]
        active = {}  # slot -> [request, steps done, admitted time]
        results = []
        steps = 0
        busy = 0.0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while pending or active:
            t = now()
            # admit arrived requests in arrival order while slots are free
            keep = []
            for r in pending:
                if realtime and r.arrival > t:
                    keep.append(r)
                    continue
                slot = self.pick_slot(r.system)
                if slot is None:
                    keep.append(r)
                    continue
                self.admit(slot, r.system, r.n_steps)
                active[slot] = [r, 0, now()]
            pending = keep
            if not active:
                if pending and realtime:
                    time.sleep(max(0.0, min(p.arrival for p in pending) - now()))
                continue
            ts = now()
            self.step()
            torch.cuda.synchronize()
            busy += now() - ts
            steps += 1
            done = []
            if self.iteration_level:
                left = self.out.scalars.view(-1, mxe.NSCALARS)[:, mxe.S_STEPS_LEFT].cpu().numpy()
                done = [slot for slot in active if left[slot] == 0]
            else:
                for slot, rec in active.items():
                    rec[1] += 1
                    if rec[1] >= rec[0].n_steps:
                        done.append(slot)
            tc = now()
            for slot in done:
                r, _, ta = active.pop(slot)
                x, q, sg, tsim, st = self.collect(slot, r.system.n)
                results.append(Result(r.rid, r.system.n, slot, r.arrival, ta, tc, x, q, sg, tsim, st))
                self.retire(slot)
                if progress is not None:
                    progress(len(results))
        makespan = now()
        lat = np.array([r.latency for r in results]) if results else np.zeros(1)
        stats = dict(systems=len(results), rejected=len(rejected), makespan_s=makespan,
                     systems_per_s=len(results) / makespan if makespan > 0 else 0.0,
                     site_steps_per_s=(sum(r.n_sites * n_steps_of[r.rid] for r in results) / makespan
                                       if makespan > 0 else 0.0),
                     p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                     gpu_steps=steps, gpu_busy_s=busy, footprint_bytes=self.footprint_bytes,
                     slots=len(self.capacities))
        return results, rejected, stats


def serve_one_at_a_time(eam: dict, params: dict, requests: list, precision: str = "fp64",
                        realtime: bool = True, device: str = "cuda", progress=None, params_for=None):
    """The plain path: each request alone on its own plan, in arrival order.
    progress: optional callable, given the number of requests done after each.
    params_for: optional callable giving the parameters for one system (e.g.
    launch shapes tuned for its size); default: params for every request."""
    import torch
    results = []
    pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    for r in pending:
        if realtime and r.arrival > now():
            time.sleep(r.arrival - now())
        ta = now()
        plan = mxe.Plan([r.system], eam, params_for(r.system) if params_for else params,
                        precision=precision)
        st, out, ws = plan.state([r.system], device), plan.out(device), plan.workspace(device)
        plan.run(st, out, ws, r.n_steps, use_graph=True)
        torch.cuda.synchronize()
        tc = now()
        sc = plan.scalars(out)[0]
        q = torch.stack([st.qx, st.qy, st.qz], 1).cpu().numpy()
        results.append(Result(r.rid, r.system.n, 0, r.arrival, ta, tc, st.x.cpu().numpy(), q,
                              st.sigma.cpu().numpy(), float(sc[mxe.S_TIME]), int(sc[mxe.S_STATUS])))
        del plan, st, out, ws
        if progress is not None:
            progress(len(results))
    makespan = now()
    lat = np.array([r.latency for r in results]) if results else np.zeros(1)
    stats = dict(systems=len(results), makespan_s=makespan,
                 systems_per_s=len(results) / makespan if makespan > 0 else 0.0,
                 p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)))
    return results, stats


def poisson_requests(systems: list, n_steps: int, rate: float, seed: int = 0) -> list:
    """Requests with exponential inter-arrival times at `rate` per second."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k, s in enumerate(systems):
        out.append(Request(k, s, n_steps, t))
        t += float(rng.exponential(1.0 / rate)) if rate > 0 else 0.0
    return out
