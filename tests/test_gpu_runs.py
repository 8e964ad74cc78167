"""Run-level parity of the staggered scheme (Sec. 4, Alg. 1) against the oracle.

* the plain-method workload (256 sites, one vacancy, 800 K) for its full 20
  diffusion steps of up to 50 FIRE updates, eager and as graph replays, with
  every step's update count, convergence flag, free energy, max |f|, time
  step and sum of x compared;
* one-step prefixes of the three large workloads at their full sizes (256,000
  vacancy sites in FP64; the 131,072-site alloy slab and the 256k-site
  nanowire in FP32-mixed, their workloads' precision), with the relaxation cut
  to 3 updates so the oracle finishes in seconds;
* a request of the serving sweep, served in a mix, against the oracle;
* a multi-step FP32-mixed run of a small alloy slab.

Increments (x - x0, q - q0, sigma - sigma0) are compared, not the values: an
error in a small change would hide in the value's norm.
"""
import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L
from paper_1910_01235_amd import serve

from tests.gpu_common import say, gpu_arrays, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    torch.cuda.set_device(0)
    return mxe


def _wrap(d, s):
    return d - np.array(s.box) * np.round(d / np.array(s.box)) * np.array(s.periodic)


KB = 8.617333262e-5


def _compare_run(tag, s, g, r, sc, tol, mx, x_floor=1e-30, dxdt_tol=None):
    """Final state of a GPU run against oracle.run, by increments.

    dx/dt is the kinetic law applied to mu: exp(beta dmu) turns a relative
    error e in mu into a relative error up to beta max|mu| e in the rates, so in
    FP32-mixed its bar is the mu bar times that condition number (dxdt_tol)."""
    errs = dict(
        dx=rel_err(g["x"] - s.x, r["x"] - s.x, x_floor),
        dq=float(np.abs(_wrap(g["q"] - r["q"], s)).max() /
                 max(np.abs(_wrap(r["q"] - s.q, s)).max(), 1e-30)),
        dsigma=rel_err(g["sigma"] - s.sigma, r["sigma"] - s.sigma, 1e-30),
        mu=rel_err(g["mu"], r["mu"], 1e-2),
    )
    err_dxdt = rel_err(g["dxdt"], r["dxdt"], 1e-30)
    kappa = np.abs(r["mu"]).max() / (KB * s.T)
    if dxdt_tol is None:
        dxdt_tol = tol if tol <= 1e-10 else tol * kappa
    say(f"[gpu] {tag}: dxdt {err_dxdt:.2e} (bar {dxdt_tol:.1e}, beta max|mu| {kappa:.1f})")
    assert err_dxdt < dxdt_tol, (tag, err_dxdt)
    say(f"[gpu] {tag}: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()) +
        f"; dt {sc[mx.S_DT]:.6e} vs {r['dt'][-1]:.6e}; updates {int(sc[mx.S_UPDATES])} vs "
        f"{int(r['updates'][-1])}")
    for k, v in errs.items():
        assert v < tol, (tag, k, v)
    assert sc[mx.S_DT] == pytest.approx(r["dt"][-1], rel=tol)
    assert int(sc[mx.S_UPDATES]) == int(r["updates"][-1])
    assert int(sc[mx.S_CONVERGED]) == int(r["converged"][-1])
    # the x integration, the conserved sum and the time step are FP64 in both precisions
    assert abs(sc[mx.S_SUMX] - s.x.sum()) <= 1e-12 * s.x.sum()
    assert abs(g["x"].sum() - s.x.sum()) <= 1e-12 * s.x.sum()
    assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0


_C0 = {}


def _c0_oracle():
    if "run" not in _C0:
        w = L.config0(0)
        s = w.systems[0]
        say("[gpu] oracle: plain-method workload, 20 steps")
        _C0["run"] = O.run(w.eam, w.params, s.box, s.periodic, s.T, w.n_steps, s.q, s.sigma, s.x,
                           s.type)
    return _C0["run"]


@pytest.mark.parametrize("use_graph", [False, True])
def test_plain_workload_full_run_matches_oracle(mx, use_graph):
    w = L.config0(0)
    s = w.systems[0]
    assert w.n_steps == 20 and w.params["max_relax"] == 50
    r = _c0_oracle()
    say(f"[gpu] plain workload, 20 steps in one call, graph={use_graph}")
    plan = mx.Plan([s], w.eam, w.params)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, w.n_steps, use_graph=use_graph)
    torch.cuda.synchronize()
    sc = plan.scalars(out)[0]
    g = gpu_arrays(plan, st, out)
    _compare_run("20 steps", s, g, r, sc, TOL["fp64"], mx)
    assert sc[mx.S_TIME] == pytest.approx(r["t"], rel=1e-10)
    # step by step: one call per step, every step's record against the oracle's
    plan = mx.Plan([s], w.eam, w.params)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    for k in range(w.n_steps):
        plan.run(st, out, ws, 1, use_graph=use_graph)
        torch.cuda.synchronize()
        sc = plan.scalars(out)[0]
        assert int(sc[mx.S_UPDATES]) == int(r["updates"][k]), k
        assert int(sc[mx.S_CONVERGED]) == int(r["converged"][k]), k
        assert sc[mx.S_F] == pytest.approx(r["F"][k], rel=1e-12, abs=1e-12), k
        assert sc[mx.S_FMAX] == pytest.approx(r["fmax"][k], rel=1e-8, abs=1e-12), k
        assert sc[mx.S_DT] == pytest.approx(r["dt"][k], rel=1e-10), k
        assert abs(sc[mx.S_SUMX] - r["sum_x"][k]) <= 1e-12 * r["sum_x"][k], k
    g = gpu_arrays(plan, st, out)
    assert rel_err(g["x"] - s.x, r["x"] - s.x, 1e-30) < TOL["fp64"]
    assert sc[mx.S_TIME] == pytest.approx(r["t"], rel=1e-10)
    say(f"    per-step records equal; updates per step {r['updates'].astype(int).tolist()}")


def _prefix_cases():
    yield "c1_vacancy_256k", L.config1(1), "fp64"
    yield "c2_alloy_slab_131k", L.config2(2), "fp32"
    yield "c3_nanowire_256k", L.config3(3), "fp32"


@pytest.mark.parametrize("name,w,precision", list(_prefix_cases()), ids=lambda v: v if isinstance(v, str) else "")
def test_full_size_one_step_prefix_matches_oracle(mx, name, w, precision):
    s = w.systems[0]
    params = dict(w.params, max_relax=3)
    say(f"[gpu] {name}: one step, 3 updates, {precision}, {s.n} sites")
    plan = mx.Plan([s], w.eam, params, precision=precision)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, 1, use_graph=False)
    torch.cuda.synchronize()
    sc = plan.scalars(out)[0]
    g = gpu_arrays(plan, st, out)
    say(f"    oracle run ({O.num_threads()} threads)")
    r = O.run(w.eam, params, s.box, s.periodic, s.T, 1, s.q, s.sigma, s.x, s.type)
    _compare_run(name, s, g, r, sc, TOL[precision], mx)


def test_served_request_matches_oracle(mx):
    """A request of the serving sweep, served beside others, equals the oracle's run."""
    reqs = L.config4_requests(4)
    order = np.argsort([s.n for s in reqs])
    pick = [reqs[k] for k in order[:6]]  # the six smallest requests of the sweep
    params = dict(L.DEFAULT_PARAMS, max_relax=50)
    n_steps = 2
    caps = [1024, 1024, 2048, 2048, 4096, 4096]
    srv = serve.Server(L.DEFAULT_EAM, params, caps)
    requests = [serve.Request(k, s, n_steps, 0.0) for k, s in enumerate(pick)]
    results, rejected, stats = srv.serve(requests, realtime=False)
    assert not rejected and len(results) == len(pick)
    for k in (0, len(pick) - 1):
        res = next(x for x in results if x.rid == k)
        s = pick[k]
        say(f"[gpu] served request {k}: {s.name}, {s.n} sites, slot {res.slot}")
        r = O.run(L.DEFAULT_EAM, params, s.box, s.periodic, s.T, n_steps, s.q, s.sigma, s.x,
                  s.type)
        assert res.status & mx.FATAL_STATUS == 0
        assert rel_err(res.x - s.x, r["x"] - s.x, 1e-30) < TOL["fp64"]
        assert np.abs(_wrap(res.q - r["q"], s)).max() < 1e-10
        assert rel_err(res.sigma, r["sigma"], 1e-30) < TOL["fp64"]
        assert res.time_simulated == pytest.approx(r["t"], rel=1e-10)


def test_fp32_mixed_multi_step_run_matches_oracle(mx):
    n = 6 * 6 * 5 * 4
    slab = L.System(L.fcc(6, 6, 5), np.full(n, 0.1), np.full(n, 0.05), np.full(n, L.ALLOY, np.int8),
                    (6 * L.A0_CU, 6 * L.A0_CU, 5 * L.A0_CU + 20.0), (True, True, False), 900.0,
                    "slab")
    s = L.jitter(slab, 5, xr=(0.02, 0.2))
    params = dict(L.DEFAULT_PARAMS, max_relax=10)
    say("[gpu] fp32-mixed slab, 4 steps")
    plan = mx.Plan([s], L.DEFAULT_EAM, params, precision="fp32")
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, 3, use_graph=True)
    torch.cuda.synchronize()
    x_pre = st.x.cpu().numpy().copy()
    plan.run(st, out, ws, 1, use_graph=True)
    torch.cuda.synchronize()
    sc = plan.scalars(out)[0]
    g = gpu_arrays(plan, st, out)
    r = O.run(L.DEFAULT_EAM, params, s.box, s.periodic, s.T, 4, s.q, s.sigma, s.x, s.type)
    _compare_run("fp32 slab 4 steps", s, g, r, sc, TOL["fp32"], mx)
    # the kinetic law itself runs in FP64: on the GPU's own mu it is the oracle's to rounding
    nb, bl = O.bonds(s.box, s.periodic, s.q, s.type, params["r_bond"])
    dxdt, dt = O.master_rates(params, s.box, s.periodic, s.T, x_pre, s.type, g["mu"], nb, bl)
    assert rel_err(g["dxdt"], dxdt, 1e-30) < 1e-12
    assert sc[mx.S_DT] == pytest.approx(dt, rel=1e-12)
    assert rel_err(g["x"], x_pre + dt * dxdt, 1e-30) < 1e-14
