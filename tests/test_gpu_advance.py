"""Free-running steps (mxe_advance): each system relaxes and takes its Euler step
at its own pace (Sec. 4, Alg. 1, per system), yet runs exactly the relaxations
and steps it would run alone under mxe_run. Every state array and scalar must
equal the alone run's bitwise:
* a batch of systems with different step budgets, in one call and in many
  short calls, eager and as graph replays;
* systems admitted into slots at different times while others run, and slots
  rebound after their systems finished;
* the iteration-level server against alone runs.
"""
import numpy as np
import pytest

from paper_1910_01235_amd import lattice as L
from paper_1910_01235_amd import serve
from tests.gpu_common import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PARAMS = dict(L.DEFAULT_PARAMS, max_relax=50, relax_chunk=4)
# scalars that the free-running scheme must reproduce (the budget aside)
KEYS = ("S_F", "S_FMAX", "S_DT", "S_TIME", "S_SUMX", "S_UPDATES", "S_CONVERGED", "S_EVALS",
        "S_STATUS", "S_REBUILDS", "S_TOTAL_EVALS", "S_PAIRS", "S_PAIR_EVALS")


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    torch.cuda.set_device(0)
    return mxe


def _systems():
    """The plain-method workload and four requests of the serving mix."""
    reqs = L.config4_requests(4)
    order = np.argsort([s.n for s in reqs])
    return [L.config0(0).systems[0]] + [reqs[k] for k in order[[0, 40, 80, 120]]]


_ALONE = {}


def _alone(mx, s, n_steps):
    key = (s.name, n_steps)
    if key not in _ALONE:
        plan = mx.Plan([s], L.DEFAULT_EAM, PARAMS)
        st, out, ws = plan.state([s]), plan.out(), plan.workspace()
        plan.run(st, out, ws, n_steps, use_graph=True)
        torch.cuda.synchronize()
        _ALONE[key] = dict(x=st.x.cpu().numpy(), qx=st.qx.cpu().numpy(), qy=st.qy.cpu().numpy(),
                           qz=st.qz.cpu().numpy(), sigma=st.sigma.cpu().numpy(),
                           mu=out.mu.cpu().numpy(), sc=plan.scalars(out)[0].copy())
    return _ALONE[key]


def _check_slot(mx, plan, st, out, k, s, n_steps, tag):
    ref = _alone(mx, s, n_steps)
    lo, hi = plan.offsets[k], plan.offsets[k] + s.n
    for name in ("x", "qx", "qy", "qz", "sigma"):
        assert np.array_equal(getattr(st, name)[lo:hi].cpu().numpy(), ref[name]), (tag, k, name)
    assert np.array_equal(out.mu[lo:hi].cpu().numpy(), ref["mu"]), (tag, k, "mu")
    sc = plan.scalars(out)[k]
    for key in KEYS:
        i = getattr(mx, key)
        assert sc[i] == ref["sc"][i], (tag, k, key, sc[i], ref["sc"][i])
    assert sc[mx.S_STEPS_LEFT] == 0
    assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("max_iters", [1000, 3])
def test_batch_with_budgets_equals_alone_runs(mx, use_graph, max_iters):
    systems = _systems()
    budgets = [3, 5, 2, 4, 1]
    say(f"[gpu] advance: {len(systems)} systems, budgets {budgets}, calls of {max_iters} "
        f"iterations, graph={use_graph}")
    plan = mx.Plan(systems, L.DEFAULT_EAM, PARAMS)
    plan.set_resume(True)
    st, out, ws = plan.state(systems), plan.out(), plan.workspace()
    for k, b in enumerate(budgets):
        plan.set_steps(k, b)
    calls = 0
    while True:
        plan.advance(st, out, ws, max_iters, use_graph=use_graph)
        calls += 1
        torch.cuda.synchronize()
        if not plan.scalars(out)[:, mx.S_STEPS_LEFT].any():
            break
        assert calls < 2000
    for k, (s, b) in enumerate(zip(systems, budgets)):
        _check_slot(mx, plan, st, out, k, s, b, f"batch/{max_iters}/{use_graph}")
    say(f"    bitwise equal to alone runs after {calls} calls")


def test_staggered_admission_and_rebinding(mx):
    """Slots start empty; systems are admitted while others run, and a slot whose
    system finished is rebound to another."""
    systems = _systems()
    caps = [8192, 8192, 8192]
    r_cap = L.DEFAULT_EAM["r_c"] + 3 * np.sqrt(2) * PARAMS.get("sigma_cap", 0.3) + PARAMS.get("skin", 0.15)
    templates = [serve._template(c, 2 * r_cap + 1.0) for c in caps]
    plan = mx.Plan(templates, L.DEFAULT_EAM, PARAMS)
    for k in range(len(caps)):
        plan.set_system(k, None)
    plan.set_resume(True)
    N = plan.n_sites
    z = lambda: torch.zeros(N, dtype=torch.float64, device="cuda")
    st = mx.DeviceState(z(), z(), z(), torch.full((N,), 0.1, dtype=torch.float64, device="cuda"), z(),
                        torch.zeros(N, dtype=torch.int8, device="cuda"))
    out, ws = plan.out(), plan.workspace()

    def admit(slot, s, n):
        off = int(plan.offsets[slot])
        plan.set_system(slot, s)
        plan.set_steps(slot, n)
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")
        st.qx[off:off + s.n] = f(s.q[:, 0])
        st.qy[off:off + s.n] = f(s.q[:, 1])
        st.qz[off:off + s.n] = f(s.q[:, 2])
        st.sigma[off:off + s.n] = f(s.sigma)
        st.x[off:off + s.n] = f(s.x)
        st.type[off:off + s.n] = torch.as_tensor(s.type.astype(np.int8), device="cuda")
        out.scalars[slot * mx.NSCALARS + mx.S_TIME] = 0.0

    # (earliest call, system, steps): admitted into the lowest free slot from then on
    queue = [(0, systems[1], 4), (0, systems[2], 2), (2, systems[0], 3), (5, systems[3], 3),
             (9, systems[4], 2)]
    n_req = len(queue)
    resident = {}
    checked = 0
    for call in range(400):
        for item in list(queue):
            free = [k for k in range(len(caps)) if k not in resident]
            if item[0] <= call and free:
                admit(free[0], item[1], item[2])
                resident[free[0]] = (item[1], item[2])
                queue.remove(item)
        plan.advance(st, out, ws, 3, use_graph=True)
        torch.cuda.synchronize()
        left = plan.scalars(out)[:, mx.S_STEPS_LEFT]
        for slot in [k for k in resident if left[k] == 0]:
            s, n = resident.pop(slot)
            _check_slot(mx, plan, st, out, slot, s, n, f"staggered/{s.name}")
            plan.set_system(slot, None)
            checked += 1
        if checked == n_req:
            break
    assert checked == n_req
    say(f"[gpu] advance: {checked} staggered systems bitwise equal to alone runs ({call + 1} calls)")


def test_iteration_level_server_equals_alone_runs(mx):
    reqs = L.config4_requests(4)
    order = np.argsort([s.n for s in reqs])
    pick = [reqs[k] for k in order[[0, 30, 60, 90, 110, 130]]]  # 500 to 8,788 sites
    srv = serve.Server(L.DEFAULT_EAM, PARAMS, [1024, 2048, 8192, 16384],
                       iteration_level=True, advance_iters=4)
    requests = [serve.Request(k, s, 3 + k % 3, 0.01 * k) for k, s in enumerate(pick)]
    results, rejected, stats = srv.serve(requests, realtime=False)
    assert not rejected and len(results) == len(pick)
    for res in results:
        s, n = pick[res.rid], requests[res.rid].n_steps
        ref = _alone(mx, s, n)
        assert np.array_equal(res.x, ref["x"]), res.rid
        assert np.array_equal(res.sigma, ref["sigma"]), res.rid
        assert np.array_equal(res.q[:, 0], ref["qx"]), res.rid
        assert res.time_simulated == ref["sc"][mx.S_TIME]
        assert res.status & mx.FATAL_STATUS == 0
    say(f"[gpu] iteration-level server: {len(results)} requests bitwise equal to alone runs, "
        f"{stats['gpu_steps']} calls")
