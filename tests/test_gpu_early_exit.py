"""Relaxations in chunks with an early exit (params.relax_chunk > 0).

The fixed launch sequence runs max_relax + 1 FIRE iterations per relaxation
(Sec. 4, Alg. 1: relax at fixed x, then one Euler step); systems that have
finished skip the rest. In chunked mode the host stops enqueueing once no
system is still relaxing. An iteration after a system has finished changes
nothing of it, so every output and scalar must equal the fixed sequence's
bitwise: eager and graph replays, a batch whose systems finish at different
iterations, chunk sizes that do and do not divide max_relax + 1, mxe_relax
alone, and FP32-mixed. The systems converge well inside the cap, so the early
exit is taken (counted launches prove it) and the runs stay valid (no status
flag that marks results invalid).
"""
import numpy as np
import pytest

from paper_1910_01235_amd import lattice as L
from tests.gpu_common import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    torch.cuda.set_device(0)
    return mxe


def _systems():
    """The plain-method workload and three requests of the serving mix (a
    vacancy crystal and two alloy crystals of 500, 864 and 2,916 sites)."""
    reqs = L.config4_requests(4)
    order = np.argsort([s.n for s in reqs])
    return [L.config0(0).systems[0]] + [reqs[k] for k in order[[0, 40, 80]]]


PARAMS = dict(L.DEFAULT_PARAMS, max_relax=50)


def _snapshot(plan, st, out):
    t = lambda a: a.cpu().numpy().copy()
    return dict(x=t(st.x), qx=t(st.qx), qy=t(st.qy), qz=t(st.qz), sigma=t(st.sigma),
                fx=t(out.fx), fy=t(out.fy), fz=t(out.fz), fs=t(out.fsigma), mu=t(out.mu),
                dxdt=t(out.dxdt), rho_bar=t(out.rho_bar), e_site=t(out.e_site),
                scalars=plan.scalars(out).copy())


def _run(mx, systems, params, n_steps, use_graph, precision="fp64", calls=1):
    plan = mx.Plan(systems, L.DEFAULT_EAM, params, precision=precision)
    st, out, ws = plan.state(systems), plan.out(), plan.workspace()
    for _ in range(calls):
        plan.run(st, out, ws, n_steps, use_graph=use_graph)
    torch.cuda.synchronize()
    snap = _snapshot(plan, st, out)
    assert np.all(snap["scalars"][:, mx.S_STATUS].astype(np.int64) & mx.FATAL_STATUS == 0)
    return snap


def _same(a, b, tag):
    for k in a:
        assert np.array_equal(a[k], b[k]), (tag, k)


@pytest.mark.parametrize("use_graph", [False, True])
@pytest.mark.parametrize("chunk", [1, 4, 7])
def test_chunked_run_equals_fixed_sequence(mx, use_graph, chunk):
    """Also the lean iterations' stalls: the chunked run enqueues no build chain
    in its chunks, so a system whose lists expire waits for an iteration with
    the chain; the lists are rebuilt inside relaxations here (the scalars,
    compared bitwise, include the build and evaluation counts)."""
    systems = _systems()
    say(f"[gpu] early exit: {len(systems)} systems, chunk {chunk}, graph={use_graph}")
    ref = _run(mx, systems, PARAMS, 3, use_graph)
    got = _run(mx, systems, dict(PARAMS, relax_chunk=chunk), 3, use_graph)
    _same(got, ref, f"chunk {chunk}")
    ev = ref["scalars"][:, mx.S_TOTAL_EVALS]
    assert ev.max() < 3 * (PARAMS["max_relax"] + 1)  # the exit is reachable
    builds = ref["scalars"][:, mx.S_REBUILDS].astype(int)
    assert builds.sum() > len(systems), builds  # builds beyond the call's first
    say(f"    bitwise equal; evaluations per system {ev.astype(int).tolist()}, builds {builds.tolist()}")


@pytest.mark.parametrize("companion", [False, True])
def test_chunked_run_large_plan_equals_fixed_sequence(mx, companion):
    """Above 65,536 occupied sites, a plan of one system still runs lean
    iterations; with a second system its chunks carry the build chain in every
    iteration. Both: bitwise the fixed sequence."""
    systems = [L.jitter(L.vacancy_bulk(26, 700, 1000.0, 7), 8, xr=(0.3, 0.95))]
    if companion:
        systems.append(L.jitter(L.vacancy_bulk(5, 1, 800.0, 9), 10, xr=(0.3, 0.95)))
    assert systems[0].n > 65536
    say(f"[gpu] early exit: {len(systems)} system(s), {sum(t.n for t in systems)} sites, chunk 4, graph")
    ref = _run(mx, systems, PARAMS, 2, True)
    got = _run(mx, systems, dict(PARAMS, relax_chunk=4), 2, True)
    _same(got, ref, "large plan")


def test_chunked_run_exits_early(mx):
    """Counted launches: the chunked run (chunks of lean iterations, and an
    iteration with the build chain after a stall) launches the pair kernel
    fewer times than the fixed sequence, and at least once per evaluation."""
    systems = _systems()
    K, n_steps = 4, 3
    plan = mx.Plan(systems, L.DEFAULT_EAM, dict(PARAMS, relax_chunk=K))
    st, out, ws = plan.state(systems), plan.out(), plan.workspace()
    plan.profile(True)
    plan.profile_read()
    plan.run(st, out, ws, n_steps, use_graph=False)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    sc = plan.scalars(out)
    per_step_max = sc[:, mx.S_EVALS].max()  # last step's evaluations, largest system count
    launches = prof["pair"][1]
    say(f"[gpu] early exit: {launches} pair launches in {n_steps} steps "
        f"(fixed sequence: {n_steps * (PARAMS['max_relax'] + 1)}); last step's evaluations "
        f"{sc[:, mx.S_EVALS].astype(int).tolist()}")
    assert launches < n_steps * (PARAMS["max_relax"] + 1)
    assert launches >= sc[:, mx.S_TOTAL_EVALS].max()
    assert per_step_max >= 1


def test_chunked_run_plain_workload_two_calls(mx):
    """The plain-method workload (20 steps of <= 50 updates), as two calls of 10
    steps on one plan: the graphs and host slots are reused by the second call."""
    w = L.config0(0)
    s = w.systems[0]
    say("[gpu] early exit: plain workload, 2 x 10 steps, chunk 4")
    ref = _run(mx, [s], w.params, 10, True, calls=2)
    got = _run(mx, [s], dict(w.params, relax_chunk=4), 10, True, calls=2)
    _same(got, ref, "plain workload")


def test_chunked_run_fp32_mixed(mx):
    systems = _systems()[1:]
    say("[gpu] early exit: fp32-mixed, chunk 3")
    ref = _run(mx, systems, PARAMS, 2, True, precision="fp32")
    got = _run(mx, systems, dict(PARAMS, relax_chunk=3), 2, True, precision="fp32")
    _same(got, ref, "fp32")


def test_chunked_relax_equals_fixed_sequence(mx):
    systems = _systems()
    say("[gpu] early exit: mxe_relax, chunk 5")
    res = []
    for p in (PARAMS, dict(PARAMS, relax_chunk=5)):
        plan = mx.Plan(systems, L.DEFAULT_EAM, p)
        st, out, ws = plan.state(systems), plan.out(), plan.workspace()
        plan.relax(st, out, ws)
        torch.cuda.synchronize()
        res.append(_snapshot(plan, st, out))
    _same(res[1], res[0], "relax")
