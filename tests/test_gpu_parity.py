"""GPU path (through the C ABI) against the FP64 CPU oracle.

Bars: FP64 1e-10 normwise relative; FP32-mixed 1e-5; sum x conserved to 1e-12.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L
from tests.gpu_common import eval_errors, gpu_arrays, oracle_eval, parity_systems, rel_err, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EAM = L.DEFAULT_EAM
P = dict(L.DEFAULT_PARAMS)


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    return mxe


def kmax_for(systems):
    """Host sites next to octahedral sites list ~122-140 neighbours; FCC hosts alone ~54-78."""
    return 160 if any((s.type == L.INTERSTITIAL).any() for s in systems) else 96


def _evaluate(mx, systems, precision="fp64", **over):
    over.setdefault("k_max", kmax_for(systems))
    plan = mx.Plan(systems, EAM, P, precision=precision, **over)
    st = plan.state(systems)
    out = plan.out()
    ws = plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    return plan, st, out, ws


@pytest.mark.parametrize("name,s", parity_systems(), ids=[n for n, _ in parity_systems()])
def test_evaluate_fp64(mx, name, s):
    say(f"[gpu] evaluate fp64 {name} n={s.n}")
    plan, st, out, ws = _evaluate(mx, [s])
    sc = plan.scalars(out)[0]
    assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0, sc
    o = oracle_eval(EAM, s)
    g = gpu_arrays(plan, st, out)
    errs = eval_errors(g, o)
    say(f"    errors {errs}")
    for k, v in errs.items():
        assert v < 1e-10, (k, v)
    assert abs(sc[mx.S_F] - o["F"]) < 1e-10 * abs(o["F"])
    assert sc[mx.S_FMAX] == pytest.approx(np.abs(o["force"]).max(), rel=1e-10, abs=1e-12)


def test_evaluate_batch_uneven_matches_single(mx):
    """Uneven systems in one plan: each equals the oracle and its own single run bitwise."""
    systems = [s for _, s in parity_systems()]
    say(f"[gpu] evaluate batch of {len(systems)} systems")
    plan, st, out, ws = _evaluate(mx, systems)
    sc = plan.scalars(out)
    for k, s in enumerate(systems):
        assert int(sc[k, mx.S_STATUS]) & mx.FATAL_STATUS == 0
        g = gpu_arrays(plan, st, out, k)
        o = oracle_eval(EAM, s)
        for key, v in eval_errors(g, o).items():
            assert v < 1e-10, (k, key, v)
        p1, st1, out1, _ = _evaluate(mx, [s])
        g1 = gpu_arrays(p1, st1, out1)
        for key in ("force", "mu", "rho_bar", "e_site"):
            assert np.array_equal(g[key], g1[key]), (k, key)
        assert plan.scalars(out)[k, mx.S_F] == p1.scalars(out1)[0, mx.S_F]


def test_evaluate_is_deterministic(mx):
    s = parity_systems()[1][1]
    _, _, out_a, _ = _evaluate(mx, [s])
    _, _, out_b, _ = _evaluate(mx, [s])
    for n in ("fx", "fy", "fz", "fsigma", "mu", "e_site"):
        assert torch.equal(getattr(out_a, n), getattr(out_b, n)), n


# Exponents alpha, gamma per pair class (host-host, host-interstitial). The
# synthetic potential's 8 : 6 and 5 : 4 take the kernels built on one
# exponential per node (both shapes as powers of it); these take the kernels
# with two exponentials: no small ratio, the ratios in one class only, and a
# ratio no kernel is compiled for.
OTHER_EXPONENTS = {
    "no_ratio": ([7.3, 5.1], [6.2, 3.9]),
    "class0_ratio_only": ([8.0, 5.2], [6.0, 4.0]),
    "ratio_3_2": ([9.0, 5.0], [6.0, 4.0]),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("rule", [0, 1], ids=["gh27", "degree3"])
@pytest.mark.parametrize("variant", list(OTHER_EXPONENTS))
def test_evaluate_other_exponents(mx, variant, rule, prec):
    al, ga = OTHER_EXPONENTS[variant]
    eam = dict(EAM, alpha=al, gamma=ga, quad_rule=rule)
    tol = 1e-10 if prec == "fp64" else 1e-5
    for name, s in (parity_systems()[3], parity_systems()[2]):  # both pair classes; hosts only
        say(f"[gpu] evaluate {prec} {variant} rule {rule} {name}")
        plan = mx.Plan([s], eam, P, precision=prec, k_max=kmax_for([s]))
        st, out, ws = plan.state([s]), plan.out(), plan.workspace()
        plan.evaluate(st, out, ws)
        torch.cuda.synchronize()
        sc = plan.scalars(out)[0]
        assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0, sc
        o = oracle_eval(eam, s)
        errs = eval_errors(gpu_arrays(plan, st, out), o)
        say(f"    errors {errs}")
        for k, v in errs.items():
            assert v < tol, (k, v)
        assert abs(sc[mx.S_F] - o["F"]) < tol * abs(o["F"])


@pytest.mark.parametrize("name,s", parity_systems()[:4], ids=[n for n, _ in parity_systems()[:4]])
def test_evaluate_fp32_mixed(mx, name, s):
    say(f"[gpu] evaluate fp32-mixed {name}")
    plan, st, out, ws = _evaluate(mx, [s], precision="fp32")
    o = oracle_eval(EAM, s)
    g = gpu_arrays(plan, st, out)
    errs = eval_errors(g, o)
    say(f"    errors {errs}")
    for k, v in errs.items():
        assert v < 1e-5, (k, v)
    sc = plan.scalars(out)[0]
    assert abs(sc[mx.S_F] - o["F"]) < 1e-5 * abs(o["F"])


def test_perfect_lattice_invariants(mx):
    s = L.vacancy_bulk(5, 0, 1000.0, 0)
    s.sigma[:] = 0.12
    plan, st, out, ws = _evaluate(mx, [s])
    g = gpu_arrays(plan, st, out)
    assert np.abs(g["force"][:, :3]).max() < 1e-12
    assert np.ptp(g["force"][:, 3]) < 1e-12
    assert np.ptp(g["mu"]) < 1e-12


def test_relax_fp64_matches_oracle(mx):
    w = L.config0(0)
    s = w.systems[0]
    say("[gpu] relax c0")
    plan = mx.Plan([s], EAM, w.params)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.relax(st, out, ws)
    torch.cuda.synchronize()
    sc = plan.scalars(out)[0]
    q, sg, info = O.relax(EAM, w.params, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    say(f"    gpu updates {sc[mx.S_UPDATES]} oracle {info['updates']}; fmax {sc[mx.S_FMAX]} vs {info['fmax']}")
    assert int(sc[mx.S_UPDATES]) == info["updates"]
    assert int(sc[mx.S_EVALS]) == info["n_evals"]
    assert bool(sc[mx.S_CONVERGED]) == info["converged"]
    g = gpu_arrays(plan, st, out)
    dq = g["q"] - q
    dq -= np.array(s.box) * np.round(dq / np.array(s.box))
    assert np.abs(dq).max() < 1e-10 * L.A0_CU
    assert rel_err(g["sigma"], sg, 1e-2) < 1e-10
    assert rel_err(g["mu"], info["mu"], 1e-2) < 1e-10
    # relaxed forces are near ftol (1e-3 eV/A): normwise error with a 1e-2 eV/A floor
    err_f = rel_err(g["force"], info["force"], 1e-2)
    say(f"    relaxed force error {err_f:.2e}")
    assert err_f < 1e-10


def test_master_step_matches_oracle(mx):
    s = L.jitter(L.alloy_bulk(5, 0.3, 900.0, 7), 8, xr=(0.05, 0.95))
    say("[gpu] master step")
    plan = mx.Plan([s], EAM, P)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    plan.step(st, out, ws)
    torch.cuda.synchronize()
    mu = out.mu.cpu().numpy()
    nb, bl = O.bonds(s.box, s.periodic, s.q, s.type, P["r_bond"])
    dxdt, dt = O.master_rates(P, s.box, s.periodic, s.T, s.x, s.type, mu, nb, bl)
    sc = plan.scalars(out)[0]
    assert rel_err(out.dxdt.cpu().numpy(), dxdt, 1e-30) < 1e-12
    assert sc[mx.S_DT] == pytest.approx(dt, rel=1e-12)
    x_new = st.x.cpu().numpy()
    assert rel_err(x_new, s.x + dt * dxdt, 1e-30) < 1e-13
    assert abs(x_new.sum() - s.x.sum()) < 1e-12 * s.x.sum()
    assert sc[mx.S_TIME] == pytest.approx(dt, rel=1e-12)
    # a forced step size
    plan.step(st, out, ws, dt_in=1e-9)
    torch.cuda.synchronize()
    assert plan.scalars(out)[0, mx.S_DT] == 1e-9


def test_step_builds_bonds_only_and_keeps_lists(mx):
    """mxe_step builds the kinetic bonds alone: in resume mode the neighbour rows of
    the previous evaluation are left as they were and the next evaluation reuses
    them; on a workspace where no lists were built, the next evaluation builds them."""
    s = L.jitter(L.alloy_bulk(5, 0.3, 900.0, 7), 18, xr=(0.05, 0.95))
    plan = mx.Plan([s], EAM, P)
    plan.set_resume(True)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    before = plan.lists(ws)
    plan.step(st, out, ws)
    torch.cuda.synchronize()
    after = plan.lists(ws)
    assert np.array_equal(before["nbr_count"], after["nbr_count"])
    assert np.array_equal(before["nbr"], after["nbr"])
    nb, bl = O.bonds(s.box, s.periodic, s.q, s.type, P["r_bond"])
    assert np.array_equal(after["bond_count"], nb)
    valid = np.arange(bl.shape[1])[None, :] < nb[:, None]
    assert np.array_equal(np.where(valid, after["bond"][:, :bl.shape[1]], -1), np.where(valid, bl, -1))
    x1 = st.x.cpu().numpy()
    assert np.abs(x1 - s.x).max() > 0
    plan.evaluate(st, out, ws)  # resume: the lists of the first evaluation
    torch.cuda.synchronize()
    o = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, x1, s.type)
    g = gpu_arrays(plan, st, out)
    assert rel_err(g["force"], o["force"], 1e-2) < 1e-10
    assert rel_err(g["mu"], o["mu"], 1e-2) < 1e-10
    # a fresh workspace: a step first (no lists), then an evaluation in resume mode
    plan2 = mx.Plan([s], EAM, P)
    plan2.set_resume(True)
    st2, out2, ws2 = plan2.state([s]), plan2.out(), plan2.workspace()
    plan2.step(st2, out2, ws2)  # mu = 0: the linear law D sum_j (x_j - x_i)
    plan2.evaluate(st2, out2, ws2)
    torch.cuda.synchronize()
    x2 = st2.x.cpu().numpy()
    o2 = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, x2, s.type)
    g2 = gpu_arrays(plan2, st2, out2)
    assert int(plan2.scalars(out2)[0, mx.S_STATUS]) & mx.FATAL_STATUS == 0
    assert rel_err(g2["force"], o2["force"], 1e-2) < 1e-10
    assert rel_err(g2["rho_bar"], o2["rho_bar"], 1.0) < 1e-10


@pytest.mark.parametrize("use_graph", [False, True])
def test_run_c0_matches_oracle(mx, use_graph):
    w = L.config0(0)
    s = w.systems[0]
    n_steps = 6
    say(f"[gpu] run c0 {n_steps} steps graph={use_graph}")
    plan = mx.Plan([s], EAM, w.params)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, n_steps, use_graph=use_graph)
    torch.cuda.synchronize()
    r = O.run(EAM, w.params, s.box, s.periodic, s.T, n_steps, s.q, s.sigma, s.x, s.type)
    g = gpu_arrays(plan, st, out)
    sc = plan.scalars(out)[0]
    say(f"    x err {rel_err(g['x'], r['x'], 1e-30)} time {sc[mx.S_TIME]} vs {r['t']}")
    assert rel_err(g["x"], r["x"], 1e-30) < 1e-10
    assert rel_err(g["sigma"], r["sigma"], 1e-30) < 1e-10
    assert sc[mx.S_TIME] == pytest.approx(r["t"], rel=1e-10)
    assert abs(sc[mx.S_SUMX] - s.x.sum()) < 1e-12 * s.x.sum()
    assert int(sc[mx.S_UPDATES]) == int(r["updates"][-1])


def test_graph_replay_equals_eager(mx):
    w = L.config0(3)
    s = w.systems[0]
    res = []
    for use_graph in (False, True):
        plan = mx.Plan([s], EAM, w.params)
        st, out, ws = plan.state([s]), plan.out(), plan.workspace()
        for rep in range(3):  # several replays with host syncs between them
            plan.run(st, out, ws, 2, use_graph=use_graph)
            torch.cuda.synchronize()
            res.append((use_graph, rep, st.x.cpu().numpy().copy(), st.qx.cpu().numpy().copy()))
    for rep in range(3):
        assert np.array_equal(res[rep][2], res[3 + rep][2])
        assert np.array_equal(res[rep][3], res[3 + rep][3])


def test_degenerate_lone_sites(mx):
    """A lone atom has no density (flagged); a lone interstitial has only its width term."""
    lone = L.System(np.array([[5.0, 5.0, 5.0]]), np.array([0.1]), np.array([1.0]),
                    np.array([L.HOST_VAC], np.int8), (20.0, 20.0, 20.0), (False,) * 3, 800.0)
    plan, st, out, ws = _evaluate(mx, [lone])
    assert int(plan.scalars(out)[0, mx.S_STATUS]) & mx.STAT_RHO
    inter = L.System(np.array([[5.0, 5.0, 5.0]]), np.array([0.1]), np.array([0.5]),
                     np.array([L.INTERSTITIAL], np.int8), (20.0, 20.0, 20.0), (False,) * 3, 800.0)
    plan, st, out, ws = _evaluate(mx, [inter])
    sc = plan.scalars(out)[0]
    assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0
    o = oracle_eval(EAM, inter)
    assert sc[mx.S_F] == pytest.approx(o["F"], rel=1e-12)
    assert out.fsigma.item() == pytest.approx(o["force"][0, 3], rel=1e-12)


def test_run_interstitial_wire_matches_oracle(mx):
    """Solute hops between the octahedral sites of a host wire (Sec. 3.1 kinetics).

    Two interstitial sites do not interact, so no neighbour row lists such a
    pair, yet they are bonded (2.56 A apart): the occupancies after the steps
    check that the bond lists hold interstitial-interstitial bonds."""
    s = L.jitter(L.nanowire(radius=9.0, n_axial=5, T=700.0), 4, xr=(0.0, 0.9))
    p = dict(P, max_relax=15, k_max=160, sigma_cap=0.5)  # widths reach 0.31 A on this thin wire
    say("[gpu] run interstitial wire, 3 steps")
    plan = mx.Plan([s], EAM, p)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, 3, use_graph=True)
    torch.cuda.synchronize()
    sc = plan.scalars(out)[0]
    assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0
    r = O.run(EAM, p, s.box, s.periodic, s.T, 3, s.q, s.sigma, s.x, s.type)
    inter = s.type == L.INTERSTITIAL
    assert np.abs(r["x"] - s.x)[inter].max() > 1e-4  # the solute does move
    g = gpu_arrays(plan, st, out)
    dq = g["q"] - r["q"]
    dq -= np.array(s.box) * np.round(dq / np.array(s.box)) * np.array(s.periodic)
    assert np.abs(dq).max() < 1e-10
    assert rel_err(g["sigma"], r["sigma"], 1e-30) < 1e-10
    assert rel_err(g["x"], r["x"], 1e-30) < 1e-10
    assert int(sc[mx.S_UPDATES]) == int(r["updates"][-1])


def test_run_multichunk_with_rebuilds(mx):
    """Eight chunks, 20 vacancies at 1000 K: lists are rebuilt inside the relaxations."""
    s = L.vacancy_bulk(8, 20, 1000.0, 1)
    p = dict(P, max_relax=30)
    say("[gpu] run 8x8x8 with rebuilds")
    plan = mx.Plan([s], EAM, p)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, 3, use_graph=True)
    torch.cuda.synchronize()
    sc = plan.scalars(out)[0]
    assert sc[mx.S_REBUILDS] >= 2
    r = O.run(EAM, p, s.box, s.periodic, s.T, 3, s.q, s.sigma, s.x, s.type)
    g = gpu_arrays(plan, st, out)
    dq = g["q"] - r["q"]
    dq -= np.array(s.box) * np.round(dq / np.array(s.box))
    assert np.abs(dq).max() < 1e-10
    assert rel_err(g["sigma"], r["sigma"], 1e-30) < 1e-10
    assert rel_err(g["x"], r["x"], 1e-30) < 1e-10
    assert int(sc[mx.S_UPDATES]) == int(r["updates"][-1])
