"""GPU reservoir sites (Sec. 4: held molar fraction, held chemical potential) against the oracle.

Held-x sites are reset after every Euler step and their uptake is booked in
the RESERVOIR scalar; held-mu sites report the held mu after the forces.
Bars: FP64 1e-10; sum x + uptake conserved to 1e-12.
"""
import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L
from tests.gpu_common import gpu_arrays, oracle_eval, rel_err, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EAM = L.DEFAULT_EAM


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    return mxe


def _with_reservoirs(mx, plan, systems, res, res_val):
    st = plan.state(systems)
    st.reservoir = torch.as_tensor(res.astype(np.int8), device="cuda")
    st.res_value = torch.as_tensor(res_val, dtype=torch.float64, device="cuda")
    return st


def _held_system(seed=3):
    s = L.jitter(L.vacancy_bulk(5, 3, 900.0, seed), seed + 1, xr=(0.3, 0.9))
    rng = np.random.default_rng(seed)
    res = np.zeros(s.n, np.int8)
    held = rng.choice(s.n, 40, replace=False)
    res[held[:20]] = O.RES_FIX_X
    res[held[20:]] = O.RES_FIX_MU
    res_val = np.zeros(s.n)
    res_val[held[:20]] = rng.uniform(0.0, 1.0, 20)
    mu0 = oracle_eval(EAM, s)["mu"]
    res_val[held[20:]] = mu0[held[20:]] + rng.uniform(-0.05, 0.05, 20)
    return s, res, res_val, held


def test_evaluate_held_mu(mx):
    s, res, res_val, held = _held_system()
    x = s.x.copy()
    x[res == O.RES_FIX_X] = res_val[res == O.RES_FIX_X]  # the call start applies held x
    s2 = s.copy()
    s2.x = x
    plan = mx.Plan([s], EAM, L.DEFAULT_PARAMS)
    st = _with_reservoirs(mx, plan, [s], res, res_val)
    out, ws = plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    g = gpu_arrays(plan, st, out)
    o = O.evaluate(EAM, s.box, s.periodic, s.T, s2.q, s2.sigma, x, s2.type, res=res, res_val=res_val)
    assert np.array_equal(g["x"], x)
    assert rel_err(g["force"], o["force"], 1e-2) < 1e-10
    assert rel_err(g["mu"], o["mu"], 1e-2) < 1e-10
    assert np.array_equal(g["mu"][held[20:]], res_val[held[20:]])


@pytest.mark.parametrize("use_graph", [False, True])
def test_run_with_reservoirs_matches_oracle(mx, use_graph):
    s, res, res_val, held = _held_system(5)
    p = dict(L.DEFAULT_PARAMS, max_relax=20)
    n_steps = 4
    say(f"[gpu] reservoir run graph={use_graph}")
    plan = mx.Plan([s], EAM, p)
    st = _with_reservoirs(mx, plan, [s], res, res_val)
    out, ws = plan.out(), plan.workspace()
    plan.run(st, out, ws, n_steps, use_graph=use_graph)
    torch.cuda.synchronize()
    r = O.run(EAM, p, s.box, s.periodic, s.T, n_steps, s.q, s.sigma, s.x, s.type, res=res,
              res_val=res_val)
    g = gpu_arrays(plan, st, out)
    sc = plan.scalars(out)[0]
    assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0
    assert int(sc[mx.S_UPDATES]) == int(r["updates"][-1])
    assert rel_err(g["x"], r["x"], 1e-30) < 1e-10
    assert rel_err(g["sigma"], r["sigma"], 1e-30) < 1e-10
    assert sc[mx.S_TIME] == pytest.approx(r["t"], rel=1e-10)
    # the uptake is a sum over held sites of x changes: rounding floor n * 1e-14
    say(f"    uptake {sc[mx.S_RESERVOIR]:.6e} vs oracle {r['uptake'][-1]:.6e}")
    assert sc[mx.S_RESERVOIR] == pytest.approx(r["uptake"][-1], rel=1e-10, abs=1e-14 * s.n)
    x0 = s.x.copy()
    x0[res == O.RES_FIX_X] = res_val[res == O.RES_FIX_X]
    assert abs(sc[mx.S_SUMX] + sc[mx.S_RESERVOIR] - x0.sum()) < 1e-12 * x0.sum()
    assert np.array_equal(g["x"][held[:20]], res_val[held[:20]])


def test_held_layers_drive_a_steady_flux(mx):
    """Slab between a full and an empty held layer: GPU run equals the oracle's."""
    q = L.fcc(4, 4, 4)
    q[:, 2] += 2.0
    n = q.shape[0]
    layer = np.rint((q[:, 2] - 2.0) / (L.A0_CU / 2)).astype(int)
    s = L.System(q, np.full(n, 0.1), np.where(layer == 0, 1.0, 0.5), np.full(n, L.HOST_VAC, np.int8),
                 (4 * L.A0_CU, 4 * L.A0_CU, 4 * L.A0_CU + 4.0), (True, True, False), 1000.0, "held_slab")
    res = np.where((layer == 0) | (layer == layer.max()), O.RES_FIX_X, O.RES_NONE).astype(np.int8)
    res_val = np.where(layer == 0, 1.0, 0.0)
    p = dict(L.DEFAULT_PARAMS, max_relax=20)
    plan = mx.Plan([s], EAM, p)
    st = _with_reservoirs(mx, plan, [s], res, res_val)
    out, ws = plan.out(), plan.workspace()
    plan.run(st, out, ws, 3, use_graph=True)
    torch.cuda.synchronize()
    r = O.run(EAM, p, s.box, s.periodic, s.T, 3, s.q, s.sigma, s.x, s.type, res=res, res_val=res_val)
    g = gpu_arrays(plan, st, out)
    assert rel_err(g["x"], r["x"], 1e-30) < 1e-10
    up = plan.scalars(out)[0, mx.S_RESERVOIR]
    say(f"    uptake {up:.6e} vs oracle {r['uptake'][-1]:.6e}")
    assert up == pytest.approx(r["uptake"][-1], rel=1e-10, abs=1e-14 * s.n)


def test_reservoir_pointers_must_come_in_pairs(mx):
    s = L.config0(0).systems[0]
    plan = mx.Plan([s], EAM, L.DEFAULT_PARAMS)
    st = plan.state([s])
    st.reservoir = torch.zeros(s.n, dtype=torch.int8, device="cuda")
    with pytest.raises(mx.MxeError, match="res_value"):
        plan.evaluate(st, plan.out(), plan.workspace())
