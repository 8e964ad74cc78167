"""GPU path with the degree-3 phase-average rule (App. A, Eq. QuadRule) against the oracle.

Same bars as the product rule: FP64 1e-10 normwise relative, FP32-mixed 1e-5,
sum x conserved to 1e-12; full size on sampled sites.
"""
import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L
from tests.gpu_common import eval_errors, gpu_arrays, oracle_eval, parity_systems, rel_err, say
from tests.test_gpu_fullsize import _sample

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EAM3 = dict(L.DEFAULT_EAM, quad_rule=1)
P = dict(L.DEFAULT_PARAMS)


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    return mxe


def _kmax(s):
    return 160 if (s.type == L.INTERSTITIAL).any() else 96


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,s", parity_systems(), ids=[n for n, _ in parity_systems()])
def test_evaluate_degree3(mx, name, s, prec):
    say(f"[gpu] evaluate degree-3 {prec} {name} n={s.n}")
    plan = mx.Plan([s], EAM3, P, precision=prec, k_max=_kmax(s))
    assert plan.params.quad_rule == mx.QUAD_DEGREE3
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    sc = plan.scalars(out)[0]
    assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0, sc
    o = oracle_eval(EAM3, s)
    errs = eval_errors(gpu_arrays(plan, st, out), o)
    say(f"    errors {errs}")
    tol = 1e-10 if prec == "fp64" else 1e-5
    for k, v in errs.items():
        assert v < tol, (k, v)
    assert abs(sc[mx.S_F] - o["F"]) < tol * abs(o["F"])


def test_rules_differ_and_product_rule_unchanged(mx):
    """The rule switch changes the physics (by O(sigma^4)), and the default stays the product rule."""
    s = parity_systems()[1][1]
    res = {}
    for rule, eam in ((0, L.DEFAULT_EAM), (1, EAM3)):
        plan = mx.Plan([s], eam, P)
        st, out, ws = plan.state([s]), plan.out(), plan.workspace()
        plan.evaluate(st, out, ws)
        torch.cuda.synchronize()
        res[rule] = gpu_arrays(plan, st, out)
    o0 = oracle_eval(L.DEFAULT_EAM, s)
    assert rel_err(res[0]["force"], o0["force"], 1e-2) < 1e-10
    d = rel_err(res[1]["force"], res[0]["force"], 1e-2)
    assert 1e-6 < d < 1e-1, d


@pytest.mark.parametrize("use_graph", [False, True])
def test_run_c0_degree3_matches_oracle(mx, use_graph):
    w = L.config0(0)
    s = w.systems[0]
    n_steps = 4
    say(f"[gpu] run c0 degree-3 {n_steps} steps graph={use_graph}")
    plan = mx.Plan([s], EAM3, w.params)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, n_steps, use_graph=use_graph)
    torch.cuda.synchronize()
    r = O.run(EAM3, w.params, s.box, s.periodic, s.T, n_steps, s.q, s.sigma, s.x, s.type)
    g = gpu_arrays(plan, st, out)
    sc = plan.scalars(out)[0]
    say(f"    x err {rel_err(g['x'], r['x'], 1e-30)} updates {sc[mx.S_UPDATES]} vs {r['updates'][-1]}")
    assert int(sc[mx.S_UPDATES]) == int(r["updates"][-1])
    assert rel_err(g["x"], r["x"], 1e-30) < 1e-10
    assert rel_err(g["sigma"], r["sigma"], 1e-30) < 1e-10
    assert sc[mx.S_TIME] == pytest.approx(r["t"], rel=1e-10)
    assert abs(sc[mx.S_SUMX] - s.x.sum()) < 1e-12 * s.x.sum()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_degree3_sampled(mx, prec):
    w = L.config1(1)
    s = L.jitter(w.systems[0], 11, dq=0.03, sig=(0.09, 0.12))
    say(f"[gpu] full-size c1 degree-3 {prec}")
    plan = mx.Plan([s], EAM3, w.params, precision=prec)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    assert int(plan.scalars(out)[0, mx.S_STATUS]) & mx.FATAL_STATUS == 0
    sel = _sample(s, np.random.default_rng(6))
    o = O.evaluate_sites(EAM3, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, sel)
    f = torch.stack([out.fx, out.fy, out.fz, out.fsigma], 1).cpu().numpy()[sel]
    tol = 1e-10 if prec == "fp64" else 1e-5
    errs = dict(force=rel_err(f, o["force"], 1e-2), mu=rel_err(out.mu.cpu().numpy()[sel], o["mu"], 1e-2),
                rho_bar=rel_err(out.rho_bar.cpu().numpy()[sel], o["rho_bar"], 1.0))
    say(f"    {len(sel)} sampled sites: {errs}")
    for k, v in errs.items():
        assert v < tol, (k, v)
