"""GPU per-site temperatures (Sec. 2: beta_i per site) against the oracle.

Bars: FP64 1e-10, FP32-mixed 1e-5, sum x conserved to 1e-12; full size on
sampled sites. A uniform T_site reproduces the uniform path bitwise.
"""
import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L
from tests.gpu_common import eval_errors, gpu_arrays, parity_systems, rel_err, say
from tests.test_gpu_fullsize import _sample

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


def _gradient(s, lo=600.0, hi=1100.0, axis=2):
    z = s.q[:, axis]
    return lo + (hi - lo) * (z - z.min()) / max(np.ptp(z), 1e-9)


def _kmax(s):
    return 160 if (s.type == L.INTERSTITIAL).any() else 96


def _state(plan, systems, T_site):
    st = plan.state(systems)
    st.T_site = torch.as_tensor(T_site, dtype=torch.float64, device="cuda")
    return st


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name,s", parity_systems(), ids=[n for n, _ in parity_systems()])
def test_evaluate_site_temperature(mx, name, s, prec):
    T_site = _gradient(s)
    say(f"[gpu] evaluate T_site {prec} {name}")
    plan = mx.Plan([s], EAM, P, precision=prec, k_max=_kmax(s))
    st = _state(plan, [s], T_site)
    out, ws = plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    sc = plan.scalars(out)[0]
    assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0
    o = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, T_site=T_site)
    errs = eval_errors(gpu_arrays(plan, st, out), o)
    tol = 1e-10 if prec == "fp64" else 1e-5
    for k, v in errs.items():
        assert v < tol, (k, v)
    assert abs(sc[mx.S_F] - o["F"]) < tol * abs(o["F"])


def test_uniform_site_temperature_matches_the_uniform_path(mx):
    """Evaluation with T_i = T is bitwise the uniform one (every weight is exactly 1);
    a run agrees to rounding (the flux forms each site's attempt rate on the device)."""
    s = parity_systems()[2][1]
    ev, rn = [], []
    for T_site in (None, np.full(s.n, s.T)):
        plan = mx.Plan([s], EAM, P)
        st = plan.state([s]) if T_site is None else _state(plan, [s], T_site)
        out, ws = plan.out(), plan.workspace()
        plan.evaluate(st, out, ws)
        torch.cuda.synchronize()
        ev.append(gpu_arrays(plan, st, out))
        plan.run(st, out, ws, 2, use_graph=True)
        torch.cuda.synchronize()
        rn.append(gpu_arrays(plan, st, out))
    for k in ("mu", "force", "e_site", "rho_bar"):
        assert np.array_equal(ev[0][k], ev[1][k]), k
    for k in ("x", "sigma"):
        assert rel_err(rn[1][k], rn[0][k], 1e-30) < 1e-12, k


@pytest.mark.parametrize("use_graph", [False, True])
def test_run_under_gradient_matches_oracle(mx, use_graph):
    s = L.jitter(L.vacancy_bulk(5, 3, 900.0, 6), 7, xr=(0.3, 0.9))
    T_site = _gradient(s, 700.0, 1000.0, axis=0)
    p = dict(P, max_relax=20)
    say(f"[gpu] run T gradient graph={use_graph}")
    plan = mx.Plan([s], EAM, p)
    st = _state(plan, [s], T_site)
    out, ws = plan.out(), plan.workspace()
    plan.run(st, out, ws, 4, use_graph=use_graph)
    torch.cuda.synchronize()
    r = O.run(EAM, p, s.box, s.periodic, s.T, 4, s.q, s.sigma, s.x, s.type, T_site=T_site)
    g = gpu_arrays(plan, st, out)
    sc = plan.scalars(out)[0]
    assert int(sc[mx.S_UPDATES]) == int(r["updates"][-1])
    assert rel_err(g["x"], r["x"], 1e-30) < 1e-10
    assert rel_err(g["sigma"], r["sigma"], 1e-30) < 1e-10
    assert sc[mx.S_TIME] == pytest.approx(r["t"], rel=1e-10)
    assert abs(sc[mx.S_SUMX] - s.x.sum()) < 1e-12 * s.x.sum()


def test_full_size_site_temperature_sampled(mx):
    w = L.config1(1)
    s = L.jitter(w.systems[0], 11, dq=0.03, sig=(0.09, 0.12))
    T_site = _gradient(s, 800.0, 1200.0, axis=2)
    say("[gpu] full-size c1 T_site")
    plan = mx.Plan([s], w.eam, w.params)
    st = _state(plan, [s], T_site)
    out, ws = plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    assert int(plan.scalars(out)[0, mx.S_STATUS]) & mx.FATAL_STATUS == 0
    sel = _sample(s, np.random.default_rng(8))
    o = O.evaluate_sites(w.eam, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, sel, T_site=T_site)
    f = torch.stack([out.fx, out.fy, out.fz, out.fsigma], 1).cpu().numpy()[sel]
    assert rel_err(f, o["force"], 1e-2) < 1e-10
    assert rel_err(out.mu.cpu().numpy()[sel], o["mu"], 1e-2) < 1e-10
    assert rel_err(out.e_site.cpu().numpy()[sel], o["e_site"], 1e-2) < 1e-10


def test_non_positive_site_temperature_is_flagged(mx):
    s = L.config0(0).systems[0]
    T_site = np.full(s.n, 800.0)
    T_site[7] = 0.0
    plan = mx.Plan([s], EAM, P)
    st = _state(plan, [s], T_site)
    out, ws = plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    assert int(plan.scalars(out)[0, mx.S_STATUS]) & mx.STAT_TEMP
