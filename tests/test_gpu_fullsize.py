"""Parity at the full workload sizes, on sampled sites the oracle computes one by one.

The GPU evaluates the whole system in the launch configuration the benchmark
uses; the oracle evaluates a sample of sites (vacancies, their neighbours,
surface and interstitial sites, random sites) from the same state.
"""
import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L
from tests.gpu_common import rel_err, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    return mxe


def _sample(s, rng, n_rand=40):
    pick = list(rng.choice(s.n, n_rand, replace=False))
    vac = np.where((s.x == 0) & (s.type == L.HOST_VAC))[0][:4].tolist()
    pick += vac
    for v in vac[:2]:
        d = s.q - s.q[v]
        per = np.array(s.periodic, dtype=bool)
        d[:, per] -= np.array(s.box)[per] * np.round(d[:, per] / np.array(s.box)[per])
        pick += np.where((np.linalg.norm(d, axis=1) < 3.0) & (np.arange(s.n) != v))[0][:4].tolist()
    if (s.type == L.INTERSTITIAL).any():
        pick += rng.choice(np.where(s.type == L.INTERSTITIAL)[0], 10, replace=False).tolist()
        pick += np.where((s.type == L.INTERSTITIAL) & (s.x > 0))[0][:5].tolist()
    if not all(s.periodic):
        z = s.q[:, 2] if not s.periodic[2] else np.hypot(s.q[:, 0] - s.box[0] / 2, s.q[:, 1] - s.box[1] / 2)
        pick += np.argsort(z)[-6:].tolist()
    return np.unique(np.array(pick, dtype=np.int32))


CASES = [("c1_vacancy_256k", lambda: L.config1(1), "fp64"),
         ("c1_vacancy_256k", lambda: L.config1(1), "fp32"),
         ("c2_alloy_slab_131k", lambda: L.config2(2), "fp32"),
         ("c2_alloy_slab_131k", lambda: L.config2(2), "fp64"),
         ("c3_nanowire_256k", lambda: L.config3(3), "fp32")]


@pytest.mark.parametrize("name,maker,prec", CASES, ids=[f"{c[0]}-{c[2]}" for c in CASES])
def test_full_size_sampled_parity(mx, name, maker, prec):
    w = maker()
    s = L.jitter(w.systems[0], 11, dq=0.03, sig=(0.09, 0.12))
    if name.startswith("c3"):
        s.x = np.where(s.type == L.INTERSTITIAL, np.clip(s.x + 0.05, 0, 1), 1.0)
    say(f"[gpu] full-size {name} {prec} n={s.n}")
    plan = mx.Plan([s], w.eam, w.params, precision=prec)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    sc = plan.scalars(out)[0]
    assert int(sc[mx.S_STATUS]) & mx.FATAL_STATUS == 0, int(sc[mx.S_STATUS])
    sel = _sample(s, np.random.default_rng(5))
    o = O.evaluate_sites(w.eam, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, sel)
    f = torch.stack([out.fx, out.fy, out.fz, out.fsigma], 1).cpu().numpy()[sel]
    tol = 1e-10 if prec == "fp64" else 1e-5
    errs = dict(force=rel_err(f, o["force"], 1e-2), mu=rel_err(out.mu.cpu().numpy()[sel], o["mu"], 1e-2),
                rho_bar=rel_err(out.rho_bar.cpu().numpy()[sel], o["rho_bar"], 1.0),
                e_site=rel_err(out.e_site.cpu().numpy()[sel], o["e_site"], 1e-2))
    say(f"    {len(sel)} sampled sites: {errs}")
    for k, v in errs.items():
        assert v < tol, (k, v)
