"""Pins of the oracle's reservoir sites (Sec. 4: setatomicfraction, setchemicalpotential).

A held-x site is reset to its value after every forward-Euler step (the
fraction fix runs after the transport fix in Algorithm 1); the matter it took
up in the step is booked as reservoir uptake. A held-mu site reports the held
chemical potential after the forces are computed. What fixes them:
  * between two held layers the linear law (constant mu) relaxes to the
    linear profile, and each held layer takes up exactly 4 D dx/dlayer per
    site, the closed-form steady flux of FCC (001) layers (4 bonds per site
    to each neighbouring layer);
  * sum x plus the reservoir uptake is conserved by a full relax + transport run;
  * holding mu changes mu only, and only on mobile held sites.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L

EAM = L.DEFAULT_EAM
P = dict(L.DEFAULT_PARAMS)
KB = 8.617333262e-5


def _slab(nc=3, nz=4):
    q = L.fcc(nc, nc, nz)
    q[:, 2] += 2.0
    n = q.shape[0]
    box = (nc * L.A0_CU, nc * L.A0_CU, nz * L.A0_CU + 4.0)
    layer = np.rint((q[:, 2] - 2.0) / (L.A0_CU / 2)).astype(int)
    return q, n, box, layer


def test_linear_steady_state_between_held_layers():
    q, n, box, layer = _slab()
    top = layer.max()
    T = 900.0
    type_ = np.full(n, L.HOST_VAC, np.int8)
    res = np.where((layer == 0) | (layer == top), O.RES_FIX_X, O.RES_NONE).astype(np.int8)
    res_val = np.where(layer == 0, 1.0, 0.0)
    x = np.full(n, 0.5)
    x[res == O.RES_FIX_X] = res_val[res == O.RES_FIX_X]
    nb, bl = O.bonds(box, (True, True, False), q, type_, P["r_bond"])
    mu = np.zeros(n)  # constant mu: the law is linear, dx_i/dt = D sum_j (x_j - x_i)
    total0 = x.sum()
    uptake = 0.0
    for _ in range(4000):
        x, dxdt, dt, up = O.master_step(P, box, (True, True, False), T, x, type_, mu, nb, bl,
                                        res=res, res_val=res_val)
        uptake += up
        assert abs(x.sum() + uptake - total0) < 1e-11 * total0
    ref = 1.0 - layer / top
    assert np.abs(x - ref).max() < 1e-9
    D = P["nu0"] * math.exp(-P["Qm"] / (KB * T))
    # held sites report their would-be rate: the steady flux 4 D (1/top) per site
    assert np.allclose(dxdt[layer == top], 4 * D / top, rtol=1e-8)
    assert np.allclose(dxdt[layer == 0], -4 * D / top, rtol=1e-8)
    # the two reservoirs exchange equal and opposite amounts at steady state
    assert abs(up) < 1e-9 * n


def test_run_conserves_matter_with_reservoir_uptake():
    s = L.jitter(L.vacancy_bulk(4, 2, 900.0, 3), 4, xr=(0.3, 0.9))
    rng = np.random.default_rng(2)
    res = np.zeros(s.n, np.int8)
    held = rng.choice(s.n, 12, replace=False)
    res[held[:6]] = O.RES_FIX_X
    res[held[6:]] = O.RES_FIX_MU
    res_val = np.zeros(s.n)
    res_val[held[:6]] = rng.uniform(0.0, 1.0, 6)
    r0 = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    res_val[held[6:]] = r0["mu"][held[6:]] + rng.uniform(-0.05, 0.05, 6)
    p = dict(P, max_relax=15)
    r = O.run(EAM, p, s.box, s.periodic, s.T, 4, s.q, s.sigma, s.x, s.type, res=res, res_val=res_val)
    x_start = s.x.copy()
    x_start[held[:6]] = res_val[held[:6]]
    total0 = x_start.sum()
    for k in range(4):
        assert abs(r["sum_x"][k] + r["uptake"][k] - total0) < 1e-12 * total0
    assert np.array_equal(r["x"][held[:6]], res_val[held[:6]])
    assert np.array_equal(r["mu"][held[6:]], res_val[held[6:]])
    assert abs(r["uptake"][-1]) > 0.0


def test_held_mu_changes_only_mu_of_mobile_held_sites():
    s = L.jitter(L.nanowire(radius=6.0, n_axial=4, T=700.0), 15, xr=(0.2, 0.9))
    res = np.zeros(s.n, np.int8)
    inter = np.where(s.type == L.INTERSTITIAL)[0][:5]
    fixed = np.where(s.type == L.HOST_FIXED)[0][:3]
    res[inter] = O.RES_FIX_MU
    res[fixed] = O.RES_FIX_MU
    res_val = np.full(s.n, -2.5)
    a = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    b = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, res=res, res_val=res_val)
    assert np.array_equal(a["force"], b["force"]) and a["F"] == b["F"]
    assert np.all(b["mu"][inter] == -2.5)
    assert np.array_equal(b["mu"][fixed], a["mu"][fixed])  # immobile sites hold no mu
    other = np.setdiff1d(np.arange(s.n), inter)
    assert np.array_equal(a["mu"][other], b["mu"][other])


def test_held_x_is_applied_before_the_first_relaxation():
    s = L.jitter(L.vacancy_bulk(4, 0, 800.0, 1), 2, xr=(0.5, 0.9))
    res = np.zeros(s.n, np.int8)
    res[:8] = O.RES_FIX_X
    res_val = np.zeros(s.n)
    p = dict(P, max_relax=5)
    r = O.run(EAM, p, s.box, s.periodic, s.T, 1, s.q, s.sigma, s.x, s.type, res=res, res_val=res_val)
    x_set = s.x.copy()
    x_set[:8] = 0.0
    r2 = O.run(EAM, p, s.box, s.periodic, s.T, 1, s.q, s.sigma, x_set, s.type, res=res, res_val=res_val)
    assert np.array_equal(r["x"], r2["x"]) and np.array_equal(r["q"], r2["q"])
