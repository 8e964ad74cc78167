"""Pins of the oracle's kinetic law (Sec. 3.1, Eqs. MassTransport, attempt_freq_mass).

  * conservation: the bond flux is antisymmetric, so sum_i dx_i/dt = 0;
  * uniform x on a perfect lattice gives uniform mu and zero flux;
  * linear limit: with mu constant, dx_i/dt = D sum_j (x_j - x_i) exactly, a lattice
    Laplacian; a Fourier mode decays at rate D sum_delta (1 - cos k.delta), whose
    long-wave limit (Z b^2 D / (2 d)) |k|^2 fixes the lattice-to-continuum relation
    of Sec. 3.1 (printed there inverted, as 2 d D_ij / (Z b^2));
  * sign: two sites with fixed mu_1 < mu_2 settle at
    x_2 (1 - x_1) / (x_1 (1 - x_2)) = exp(2 c beta (mu_1 - mu_2)), so the lower-mu site
    holds more matter;
  * the time-step rule keeps x inside [0, 1] whatever the mu field.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L

KB = 8.617333262e-5
P = dict(L.DEFAULT_PARAMS)


def _D(T, p=P):
    return p["nu0"] * math.exp(-p["Qm"] / (KB * T))


def _bulk(n=4, T=800.0):
    s = L.vacancy_bulk(n, 0, T, 0)
    nb, bl = O.bonds(s.box, s.periodic, s.q, s.type, P["r_bond"])
    return s, nb, bl


def test_bonds_are_the_twelve_nearest_neighbours():
    s, nb, bl = _bulk()
    assert np.all(nb == 12)
    for i in (0, 77, 255):
        for j in bl[i, :12]:
            d = s.q[j] - s.q[i]
            d -= np.array(s.box) * np.round(d / np.array(s.box))
            assert abs(np.linalg.norm(d) - L.A0_CU / math.sqrt(2)) < 1e-12


def test_flux_conserves_matter():
    s, nb, bl = _bulk()
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, s.n)
    mu = rng.normal(-1.7, 0.1, s.n)
    dxdt, dt = O.master_rates(P, s.box, s.periodic, s.T, x, s.type, mu, nb, bl)
    scale = np.abs(dxdt).sum()
    assert abs(dxdt.sum()) < 1e-12 * scale


def test_uniform_field_has_zero_flux():
    s, nb, bl = _bulk(T=1000.0)
    out = O.evaluate(L.DEFAULT_EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    dxdt, dt = O.master_rates(P, s.box, s.periodic, s.T, s.x, s.type, out["mu"], nb, bl)
    assert np.abs(dxdt).max() <= 1e-12 * _D(s.T)
    a = L.alloy_bulk(4, 0.07, 900.0, 0)
    a.x[:] = 0.07
    out = O.evaluate(L.DEFAULT_EAM, a.box, a.periodic, a.T, a.q, a.sigma, a.x, a.type)
    dxdt, dt = O.master_rates(P, a.box, a.periodic, a.T, a.x, a.type, out["mu"], nb, bl)
    assert np.abs(dxdt).max() <= 1e-12 * _D(a.T)


def test_constant_mu_gives_lattice_laplacian():
    s, nb, bl = _bulk()
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, s.n)
    mu = np.full(s.n, -1.3)
    dxdt, dt = O.master_rates(P, s.box, s.periodic, s.T, x, s.type, mu, nb, bl)
    D = _D(s.T)
    lap = np.array([D * (x[bl[i, :nb[i]]] - x[i]).sum() for i in range(s.n)])
    assert np.allclose(dxdt, lap, rtol=1e-12, atol=1e-12 * D)


@pytest.mark.parametrize("mode", [(1, 0, 0), (1, 1, 0), (2, 1, 1)])
def test_fourier_mode_decay_rate(mode):
    n = 6
    s, nb, bl = _bulk(n)
    Lb = n * L.A0_CU
    k = 2 * math.pi * np.array(mode) / Lb
    eps = 1e-3
    x = 0.5 + eps * np.cos(s.q @ k)
    mu = np.full(s.n, -1.0)
    dxdt, dt = O.master_rates(P, s.box, s.periodic, s.T, x, s.type, mu, nb, bl)
    b = L.A0_CU / math.sqrt(2)
    deltas = np.array([(a, c, 0) for a in (-1, 1) for c in (-1, 1)] +
                      [(a, 0, c) for a in (-1, 1) for c in (-1, 1)] +
                      [(0, a, c) for a in (-1, 1) for c in (-1, 1)]) * (L.A0_CU / 2)
    rate = _D(s.T) * np.sum(1 - np.cos(deltas @ k))
    assert np.allclose(dxdt, -rate * eps * np.cos(s.q @ k), rtol=1e-9, atol=1e-12 * rate)
    # long-wave limit: D_macro = Z b^2 D_ij / (2 d) = 2 b^2 D_ij for FCC
    kk = 1e-3 * np.array(mode, dtype=float)
    rate_small = _D(s.T) * np.sum(1 - np.cos(deltas @ kk))
    D_macro = 12 * b ** 2 * _D(s.T) / (2 * 3)
    assert abs(rate_small / (D_macro * (kk @ kk)) - 1) < 1e-5


def _two_sites():
    q = np.array([[10.0, 10.0, 10.0], [10.0 + 2.556, 10.0, 10.0]])
    t = np.array([L.ALLOY, L.ALLOY], np.int8)
    box, per = (30.0, 30.0, 30.0), (False, False, False)
    nb, bl = O.bonds(box, per, q, t, P["r_bond"])
    return q, t, box, per, nb, bl


@pytest.mark.parametrize("kin_c", [1.0, 0.5])
def test_two_site_fixed_point(kin_c):
    """Matter flows downhill in mu; the fixed point is exp(2 c beta (mu_1 - mu_2))."""
    q, t, box, per, nb, bl = _two_sites()
    T = 600.0
    p = dict(P, kin_c=kin_c)
    mu = np.array([-1.50, -1.45])
    x = np.array([0.3, 0.3])
    for _ in range(4000):
        dxdt, dt = O.master_rates(p, box, per, T, x, t, mu, nb, bl)
        x = x + dt * dxdt
    assert abs(x.sum() - 0.6) < 1e-12
    ratio = x[1] * (1 - x[0]) / (x[0] * (1 - x[1]))
    target = math.exp(2 * kin_c * (mu[0] - mu[1]) / (KB * T))
    assert abs(ratio / target - 1) < 1e-8
    assert x[0] > x[1]


def test_step_rule_keeps_x_in_unit_interval():
    s, nb, bl = _bulk()
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, s.n)
    x[rng.choice(s.n, 40, replace=False)] = 0.0
    x[rng.choice(s.n, 40, replace=False)] = 1.0
    for it in range(50):
        mu = rng.normal(-1.7, 0.05, s.n)
        mu[rng.choice(s.n, 5, replace=False)] += rng.normal(0, 1.0, 5)  # spikes
        dxdt, dt = O.master_rates(P, s.box, s.periodic, s.T, x, s.type, mu, nb, bl)
        assert dt > 0
        x = x + dt * dxdt
        assert x.min() >= -1e-15 and x.max() <= 1 + 1e-15


def test_arrhenius_rate_sets_time_not_path():
    """With the adaptive step, dt * D is invariant: x(step) does not depend on D."""
    s, nb, bl = _bulk()
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, s.n)
    mu = rng.normal(-1.7, 0.05, s.n)
    d1, dt1 = O.master_rates(P, s.box, s.periodic, s.T, x, s.type, mu, nb, bl)
    p2 = dict(P, Qm=P["Qm"] + 0.1)
    d2, dt2 = O.master_rates(p2, s.box, s.periodic, s.T, x, s.type, mu, nb, bl)
    assert np.allclose(dt1 * d1, dt2 * d2, rtol=1e-10, atol=1e-15)
    assert abs(dt2 / dt1 - math.exp(0.1 / (KB * s.T))) < 1e-9 * dt2 / dt1


def test_run_conserves_total_occupancy():
    w = L.config0(0)
    s = w.systems[0]
    r = O.run(w.eam, w.params, s.box, s.periodic, s.T, 4, s.q, s.sigma, s.x, s.type)
    assert np.all(np.abs(r["sum_x"] - s.x.sum()) < 1e-12 * s.x.sum())
    assert r["x"].min() >= 0.0 and r["x"].max() <= 1.0
    assert np.all(r["dt"] > 0)
    # the vacancy fills from its neighbours
    v = int(np.where(s.x == 0)[0][0])
    assert r["x"][v] > 0.0
