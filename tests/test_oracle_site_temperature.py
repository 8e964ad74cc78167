"""Pins of the oracle's per-site temperatures (Sec. 2: the beta_i of each site).

With site temperatures T_i the relaxed functional is k_B T (T the system's
reference temperature) times the mean-field free entropy of Eq.
(Grand-Canonical-Free-Energy): each site's energy share carries beta_i, i.e.
the weight theta_i = T / T_i; the chemical potential is mu_i = gamma_i / beta_i;
each hop of the kinetic law runs at its source site's temperature. What fixes it:
  * T_i = T everywhere reproduces the uniform-temperature oracle;
  * T_i = T' everywhere gives exactly the uniform-T' chemical potentials, and
    forces and site shares T / T' times the uniform-T' ones (the functional is
    the uniform one at T', rescaled);
  * gradients and theta_i mu_i equal finite differences of the functional
    under a temperature gradient;
  * two bonded sites at different temperatures relax to the closed-form fixed
    point of the source-site kinetic law, conserving matter.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L

EAM = L.DEFAULT_EAM
P = dict(L.DEFAULT_PARAMS)
KB = 8.617333262e-5


def _sys():
    return L.jitter(L.alloy_bulk(4, 0.3, 900.0, 2), 7, xr=(0.1, 0.9))


def _wire():
    return L.jitter(L.nanowire(radius=6.0, n_axial=4, T=700.0), 15, xr=(0.2, 0.9))


@pytest.mark.parametrize("maker", [_sys, _wire])
def test_uniform_site_temperature_is_the_uniform_oracle(maker):
    s = maker()
    a = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    b = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, T_site=np.full(s.n, s.T))
    for k in ("force", "mu", "e_site", "rho_bar"):
        assert np.allclose(a[k], b[k], rtol=1e-14, atol=1e-15), k
    nb, bl = O.bonds(s.box, s.periodic, s.q, s.type, P["r_bond"])
    r1 = O.master_rates(P, s.box, s.periodic, s.T, s.x, s.type, a["mu"], nb, bl)
    r2 = O.master_rates(P, s.box, s.periodic, s.T, s.x, s.type, a["mu"], nb, bl, T_site=np.full(s.n, s.T))
    assert np.allclose(r1[0], r2[0], rtol=1e-13, atol=1e-14 * np.abs(r1[0]).max())
    assert r1[1] == pytest.approx(r2[1], rel=1e-13)


@pytest.mark.parametrize("maker", [_sys, _wire])
def test_site_temperature_shift_is_the_uniform_functional_rescaled(maker):
    s = maker()
    T2 = 650.0
    lam = s.T / T2
    u = O.evaluate(EAM, s.box, s.periodic, T2, s.q, s.sigma, s.x, s.type)
    v = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, T_site=np.full(s.n, T2))
    mob = s.type != L.HOST_FIXED
    assert np.allclose(v["mu"][mob], u["mu"][mob], rtol=1e-12, atol=1e-13)
    assert np.allclose(v["force"], lam * u["force"], rtol=1e-12, atol=1e-13)
    assert np.allclose(v["e_site"], lam * u["e_site"], rtol=1e-12, atol=1e-13)
    assert v["F"] == pytest.approx(lam * u["F"], rel=1e-12)


def test_gradients_and_mu_match_finite_differences_under_a_gradient():
    s = _wire()
    T_site = 500.0 + 400.0 * (s.q[:, 2] - s.q[:, 2].min()) / np.ptp(s.q[:, 2])
    kT = KB * s.T
    out = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, T_site=T_site)
    theta = s.T / T_site
    h = 1e-5
    rng = np.random.default_rng(4)
    gmax = np.abs(out["grad"]).max()
    for _ in range(10):
        i = int(rng.integers(s.n))
        a = int(rng.integers(4))

        def F(d):
            q = s.q.copy()
            sg = s.sigma.copy()
            if a < 3:
                q[i, a] += d
            else:
                sg[i] += d
            return O.free_energy(EAM, s.box, s.periodic, s.T, q, sg, s.x, s.type, T_site=T_site)

        fd = (F(h) - F(-h)) / (2 * h)
        assert abs(fd - out["grad"][i, a]) < 1e-7 * gmax, (i, a)
    mob = np.where(s.type != L.HOST_FIXED)[0]
    mumax = np.abs(out["mu"][mob] * theta[mob]).max()
    for _ in range(10):
        i = int(rng.choice(mob))

        def G(d):
            x = s.x.copy()
            x[i] += d
            xi = x[i]
            mix = kT * (xi * math.log(xi) + (1 - xi) * math.log(1 - xi))
            return O.free_energy(EAM, s.box, s.periodic, s.T, s.q, s.sigma, x, s.type, T_site=T_site) - mix

        fd = (G(h) - G(-h)) / (2 * h)
        assert abs(fd - theta[i] * out["mu"][i]) < 1e-7 * mumax, i


def test_two_sites_at_different_temperatures_reach_the_closed_form_fixed_point():
    d = L.A0_CU / math.sqrt(2)
    q = np.array([[10.0, 10.0, 10.0], [10.0 + d, 10.0, 10.0]])
    type_ = np.full(2, L.HOST_VAC, np.int8)
    box, per = (40.0, 40.0, 40.0), (False, False, False)
    nb, bl = O.bonds(box, per, q, type_, P["r_bond"])
    assert list(nb) == [1, 1]
    T_site = np.array([700.0, 1100.0])
    mu = np.array([-0.02, 0.03])
    x = np.array([0.3, 0.6])
    for c in (1.0, 0.5):
        p = dict(P, kin_c=c)
        xs = x.copy()
        for _ in range(3000):
            xs, dxdt, dt, _ = O.master_step(p, box, per, 900.0, xs, type_, mu, nb, bl, T_site=T_site)
            assert abs(xs.sum() - x.sum()) < 1e-14
        b1, b2 = 1 / (KB * T_site[0]), 1 / (KB * T_site[1])
        D1 = P["nu0"] * math.exp(-b1 * P["Qm"])
        D2 = P["nu0"] * math.exp(-b2 * P["Qm"])
        # D1 x1 (1 - x2) e^{c b1 (mu1 - mu2)} = D2 x2 (1 - x1) e^{c b2 (mu2 - mu1)}
        K = (D1 / D2) * math.exp(c * (b1 + b2) * (mu[0] - mu[1]))
        got = xs[1] * (1 - xs[0]) / (xs[0] * (1 - xs[1]))
        assert got == pytest.approx(K, rel=1e-10)


def test_run_under_a_temperature_gradient_conserves_matter():
    s = L.jitter(L.vacancy_bulk(4, 2, 900.0, 3), 4, xr=(0.3, 0.9))
    T_site = 700.0 + 300.0 * s.q[:, 0] / s.box[0]
    p = dict(P, max_relax=12)
    r = O.run(EAM, p, s.box, s.periodic, s.T, 3, s.q, s.sigma, s.x, s.type, T_site=T_site)
    for k in range(3):
        assert abs(r["sum_x"][k] - s.x.sum()) < 1e-12 * s.x.sum()
    u = O.run(EAM, p, s.box, s.periodic, s.T, 3, s.q, s.sigma, s.x, s.type)
    assert np.abs(r["x"] - u["x"]).max() > 1e-6  # the gradient changes the kinetics
