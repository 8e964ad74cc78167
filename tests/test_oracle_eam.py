"""Pins of the oracle's mean-field EAM free energy, forces and chemical potentials.

Sec. 2.1 Eq. (Grand-Canonical-Free-Energy) with the EAM thermalisation of
App. B.2 (Eqs. EAM_mxe, F_taylor_mxe) and the occupancy form of App. B.2.1.
What fixes the oracle here, independently of its own formulas:
  * sigma -> 0 reduces to plain EAM: a brute-force plain-EAM sum and the
    closed-form FCC shell sum;
  * the sigma^2 coefficient of E(sigma) equals the Laplacian lattice sum (the
    rule is exact to degree 5, so the harmonic term is exact), which also
    fixes the harmonic width sigma_eq^2 = 3 kT / (2 K);
  * a perfect periodic lattice has zero position forces and uniform sigma
    forces and mu (inversion and translation symmetry);
  * analytic forces, sigma-forces and mu equal central finite differences of
    the free energy.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L

EAM = L.DEFAULT_EAM
KB = 8.617333262e-5
A0 = L.A0_CU
SHELLS = [(A0 / math.sqrt(2), 12), (A0, 6), (A0 * math.sqrt(1.5), 24), (A0 * math.sqrt(2), 12)]


def _shape(r, re, a):
    """Input potential's radial shape: exp(-a (r/re - 1)) with the cosine taper."""
    r = np.asarray(r, dtype=float)
    ex = np.exp(-a * (r / re - 1.0))
    t = np.clip((r - EAM["r_s"]) / (EAM["r_c"] - EAM["r_s"]), 0.0, 1.0)
    S = np.where(r <= EAM["r_s"], 1.0, 0.5 * (1.0 + np.cos(np.pi * t)))
    return np.where(r >= EAM["r_c"], 0.0, ex * S)


def _d_shape(r, re, a, order):
    h = 1e-4
    if order == 1:
        return (_shape(r + h, re, a) - _shape(r - h, re, a)) / (2 * h)
    return (_shape(r + h, re, a) - 2 * _shape(r, re, a) + _shape(r - h, re, a)) / h ** 2


def plain_eam_energy(q, box):
    """Brute-force plain EAM of a pure-A periodic system: sum_{i<j} phi + sum_i F(rho_i)."""
    n = q.shape[0]
    d = q[None, :, :] - q[:, None, :]
    d -= np.asarray(box) * np.round(d / np.asarray(box))
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, 1e9)
    phi = 0.3 * _shape(r, 2.556, 8.0)
    rho = _shape(r, 2.556, 6.0).sum(1)
    return 0.5 * phi.sum() - np.sqrt(rho).sum(), rho


def test_sigma_to_zero_is_plain_eam():
    s = L.vacancy_bulk(4, 0, 800.0, 0)
    sig = 1e-7
    out = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, np.full(s.n, sig), s.x, s.type)
    e_vib = -3 * KB * s.T * s.n * math.log(sig)
    E_brute, rho = plain_eam_energy(s.q, s.box)
    assert abs((out["F"] - e_vib) - E_brute) < 1e-9 * abs(E_brute)
    assert np.allclose(out["rho0"], rho, rtol=1e-13)
    # closed-form FCC shell sum
    phi = sum(n * 0.3 * _shape(r, 2.556, 8.0) for r, n in SHELLS)
    rho0 = sum(n * _shape(r, 2.556, 6.0) for r, n in SHELLS)
    e_site = 0.5 * phi - math.sqrt(rho0)
    assert abs((out["F"] - e_vib) / s.n - e_site) < 1e-11
    assert abs(e_site - (-1.7344951)) < 1e-6
    # interaction part of mu at x = 1: sum phi + F(rho) + F'(rho) rho
    mu_int = phi - math.sqrt(rho0) - 0.5 / math.sqrt(rho0) * rho0
    mu_vib = -3 * KB * s.T * math.log(sig)
    assert np.allclose(out["mu"] - mu_vib, mu_int, atol=1e-9)


def _laplacian_K():
    """E/site = E0 + K sigma^2 + O(sigma^4) on the perfect lattice (all widths equal).

    Each pair has s^2 = 2 sigma^2 and <g(|r + s Z|)> = g + (s^2/2) lap g + O(s^4);
    lap g = g'' + 2 g'/r for a radial function. Embedding: F'(rho0) (rho_bar - rho0)."""
    lap_phi = sum(n * 0.3 * (_d_shape(r, 2.556, 8.0, 2) + 2 * _d_shape(r, 2.556, 8.0, 1) / r)
                  for r, n in SHELLS)
    lap_f = sum(n * (_d_shape(r, 2.556, 6.0, 2) + 2 * _d_shape(r, 2.556, 6.0, 1) / r)
                for r, n in SHELLS)
    rho0 = sum(n * _shape(r, 2.556, 6.0) for r, n in SHELLS)
    return 0.5 * lap_phi + (-0.5 / math.sqrt(rho0)) * lap_f


def test_harmonic_coefficient_matches_lattice_laplacian():
    s = L.vacancy_bulk(4, 0, 800.0, 0)
    K = _laplacian_K()
    e = []
    for sig in (1e-7, 0.01):
        out = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, np.full(s.n, sig), s.x, s.type)
        e.append(out["F"] / s.n + 3 * KB * s.T * math.log(sig))
    K_oracle = (e[1] - e[0]) / 0.01 ** 2
    assert abs(K_oracle - K) < 2e-3 * abs(K), (K_oracle, K)


def test_relaxed_width_matches_harmonic_estimate():
    """At low T the relaxed width obeys 2 K sigma = 3 kT / sigma."""
    T = 40.0
    s = L.vacancy_bulk(4, 0, T, 0)
    K = _laplacian_K()
    sig_eq = math.sqrt(3 * KB * T / (2 * K))
    p = dict(L.DEFAULT_PARAMS, max_relax=400, ftol=1e-6)
    q, sg, info = O.relax(EAM, p, s.box, s.periodic, T, s.q, np.full(s.n, 0.03), s.x, s.type)
    assert info["converged"]
    assert np.ptp(sg) < 1e-9
    assert abs(sg[0] / sig_eq - 1.0) < 5e-3, (sg[0], sig_eq)


@pytest.mark.parametrize("sig", [0.05, 0.1, 0.13])
def test_perfect_lattice_symmetry(sig):
    s = L.vacancy_bulk(4, 0, 1000.0, 0)
    out = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, np.full(s.n, sig), s.x, s.type)
    assert np.abs(out["force"][:, :3]).max() < 1e-12
    assert np.abs(out["grad"][:, :3]).max() < 1e-12
    assert np.ptp(out["force"][:, 3]) < 1e-12
    assert np.ptp(out["mu"]) < 1e-12
    assert np.ptp(out["e_site"]) < 1e-12
    assert abs(out["F"] - out["e_site"].sum()) < 1e-9


def _fd_errors(s, h=1e-5, nprobe=10, seed=0, eam=EAM):
    out = O.evaluate(eam, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    kT = KB * s.T
    rng = np.random.default_rng(seed)
    gmax = np.abs(out["grad"]).max()
    err_g = 0.0
    for _ in range(nprobe):
        i = int(rng.integers(s.n))
        a = int(rng.integers(4))

        def F(delta):
            q = s.q.copy()
            sg = s.sigma.copy()
            if a < 3:
                q[i, a] += delta
            else:
                sg[i] += delta
            return O.free_energy(eam, s.box, s.periodic, s.T, q, sg, s.x, s.type)

        fd = (F(h) - F(-h)) / (2 * h)
        err_g = max(err_g, abs(fd - out["grad"][i, a]) / gmax)
    mob = np.where(s.type != L.HOST_FIXED)[0]
    mumax = np.abs(out["mu"][mob]).max()
    err_mu = 0.0
    for _ in range(nprobe):
        i = int(rng.choice(mob))

        def Fm(delta):
            x = s.x.copy()
            x[i] += delta
            xi = x[i]
            mix = kT * (xi * math.log(xi) + (1 - xi) * math.log(1 - xi))
            return O.free_energy(eam, s.box, s.periodic, s.T, s.q, s.sigma, x, s.type) - mix

        fd = (Fm(h) - Fm(-h)) / (2 * h)
        err_mu = max(err_mu, abs(fd - out["mu"][i]) / mumax)
    return err_g, err_mu, out


def _systems():
    yield "cluster13", L.jitter(L.cluster(1), 11, xr=(0.2, 0.9))
    yield "cluster43", L.jitter(L.cluster(3), 12, xr=(0.2, 0.9))
    yield "periodic256", L.jitter(L.vacancy_bulk(4, 0, 800.0, 0), 13, xr=(0.2, 0.9))
    a = L.jitter(L.alloy_bulk(4, 0.3, 900.0, 0), 14, xr=(0.2, 0.9))
    yield "alloy256", a
    w = L.jitter(L.nanowire(radius=6.0, n_axial=4, T=700.0), 15, xr=(0.2, 0.9))
    yield "wire_interstitial", w


@pytest.mark.parametrize("name,sys_", list(_systems()))
def test_gradients_and_mu_match_finite_differences(name, sys_):
    err_g, err_mu, out = _fd_errors(sys_)
    assert err_g < 1e-7, (name, err_g)
    assert err_mu < 1e-7, (name, err_mu)


def test_normalised_force_is_gradient_over_occupancy():
    s = L.jitter(L.nanowire(radius=6.0, n_axial=4, T=700.0), 21, xr=(0.2, 0.9))
    out = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    w = np.where((s.type == L.HOST_VAC) | (s.type == L.INTERSTITIAL), s.x, 1.0)
    assert np.abs(-out["force"] * w[:, None] - out["grad"]).max() < 1e-13 * np.abs(out["grad"]).max()
    # at an empty site it is the limit of -grad / x as x -> 0 (a "virtual" particle)
    i = int(np.where(s.type == L.INTERSTITIAL)[0][3])
    x0 = s.x.copy()
    x0[i] = 0.0
    out0 = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, x0, s.type)
    eps = 1e-7
    xe = s.x.copy()
    xe[i] = eps
    oute = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, xe, s.type)
    assert np.allclose(out0["force"][i], -oute["grad"][i] / eps, rtol=1e-6, atol=1e-9)
    assert np.all(out0["grad"][i] == 0.0)


def test_vacancy_site_has_zero_raw_force():
    s = L.jitter(L.vacancy_bulk(4, 1, 800.0, 3), 5)
    out = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    v = int(np.where(s.x == 0.0)[0][0])
    assert np.all(out["grad"][v] == 0.0)
    assert np.abs(out["force"][v]).max() > 1e-3  # the virtual atom still relaxes


def test_free_energy_is_sum_of_site_shares():
    s = L.jitter(L.alloy_bulk(4, 0.3, 900.0, 1), 9, xr=(0.1, 0.9))
    out = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    assert abs(out["F"] - out["e_site"].sum()) < 1e-10 * abs(out["F"])


def test_evaluate_sites_equals_full_evaluation():
    s = L.jitter(L.vacancy_bulk(6, 8, 900.0, 2), 4)
    out = O.evaluate(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    sel = np.array([0, 5, 17, 400, s.n - 1])
    sub = O.evaluate_sites(EAM, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type, sel)
    for k in ("rho_bar", "rho0", "mu", "e_site"):
        assert np.allclose(sub[k], out[k][sel], rtol=1e-14, atol=1e-14)
    assert np.allclose(sub["force"], out["force"][sel], rtol=1e-13, atol=1e-14)
