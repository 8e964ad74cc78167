"""Pins of the oracle's occupancy-weighted functional (App. B.2.1).

The functional of Eqs. (EAM-Substitutional-ave) and
(EAM-density-substitutional-ave), with the Taylor embedding of App. B.2,
Eq. (F_taylor_mxe), is fixed here by things other than the oracle itself:

* an independent NumPy statement of the equations over species pairs
  (tests/occupancy_reference.py: per-site species fractions x_ik, shape classes
  by species pair, numpy's Gauss-Hermite nodes), compared element by element
  on alloy, vacancy and interstitial systems with fractional occupancies; mu and
  the gradients come from complex-step derivatives of that statement, not from
  a retyped derivative formula;
* the discrete limit: with every x in {0, 1} and sigma -> 0 the functional must
  be plain EAM of the discrete configuration (species-resolved pair and
  embedding functions, vacancies removed), and pure-A / pure-B crystals the
  closed-form FCC shell sums;
* the meaning of the occupancy average: the pair energy and the densities are
  the expectations over independent site occupations with probabilities x_ik,
  enumerated over every configuration of a small cluster;
* the quadrature: the same functional with a 40-point-per-axis rule (the
  Gaussian average itself, up to 1e-9) differs from the 27-node rule by the
  rule's error, which shrinks as sigma shrinks.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L
from occupancy_reference import (KB, functional, gradient, chemical_potentials, pair_tables,
                                 species_fractions, shape_class)

EAM = L.DEFAULT_EAM
A0 = L.A0_CU


def _oracle(s, eam=EAM):
    return O.evaluate(eam, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)


def _rel(a, b, floor=1e-30):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))


def _alloy():
    return L.jitter(L.alloy_bulk(4, 0.3, 900.0, 5), 31, xr=(0.05, 0.95))


def _vacancy():
    s = L.jitter(L.vacancy_bulk(4, 0, 800.0, 0), 32, xr=(0.3, 1.0))
    rng = np.random.default_rng(33)
    s.x[rng.choice(s.n, 5, replace=False)] = 0.0  # vacancies beside partly filled sites
    s.x[rng.choice(s.n, 5, replace=False)] = 1.0
    return s


def _wire():
    s = L.jitter(L.nanowire(radius=6.0, n_axial=4, T=700.0), 34, xr=(0.05, 0.9))
    return s


SYSTEMS = {"alloy": _alloy, "vacancy": _vacancy, "wire_interstitial": _wire}


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_functional_matches_independent_statement(name):
    """F, e_i, rho_bar, rho0 element by element against the species-pair statement."""
    s = SYSTEMS[name]()
    o = _oracle(s)
    r = functional(EAM, s)
    assert abs(o["F"] - r["F"]) < 1e-12 * abs(r["F"]), (name, o["F"], r["F"])
    assert _rel(o["e_site"], r["e_site"]) < 1e-12, name
    host = s.type != L.INTERSTITIAL  # interstitial sites carry no embedding: compare anyway
    assert _rel(o["rho_bar"][host], r["rho_bar"][host]) < 1e-12, name
    assert _rel(o["rho0"][host], r["rho0"][host]) < 1e-12, name
    if np.any(~host):
        assert _rel(o["rho_bar"][~host], r["rho_bar"][~host]) < 1e-12, name
        assert _rel(o["rho0"][~host], r["rho0"][~host]) < 1e-12, name


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_mu_is_complex_step_derivative_of_independent_statement(name):
    """mu_i = d(F - E_mix)/dx_i, with the derivative taken numerically exactly."""
    s = SYSTEMS[name]()
    o = _oracle(s)
    mu = chemical_potentials(EAM, s)
    mob = s.type != L.HOST_FIXED
    assert _rel(o["mu"][mob], mu[mob]) < 1e-12, name
    assert np.all(o["mu"][~mob] == 0.0)


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_gradient_is_complex_step_derivative_of_independent_statement(name):
    s = SYSTEMS[name]()
    o = _oracle(s)
    rng = np.random.default_rng(7)
    sites = list(rng.choice(s.n, 6, replace=False))
    if name == "wire_interstitial":  # include interstitial sites and fixed hosts
        sites += list(np.where(s.type == L.INTERSTITIAL)[0][:3])
        sites += list(np.where(s.type == L.HOST_FIXED)[0][:2])
    g = gradient(EAM, s, sites)
    scale = np.abs(o["grad"]).max()
    assert np.abs(o["grad"][sites] - g).max() < 1e-11 * scale, name


# ---------------------------------------------------------------------------
# Discrete limit: x in {0, 1}, sigma -> 0 is plain EAM of the configuration.
# ---------------------------------------------------------------------------
def _g(r, re, a):
    """Radial shape with the taper, written out again for the plain EAM sums."""
    r = np.asarray(r, dtype=float)
    t = np.clip((r - EAM["r_s"]) / (EAM["r_c"] - EAM["r_s"]), 0.0, 1.0)
    S = 0.5 * (1.0 + np.cos(np.pi * t))
    return np.where(r >= EAM["r_c"], 0.0, np.exp(-a * (r / re - 1.0)) * S)


# species of the discrete configuration: 0 A, 1 B, 2 S, -1 nothing
def _species(s):
    sp = np.full(s.n, -1)
    on = s.x > 0.5
    sp[(s.type == L.HOST_VAC) & on] = 0
    sp[(s.type == L.ALLOY) & ~on] = 0
    sp[(s.type == L.ALLOY) & on] = 1
    sp[(s.type == L.INTERSTITIAL) & on] = 2
    sp[s.type == L.HOST_FIXED] = 0
    return sp


def plain_eam(s):
    """Plain EAM of the atoms present: per-atom energy 1/2 sum phi_kl + F_k(rho).

    phi_kl = a_kl exp(-alpha (r/r_e - 1)) S(r) with the host-host shape for A, B
    pairs and the host-solute shape for pairs with one S (no S-S pair);
    rho = sum_l b_l f(r) with the shape of the pair's class; F_k = -c_k sqrt(rho)."""
    sp = _species(s)
    atoms = np.where(sp >= 0)[0]
    q = s.q[atoms]
    d = q[None, :, :] - q[:, None, :]
    for a in range(3):
        if s.periodic[a]:
            d[..., a] -= s.box[a] * np.round(d[..., a] / s.box[a])
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, 1e9)
    k = sp[atoms]
    solute = (k[:, None] == 2).astype(int) + (k[None, :] == 2).astype(int)
    a_kl = np.asarray(EAM["pair_a"])[k[:, None], k[None, :]]
    b = np.asarray(EAM["emit_b"])[k]
    c = np.asarray(EAM["embed_c"])[k]
    phi = np.where(solute == 0, _g(r, 2.556, 8.0), _g(r, 1.8, 5.0))
    f = np.where(solute == 0, _g(r, 2.556, 6.0), _g(r, 1.8, 4.0))
    phi = np.where(solute == 2, 0.0, a_kl * phi)
    f = np.where(solute == 2, 0.0, f)
    rho = (f * b[None, :]).sum(1)
    e = 0.5 * phi.sum(1) - c * np.sqrt(rho)
    return atoms, e, rho


def _discrete_cases():
    rng = np.random.default_rng(40)
    # a single B substituted into A
    s = L.alloy_bulk(4, 0.0, 900.0, 0)
    s.x[:] = 0.0
    s.x[37] = 1.0
    yield "B_in_A", s
    # ordered L1_0 AB: the (001) planes alternate A and B
    s = L.alloy_bulk(4, 0.0, 900.0, 0)
    s.x = np.where(np.isclose(np.mod(s.q[:, 2], A0), 0.0), 0.0, 1.0)
    yield "L10_AB", s
    # random AB
    s = L.alloy_bulk(4, 0.0, 900.0, 0)
    s.x = (rng.random(s.n) < 0.4).astype(float)
    yield "random_AB", s
    # vacancies: x = 0 removes the atom
    s = L.vacancy_bulk(4, 9, 800.0, 41)
    yield "vacancies", s
    # host wire with some occupied octahedral sites
    s = L.nanowire(radius=6.0, n_axial=4, T=700.0)
    inter = np.where(s.type == L.INTERSTITIAL)[0]
    s.x[:] = np.where(s.type == L.HOST_FIXED, 1.0, 0.0)
    s.x[rng.choice(inter, 7, replace=False)] = 1.0
    yield "wire_octahedral", s


@pytest.mark.parametrize("name,s", list(_discrete_cases()))
def test_discrete_occupancy_at_zero_width_is_plain_eam(name, s):
    sig = 1e-7
    s.sigma = np.full(s.n, sig)
    o = _oracle(s)
    kT = KB * s.T
    w = np.where((s.type == L.HOST_VAC) | (s.type == L.INTERSTITIAL), s.x, 1.0)
    e_vib = -3.0 * kT * w * math.log(sig)
    atoms, e, rho = plain_eam(s)
    e_or = o["e_site"] - e_vib
    assert abs(e_or.sum() - e.sum()) < 1e-12 * abs(e.sum()) * 10, (name, e_or.sum(), e.sum())
    assert np.abs(e_or[atoms] - e).max() < 1e-11, name
    empty = np.setdiff1d(np.arange(s.n), atoms)
    assert np.all(np.abs(e_or[empty]) < 1e-12), name  # an empty site holds no energy
    host_atoms = atoms[s.type[atoms] != L.INTERSTITIAL]
    sel = np.isin(atoms, host_atoms)
    assert np.abs(o["rho0"][host_atoms] - rho[sel]).max() < 1e-12 * rho.max(), name
    assert np.abs(o["rho_bar"][host_atoms] - rho[sel]).max() < 1e-9 * rho.max(), name


SHELLS = [(A0 / math.sqrt(2), 12), (A0, 6), (A0 * math.sqrt(1.5), 24), (A0 * math.sqrt(2), 12)]


@pytest.mark.parametrize("xB,a_pair,b,c", [(0.0, 0.3, 1.0, 1.0), (1.0, 0.36, 1.2, 1.1)])
def test_pure_alloy_crystal_is_closed_form_shell_sum(xB, a_pair, b, c):
    """x_B = 0 and 1 on an ALLOY crystal: pure A and pure B per-site energies."""
    s = L.alloy_bulk(4, xB, 900.0, 0)
    s.x[:] = xB
    sig = 1e-7
    s.sigma = np.full(s.n, sig)
    o = _oracle(s)
    phi = sum(n * a_pair * _g(r, 2.556, 8.0) for r, n in SHELLS)
    rho = sum(n * b * _g(r, 2.556, 6.0) for r, n in SHELLS)
    e = 0.5 * phi - c * math.sqrt(rho)
    e_vib = -3.0 * KB * s.T * math.log(sig)
    assert np.abs(o["e_site"] - e_vib - e).max() < 1e-11
    assert np.abs(o["rho0"] - rho).max() < 1e-12 * rho


# ---------------------------------------------------------------------------
# The occupancy average is the expectation over independent site occupations.
# ---------------------------------------------------------------------------
def test_occupancy_average_is_expectation_over_configurations():
    s = L.jitter(L.cluster(1), 50, xr=(0.1, 0.9))  # 13 sites, 8192 configurations
    s.type[:] = L.ALLOY
    s.type[[2, 5, 11]] = L.HOST_VAC  # mixed: A/B sites and A/vacancy sites
    tab = pair_tables(EAM, s.q, s.sigma, s.box, s.periodic)
    r = functional(EAM, s, tables=tab)
    o = _oracle(s)
    a = np.asarray(EAM["pair_a"])
    b = np.asarray(EAM["emit_b"])
    cvec = np.asarray(EAM["embed_c"])
    n = s.n
    E_pair = 0.0
    rho = np.zeros(n)
    c_mean = np.zeros(n)
    for bits in itertools.product((0, 1), repeat=n):
        bits = np.array(bits)
        # species of each site in this configuration (-1: empty)
        sp = np.where(s.type == L.ALLOY, bits, np.where(bits == 1, 0, -1))
        p = np.prod(np.where(bits == 1, s.x, 1.0 - s.x))
        occ = sp >= 0
        k = np.where(occ, sp, 0)
        cls0_phi, cls0_f = tab[0][0], tab[0][1]
        amp = np.where(occ[:, None] & occ[None, :], a[k[:, None], k[None, :]], 0.0)
        E_pair += p * 0.5 * (amp * cls0_phi).sum()
        rho += p * (cls0_f * np.where(occ, b[k], 0.0)[None, :]).sum(1)
        c_mean += p * np.where(occ, cvec[k], 0.0)
    assert abs(E_pair - r["E_pair"]) < 1e-12 * abs(E_pair)
    assert np.abs(rho - r["rho_bar"]).max() < 1e-12 * rho.max()
    assert np.abs(rho - o["rho_bar"]).max() < 1e-12 * rho.max()
    # the embedding share is the mean embedding strength times the Taylor form at the mean density
    X = species_fractions(s.type, s.x)
    assert np.abs(c_mean - X @ cvec).max() < 1e-14


# ---------------------------------------------------------------------------
# The 27-node rule against the Gaussian average itself.
# ---------------------------------------------------------------------------
def test_rule_error_against_forty_point_average():
    base = L.jitter(L.cluster(1), 60, xr=(0.1, 0.9))
    base.type[:] = L.ALLOY
    errs = []
    for sig in (0.1, 0.05):
        s = base.copy()
        s.sigma = base.sigma * (sig / 0.1)
        o = _oracle(s)
        ref = functional(EAM, s, n_rule=40)
        kT = KB * s.T
        # compare the interaction part (the entropy terms do not involve the rule)
        vib_mix = functional(EAM, s)["E_vib"] + functional(EAM, s)["E_mix"]
        e_int_o = o["F"] - vib_mix
        e_int_r = ref["F"] - ref["E_vib"] - ref["E_mix"]
        errs.append(abs(e_int_o - e_int_r) / abs(e_int_r))
        assert _rel(o["rho_bar"], ref["rho_bar"]) < 2e-4
    assert errs[0] < 2e-5, errs
    assert errs[1] < errs[0] / 8, errs  # the error falls much faster than sigma^2
