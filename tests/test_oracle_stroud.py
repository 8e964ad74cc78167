"""Pins of the oracle's degree-3 phase-average rule (App. A, Eq. QuadRule).

For the N_q = 6 coordinates of a pair the rule has M = 2 N_q = 12 nodes at
+-r on each axis of the scaled coordinates chi = (q - qbar)/(sqrt(2) sigma),
r^2 = N_q / 2, all with the same weight. What fixes it:
  * the node set and weights as the appendix states them;
  * exactness for every polynomial of total degree <= 3 in the six
    coordinates against the closed-form Gaussian moments, and failure at
    degree 4 (so it is the degree-3 rule and not a richer one);
  * pair averages of the potential's analytic shapes converge to a
    40-point-per-axis Gauss-Hermite reference as sigma^4;
  * the rule's own value, gradient and per-end width derivatives agree with
    central differences, and the full free energy's gradients and mu agree
    with finite differences under this rule.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L
from tests.test_oracle_eam import _fd_errors, _systems
from tests.test_oracle_quadrature import _reference_average

EAM3 = dict(L.DEFAULT_EAM, quad_rule=1)


def gauss_moment(p, sig):
    """E[X^p] for X ~ N(0, sig^2)."""
    if p % 2:
        return 0.0
    return float(np.prod(np.arange(p - 1, 0, -2))) * sig ** p if p > 0 else 1.0


def test_nodes_and_weights_follow_the_appendix():
    si, sj = 0.08, 0.13
    off, w = O.stroud_nodes(si, sj)
    assert off.shape == (12, 6) and np.allclose(w, 1.0 / 12.0, rtol=0, atol=1e-16)
    sig = np.array([si] * 3 + [sj] * 3)
    chi = off / (math.sqrt(2.0) * sig)
    # each node lies on one coordinate axis at |chi| = r, r^2 = N_q / 2 = 3
    assert np.all((np.abs(chi) > 1e-12).sum(axis=1) == 1)
    assert np.allclose((chi ** 2).sum(axis=1), 3.0, rtol=0, atol=1e-13)
    # both signs on every axis
    for a in range(6):
        v = chi[np.abs(chi[:, a]) > 0, a]
        assert sorted(np.sign(v)) == [-1.0, 1.0]


def test_exact_to_total_degree_three_only():
    si, sj = 0.07, 0.11
    off, w = O.stroud_nodes(si, sj)
    sig = [si] * 3 + [sj] * 3
    for deg in range(4):
        for combo in itertools.combinations_with_replacement(range(6), deg):
            p = np.bincount(np.array(combo, dtype=int), minlength=6) if deg else np.zeros(6, int)
            got = float(np.sum(w * np.prod(off ** p, axis=1)))
            ref = float(np.prod([gauss_moment(int(p[a]), sig[a]) for a in range(6)]))
            assert abs(got - ref) < 1e-16 + 1e-12 * abs(ref), (combo, got, ref)
    # degree 4 fails: E[x^4] = 3 s^4 but the rule gives 6 s^4; E[x_i^2 x_j^2] = si^2 sj^2, rule 0
    assert abs(np.sum(w * off[:, 0] ** 4) - 6 * si ** 4) < 1e-18
    assert np.sum(w * off[:, 0] ** 2 * off[:, 3] ** 2) == 0.0


@pytest.mark.parametrize("rbar", [(2.5, 0.0, 0.0), (2.556 / math.sqrt(2), 2.556 / math.sqrt(2), 0.0)])
def test_pair_average_error_scales_as_sigma4(rbar):
    """Away from the taper the shapes are analytic: a degree-3 rule errs as sigma^4."""
    rbar = np.array(rbar)
    errs = []
    for sc in (0.06, 0.03):
        si, sj = sc, 1.3 * sc
        s = math.hypot(si, sj)
        m = O.pair_moments(EAM3, 0, rbar, si, sj)
        e = []
        for val, a in ((m[0], 8.0), (m[5], 6.0)):
            ref = _reference_average(rbar, s, 2.556, a)
            e.append(abs(val - ref))
            assert abs(val - ref) < 1e-3 * abs(ref)
        errs.append(e)
    for k in range(2):
        ratio = errs[0][k] / errs[1][k]
        assert 14.0 < ratio < 18.5, ratio  # 2^4 = 16


def test_product_rule_is_more_accurate_at_the_same_width():
    rbar = np.array([2.3, 0.9, -0.4])
    si = sj = 0.1
    s = math.hypot(si, sj)
    ref = _reference_average(rbar, s, 2.556, 8.0)
    e27 = abs(O.pair_moments(L.DEFAULT_EAM, 0, rbar, si, sj)[0] - ref)
    e12 = abs(O.pair_moments(EAM3, 0, rbar, si, sj)[0] - ref)
    assert e27 < e12


def test_moment_derivatives_match_finite_differences():
    rng = np.random.default_rng(11)
    h = 1e-6
    for cls in (0, 1):
        for _ in range(6):
            rbar = rng.normal(size=3)
            rbar *= rng.uniform(2.0, 5.2) / np.linalg.norm(rbar)
            si, sj = rng.uniform(0.06, 0.15, 2)
            m = O.pair_moments(EAM3, cls, rbar, si, sj)
            for a in range(3):
                e = np.zeros(3)
                e[a] = h
                p = O.pair_moments(EAM3, cls, rbar + e, si, sj)
                q = O.pair_moments(EAM3, cls, rbar - e, si, sj)
                for base, grad in ((0, 1), (5, 6), (10, 11)):
                    fd = (p[base] - q[base]) / (2 * h)
                    assert abs(fd - m[grad + a]) < 1e-7 * max(1.0, abs(m[grad + a])), (cls, a, base)
            for which, (dphi, df) in ((0, (4, 9)), (1, (14, 15))):
                dp = np.array([h, 0.0]) if which == 0 else np.array([0.0, h])
                p = O.pair_moments(EAM3, cls, rbar, si + dp[0], sj + dp[1])
                q = O.pair_moments(EAM3, cls, rbar, si - dp[0], sj - dp[1])
                assert abs((p[0] - q[0]) / (2 * h) - m[dphi]) < 1e-7
                assert abs((p[5] - q[5]) / (2 * h) - m[df]) < 1e-7
                assert p[10] == q[10] == m[10]


def test_equal_widths_make_the_ends_symmetric():
    """Swapping the ends (rbar -> -rbar, sigma_i <-> sigma_j) swaps the width derivatives."""
    rbar = np.array([2.1, -1.2, 0.7])
    a = O.pair_moments(EAM3, 0, rbar, 0.09, 0.12)
    b = O.pair_moments(EAM3, 0, -rbar, 0.12, 0.09)
    assert abs(a[0] - b[0]) < 1e-15 and abs(a[5] - b[5]) < 1e-15
    assert np.allclose(a[1:4], -b[1:4], rtol=0, atol=1e-15)
    assert abs(a[4] - b[14]) < 1e-15 and abs(a[14] - b[4]) < 1e-15
    assert abs(a[9] - b[15]) < 1e-15 and abs(a[15] - b[9]) < 1e-15


@pytest.mark.parametrize("name,sys_", list(_systems()))
def test_gradients_and_mu_match_finite_differences_degree3(name, sys_):
    err_g, err_mu, _ = _fd_errors(sys_, eam=EAM3)
    assert err_g < 1e-7, (name, err_g)
    assert err_mu < 1e-7, (name, err_mu)
