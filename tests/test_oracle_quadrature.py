"""Pins of the oracle's quadrature and pair averages (App. A, Eq. QuadRule).

The 3-point-per-axis Gauss-Hermite product rule integrates every polynomial of
per-axis degree <= 5 exactly against the standard normal density. Its nodes
are checked against numpy's Gauss-Hermite routine, its moments against the
normal distribution's, and its pair averages against a 40-point-per-axis
reference, whose difference must shrink as s^6.
"""
import itertools
import math

import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss

import oracle as O
from paper_1910_01235_amd.lattice import DEFAULT_EAM

EAM = DEFAULT_EAM


def normal_moment(p):
    """E[Z^p] for Z ~ N(0,1): (p-1)!! for even p, 0 for odd p."""
    if p % 2:
        return 0.0
    return float(np.prod(np.arange(p - 1, 0, -2))) if p > 0 else 1.0


def test_nodes_match_numpy_gauss_hermite():
    z, w = O.quadrature()
    t, wt = hermegauss(3)
    wt = wt / wt.sum()
    ref = sorted((tuple(np.round([t[a], t[b], t[c]], 14)), wt[a] * wt[b] * wt[c])
                 for a, b, c in itertools.product(range(3), repeat=3))
    got = sorted((tuple(np.round(z[k], 14)), w[k]) for k in range(27))
    for (pr, wr), (pg, wg) in zip(ref, got):
        assert np.allclose(pr, pg, atol=1e-13)
        assert abs(wr - wg) < 1e-15


def test_moments_exact_to_degree_five_per_axis():
    z, w = O.quadrature()
    for px, py, pz in itertools.product(range(6), repeat=3):
        got = np.sum(w * z[:, 0] ** px * z[:, 1] ** py * z[:, 2] ** pz)
        ref = normal_moment(px) * normal_moment(py) * normal_moment(pz)
        assert abs(got - ref) < 1e-12, (px, py, pz, got, ref)
    # degree 6 per axis is not exact: E[Z^6] = 15, the rule gives 9
    assert abs(np.sum(w * z[:, 0] ** 6) - 9.0) < 1e-12


def _shape(r, re, a):
    """The potential's radial shape (input model): exp(-a (r/re - 1)) * taper."""
    r = np.asarray(r, dtype=float)
    ex = np.exp(-a * (r / re - 1.0))
    t = np.clip((r - EAM["r_s"]) / (EAM["r_c"] - EAM["r_s"]), 0.0, 1.0)
    S = np.where(r <= EAM["r_s"], 1.0, 0.5 * (1.0 + np.cos(np.pi * t)))
    return np.where(r >= EAM["r_c"], 0.0, ex * S)


def _reference_average(rbar, s, re, a, npts=40):
    t, wt = hermegauss(npts)
    wt = wt / wt.sum()
    X, Y, Z = np.meshgrid(t, t, t, indexing="ij")
    W = wt[:, None, None] * wt[None, :, None] * wt[None, None, :]
    d = np.stack([rbar[0] + s * X, rbar[1] + s * Y, rbar[2] + s * Z])
    r = np.sqrt((d ** 2).sum(0))
    return float((W * _shape(r, re, a)).sum())


@pytest.mark.parametrize("rbar", [(2.5, 0.0, 0.0), (2.556 / math.sqrt(2), 2.556 / math.sqrt(2), 0.0)])
def test_pair_average_error_scales_as_s6(rbar):
    """Away from the taper the shape is analytic: the rule's error is O(s^6)."""
    rbar = np.array(rbar)
    errs = []
    for s in (0.06, 0.03):
        m = O.pair_average(EAM, 0, rbar, s)
        ref_phi = _reference_average(rbar, s, 2.556, 8.0)
        ref_f = _reference_average(rbar, s, 2.556, 6.0)
        errs.append((abs(m[0] - ref_phi), abs(m[5] - ref_f)))
        assert abs(m[0] - ref_phi) < 1e-4 * abs(ref_phi)
    for k in range(2):
        ratio = errs[0][k] / errs[1][k]
        assert 55.0 < ratio < 75.0, ratio  # 2^6 = 64


def test_pair_average_gradients_match_finite_differences():
    """grad<g> and d<g>/ds of the rule are the derivatives of its own average."""
    rng = np.random.default_rng(7)
    for cls in (0, 1):
        for _ in range(6):
            rbar = rng.normal(size=3)
            rbar *= rng.uniform(2.0, 5.2) / np.linalg.norm(rbar)
            s = rng.uniform(0.08, 0.2)
            m = O.pair_average(EAM, cls, rbar, s)
            h = 1e-6
            for a in range(3):
                e = np.zeros(3)
                e[a] = h
                p = O.pair_average(EAM, cls, rbar + e, s)
                q = O.pair_average(EAM, cls, rbar - e, s)
                for base, grad in ((0, 1), (5, 6), (10, 11)):
                    fd = (p[base] - q[base]) / (2 * h)
                    assert abs(fd - m[grad + a]) < 1e-7 * max(1.0, abs(m[grad + a])), (cls, a, base)
            p = O.pair_average(EAM, cls, rbar, s + h)
            q = O.pair_average(EAM, cls, rbar, s - h)
            assert abs((p[0] - q[0]) / (2 * h) - m[4]) < 1e-7
            assert abs((p[5] - q[5]) / (2 * h) - m[9]) < 1e-7
            # the density at mean positions does not depend on s
            assert p[10] == q[10] == m[10]


def test_centre_value_is_shape_at_mean_distance():
    rbar = np.array([2.1, 1.2, -0.4])
    m = O.pair_average(EAM, 0, rbar, 0.1)
    g, _ = O.shape(EAM, float(np.linalg.norm(rbar)), 2.556, 6.0)
    assert m[10] == g
    assert abs(g - _shape(np.linalg.norm(rbar), 2.556, 6.0)) < 1e-15


def test_pair_beyond_reach_is_zero():
    """All nodes lie within 3 s of the mean: |rbar| >= r_c + 3 s gives zero."""
    s = 0.15
    rbar = np.array([EAM["r_c"] + 3 * s + 1e-9, 0.0, 0.0])
    assert np.all(O.pair_average(EAM, 0, rbar, s)[:10] == 0.0)
    rbar = np.array([EAM["r_c"] + 3 * s - 1e-3, 0.0, 0.0]) / math.sqrt(1.0)
    # the corner node (-1,-1,-1) direction only reaches inside along a diagonal
    rd = np.ones(3) / math.sqrt(3) * (EAM["r_c"] + 3 * s - 1e-3)
    assert O.pair_average(EAM, 0, rd, s)[0] > 0.0


def test_taper_is_c1():
    re, a = 2.556, 8.0
    for r0 in (EAM["r_s"], EAM["r_c"]):
        gl, dgl = O.shape(EAM, r0 - 1e-9, re, a)
        gr, dgr = O.shape(EAM, r0 + 1e-9, re, a)
        assert abs(gl - gr) < 1e-10 and abs(dgl - dgr) < 1e-8
    g, dg = O.shape(EAM, 4.7, re, a)
    h = 1e-6
    fd = (O.shape(EAM, 4.7 + h, re, a)[0] - O.shape(EAM, 4.7 - h, re, a)[0]) / (2 * h)
    assert abs(fd - dg) < 1e-9
