"""Point-source vacancy spreading in the oracle (Sec. 5.1; D relation of Sec. 3.1).

Under the linear law (constant mu) the vacancy's second moment grows by
exactly Z b^2 D_ij dt per Euler step, whatever dt the stability rule picks,
which fixes the macroscopic diffusivity D = Z b^2 D_ij / (2 d) = 2 b^2 D_ij of
FCC (reading of the printed relation); the profile then approaches the
continuum point-source solution compared with in Sec. 5.1.
"""
import math

import numpy as np

import oracle as O
from paper_1910_01235_amd import lattice as L
from tests.vacancy_spread import B_NN, Z_FCC, continuum, distances, profile_error, second_moment, \
    single_vacancy

P = dict(L.DEFAULT_PARAMS)
KB = 8.617333262e-5


def _spread(n_steps, n_cells=16, T=1000.0):
    s, v0 = single_vacancy(n_cells, T)
    nb, bl = O.bonds(s.box, s.periodic, s.q, s.type, P["r_bond"])
    mu = np.zeros(s.n)
    x, t = s.x.copy(), 0.0
    moments = []
    for _ in range(n_steps):
        x, _, dt, _ = O.master_step(P, s.box, s.periodic, s.T, x, s.type, mu, nb, bl)
        t += dt
        moments.append((t, second_moment(1.0 - x, distances(s, v0))))
    return s, v0, x, t, moments


def test_second_moment_grows_by_z_b2_dij_dt():
    s, v0, x, t, moments = _spread(20)
    Dij = P["nu0"] * math.exp(-P["Qm"] / (KB * s.T))
    for tk, m2 in moments:
        assert abs(m2 - Z_FCC * B_NN ** 2 * Dij * tk) < 1e-8 * m2
    assert abs((1.0 - x).sum() - 1.0) < 1e-12


def test_profile_approaches_the_continuum_point_source():
    s, v0, x, t, _ = _spread(40)
    Dij = P["nu0"] * math.exp(-P["Qm"] / (KB * s.T))
    D_macro = Z_FCC * B_NN ** 2 * Dij / 6.0
    r = distances(s, v0)
    err = profile_error(1.0 - x, r, t, D_macro)
    assert err < 0.02, err
    # the printed relation 2 d D_ij / (Z b^2) would be wrong by orders of magnitude
    wrong = 6.0 * Dij / (Z_FCC * B_NN ** 2)
    assert profile_error(1.0 - x, r, t, wrong) > 0.5
