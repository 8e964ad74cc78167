"""Oracle neighbour search (cell list vs all pairs) and FIRE relaxation checks.

The relaxer is FIRE (Bitzek et al. 2006) on the occupancy-normalised forces; the
paper relaxes by damped dynamics (Sec. 4). Parity unpinned by the paper: FIRE's
iteration counts are only compared between the oracle and the GPU path. What is
checked here is that relaxation lowers F and reaches the force tolerance.
"""
import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L


def _slab():
    n = 8 * 8 * 6 * 4
    s = L.System(L.fcc(8, 8, 6), np.full(n, 0.1), np.full(n, 0.05), np.full(n, L.ALLOY, np.int8),
                 (8 * L.A0_CU, 8 * L.A0_CU, 6 * L.A0_CU + 20), (True, True, False), 900.0)
    return L.jitter(s, 2, dq=0.2)


@pytest.mark.parametrize("maker", [
    lambda: L.jitter(L.vacancy_bulk(6, 0, 800.0, 0), 1, dq=0.3),
    _slab,
    lambda: L.nanowire(radius=9.0, n_axial=5, T=600.0),
])
def test_cell_list_matches_all_pairs(maker):
    s = maker()
    for radius in (3.09, 5.6):
        c0, l0 = O.neighbors(s.box, s.periodic, s.q, radius, 0)
        c1, l1 = O.neighbors(s.box, s.periodic, s.q, radius, 1)
        assert np.array_equal(c0, c1)
        assert np.array_equal(l0, l1)
    assert c0.max() > 40


def test_small_periodic_box_has_no_duplicate_images():
    s = L.vacancy_bulk(4, 0, 800.0, 0)  # 14.46 A box: 2 cells per axis
    c0, l0 = O.neighbors(s.box, s.periodic, s.q, 5.6, 0)
    c1, l1 = O.neighbors(s.box, s.periodic, s.q, 5.6, 1)
    assert np.all(c0 == 54) and np.array_equal(l0, l1)
    for i in range(s.n):
        row = l1[i, :c1[i]]
        assert len(set(row.tolist())) == row.size


def test_relax_lowers_free_energy_and_converges():
    w = L.config0(0)
    s = w.systems[0]
    p = dict(w.params, max_relax=200)
    F0 = O.free_energy(w.eam, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    q, sg, info = O.relax(w.eam, p, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    assert info["converged"] and info["fmax"] <= p["ftol"]
    assert info["F"] < F0
    assert info["n_evals"] == info["updates"] + 1
    # relaxed widths grow above the initial 0.1 A at 800 K
    assert 0.105 < np.median(sg) < 0.125


def test_relax_cap_is_respected():
    w = L.config0(0)
    s = w.systems[0]
    p = dict(w.params, max_relax=7)
    q, sg, info = O.relax(w.eam, p, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    assert info["updates"] == 7 and info["n_evals"] == 8 and not info["converged"]


def test_sigma_floor():
    s = L.vacancy_bulk(4, 0, 5.0, 0)
    p = dict(L.DEFAULT_PARAMS, max_relax=30, sigma_min=0.02)
    q, sg, info = O.relax(L.DEFAULT_EAM, p, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)
    assert sg.min() >= 0.02
