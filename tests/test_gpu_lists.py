"""Index work compared exactly: neighbour rows and kinetic bonds at full size.

The GPU's neighbour rows (Sec. 4, Alg. 1: neighbour lists) and nearest-neighbour
bonds (Sec. 3.1, the bonds of the kinetic law) are read back from the
workspace after a call that built them and compared with the oracle's
neighbour search and bond builder:
* bonds bit-exactly (count and sorted row of every mobile site);
* neighbour rows as sets: a row holds every pair with
  |rbar| < r_c + 3 s_ij + skin - 1e-5 and none with |rbar| >= r_c + 3 s_ij +
  skin + 1e-5 or between two interstitial sites (the list test pads its radius
  by 1e-6 A; pairs in the 2e-5 A band may go either way), rows are strictly
  ascending, and the row lengths are exact where no pair lies in the band.
"""
import numpy as np
import pytest

import oracle as O
from paper_1910_01235_amd import lattice as L

from tests.gpu_common import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BAND = 1e-5


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    torch.cuda.set_device(0)
    return mxe


def _cases():
    w1 = L.config1(1)
    yield "c1_vacancy_256k", w1.systems[0], w1, 0
    yield "c1_jittered", L.jitter(w1.systems[0], 11, dq=0.05, sig=(0.07, 0.13)), w1, 0
    yield "c1_jittered_degree3", L.jitter(w1.systems[0], 12, dq=0.05, sig=(0.07, 0.13)), w1, 1
    w3 = L.config3(3)
    yield "c3_nanowire_256k", w3.systems[0], w3, 0


@pytest.mark.parametrize("name,s,w,rule", list(_cases()), ids=lambda v: v if isinstance(v, str) else "")
def test_lists_and_bonds_match_oracle(mx, name, s, w, rule):
    """The list radius is r_c + skin + the rule's farthest node from the mean:
    3 s_ij (27-node product rule) or sqrt(6) max(sigma_i, sigma_j) (degree-3)."""
    p = w.params
    say(f"[gpu] lists of {name}: {s.n} sites")
    plan = mx.Plan([s], dict(w.eam, quad_rule=rule), p)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, 0, use_graph=False)  # builds lists and bonds, runs no step
    torch.cuda.synchronize()
    assert int(plan.scalars(out)[0, mx.S_STATUS]) & mx.FATAL_STATUS == 0
    g = plan.lists(ws)
    n = s.n
    K = plan.params.k_max

    # bonds: exact
    mobile = s.type != L.HOST_FIXED
    nb, bl = O.bonds(s.box, s.periodic, s.q, s.type, p["r_bond"], bmax=plan.params.bond_max)
    assert np.array_equal(g["bond_count"][mobile], nb[mobile]), name
    B = plan.params.bond_max
    col = np.arange(B)[None, :]
    valid = col < nb[:, None]
    assert np.array_equal(np.where(valid, g["bond"], -1)[mobile], np.where(valid, bl, -1)[mobile])
    say(f"    bonds equal: {int(nb[mobile].sum())} over {int(mobile.sum())} mobile sites")

    # neighbour rows
    cnt = g["nbr_count"]
    assert cnt.min() >= 0 and cnt.max() <= K
    rows = g["nbr"]
    colk = np.arange(K)[None, :]
    inrow = colk < cnt[:, None]
    gi = np.repeat(np.arange(n), cnt)
    gj = rows[inrow]
    assert np.all(np.diff(np.where(inrow, rows, np.iinfo(np.int32).max), axis=1)[inrow[:, 1:]] > 0)
    r_list = w.eam["r_c"] + p.get("skin", 0.15)
    radius = r_list + 3.0 * np.sqrt(2.0) * s.sigma.max() + 2 * BAND
    oc, ol = O.neighbors(s.box, s.periodic, s.q, radius, 1, kmax=256)
    oi = np.repeat(np.arange(n), oc)
    oj = ol[np.arange(256)[None, :] < oc[:, None]]
    d = s.q[oj] - s.q[oi]
    box = np.array(s.box)
    per = np.array(s.periodic, dtype=float)
    d -= per * box * np.round(d / box)
    r = np.sqrt((d * d).sum(1))
    if rule == 0:
        R = r_list + 3.0 * np.sqrt(s.sigma[oi] ** 2 + s.sigma[oj] ** 2)
    else:
        R = r_list + np.sqrt(6.0) * np.maximum(s.sigma[oi], s.sigma[oj])
    ii = (s.type[oi] == L.INTERSTITIAL) & (s.type[oj] == L.INTERSTITIAL)
    must = (r < R - BAND) & ~ii
    allowed = (r < R + BAND) & ~ii
    key = lambda a, b: a.astype(np.int64) * n + b
    gk = key(gi, gj)
    assert np.all(np.isin(key(oi[must], oj[must]), gk)), f"{name}: a required pair is missing"
    assert np.all(np.isin(gk, key(oi[allowed], oj[allowed]))), f"{name}: a row holds a pair it should not"
    band = allowed & ~must
    if not band.any():
        assert np.array_equal(cnt, np.bincount(oi[must], minlength=n)), name
    say(f"    rows equal as sets: {gk.size} entries, {int(band.sum())} pairs in the band, "
        f"row lengths {cnt.min()}..{cnt.max()}")
