"""Point-source vacancy spreading on the 256,000-site FCC crystal, whole GPU hot path (Sec. 5.1).

One vacancy at the centre of the 40^3-cell crystal, T = 1000 K; every step
relaxes positions and widths (FIRE) and takes one Euler step of the kinetic law.
  * c = 0 (linear law): the x trajectory does not depend on mu, so the second
    moment must equal Z b^2 D_ij t exactly and the profile must follow the
    continuum point-source solution with D = Z b^2 D_ij / 6.
  * c = 1 (the paper's law): mu at the vacancy lies above the bulk, so the
    vacancy is held at first; at 1000 K it escapes and, once dilute (uniform
    mu), spreads at the lattice rate with a point-source profile; at 600 K it
    stays (the paper reports the same contrast between low and higher T).
    These are properties of the stand-in potential: parity unpinned.
"""
import math

import numpy as np
import pytest

from paper_1910_01235_amd import lattice as L
from tests.gpu_common import say
from tests.vacancy_spread import B_NN, Z_FCC, distances, profile_error, second_moment, single_vacancy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KB = 8.617333262e-5


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    return mxe


def _spread(mx, kin_c, n_steps):
    s, v0 = single_vacancy(40, 1000.0)
    p = dict(L.DEFAULT_PARAMS, max_relax=30, kin_c=kin_c)
    plan = mx.Plan([s], L.DEFAULT_EAM, p)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    r = distances(s, v0)
    hist = []
    for k in range(n_steps):
        plan.run(st, out, ws, 1, use_graph=True)
        torch.cuda.synchronize()
        sc = plan.scalars(out)[0]
        v = 1.0 - st.x.cpu().numpy()
        hist.append((float(sc[mx.S_TIME]), second_moment(v, r), float(sc[mx.S_SUMX]), int(sc[mx.S_STATUS])))
    Dij = p["nu0"] * math.exp(-p["Qm"] / (KB * s.T))
    return s, r, v, hist, Dij


def test_linear_law_spreads_exactly_on_the_lattice(mx):
    say("[gpu] vacancy point source, c = 0, 60 steps on 256k sites")
    s, r, v, hist, Dij = _spread(mx, 0.0, 60)
    for t, m2, sv, st in hist:
        assert st & mx.FATAL_STATUS == 0
        assert abs(m2 - Z_FCC * B_NN ** 2 * Dij * t) < 1e-9 * m2
        assert abs(sv - (s.n - 1)) < 1e-12 * s.n  # sum x conserved
    t = hist[-1][0]
    err = profile_error(v, r, t, Z_FCC * B_NN ** 2 * Dij / 6.0)
    say(f"    continuum profile error {err:.4f}")
    assert err < 0.02


def test_full_law_vacancy_escapes_then_spreads_at_the_lattice_rate(mx):
    """At 1000 K the vacancy leaves its site after a delay (mu at the vacancy lies
    above the bulk, which slows the first hops); once dilute, mu is uniform and
    the second moment grows at the linear-law rate Z b^2 D_ij."""
    say("[gpu] vacancy point source, c = 1, 1000 K, 200 steps on 256k sites")
    s, r, v, hist, Dij = _spread(mx, 1.0, 200)
    for t, m2, sv, st in hist:
        assert st & mx.FATAL_STATUS == 0
        assert abs(sv - (s.n - 1)) < 1e-12 * s.n
    t = np.array([h[0] for h in hist])
    m2 = np.array([h[1] for h in hist])
    assert np.all(np.diff(m2) > 0)
    late = slice(150, 200)
    slope = np.polyfit(t[late], m2[late], 1)[0]
    ratio = slope / (Z_FCC * B_NN ** 2 * Dij)
    D_fit = slope / 6.0
    t_eff = m2[-1] / (6.0 * D_fit)  # time origin of the equivalent point source
    err = profile_error(v, r, t_eff, D_fit)
    say(f"    late spreading rate / Z b^2 D_ij = {ratio:.4f}; point-source profile error {err:.4f}; "
        f"fraction left at the origin {v[np.argmin(r)]:.2e}")
    assert 0.9 < ratio < 1.1
    assert err < 0.05
    assert v[np.argmin(r)] < 1e-2


def test_full_law_vacancy_stays_at_low_temperature(mx):
    """At 600 K the same vacancy stays on its site (Sec. 5.1: at low temperature the
    vacancy lacks the entropic drive to leave)."""
    say("[gpu] vacancy point source, c = 1, 600 K, 60 steps")
    s, v0 = single_vacancy(40, 600.0)
    p = dict(L.DEFAULT_PARAMS, max_relax=30, kin_c=1.0)
    plan = mx.Plan([s], L.DEFAULT_EAM, p)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, 60, use_graph=True)
    torch.cuda.synchronize()
    v = 1.0 - st.x.cpu().numpy()
    assert int(plan.scalars(out)[0, mx.S_STATUS]) & mx.FATAL_STATUS == 0
    say(f"    fraction left at the origin {v[v0]:.4f}")
    assert v[v0] > 0.9
