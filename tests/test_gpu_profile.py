"""Profiling instrumentation: every kernel family bracketed by HIP events, or
only the pair kernel (the least instrumentation that times the dominant
kernel). Either way the results are those of an unprofiled run."""
import numpy as np
import pytest

from paper_1910_01235_amd import lattice as L
from tests.gpu_common import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    return mxe


def _run(mx, w, mode):
    plan = mx.Plan(w.systems, w.eam, w.params)
    st, out, ws = plan.state(w.systems), plan.out(), plan.workspace()
    plan.profile(mode)
    if mode:
        plan.profile_read()
    plan.run(st, out, ws, 1, use_graph=True)  # profiling launches eagerly
    torch.cuda.synchronize()
    pr = plan.profile_read() if mode else None
    plan.profile(False)
    return pr, st.x.cpu().numpy(), st.qx.cpu().numpy()


def test_profile_modes(mx):
    w = L.config0(0)
    say("[gpu] profiling modes on the small workload")
    _, x0, q0 = _run(mx, w, False)
    every, x1, q1 = _run(mx, w, True)
    pair, x2, q2 = _run(mx, w, "pair")
    n_eval = w.params["max_relax"] + 1  # one diffusion step
    for fam in ("pair", "density", "force", "fire"):
        assert every[fam][1] == n_eval and every[fam][0] > 0.0, (fam, every[fam])
    assert every["master"][1] == 1
    assert pair["pair"][1] == n_eval and pair["pair"][0] > 0.0
    for fam in ("density", "force", "build", "fire", "master"):
        assert pair[fam] == (0.0, 0), (fam, pair[fam])
    for a, b in ((x0, x1), (x0, x2), (q0, q1), (q0, q2)):
        assert np.array_equal(a, b)
