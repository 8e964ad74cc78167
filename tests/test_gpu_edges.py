"""Edge cases of the GPU path: empty systems in a batch, row overflow, the
largest row length, and an all-empty plan.

Every case either reproduces the oracle / the system's solo run or reports
its condition through the status bits; none may fault."""
import numpy as np
import pytest

from paper_1910_01235_amd import lattice as L
from tests.gpu_common import eval_errors, gpu_arrays, oracle_eval, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EAM = L.DEFAULT_EAM
P = dict(L.DEFAULT_PARAMS)


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    return mxe


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_empty_system_in_a_batch(mx, prec):
    """A slot emptied between calls: the other systems keep their solo results bitwise."""
    a = L.jitter(L.vacancy_bulk(5, 2, 900.0, 1), 2, xr=(0.3, 0.9))
    b = L.jitter(L.alloy_bulk(5, 0.2, 800.0, 3), 4, xr=(0.1, 0.9))
    c = L.jitter(L.vacancy_bulk(6, 1, 1000.0, 5), 6, xr=(0.3, 0.9))
    say(f"[gpu] batch with an empty slot {prec}")
    plan = mx.Plan([a, b, c], EAM, P, precision=prec)
    st, out, ws = plan.state([a, b, c]), plan.out(), plan.workspace()
    plan.set_system(1, None)
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    sc = plan.scalars(out)
    assert sc[1, mx.S_F] == 0.0 and sc[1, mx.S_TOTAL_EVALS] == 0.0
    for k, s in ((0, a), (2, c)):
        solo = mx.Plan([s], EAM, P, precision=prec)
        st1, out1, ws1 = solo.state([s]), solo.out(), solo.workspace()
        solo.evaluate(st1, out1, ws1)
        torch.cuda.synchronize()
        g, g1 = gpu_arrays(plan, st, out, k), gpu_arrays(solo, st1, out1)
        for key in ("force", "mu", "e_site", "rho_bar"):
            assert np.array_equal(g[key], g1[key]), (k, key)
        assert sc[k, mx.S_F] == solo.scalars(out1)[0, mx.S_F]
        assert int(sc[k, mx.S_STATUS]) & mx.FATAL_STATUS == 0


def test_all_slots_empty_is_a_no_op(mx):
    s = L.vacancy_bulk(4, 0, 800.0, 0)
    plan = mx.Plan([s], EAM, P)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.set_system(0, None)
    plan.run(st, out, ws, 2, use_graph=True)
    plan.run(st, out, ws, 1, use_graph=False)
    torch.cuda.synchronize()
    assert np.array_equal(st.x.cpu().numpy(), s.x)


def test_row_overflow_is_reported(mx):
    """k_max below the neighbour count: the build reports KMAX (results invalid) and nothing faults."""
    s = L.vacancy_bulk(5, 0, 800.0, 0)
    plan = mx.Plan([s], EAM, P, k_max=20)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    plan.run(st, out, ws, 1, use_graph=False)
    torch.cuda.synchronize()
    assert int(plan.scalars(out)[0, mx.S_STATUS]) & mx.STAT_KMAX


def test_largest_row_length(mx):
    """k_max at its limit (256, four entries per lane in the row sort) gives the oracle's results."""
    s = L.jitter(L.nanowire(radius=9.0, n_axial=5, T=700.0), 4, xr=(0.0, 0.9))
    plan = mx.Plan([s], EAM, P, k_max=256)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    assert int(plan.scalars(out)[0, mx.S_STATUS]) & mx.FATAL_STATUS == 0
    for k, v in eval_errors(gpu_arrays(plan, st, out), oracle_eval(EAM, s)).items():
        assert v < 1e-10, (k, v)
    with pytest.raises(mx.MxeError, match="k_max"):
        mx.Plan([s], EAM, P, k_max=257)
