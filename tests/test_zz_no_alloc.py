"""The allocation-free entry point mxe_run_noalloc against mxe_run on a caller workspace.

mxe_run_noalloc runs the same launch sequence on the library's per-device
scratch. Two calls in a row, the second on a smaller system (the scratch then
holds the first call's lists and tables), and a third on the first plan again
after the second plan overwrote the scratch, must each equal mxe_run on a
workspace of their own.
"""
import numpy as np
import pytest

from paper_1910_01235_amd import lattice as L
from paper_1910_01235_amd import mxe

from tests.gpu_common import say, gpu_arrays, rel_err

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def _pair(plan, s, n_steps):
    import torch
    st_w, out_w, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st_w, out_w, ws, n_steps, use_graph=False)
    st_n, out_n = plan.state([s]), plan.out()
    plan.run_noalloc(st_n, out_n, n_steps)
    torch.cuda.synchronize()
    return (gpu_arrays(plan, st_w, out_w), plan.scalars(out_w),
            gpu_arrays(plan, st_n, out_n), plan.scalars(out_n))


def _compare(tag, a, sa, b, sb):
    errs = {k: rel_err(b[k], a[k], 1e-2) for k in a}
    bitwise = all(np.array_equal(a[k], b[k]) for k in a) and np.array_equal(sa, sb)
    say(f"[no_alloc] {tag}: max rel err {max(errs.values()):.2e}, bitwise {bitwise}")
    for k, e in errs.items():
        assert e <= 1e-10, (tag, k, e)
    # iteration counts, rebuilds and convergence equal; F, FMAX, dt, time, sum x to 1e-12
    for k in (mxe.S_UPDATES, mxe.S_CONVERGED, mxe.S_EVALS, mxe.S_REBUILDS, mxe.S_TOTAL_EVALS,
              mxe.S_PAIRS, mxe.S_STATUS):
        assert np.array_equal(sa[:, k], sb[:, k]), (tag, k)
    for k in (mxe.S_F, mxe.S_FMAX, mxe.S_DT, mxe.S_TIME, mxe.S_SUMX):
        assert np.all(np.abs(sa[:, k] - sb[:, k]) <= 1e-12 * np.abs(sa[:, k])), (tag, k)


def test_noalloc_run_matches_workspace_run_on_consecutive_calls():
    import torch
    torch.cuda.set_device(0)
    w = L.config0(0)
    big = w.systems[0]                                        # 256 sites
    small = L.jitter(L.cluster(3), 70, xr=(0.3, 0.95))        # 43 sites, open box
    params = dict(w.params, max_relax=15)
    plan_big = mxe.Plan([big], w.eam, params)
    plan_small = mxe.Plan([small], w.eam, params)
    assert plan_big.ws_bytes <= SCRATCH_BYTES and plan_small.ws_bytes < plan_big.ws_bytes
    say(f"[no_alloc] workspaces: {plan_big.ws_bytes} and {plan_small.ws_bytes} bytes")
    _compare("first call, 256 sites", *_pair(plan_big, big, 2))
    _compare("second call, 43 sites", *_pair(plan_small, small, 2))
    _compare("third call, 256 sites again", *_pair(plan_big, big, 1))


def test_noalloc_rejects_a_plan_larger_than_the_scratch():
    w = L.config1(1)
    plan = mxe.Plan(w.systems, w.eam, w.params)
    assert plan.ws_bytes > SCRATCH_BYTES
    st, out = plan.state(w.systems), plan.out()
    with pytest.raises(mxe.MxeError, match="allocation-free"):
        plan.run_noalloc(st, out, 1)
