"""The C-ABI library loads and exports every entry point include/mxe.h declares.

No compute call is made here (no GPU in this check)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "mxe.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mxe_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("mxe_plan_create", "mxe_evaluate", "mxe_relax", "mxe_step", "mxe_run",
              "mxe_workspace_bytes", "mxe_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1910_01235_amd import mxe
    if not os.path.exists(mxe.LIB_PATH):
        pytest.skip("libmxe.so not built")
    lib = ctypes.CDLL(mxe.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert sorted(mxe.EXPORTED) == declared_functions()


def test_plan_validation_needs_no_gpu():
    """Plan creation is host-only: argument checks and workspace sizing."""
    from paper_1910_01235_amd import lattice as L
    from paper_1910_01235_amd import mxe
    if not os.path.exists(mxe.LIB_PATH):
        pytest.skip("libmxe.so not built")
    w = L.config0(0)
    plan = mxe.Plan(w.systems, w.eam, w.params)
    assert plan.n_sites == 256 and plan.ws_bytes > 0
    # a periodic box shorter than twice the list radius is rejected
    s = L.vacancy_bulk(3, 0, 800.0, 0)
    with pytest.raises(mxe.MxeError, match="periodic box"):
        mxe.Plan([s], w.eam, w.params)
    # an empty system is rejected
    e = s.copy()
    e.q = e.q[:0]
    with pytest.raises(mxe.MxeError, match="n_sites"):
        mxe.Plan([e], w.eam, w.params)
    with pytest.raises(mxe.MxeError, match="symmetric"):
        bad = dict(w.eam, pair_a=[[0.3, 0.1, 0.2], [0.2, 0.36, 0.2], [0.2, 0.2, 0.0]])
        mxe.Plan(w.systems, bad, w.params)
    # row and bond lengths are bounded (rows sort in registers, bond rows sit in LDS)
    with pytest.raises(mxe.MxeError, match="k_max"):
        mxe.Plan(w.systems, w.eam, dict(w.params, k_max=257))
    with pytest.raises(mxe.MxeError, match="bond_max"):
        mxe.Plan(w.systems, w.eam, dict(w.params, bond_max=65))
    assert mxe.Plan(w.systems, w.eam, dict(w.params, bond_max=64)).n_sites == 256
    # the relaxation chunk is bounded; creating a chunked plan touches no device
    for bad in (-1, 1025):
        with pytest.raises(mxe.MxeError, match="relax_chunk"):
            mxe.Plan(w.systems, w.eam, dict(w.params, relax_chunk=bad))
    assert mxe.Plan(w.systems, w.eam, dict(w.params, relax_chunk=4)).params.relax_chunk == 4
    # free-running steps: argument checks precede any device work
    L_ = mxe.lib()
    p0 = mxe.Plan(w.systems, w.eam, w.params)
    assert L_.mxe_advance(p0._h, None, None, 10, 1, None, 0, None) == -1  # relax_chunk 0
    assert b"relax_chunk" in L_.mxe_last_error()
    p4 = mxe.Plan(w.systems, w.eam, dict(w.params, relax_chunk=4))
    assert L_.mxe_advance(p4._h, None, None, 10, 1, None, 0, None) == -1  # resume mode off
    assert b"resume" in L_.mxe_last_error()
    p4.set_resume(True)
    assert L_.mxe_advance(p4._h, None, None, -1, 1, None, 0, None) == -1
    with pytest.raises(mxe.MxeError, match="slot"):
        p4.set_steps(5, 3)
    with pytest.raises(mxe.MxeError, match="n_steps"):
        p4.set_steps(0, -1)
    p4.set_steps(0, 3)
    # fp32 workspace is smaller (FP32 moments)
    p32 = mxe.Plan(w.systems, w.eam, w.params, precision="fp32")
    assert p32.ws_bytes < plan.ws_bytes


def test_host_only_queries():
    """Slot checks, workspace layout and the scratch limit need no GPU."""
    from paper_1910_01235_amd import lattice as L
    from paper_1910_01235_amd import mxe
    if not os.path.exists(mxe.LIB_PATH):
        pytest.skip("libmxe.so not built")
    w = L.config0(0)
    plan = mxe.Plan(w.systems, w.eam, w.params)
    # layout: rows of k_max ints, counts, bonds of bond_max ints, inside the workspace
    items = [(mxe.L_NBR, 256 * 96 * 4), (mxe.L_NBR_COUNT, 256 * 4), (mxe.L_BOND, 256 * 16 * 4),
             (mxe.L_BOND_COUNT, 256 * 4)]
    for item, size in items:
        off, nb = plan.layout(item)
        assert nb == size and off % 256 == 0 and off + nb <= plan.ws_bytes
    with pytest.raises(mxe.MxeError, match="layout"):
        plan.layout(7)
    # slot checks: sites, then cells of the box; the plan is left unchanged
    small = L.vacancy_bulk(4, 0, 800.0, 1)
    assert plan.check_system(0, small)
    big = L.vacancy_bulk(5, 0, 800.0, 1)
    assert not plan.check_system(0, big)
    rod = small.copy()
    rod.q = rod.q[:200]
    rod.box = (14.46, 14.46, 2000.0)  # few sites, far more cells than the slot holds
    rod.periodic = (True, True, False)
    assert not plan.check_system(0, rod)
    bad = small.copy()
    bad.T = -1.0
    with pytest.raises(mxe.MxeError, match="T must be positive"):
        plan.check_system(0, bad)
    assert plan.n_sites == 256


def test_noalloc_rejects_oversized_plan_before_any_device_call():
    """mxe_run_noalloc checks the plan against its fixed scratch first (no GPU touched)."""
    import ctypes as C
    from paper_1910_01235_amd import lattice as L
    from paper_1910_01235_amd import mxe
    if not os.path.exists(mxe.LIB_PATH):
        pytest.skip("libmxe.so not built")
    w = L.config1(1)
    plan = mxe.Plan(w.systems, w.eam, w.params)
    assert plan.ws_bytes > (64 << 20)
    st, out = mxe.State(), mxe.Out()
    code = mxe.lib().mxe_run_noalloc(plan._h, C.byref(st), C.byref(out), 1, None)
    assert code == -2  # MXE_ENOMEM
    assert b"allocation-free" in mxe.lib().mxe_last_error()
