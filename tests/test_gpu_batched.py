"""Batched systems of uneven size in one launch sequence, slots, continuous batching.

Each system's results must equal its single-system run bitwise: the kernels are
deterministic and a system's reductions do not depend on its slot, capacity or
batch-mates."""
import numpy as np
import pytest

from paper_1910_01235_amd import lattice as L
from paper_1910_01235_amd import serve
from tests.gpu_common import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    from paper_1910_01235_amd import mxe
    mxe.lib()
    assert torch.cuda.is_available(), "no HIP device"
    return mxe


def _mixed_systems():
    return [L.vacancy_bulk(5, 1, 700.0, 1, name="vac5"),
            L.alloy_bulk(6, 0.06, 1100.0, 2, name="alloy6"),
            L.vacancy_bulk(7, 1, 950.0, 3, name="vac7"),
            L.alloy_bulk(5, 0.02, 620.0, 4, name="alloy5")]


def _run_alone(mx, s, params, n_steps, precision="fp64"):
    plan = mx.Plan([s], L.DEFAULT_EAM, params, precision=precision)
    st, out, ws = plan.state([s]), plan.out(), plan.workspace()
    plan.run(st, out, ws, n_steps, use_graph=True)
    torch.cuda.synchronize()
    return (st.x.cpu().numpy(), torch.stack([st.qx, st.qy, st.qz], 1).cpu().numpy(),
            st.sigma.cpu().numpy(), plan.scalars(out)[0])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_plan_equals_single_runs_bitwise(mx, precision):
    systems = _mixed_systems()
    params = dict(L.DEFAULT_PARAMS, max_relax=20)
    say(f"[gpu] batched {len(systems)} systems {precision}")
    plan = mx.Plan(systems, L.DEFAULT_EAM, params, precision=precision)
    st, out, ws = plan.state(systems), plan.out(), plan.workspace()
    plan.run(st, out, ws, 3, use_graph=True)
    torch.cuda.synchronize()
    sc = plan.scalars(out)
    for k, s in enumerate(systems):
        lo, hi = plan.offsets[k], plan.offsets[k + 1]
        x, q, sg, sc1 = _run_alone(mx, s, params, 3, precision)
        assert np.array_equal(st.x[lo:hi].cpu().numpy(), x), s.name
        assert np.array_equal(st.sigma[lo:hi].cpu().numpy(), sg), s.name
        assert np.array_equal(st.qx[lo:hi].cpu().numpy(), q[:, 0]), s.name
        assert sc[k, mx.S_TIME] == sc1[mx.S_TIME]
        assert int(sc[k, mx.S_STATUS]) & mx.FATAL_STATUS == 0


def test_slots_rebind_with_resume(mx):
    """Slots larger than their systems, rebound between calls, in resume mode."""
    a, b, c = _mixed_systems()[:3]
    params = dict(L.DEFAULT_PARAMS, max_relax=15)
    tmpl = [L.vacancy_bulk(8, 0, 300.0, 0), L.vacancy_bulk(8, 0, 300.0, 0)]  # 2048-site slots
    plan = mx.Plan(tmpl, L.DEFAULT_EAM, params)
    plan.set_resume(True)
    N = plan.n_sites
    st = mx.DeviceState(*[torch.zeros(N, dtype=torch.float64, device="cuda") for _ in range(5)],
                        torch.zeros(N, dtype=torch.int8, device="cuda"))
    st.sigma.fill_(0.1)
    out, ws = plan.out(), plan.workspace()

    def load(slot, s):
        plan.set_system(slot, s)
        off = int(plan.offsets[slot])
        for name, arr in (("qx", s.q[:, 0]), ("qy", s.q[:, 1]), ("qz", s.q[:, 2]), ("sigma", s.sigma),
                          ("x", s.x)):
            getattr(st, name)[off:off + s.n] = torch.as_tensor(arr, device="cuda")
        st.type[off:off + s.n] = torch.as_tensor(s.type, device="cuda")
        out.scalars[slot * mx.NSCALARS + mx.S_TIME] = 0.0

    load(0, a)
    load(1, b)
    for _ in range(2):
        plan.run(st, out, ws, 1, use_graph=True)
    plan.set_system(0, None)         # slot 0 retires a; slot 1 keeps b
    load(0, c)
    plan.run(st, out, ws, 2, use_graph=True)
    torch.cuda.synchronize()
    xb, _, _, _ = _run_alone(mx, b, params, 4)
    xc, _, sgc, _ = _run_alone(mx, c, params, 2)
    o0, o1 = int(plan.offsets[0]), int(plan.offsets[1])
    assert np.array_equal(st.x[o1:o1 + b.n].cpu().numpy(), xb)
    assert np.array_equal(st.x[o0:o0 + c.n].cpu().numpy(), xc)
    assert np.array_equal(st.sigma[o0:o0 + c.n].cpu().numpy(), sgc)
    with pytest.raises(mx.MxeError, match="holds at most"):
        plan.set_system(0, L.vacancy_bulk(9, 0, 300.0, 0))


def test_served_results_equal_alone(mx):
    params = dict(L.DEFAULT_PARAMS, max_relax=15)
    rng = np.random.default_rng(7)
    systems = []
    for k in range(7):
        cells = int(rng.integers(5, 9))
        T = float(rng.uniform(600, 1200))
        systems.append(L.vacancy_bulk(cells, 1, T, k) if k % 2 else L.alloy_bulk(cells, 0.05, T, k))
    systems.append(L.vacancy_bulk(12, 1, 800.0, 99))  # 6912 sites: too large for the pool
    reqs = serve.poisson_requests(systems, n_steps=3, rate=0.0)
    per_site = serve.bytes_per_site(L.DEFAULT_EAM, params)
    caps = [1024, 1024, 2048, 2048]
    budget = sum(caps) * per_site * 1.05
    say("[gpu] serving 8 requests on 4 slots")
    srv = serve.Server(L.DEFAULT_EAM, params, caps)
    assert srv.footprint_bytes <= budget
    results, rejected, stats = srv.serve(reqs, realtime=False)
    assert rejected == [7]
    assert len(results) == 7 and stats["gpu_steps"] >= 6
    alone, _ = serve.serve_one_at_a_time(L.DEFAULT_EAM, params, reqs[:7], realtime=False)
    by_id = {r.rid: r for r in alone}
    for r in results:
        a = by_id[r.rid]
        assert r.status & mx.FATAL_STATUS == 0
        assert np.array_equal(r.x, a.x), r.rid
        assert np.array_equal(r.q, a.q), r.rid
        assert np.array_equal(r.sigma, a.sigma), r.rid
        assert r.time_simulated == a.time_simulated


def test_autotuned_shapes_keep_results(mx, tmp_path):
    """Every launch shape gives the same physics (to rounding); the tuner picks one."""
    from paper_1910_01235_amd import autotune
    s = L.jitter(L.vacancy_bulk(6, 4, 900.0, 5), 6, xr=(0.3, 0.9))
    p = dict(L.DEFAULT_PARAMS)
    # FP64 shapes agree to rounding; FP32-mixed shapes store the moments in FP32
    # (two lanes per force-gather entry) and agree to that precision
    for prec, tol in (("fp64", 1e-13), ("fp32", 1e-6)):
        ref = None
        for g in autotune.GATHER_LANES:
            for b in autotune.PAIR_BLOCKS:
                f = autotune.GATHER_LANES[(autotune.GATHER_LANES.index(g) + 1) % len(autotune.GATHER_LANES)]
                plan = mx.Plan([s], L.DEFAULT_EAM, p, precision=prec, gather_lanes=g, force_lanes=f,
                               pair_block=b)
                st, out, ws = plan.state([s]), plan.out(), plan.workspace()
                plan.evaluate(st, out, ws)
                f = torch.stack([out.fx, out.fy, out.fz, out.fsigma, out.mu], 1).cpu().numpy()
                if ref is None:
                    ref = f
                assert np.abs(f - ref).max() <= tol * np.abs(ref).max(), (prec, g, b)
    cache = autotune.Cache(str(tmp_path / "tune.json"))
    params, hit = autotune.tuned_params([s], L.DEFAULT_EAM, p, "fp64", cache=cache, reps=2)
    assert params["gather_lanes"] in autotune.GATHER_LANES
    assert params["force_lanes"] in autotune.GATHER_LANES
    assert params["pair_block"] in autotune.PAIR_BLOCKS
    assert cache.get(autotune.bucket([s], "fp64", 0)) == hit
    assert params["gather_stride"] >= 1
    assert params["pair_split"] in autotune.PAIR_SPLITS


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_gather_stride_and_pair_split_keep_results_bitwise(mx, precision):
    """The gathers' chunk visit order changes no sum, and which pair-kernel block
    takes a pair changes none of its moments: every stride and every split gives
    the same bits, on one multi-chunk system and on a batch whose systems
    straddle XCD ranges."""
    one = [L.jitter(L.vacancy_bulk(8, 6, 900.0, 5), 7, xr=(0.3, 0.9))]  # 2048 sites, 8 chunks
    batch = _mixed_systems() + [L.vacancy_bulk(9, 2, 800.0, 9)]
    p = dict(L.DEFAULT_PARAMS, max_relax=4)
    for systems in (one, batch):
        ref = None
        shapes = [dict(gather_stride=st) for st in (1, 2, 3, 7, 26, 4096)] + \
                 [dict(pair_split=sp, pair_block=b) for sp in (1, 4, 8, 16) for b in (64, 256)]
        for shape in shapes:
            plan = mx.Plan(systems, L.DEFAULT_EAM, p, precision=precision, **shape)
            st, out, ws = plan.state(systems), plan.out(), plan.workspace()
            plan.run(st, out, ws, 2, use_graph=False)
            torch.cuda.synchronize()
            got = [torch.stack([out.fx, out.fy, out.fz, out.fsigma, out.mu, out.rho_bar], 1).cpu().numpy(),
                   st.x.cpu().numpy(), st.qx.cpu().numpy(), plan.scalars(out)]
            assert int(np.bitwise_or.reduce(got[3][:, mx.S_STATUS].astype(np.int64))) & mx.FATAL_STATUS == 0
            if ref is None:
                ref = got
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), (precision, len(systems), shape)



@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_row_fold_paths_agree_bitwise(mx, precision):
    """The FIRE control folds the force gather's partial rows itself, unless a
    system of the plan has more than 256 site chunks (then a launch of its own
    folds them, in the same order): a small system gives the same bits alone
    and beside a 70k-site system."""
    small = L.vacancy_bulk(6, 1, 900.0, 5, name="vac6")
    big = L.vacancy_bulk(26, 700, 1000.0, 7, name="vac26")
    assert big.n > 256 * 256
    params = dict(L.DEFAULT_PARAMS, max_relax=12)
    say(f"[gpu] row fold paths {precision}: {small.n} alone and beside {big.n}")
    x, q, sg, sc1 = _run_alone(mx, small, params, 2, precision)
    plan = mx.Plan([big, small], L.DEFAULT_EAM, params, precision=precision)
    st, out, ws = plan.state([big, small]), plan.out(), plan.workspace()
    plan.run(st, out, ws, 2, use_graph=True)
    torch.cuda.synchronize()
    lo, hi = plan.offsets[1], plan.offsets[2]
    sc = plan.scalars(out)
    assert np.array_equal(st.x[lo:hi].cpu().numpy(), x)
    assert np.array_equal(st.sigma[lo:hi].cpu().numpy(), sg)
    assert np.array_equal(st.qx[lo:hi].cpu().numpy(), q[:, 0])
    for key in (mx.S_TIME, mx.S_F, mx.S_FMAX, mx.S_SUMX, mx.S_UPDATES):
        assert sc[1, key] == sc1[key], key
    assert int(sc[0, mx.S_STATUS]) & mx.FATAL_STATUS == 0
