"""Autotuner host logic: buckets, cache round trip, shape validation by the plan."""
import pytest

from paper_1910_01235_amd import autotune
from paper_1910_01235_amd import lattice as L
from paper_1910_01235_amd import mxe


def test_bucket_names():
    a = [L.vacancy_bulk(4, 0, 800.0, 0)]
    assert autotune.bucket(a, "fp64") == "fp64/gh27/host/2^8"
    assert autotune.bucket(a, "fp64", quad_rule=1) == "fp64/deg3/host/2^8"
    w = L.nanowire(radius=6.0, n_axial=4)
    assert autotune.bucket([w], "fp32").startswith("fp32/gh27/interstitial/")


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "cache.json")
    c = autotune.Cache(p)
    assert c.get("k") is None
    c.put("k", {"gather_lanes": 32, "pair_block": 128})
    assert autotune.Cache(p).get("k") == {"gather_lanes": 32, "pair_block": 128}


def test_plan_validates_launch_shapes():
    import os
    if not os.path.exists(mxe.LIB_PATH):
        pytest.skip("libmxe.so not built")
    w = L.config0(0)
    for g in autotune.GATHER_LANES:
        mxe.Plan(w.systems, w.eam, w.params, gather_lanes=g, force_lanes=g)
    for b in autotune.PAIR_BLOCKS:
        mxe.Plan(w.systems, w.eam, w.params, pair_block=b)
    with pytest.raises(mxe.MxeError, match="gather_lanes"):
        mxe.Plan(w.systems, w.eam, w.params, gather_lanes=12)
    with pytest.raises(mxe.MxeError, match="force_lanes"):
        mxe.Plan(w.systems, w.eam, w.params, force_lanes=24)
    with pytest.raises(mxe.MxeError, match="pair_block"):
        mxe.Plan(w.systems, w.eam, w.params, pair_block=512)
    for st in (0, 1, 25, 4096):
        mxe.Plan(w.systems, w.eam, w.params, gather_stride=st)
    with pytest.raises(mxe.MxeError, match="gather_stride"):
        mxe.Plan(w.systems, w.eam, w.params, gather_stride=-1)
    for sp in autotune.PAIR_SPLITS:
        mxe.Plan(w.systems, w.eam, w.params, pair_split=sp)
    for bad in (3, 32, -1):
        with pytest.raises(mxe.MxeError, match="pair_split"):
            mxe.Plan(w.systems, w.eam, w.params, pair_split=bad)


def test_layer_stride_from_site_order():
    """FCC cells in lattice order: one layer of 40 x 40 cells is 6,400 sites, of
    32 x 32 cells 4,096 (25 and 16 chunks of 256; the farthest first-shell
    neighbour sits a few sites further)."""
    assert autotune.layer_stride(L.config1(1).systems) == 26
    assert autotune.layer_stride(L.config2(2).systems) == 16
    assert autotune.layer_stride([L.vacancy_bulk(4, 0, 800.0, 0)]) == 1  # one chunk
    assert autotune.stride_candidates(L.config1(1).systems) == [1, 13, 26, 39]


def test_profile_modes_are_validated():
    import os
    if not os.path.exists(mxe.LIB_PATH):
        pytest.skip("libmxe.so not built")
    w = L.config0(0)
    plan = mxe.Plan(w.systems, w.eam, w.params)
    for mode in (mxe.PROFILE_OFF, mxe.PROFILE_ALL, mxe.PROFILE_PAIR):
        assert mxe.lib().mxe_profile(plan._h, mode) == 0
    assert mxe.lib().mxe_profile(plan._h, 3) != 0
    assert mxe.lib().mxe_profile(plan._h, -1) != 0
    plan.profile("pair")
    plan.profile(True)
    plan.profile(False)


@pytest.mark.parametrize("t64,expect", [(0.99, 256), (0.90, 64), (1.02, 256)])
def test_pair_block_near_ties_keep_the_largest(monkeypatch, t64, expect):
    """Pair blocks within the tie margin of the fastest: the largest is kept
    (more threads per chunk); a clearly faster smaller block still wins."""
    def fake(systems, eam, params, precision, reps, **shape):
        b = shape.get("pair_block", 256)
        pair = {64: t64, 128: 1.005, 256: 1.0}[b] * (1.0 + 0.01 * shape.get("pair_split", 1))
        return dict(density=1.0, force=1.0, pair=pair)
    monkeypatch.setattr(autotune, "_time_kernels", fake)
    w = L.config0(0)
    got = autotune.tune(w.systems, w.eam, w.params, reps=1)
    assert got["pair_block"] == expect
    assert got["pair_split"] == 1
