"""Launch-shape autotuner for the evaluation kernels.

Five launch shapes change speed but not the method: the lanes per site of
the density gather and of the force gather (8, 16, 32, 64 each), the block
size of the pair quadrature kernel (64, 128, 256) and its blocks per chunk of
4096 pair slots (1 to 16: small systems want more, shorter blocks), and the
gathers' chunk visit stride. The tuner times every candidate on the workload at hand (HIP
events around each kernel launch, through the library's profiling switch),
keeps the fastest of each, and caches the choice per size bucket, precision
and lattice kind in a JSON file. Pair blocks within 3 % of the fastest count as
tied and the largest of them is kept: the grid has a fixed number of blocks
per chunk, so a smaller block means fewer threads per launch, which a large
batch hides and a plan of a few chunks does not (one small system with the
64-thread block of a large batch's tie takes half as long again per step).

Stride candidates come from the systems' own site order: the index distance
from a site to its nearest neighbours one lattice layer away, in chunks of
256 sites (the gathers then read a pair block from its second end while it is
still cached), with half and one and a half times that, and 1 (plain order).
"""
from __future__ import annotations

import json
import math
import os

from . import lattice as L
from . import mxe

GATHER_LANES = (8, 16, 32, 64)
CHUNK = 256  # sites per chunk of the gathers
PAIR_BLOCKS = (64, 128, 256)
PAIR_SPLITS = (1, 2, 4, 8, 16)
PAIR_BLOCK_TIE = 0.03  # relative time within which pair blocks count as tied
SHAPES = ("gather_lanes", "force_lanes", "pair_block", "pair_split", "gather_stride")
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mxe_autotune.json")


def bucket(systems, precision: str, quad_rule: int = 0) -> str:
    """Size bucket (power of two of the total sites), precision, quadrature rule and lattice kind."""
    n = sum(int(s.n) for s in systems)
    kind = "interstitial" if any((s.type == L.INTERSTITIAL).any() for s in systems) else "host"
    rule = "deg3" if quad_rule == mxe.QUAD_DEGREE3 else "gh27"
    return f"{precision}/{rule}/{kind}/2^{int(round(math.log2(max(n, 1))))}"


class Cache:
    def __init__(self, path: str = DEFAULT_CACHE):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key: str):
        return self.data.get(key)

    def put(self, key: str, value: dict):
        self.data[key] = value
        if self.path:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _time_kernels(systems, eam, params, precision, reps, **shape):
    import torch
    plan = mxe.Plan(systems, eam, params, precision=precision, **shape)
    st, out, ws = plan.state(systems), plan.out(), plan.workspace()
    plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.profile_read()
    for _ in range(reps):
        plan.evaluate(st, out, ws)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    ms = {k: v[0] / max(v[1], 1) for k, v in prof.items()}
    del plan, st, out, ws
    torch.cuda.empty_cache()
    return ms


def layer_stride(systems, n_probe: int = 512, seed: int = 0) -> int:
    """Chunks between a site and its farthest first-shell neighbour in index order
    (neighbours across a periodic wrap excluded): the 90th percentile over probe
    sites of the largest system (in a lattice order with a basis, only some
    basis sites reach into the next layer); 1 if it has fewer than two chunks."""
    import numpy as np
    from scipy.spatial import cKDTree
    s = max(systems, key=lambda t: t.n)
    if s.n < 2 * CHUNK:
        return 1
    box = np.array([b if p else 0.0 for b, p in zip(s.box, s.periodic)])
    q = s.q - np.floor(s.q / np.where(box > 0, box, 1.0)) * box if box.any() else s.q
    tree = cKDTree(q, boxsize=np.where(box > 0, box, np.ptp(s.q, axis=0) * 4 + 100.0))
    rng = np.random.default_rng(seed)
    probe = rng.choice(s.n, min(n_probe, s.n), replace=False)
    d, nb = tree.query(q[probe], k=13)
    off = nb - probe[:, None]
    off = np.where((off > 0) & (off < s.n // 2) & (d < 1.25 * d[:, 1:2]), off, 0).max(axis=1)
    return max(1, int(round(float(np.percentile(off, 90)) / CHUNK)))


def stride_candidates(systems):
    s0 = layer_stride(systems)
    return sorted({1, max(1, s0 // 2), s0, s0 + s0 // 2})


def tune(systems, eam: dict, params: dict, precision: str = "fp64", reps: int = 5) -> dict:
    """Time every candidate shape on these systems; return the fastest and the timings."""
    timings = {"gather_lanes": {}, "force_lanes": {}, "pair_block": {}, "pair_split": {},
               "gather_stride": {}}
    for g in GATHER_LANES:  # both gathers at once: each is timed on its own
        ms = _time_kernels(systems, eam, params, precision, reps, gather_lanes=g, force_lanes=g)
        timings["gather_lanes"][g] = ms["density"]
        timings["force_lanes"][g] = ms["force"]
    for b in PAIR_BLOCKS:
        ms = _time_kernels(systems, eam, params, precision, reps, pair_block=b)
        timings["pair_block"][b] = ms["pair"]
    best_g = min(timings["gather_lanes"], key=timings["gather_lanes"].get)
    best_f = min(timings["force_lanes"], key=timings["force_lanes"].get)
    t_b = min(timings["pair_block"].values())
    best_b = max(b for b, t in timings["pair_block"].items() if t <= t_b * (1.0 + PAIR_BLOCK_TIE))
    for sp in PAIR_SPLITS:  # with the tuned block
        ms = _time_kernels(systems, eam, params, precision, reps, pair_block=best_b, pair_split=sp)
        timings["pair_split"][sp] = ms["pair"]
    best_p = min(timings["pair_split"], key=timings["pair_split"].get)
    for st in stride_candidates(systems):  # with the tuned widths; both gathers together
        ms = _time_kernels(systems, eam, params, precision, reps, gather_lanes=best_g,
                           force_lanes=best_f, gather_stride=st)
        timings["gather_stride"][st] = ms["density"] + ms["force"]
    best_s = min(timings["gather_stride"], key=timings["gather_stride"].get)
    return dict(gather_lanes=int(best_g), force_lanes=int(best_f), pair_block=int(best_b),
                pair_split=int(best_p), gather_stride=int(best_s),
                timings_ms={k: {str(a): round(b, 5) for a, b in v.items()} for k, v in timings.items()})


def tuned_params(systems, eam: dict, params: dict, precision: str = "fp64", cache: Cache = None,
                 retune: bool = False, reps: int = 5):
    """params with the tuned launch shapes (tuned now, or taken from the cache)."""
    key = bucket(systems, precision, int(params.get("quad_rule", eam.get("quad_rule", 0))))
    hit = None if (cache is None or retune) else cache.get(key)
    if hit is not None and any(k not in hit for k in SHAPES):
        hit = None  # written before these shapes existed
    if hit is None:
        hit = tune(systems, eam, params, precision, reps)
        if cache is not None:
            cache.put(key, hit)
    return dict(params, **{k: hit[k] for k in SHAPES}), hit
