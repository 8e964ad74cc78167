"""Host logic of the serving loop: pool sizing against an HBM budget, admission."""
import pytest

from paper_1910_01235_amd import lattice as L
from paper_1910_01235_amd import serve


def test_pool_fits_budget():
    per_site = 9000.0
    budget = 32e9
    caps = serve.pool_capacities(budget, per_site)
    assert sum(caps) * per_site <= budget
    classes = sorted(set(caps))
    counts = [caps.count(c) for c in classes]
    assert len(set(counts)) == 1 and counts[0] >= 1
    # one more slot per class would exceed the budget
    assert (sum(caps) + sum(classes)) * per_site > budget
    with pytest.raises(ValueError):
        serve.pool_capacities(1e6, per_site)


def test_smallest_free_slot_that_fits():
    caps = [1024, 1024, 4096, 65536]
    assert serve.pick_slot(caps, {0, 1, 2, 3}, 500) == 0
    assert serve.pick_slot(caps, {1, 2, 3}, 500) == 1
    assert serve.pick_slot(caps, {2, 3}, 3000) == 2
    assert serve.pick_slot(caps, {3}, 3000) == 3
    assert serve.pick_slot(caps, {0, 1, 2}, 5000) is None
    assert serve.pick_slot(caps, set(), 10) is None


def test_bytes_per_site_probe_is_host_only():
    w = L.config0(0)
    b64 = serve.bytes_per_site(w.eam, w.params)
    b32 = serve.bytes_per_site(w.eam, w.params, precision="fp32")
    assert 2000 < b32 < b64 < 20000


def test_poisson_arrivals_are_ordered_and_seeded():
    systems = [L.vacancy_bulk(5, 1, 800.0, k) for k in range(5)]
    a = serve.poisson_requests(systems, 3, rate=10.0, seed=1)
    b = serve.poisson_requests(systems, 3, rate=10.0, seed=1)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    assert all(x.arrival <= y.arrival for x, y in zip(a, a[1:]))
    assert a[0].arrival == 0.0
