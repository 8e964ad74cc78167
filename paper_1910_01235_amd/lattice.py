"""Seeded synthetic inputs: lattices, site types, occupancy fields, parameters.

This module builds geometry and parameter values only. It holds none of the
method's arithmetic, so the GPU path and the CPU oracle can both take their
inputs from it without sharing any computation.

The workloads stand in for the paper's applications (Sec. 5), whose potentials
and data are not available: the vacancy in fcc Cu (Sec. 5.1), the surface
segregation slabs (Sec. 5.3) and the H-in-Pd nanowire (Sec. 5.5). They use the
single-species analytic EAM below in place of the paper's tabulated potentials.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

HOST_VAC, ALLOY, INTERSTITIAL, HOST_FIXED = 0, 1, 2, 3
A0_CU = 3.615  # lattice parameter, Angstrom (Sec. 5.1)

# Analytic EAM: phi(r) = 0.3 exp(-8 (r/2.556 - 1)) eV, f(r) = exp(-6 (r/2.556 - 1)),
# F(rho) = -sqrt(rho) eV, cosine taper 4.5-5.0 A. Species B: phi amplitude 0.36,
# f prefactor 1.2, F = -1.1 sqrt(rho), phi_AB = sqrt(phi_A phi_B). Interstitial
# solute S: host-solute phi = 0.2 exp(-5 (r/1.8 - 1)), f = 0.5 exp(-4 (r/1.8 - 1)),
# no solute-solute interaction, no solute embedding.
# Species order A, B, S; pair classes host-host, host-interstitial.
DEFAULT_EAM = dict(
    embed_c=[1.0, 1.1, 0.0],
    emit_b=[1.0, 1.2, 0.5],
    pair_a=[[0.3, math.sqrt(0.3 * 0.36), 0.2],
            [math.sqrt(0.3 * 0.36), 0.36, 0.2],
            [0.2, 0.2, 0.0]],
    r_e=[2.556, 1.8],
    alpha=[8.0, 5.0],
    gamma=[6.0, 4.0],
    r_s=4.5,
    r_c=5.0,
)

# Kinetic and relaxation parameters. nu0, Qm: Cu values of Sec. 5.1; the
# Pd-H values of Sec. 5.5 are used for the interstitial nanowire.
DEFAULT_PARAMS = dict(
    nu0=1.0e13, Qm=0.69, kin_c=1.0, dt_safety=0.5,
    max_relax=50, ftol=1.0e-3,
    dt0=0.05, dtmax=0.15, alpha0=0.1, finc=1.1, fdec=0.5, falpha=0.99, nmin=5,
    sigma_min=0.01, r_bond=3.09,
)
PDH_KINETICS = dict(nu0=8.1e12, Qm=0.294)


@dataclass
class System:
    """One periodic or open system of sites (SoA-friendly numpy arrays)."""
    q: np.ndarray          # (n, 3) float64 mean positions, Angstrom
    sigma: np.ndarray      # (n,) float64 per-axis width, Angstrom
    x: np.ndarray          # (n,) float64 molar fraction of the site's mobile species
    type: np.ndarray       # (n,) int8 site type
    box: tuple             # box lengths (periodic axes) / extents (open axes)
    periodic: tuple        # (3,) bools
    T: float               # temperature, K
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.q.shape[0])

    def copy(self) -> "System":
        return System(self.q.copy(), self.sigma.copy(), self.x.copy(), self.type.copy(),
                      tuple(self.box), tuple(self.periodic), float(self.T), self.name)


@dataclass
class Workload:
    name: str
    systems: list
    eam: dict = field(default_factory=lambda: dict(DEFAULT_EAM))
    params: dict = field(default_factory=lambda: dict(DEFAULT_PARAMS))
    n_steps: int = 1
    precision: str = "fp64"


def fcc(nx: int, ny: int, nz: int, a0: float = A0_CU) -> np.ndarray:
    """FCC sites, cell by cell, 4 basis sites per cubic cell (lattice order)."""
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    q = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a0
    return np.ascontiguousarray(q)


def octahedral(nx: int, ny: int, nz: int, a0: float = A0_CU) -> np.ndarray:
    """Octahedral interstitial sites of the FCC lattice, 4 per cubic cell."""
    basis = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5], [0.5, 0.5, 0.5]])
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    q = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a0
    return np.ascontiguousarray(q)


def vacancy_bulk(n_cells: int, n_vac: int, T: float, seed: int, sigma0: float = 0.1,
                 a0: float = A0_CU, name: str = "") -> System:
    q = fcc(n_cells, n_cells, n_cells, a0)
    n = q.shape[0]
    rng = np.random.default_rng(seed)
    x = np.ones(n)
    if n_vac == 1:
        x[int(rng.integers(n))] = 0.0
    elif n_vac > 1:
        x[rng.choice(n, n_vac, replace=False)] = 0.0
    L = n_cells * a0
    return System(q, np.full(n, sigma0), x, np.full(n, HOST_VAC, np.int8), (L, L, L),
                  (True, True, True), float(T), name)


def alloy_bulk(n_cells: int, xbar: float, T: float, seed: int, sigma0: float = 0.1,
               a0: float = A0_CU, name: str = "") -> System:
    q = fcc(n_cells, n_cells, n_cells, a0)
    n = q.shape[0]
    rng = np.random.default_rng(seed)
    x = np.clip(xbar + rng.uniform(-0.01, 0.01, n), 0.0, 1.0)
    L = n_cells * a0
    return System(q, np.full(n, sigma0), x, np.full(n, ALLOY, np.int8), (L, L, L),
                  (True, True, True), float(T), name)


def config0(seed: int = 0) -> Workload:
    """Plain method, FP64: 4x4x4 periodic FCC (256 sites), one vacancy, T = 800 K."""
    s = vacancy_bulk(4, 1, 800.0, seed, name="c0_vacancy_256")
    p = dict(DEFAULT_PARAMS, max_relax=50)
    return Workload("c0_vacancy_256", [s], params=p, n_steps=20)


def config1(seed: int = 1) -> Workload:
    """Single large system: 40^3 periodic cells (256,000 sites), 1% vacancies, T = 1000 K."""
    s = vacancy_bulk(40, 2560, 1000.0, seed, name="c1_vacancy_256k")
    p = dict(DEFAULT_PARAMS, max_relax=30)
    return Workload("c1_vacancy_256k", [s], params=p, n_steps=100)


# FCC spacing at which the analytic EAM's energy per atom of species A is lowest
# at T = 0 (3.813 A for pair 0.3 exp(-8 (r/2.556 - 1)), density
# exp(-6 (r/2.556 - 1)), F = -sqrt(rho), cosine taper 4.5-5.0 A): a free surface
# needs the crystal near its own spacing
A0_EAM = 3.81


def config2(seed: int = 2) -> Workload:
    """Binary alloy slab: 32^3 cells (131,072 sites), periodic x,y, 20 A vacuum in z
    (10 A on each side), T = 900 K, at the potential's own FCC spacing A0_EAM."""
    n_c = 32
    q = fcc(n_c, n_c, n_c, A0_EAM)
    q[:, 2] += 10.0
    n = q.shape[0]
    rng = np.random.default_rng(seed)
    x = 0.05 + rng.uniform(-0.01, 0.01, n)
    L = n_c * A0_EAM
    s = System(q, np.full(n, 0.1), x, np.full(n, ALLOY, np.int8), (L, L, L + 20.0),
               (True, True, False), 900.0, "c2_alloy_slab_131k")
    p = dict(DEFAULT_PARAMS, max_relax=30)
    return Workload("c2_alloy_slab_131k", [s], params=p, n_steps=500, precision="fp32")


def nanowire(radius: float = 50.0, n_axial: int = 55, x_shell: float = 0.1, T: float = 600.0,
             a0: float = A0_CU, name: str = "c3_nanowire", caged: bool = False) -> System:
    """FCC host cylinder along [001] (fixed host atoms) plus its octahedral sites.

    Octahedral sites with r_perp > radius - a0 start at x = x_shell, the rest at 0.
    caged: keep only octahedral sites whose six host neighbours (a0/2 away along
    x, y, z) all lie in the cylinder; otherwise every octahedral position within
    the radius, as the paper counts them for its Pd wire.
    """
    n_lat = int(math.ceil(2.0 * radius / a0)) + 2
    Lxy = n_lat * a0
    c = 0.5 * Lxy
    host = fcc(n_lat, n_lat, n_axial, a0)
    octa = octahedral(n_lat, n_lat, n_axial, a0)
    rh = np.hypot(host[:, 0] - c, host[:, 1] - c)
    ro = np.hypot(octa[:, 0] - c, octa[:, 1] - c)
    host = host[rh <= radius]
    keep = ro <= radius
    if caged:
        for dx, dy in ((0.5 * a0, 0.0), (-0.5 * a0, 0.0), (0.0, 0.5 * a0), (0.0, -0.5 * a0)):
            keep &= np.hypot(octa[:, 0] + dx - c, octa[:, 1] + dy - c) <= radius
    octa = octa[keep]
    ro = ro[keep]
    q = np.concatenate([host, octa], axis=0)
    t = np.concatenate([np.full(host.shape[0], HOST_FIXED, np.int8),
                        np.full(octa.shape[0], INTERSTITIAL, np.int8)])
    x = np.concatenate([np.ones(host.shape[0]), np.where(ro > radius - a0, x_shell, 0.0)])
    return System(np.ascontiguousarray(q), np.full(q.shape[0], 0.1), x, t,
                  (Lxy, Lxy, n_axial * a0), (False, False, True), float(T), name)


def config3(seed: int = 3) -> Workload:
    """Interstitial solute in a host nanowire: R = 50 A, 55 cells along the axis, T = 600 K.
    Octahedral sites with complete host cages only: with no solute-solute pair,
    nothing confines a solute on a site whose cage the surface cuts, and its
    width would grow without bound."""
    s = nanowire(name="c3_nanowire_256k", caged=True)
    # host sites see ~54 host and ~68-86 octahedral neighbours inside the list radius
    p = dict(DEFAULT_PARAMS, max_relax=30, k_max=160, **PDH_KINETICS)
    return Workload("c3_nanowire_256k", [s], params=p, n_steps=300, precision="fp32")


def config4_requests(seed: int = 4, n_requests: int = 256, n_min: int = 500,
                     n_max: int = 50_000) -> list:
    """Serving sweep: vacancy or alloy systems, cubic sizes log-uniform in [n_min, n_max]."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_requests):
        n_target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        cells = max(5, int(round((n_target / 4.0) ** (1.0 / 3.0))))
        T = float(rng.uniform(600.0, 1200.0))
        sub = int(rng.integers(1 << 30))
        if rng.random() < 0.5:
            s = vacancy_bulk(cells, 1, T, sub, name=f"req{r}_vac{cells}")
        else:
            xbar = float(rng.uniform(0.0, 0.1))
            s = alloy_bulk(cells, xbar, T, sub, name=f"req{r}_alloy{cells}")
        out.append(s)
    return out


def cluster(n_shells: int, T: float = 800.0, a0: float = A0_CU) -> System:
    """Open FCC cluster: a centre site plus its first 1 (13 sites) or 3 (43 sites) shells."""
    q = fcc(5, 5, 5, a0)
    c = q[(q.shape[0] // 2)]
    c = np.array([2.0, 2.0, 2.0]) * a0
    d = np.linalg.norm(q - c, axis=1)
    shells = {1: 0.75, 2: 1.05, 3: 1.3}
    keep = d < shells[n_shells] * a0 + 1e-9
    q = q[keep] - c + 20.0
    n = q.shape[0]
    return System(np.ascontiguousarray(q), np.full(n, 0.1), np.ones(n),
                  np.full(n, HOST_VAC, np.int8), (40.0 + a0, 40.0 + a0, 40.0 + a0),
                  (False, False, False), float(T), f"cluster{n}")


def jitter(s: System, seed: int, dq: float = 0.05, sig=(0.07, 0.13), xr=None) -> System:
    """Random perturbation of a system: q +- dq, sigma uniform in sig, x uniform in xr."""
    rng = np.random.default_rng(seed)
    t = s.copy()
    t.q = t.q + rng.uniform(-dq, dq, t.q.shape)
    t.sigma = rng.uniform(sig[0], sig[1], t.n)
    if xr is not None:
        mob = t.type != HOST_FIXED
        t.x = np.where(mob, rng.uniform(xr[0], xr[1], t.n), 1.0)
    return t


def concat(systems: list):
    """Concatenate systems into flat SoA arrays plus per-system offsets."""
    q = np.concatenate([s.q for s in systems], axis=0)
    sigma = np.concatenate([s.sigma for s in systems])
    x = np.concatenate([s.x for s in systems])
    t = np.concatenate([s.type for s in systems])
    off = np.cumsum([0] + [s.n for s in systems])
    return q, sigma, x, t, off
