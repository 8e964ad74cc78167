"""Point-source vacancy spreading (Sec. 5.1): measures and the continuum solution.

A single vacancy (x = 0 at one site of a full FCC crystal) spreads under the
kinetic law. Its continuum limit is the point-source solution of the diffusion
equation used in Sec. 5.1, c(d, t) = Omega (4 pi D t)^(-3/2) exp(-d^2 / (4 D t))
per site, Omega the volume per site, with the macroscopic diffusivity
D = Z b^2 D_ij / (2 d_dim) (Sec. 3.1, dimensionally corrected). For the linear
law the second moment of the vacancy distribution grows by exactly
Z b^2 D_ij dt per Euler step.
"""
import math

import numpy as np

from paper_1910_01235_amd import lattice as L

Z_FCC = 12
B_NN = L.A0_CU / math.sqrt(2.0)
OMEGA = L.A0_CU ** 3 / 4.0


def single_vacancy(n_cells: int, T: float):
    q = L.fcc(n_cells, n_cells, n_cells)
    n = q.shape[0]
    box = np.array([n_cells * L.A0_CU] * 3)
    d = q - box / 2
    v0 = int(np.argmin(np.linalg.norm(d, axis=1)))
    x = np.ones(n)
    x[v0] = 0.0
    s = L.System(q, np.full(n, 0.1), x, np.full(n, L.HOST_VAC, np.int8), tuple(box), (True,) * 3, T,
                 f"vacancy_point_source_{n}")
    return s, v0


def distances(s, v0):
    d = s.q - s.q[v0]
    box = np.array(s.box)
    d -= box * np.round(d / box)
    return np.linalg.norm(d, axis=1)


def second_moment(v, r):
    return float((v * r ** 2).sum())


def continuum(r, t, D_macro):
    return OMEGA * (4 * math.pi * D_macro * t) ** -1.5 * np.exp(-r ** 2 / (4 * D_macro * t))


def profile_error(v, r, t, D_macro, within=2.0):
    """Relative L2 difference between the lattice and continuum profiles within `within` rms radii."""
    c = continuum(r, t, D_macro)
    rms = math.sqrt(6 * D_macro * t)
    w = r < within * rms
    return float(np.sqrt(((v - c) ** 2)[w].sum() / (c ** 2)[w].sum()))
