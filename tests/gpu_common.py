"""Shared helpers of the GPU tests: oracle references and error measures."""
import sys

import numpy as np

import oracle as O
from paper_1910_01235_amd import lattice as L


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a, b, floor):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))


def oracle_eval(eam, s):
    return O.evaluate(eam, s.box, s.periodic, s.T, s.q, s.sigma, s.x, s.type)


def gpu_arrays(plan, st, out, k=None):
    """Host copies of the outputs, optionally of system k only."""
    lo, hi = (0, plan.n_sites) if k is None else (plan.offsets[k], plan.offsets[k + 1])
    g = lambda t: t[lo:hi].cpu().numpy()
    return dict(force=np.stack([g(out.fx), g(out.fy), g(out.fz), g(out.fsigma)], axis=1),
                mu=g(out.mu), rho_bar=g(out.rho_bar), rho0=g(out.rho0), e_site=g(out.e_site),
                dxdt=g(out.dxdt), q=np.stack([g(st.qx), g(st.qy), g(st.qz)], axis=1),
                sigma=g(st.sigma), x=g(st.x))


def eval_errors(g, o, mobile=None):
    """Normwise relative errors per output (absolute floor for near-zero arrays)."""
    errs = dict(
        force_q=rel_err(g["force"][:, :3], o["force"][:, :3], 1e-2),
        force_s=rel_err(g["force"][:, 3], o["force"][:, 3], 1e-2),
        mu=rel_err(g["mu"], o["mu"], 1e-2),
        rho_bar=rel_err(g["rho_bar"], o["rho_bar"], 1.0),
        rho0=rel_err(g["rho0"], o["rho0"], 1.0),
        e_site=rel_err(g["e_site"], o["e_site"], 1e-2),
    )
    return errs


def parity_systems():
    """Small systems spanning several chunks and tiles with ragged tails."""
    out = []
    out.append(("c0_vacancy", L.config0(0).systems[0]))
    out.append(("bulk5_jitter", L.jitter(L.vacancy_bulk(5, 3, 900.0, 1), 2, xr=(0.2, 0.9))))
    a = L.jitter(L.alloy_bulk(6, 0.3, 900.0, 2), 3, xr=(0.05, 0.95))
    out.append(("alloy6_jitter", a))
    w = L.jitter(L.nanowire(radius=9.0, n_axial=5, T=700.0), 4, xr=(0.0, 0.9))
    out.append(("wire_interstitial", w))
    n = 6 * 6 * 5 * 4
    slab = L.System(L.fcc(6, 6, 5), np.full(n, 0.1), np.full(n, 0.05), np.full(n, L.ALLOY, np.int8),
                    (6 * L.A0_CU, 6 * L.A0_CU, 5 * L.A0_CU + 20.0), (True, True, False), 900.0, "slab")
    out.append(("slab_open_z", L.jitter(slab, 5, xr=(0.02, 0.2))))
    c = L.jitter(L.cluster(3), 6, xr=(0.2, 0.9))
    out.append(("cluster43", c))
    return out
