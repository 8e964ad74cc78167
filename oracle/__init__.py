"""Plain FP64 CPU oracle of the MXE method (arXiv:1910.01235) -- ctypes wrapper.

TEST INFRASTRUCTURE ONLY. Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU product path (``paper_1910_01235_amd``) and imports nothing from
it; both sides receive the same seeded inputs from the input generators.

What each function computes, and the passage of the paper it follows, is
stated in ``mxe_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmxe_oracle.so")
_SRC = os.path.join(_HERE, "mxe_oracle.c")

OK = 0

SITE_HOST_VAC, SITE_ALLOY, SITE_INTERSTITIAL, SITE_HOST_FIXED = 0, 1, 2, 3


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math), OpenMP over sites."""
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Eam(C.Structure):
    _fields_ = [("embed_c", C.c_double * 3), ("emit_b", C.c_double * 3),
                ("pair_a", (C.c_double * 3) * 3), ("r_e", C.c_double * 2),
                ("alpha", C.c_double * 2), ("gamma", C.c_double * 2),
                ("r_s", C.c_double), ("r_c", C.c_double), ("quad_rule", C.c_int)]


RES_NONE, RES_FIX_X, RES_FIX_MU = 0, 1, 2


class _Box(C.Structure):
    _fields_ = [("n", C.c_int), ("box", C.c_double * 3), ("periodic", C.c_int * 3),
                ("T", C.c_double), ("res", C.POINTER(C.c_int8)), ("res_val", C.POINTER(C.c_double)),
                ("T_site", C.POINTER(C.c_double))]


class _Params(C.Structure):
    _fields_ = [("nu0", C.c_double), ("Qm", C.c_double), ("kin_c", C.c_double),
                ("dt_safety", C.c_double), ("max_relax", C.c_int), ("ftol", C.c_double),
                ("dt0", C.c_double), ("dtmax", C.c_double), ("alpha0", C.c_double),
                ("finc", C.c_double), ("fdec", C.c_double), ("falpha", C.c_double),
                ("nmin", C.c_int), ("sigma_min", C.c_double), ("r_bond", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _lib.oref_num_threads.restype = C.c_int
        _lib.oref_set_num_threads.argtypes = [C.c_int]
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int)) if a is not None else None


def _bp(a):
    return a.ctypes.data_as(C.POINTER(C.c_int8)) if a is not None else None


def make_eam(eam: dict) -> _Eam:
    e = _Eam()
    for k in range(3):
        e.embed_c[k] = eam["embed_c"][k]
        e.emit_b[k] = eam["emit_b"][k]
        for l in range(3):
            e.pair_a[k][l] = eam["pair_a"][k][l]
    for c in range(2):
        e.r_e[c] = eam["r_e"][c]
        e.alpha[c] = eam["alpha"][c]
        e.gamma[c] = eam["gamma"][c]
    e.r_s = eam["r_s"]
    e.r_c = eam["r_c"]
    e.quad_rule = int(eam.get("quad_rule", 0))
    return e


def make_box(n, box, periodic, T, res=None, res_val=None, T_site=None) -> _Box:
    """System description; res / res_val: optional per-site reservoir kinds and held values;
    T_site: optional per-site temperatures (T is then the reference temperature)."""
    b = _Box()
    b.n = int(n)
    for a in range(3):
        b.box[a] = float(box[a])
        b.periodic[a] = int(bool(periodic[a]))
    b.T = float(T)
    b._keep = []
    if res is not None:
        r = np.ascontiguousarray(res, dtype=np.int8)
        v = np.ascontiguousarray(res_val, dtype=np.float64)
        assert r.shape == (n,) and v.shape == (n,)
        b._keep += [r, v]
        b.res = _bp(r)
        b.res_val = _dp(v)
    if T_site is not None:
        t = np.ascontiguousarray(T_site, dtype=np.float64)
        assert t.shape == (n,)
        b._keep.append(t)
        b.T_site = _dp(t)
    return b


def make_params(p: dict) -> _Params:
    q = _Params()
    for name, _ in _Params._fields_:
        setattr(q, name, p[name])
    return q


def num_threads() -> int:
    return lib().oref_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops (CPU-baseline timing)."""
    lib().oref_set_num_threads(int(n))


def quadrature():
    z = np.zeros((27, 3))
    w = np.zeros(27)
    lib().oref_quadrature(_dp(z), _dp(w))
    return z, w


def shape(eam: dict, r: float, r_e: float, a: float):
    g = C.c_double()
    dg = C.c_double()
    e = make_eam(eam)
    lib().oref_shape(C.byref(e), C.c_double(r), C.c_double(r_e), C.c_double(a),
                     C.byref(g), C.byref(dg))
    return g.value, dg.value


def pair_average(eam: dict, cls: int, rbar, s: float) -> np.ndarray:
    """14 moments: <phi>, grad<phi>(3), d<phi>/ds, <f>, grad<f>(3), d<f>/ds, f0, grad f0(3)."""
    e = make_eam(eam)
    rb = np.ascontiguousarray(rbar, dtype=np.float64)
    out = np.zeros(14)
    lib().oref_pair_average(C.byref(e), C.c_int(cls), _dp(rb), C.c_double(s), _dp(out))
    return out


def stroud_nodes(sigma_i: float, sigma_j: float):
    """Degree-3 rule of the pair: (12, 6) displacements (dq_i, dq_j) and 12 weights."""
    off = np.zeros((12, 6))
    w = np.zeros(12)
    lib().oref_stroud_nodes(C.c_double(sigma_i), C.c_double(sigma_j), _dp(off), _dp(w))
    return off, w


def pair_moments(eam: dict, cls: int, rbar, sigma_i: float, sigma_j: float) -> np.ndarray:
    """16 moments under eam["quad_rule"]: <phi>, grad<phi>(3), d<phi>/dsigma_i, <f>,
    grad<f>(3), d<f>/dsigma_i, f0, grad f0(3), d<phi>/dsigma_j, d<f>/dsigma_j."""
    e = make_eam(eam)
    rb = np.ascontiguousarray(rbar, dtype=np.float64)
    out = np.zeros(16)
    lib().oref_pair_moments(C.byref(e), C.c_int(cls), _dp(rb), C.c_double(sigma_i),
                            C.c_double(sigma_j), _dp(out))
    return out


def _state(q, sigma, x, type_):
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    type_ = np.ascontiguousarray(type_, dtype=np.int8)
    n = q.shape[0]
    assert sigma.shape == (n,) and x.shape == (n,) and type_.shape == (n,)
    return q, sigma, x, type_, n


def evaluate(eam, box, periodic, T, q, sigma, x, type_, res=None, res_val=None, T_site=None):
    """Full evaluation. Returns a dict of numpy arrays and the total F."""
    q, sigma, x, type_, n = _state(q, sigma, x, type_)
    e = make_eam(eam)
    b = make_box(n, box, periodic, T, res, res_val, T_site)
    out = {k: np.zeros(n) for k in ("rho_bar", "rho0", "mu", "e_site")}
    out["grad"] = np.zeros((n, 4))
    out["force"] = np.zeros((n, 4))
    F = C.c_double()
    st = lib().oref_evaluate(C.byref(e), C.byref(b), _dp(q), _dp(sigma), _dp(x), _bp(type_),
                             _dp(out["rho_bar"]), _dp(out["rho0"]), _dp(out["grad"]),
                             _dp(out["force"]), _dp(out["mu"]), _dp(out["e_site"]), C.byref(F))
    if st != OK:
        raise RuntimeError(f"oracle evaluate failed: status {st}")
    out["F"] = F.value
    return out


def free_energy(eam, box, periodic, T, q, sigma, x, type_, res=None, res_val=None, T_site=None) -> float:
    q, sigma, x, type_, n = _state(q, sigma, x, type_)
    e = make_eam(eam)
    b = make_box(n, box, periodic, T, res, res_val, T_site)
    F = C.c_double()
    st = lib().oref_evaluate(C.byref(e), C.byref(b), _dp(q), _dp(sigma), _dp(x), _bp(type_),
                             None, None, None, None, None, None, C.byref(F))
    if st != OK:
        raise RuntimeError(f"oracle evaluate failed: status {st}")
    return F.value


def evaluate_sites(eam, box, periodic, T, q, sigma, x, type_, sel, res=None, res_val=None, T_site=None):
    q, sigma, x, type_, n = _state(q, sigma, x, type_)
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    m = sel.shape[0]
    e = make_eam(eam)
    b = make_box(n, box, periodic, T, res, res_val, T_site)
    out = {k: np.zeros(m) for k in ("rho_bar", "rho0", "mu", "e_site")}
    out["force"] = np.zeros((m, 4))
    st = lib().oref_evaluate_sites(C.byref(e), C.byref(b), _dp(q), _dp(sigma), _dp(x),
                                   _bp(type_), C.c_int(m), _ip(sel), _dp(out["rho_bar"]),
                                   _dp(out["rho0"]), _dp(out["force"]), _dp(out["mu"]),
                                   _dp(out["e_site"]))
    if st != OK:
        raise RuntimeError(f"oracle evaluate_sites failed: status {st}")
    return out


def neighbors(box, periodic, q, radius, method, kmax=256):
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    n = q.shape[0]
    b = make_box(n, box, periodic, 300.0)
    counts = np.zeros(n, dtype=np.int32)
    lst = np.full((n, kmax), -1, dtype=np.int32)
    tot = lib().oref_neighbors(C.byref(b), _dp(q), C.c_double(radius), C.c_int(method),
                               C.c_int(kmax), _ip(counts), _ip(lst))
    if tot < 0:
        raise RuntimeError(f"oracle neighbors failed: {tot}")
    return counts, lst


def bonds(box, periodic, q, type_, r_bond, bmax=16):
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1, 3)
    type_ = np.ascontiguousarray(type_, dtype=np.int8)
    n = q.shape[0]
    b = make_box(n, box, periodic, 300.0)
    nb = np.zeros(n, dtype=np.int32)
    bl = np.full((n, bmax), -1, dtype=np.int32)
    st = lib().oref_bonds(C.byref(b), _dp(q), _bp(type_), C.c_double(r_bond), C.c_int(bmax),
                          _ip(nb), _ip(bl))
    if st != OK:
        raise RuntimeError(f"oracle bonds failed: {st}")
    return nb, bl


def master_rates(params, box, periodic, T, x, type_, mu, nbond, bond_list, res=None, res_val=None, T_site=None):
    x = np.ascontiguousarray(x, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    type_ = np.ascontiguousarray(type_, dtype=np.int8)
    nbond = np.ascontiguousarray(nbond, dtype=np.int32)
    bond_list = np.ascontiguousarray(bond_list, dtype=np.int32)
    n = x.shape[0]
    b = make_box(n, box, periodic, T, res, res_val, T_site)
    p = make_params(params)
    dxdt = np.zeros(n)
    dt = C.c_double()
    lib().oref_master_rates(C.byref(b), C.byref(p), _dp(x), _bp(type_), _dp(mu),
                            C.c_int(bond_list.shape[1]), _ip(nbond), _ip(bond_list), _dp(dxdt),
                            C.byref(dt))
    return dxdt, dt.value


def master_step(params, box, periodic, T, x, type_, mu, nbond, bond_list, dt_in=0.0, res=None,
                res_val=None, T_site=None):
    """One Euler step of x with held reservoir sites; returns (x, dxdt, dt, uptake)."""
    x = np.ascontiguousarray(x, dtype=np.float64).copy()
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    type_ = np.ascontiguousarray(type_, dtype=np.int8)
    nbond = np.ascontiguousarray(nbond, dtype=np.int32)
    bond_list = np.ascontiguousarray(bond_list, dtype=np.int32)
    n = x.shape[0]
    b = make_box(n, box, periodic, T, res, res_val, T_site)
    p = make_params(params)
    dxdt = np.zeros(n)
    dt = C.c_double()
    up = C.c_double(0.0)
    st = lib().oref_master_step(C.byref(b), C.byref(p), _dp(x), _bp(type_), _dp(mu),
                                C.c_int(bond_list.shape[1]), _ip(nbond), _ip(bond_list),
                                C.c_double(dt_in), _dp(dxdt), C.byref(dt), C.byref(up))
    if st != OK:
        raise RuntimeError(f"oracle master_step failed: {st}")
    return x, dxdt, dt.value, up.value


def relax(eam, params, box, periodic, T, q, sigma, x, type_, res=None, res_val=None, T_site=None):
    """FIRE relaxation; returns (q, sigma, info dict) with the last evaluation's outputs."""
    q, sigma, x, type_, n = _state(q, sigma, x, type_)
    q = q.copy()
    sigma = sigma.copy()
    e = make_eam(eam)
    b = make_box(n, box, periodic, T, res, res_val, T_site)
    p = make_params(params)
    force = np.zeros((n, 4))
    mu = np.zeros(n)
    es = np.zeros(n)
    F = C.c_double()
    fmax = C.c_double()
    conv = C.c_int()
    nev = C.c_int()
    upd = lib().oref_relax(C.byref(e), C.byref(b), C.byref(p), _dp(q), _dp(sigma), _dp(x),
                           _bp(type_), _dp(force), _dp(mu), _dp(es), C.byref(F), C.byref(fmax),
                           C.byref(conv), C.byref(nev))
    if upd < 0:
        raise RuntimeError(f"oracle relax failed: {upd}")
    return q, sigma, dict(updates=upd, converged=bool(conv.value), n_evals=nev.value,
                          force=force, mu=mu, e_site=es, F=F.value, fmax=fmax.value)


def run(eam, params, box, periodic, T, n_steps, q, sigma, x, type_, t0=0.0, res=None, res_val=None, T_site=None):
    """Staggered relax + master-equation run. Returns final state and per-step records."""
    q, sigma, x, type_, n = _state(q, sigma, x, type_)
    q = q.copy()
    sigma = sigma.copy()
    x = x.copy()
    e = make_eam(eam)
    b = make_box(n, box, periodic, T, res, res_val, T_site)
    p = make_params(params)
    mu = np.zeros(n)
    dxdt = np.zeros(n)
    t = C.c_double(t0)
    rec = np.zeros((n_steps, 7))
    st = lib().oref_run(C.byref(e), C.byref(b), C.byref(p), C.c_int(n_steps), _dp(q),
                        _dp(sigma), _dp(x), _bp(type_), _dp(mu), _dp(dxdt), C.byref(t), _dp(rec))
    if st != OK:
        raise RuntimeError(f"oracle run failed: {st}")
    return dict(q=q, sigma=sigma, x=x, mu=mu, dxdt=dxdt, t=t.value, updates=rec[:, 0],
                converged=rec[:, 1], F=rec[:, 2], fmax=rec[:, 3], dt=rec[:, 4], sum_x=rec[:, 5],
                uptake=rec[:, 6])
