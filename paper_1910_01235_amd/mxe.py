"""ctypes binding of the C ABI in include/mxe.h.

Argument marshalling only: every step of the hot path runs in the HIP library.
PyTorch supplies device memory and the stream. Importing this module does not
touch the GPU; loading the library fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmxe.so")

FP64, FP32_MIXED = 0, 1
QUAD_GH27, QUAD_DEGREE3 = 0, 1
RES_NONE, RES_FIX_X, RES_FIX_MU = 0, 1, 2
NSCALARS = 16
S_F, S_FMAX, S_DT, S_TIME, S_SUMX, S_UPDATES, S_CONVERGED, S_EVALS, S_STATUS, S_REBUILDS, \
    S_TOTAL_EVALS, S_PAIRS, S_PAIR_EVALS, S_RESERVOIR, S_STEPS_LEFT = range(15)
K_PAIR, K_DENSITY, K_FORCE, K_BUILD, K_FIRE, K_MASTER = range(6)
KERNEL_FAMILIES = ["pair", "density", "force", "build", "fire", "master"]
PROFILE_OFF, PROFILE_ALL, PROFILE_PAIR = 0, 1, 2  # mxe_profile modes
L_NBR, L_NBR_COUNT, L_BOND, L_BOND_COUNT = range(4)  # mxe_plan_layout items
STAT_NONFINITE, STAT_X_RANGE, STAT_RHO, STAT_SIGMA_MIN, STAT_KMAX, STAT_TEMP, STAT_PAIRS, \
    STAT_BONDS, STAT_SIGMA_CAP = (1 << k for k in range(9))
FATAL_STATUS = STAT_NONFINITE | STAT_X_RANGE | STAT_RHO | STAT_KMAX | STAT_PAIRS | STAT_BONDS | \
    STAT_SIGMA_CAP | STAT_TEMP

EXPORTED = ["mxe_default_params", "mxe_plan_create", "mxe_plan_destroy", "mxe_workspace_bytes",
            "mxe_plan_sites", "mxe_plan_set_system", "mxe_plan_check_system", "mxe_plan_slot_offset",
            "mxe_plan_set_resume", "mxe_plan_layout", "mxe_plan_set_steps",
            "mxe_evaluate", "mxe_relax", "mxe_step", "mxe_run", "mxe_advance", "mxe_run_noalloc",
            "mxe_profile", "mxe_profile_read",
            "mxe_status_string", "mxe_last_error"]


class Eam(C.Structure):
    _fields_ = [("embed_c", C.c_double * 3), ("emit_b", C.c_double * 3),
                ("pair_a", (C.c_double * 3) * 3), ("r_e", C.c_double * 2),
                ("alpha", C.c_double * 2), ("gamma", C.c_double * 2),
                ("r_s", C.c_double), ("r_c", C.c_double)]


class Params(C.Structure):
    _fields_ = [("nu0", C.c_double), ("Qm", C.c_double), ("kin_c", C.c_double),
                ("dt_safety", C.c_double), ("max_relax", C.c_int), ("ftol", C.c_double),
                ("fire_dt0", C.c_double), ("fire_dtmax", C.c_double), ("fire_alpha0", C.c_double),
                ("fire_finc", C.c_double), ("fire_fdec", C.c_double), ("fire_falpha", C.c_double),
                ("fire_nmin", C.c_int), ("sigma_min", C.c_double), ("sigma_cap", C.c_double),
                ("skin", C.c_double), ("r_bond", C.c_double), ("k_max", C.c_int),
                ("bond_max", C.c_int), ("precision", C.c_int), ("gather_lanes", C.c_int),
                ("pair_block", C.c_int), ("quad_rule", C.c_int), ("force_lanes", C.c_int),
                ("gather_stride", C.c_int), ("relax_chunk", C.c_int),
                ("pair_split", C.c_int)]


class System(C.Structure):
    _fields_ = [("n_sites", C.c_int64), ("box", C.c_double * 3), ("periodic", C.c_int * 3),
                ("T", C.c_double)]


class State(C.Structure):
    _fields_ = [("qx", C.c_void_p), ("qy", C.c_void_p), ("qz", C.c_void_p),
                ("sigma", C.c_void_p), ("x", C.c_void_p), ("type", C.c_void_p),
                ("reservoir", C.c_void_p), ("res_value", C.c_void_p), ("T_site", C.c_void_p)]


class Out(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("fx", "fy", "fz", "fsigma", "mu", "dxdt", "rho_bar",
                                          "rho0", "e_site", "scalars")]


_lib = None


def lib():
    """Load libmxe.so (raises if it was not built: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_1910_01235_amd.build")
        L = C.CDLL(LIB_PATH)
        L.mxe_plan_create.argtypes = [C.POINTER(Params), C.POINTER(Eam), C.c_int,
                                      C.POINTER(System), C.POINTER(C.c_void_p)]
        L.mxe_plan_create.restype = C.c_int
        L.mxe_plan_destroy.argtypes = [C.c_void_p]
        L.mxe_workspace_bytes.argtypes = [C.c_void_p, C.POINTER(C.c_size_t)]
        L.mxe_workspace_bytes.restype = C.c_int
        L.mxe_plan_sites.argtypes = [C.c_void_p]
        L.mxe_plan_sites.restype = C.c_int64
        L.mxe_plan_set_system.argtypes = [C.c_void_p, C.c_int, C.POINTER(System)]
        L.mxe_plan_set_system.restype = C.c_int
        L.mxe_plan_check_system.argtypes = [C.c_void_p, C.c_int, C.POINTER(System)]
        L.mxe_plan_check_system.restype = C.c_int
        L.mxe_plan_layout.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_size_t),
                                      C.POINTER(C.c_size_t)]
        L.mxe_plan_layout.restype = C.c_int
        L.mxe_plan_slot_offset.argtypes = [C.c_void_p, C.c_int]
        L.mxe_plan_slot_offset.restype = C.c_int64
        L.mxe_plan_set_resume.argtypes = [C.c_void_p, C.c_int]
        L.mxe_plan_set_resume.restype = C.c_int
        for name in ("mxe_evaluate", "mxe_relax"):
            getattr(L, name).argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(Out), C.c_void_p,
                                         C.c_size_t, C.c_void_p]
            getattr(L, name).restype = C.c_int
        L.mxe_step.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(Out), C.c_double,
                               C.c_void_p, C.c_size_t, C.c_void_p]
        L.mxe_step.restype = C.c_int
        L.mxe_run.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(Out), C.c_int, C.c_int,
                              C.c_void_p, C.c_size_t, C.c_void_p]
        L.mxe_run.restype = C.c_int
        L.mxe_advance.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(Out), C.c_int, C.c_int,
                                  C.c_void_p, C.c_size_t, C.c_void_p]
        L.mxe_advance.restype = C.c_int
        L.mxe_plan_set_steps.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.mxe_plan_set_steps.restype = C.c_int
        L.mxe_run_noalloc.argtypes = [C.c_void_p, C.POINTER(State), C.POINTER(Out), C.c_int,
                                      C.c_void_p]
        L.mxe_run_noalloc.restype = C.c_int
        L.mxe_status_string.argtypes = [C.c_int]
        L.mxe_status_string.restype = C.c_char_p
        L.mxe_last_error.restype = C.c_char_p
        L.mxe_default_params.argtypes = [C.POINTER(Params)]
        L.mxe_profile.argtypes = [C.c_void_p, C.c_int]
        L.mxe_profile.restype = C.c_int
        L.mxe_profile_read.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.mxe_profile_read.restype = C.c_int
        _lib = L
    return _lib


class MxeError(RuntimeError):
    pass


def _check(code: int):
    if code != 0:
        L = lib()
        raise MxeError(f"{L.mxe_status_string(code).decode()}: {L.mxe_last_error().decode()}")


def default_params() -> Params:
    p = Params()
    lib().mxe_default_params(C.byref(p))
    return p


# keys of the workload parameter dicts and their ABI names
_PARAM_MAP = dict(nu0="nu0", Qm="Qm", kin_c="kin_c", dt_safety="dt_safety",
                  max_relax="max_relax", ftol="ftol", dt0="fire_dt0", dtmax="fire_dtmax",
                  alpha0="fire_alpha0", finc="fire_finc", fdec="fire_fdec", falpha="fire_falpha",
                  nmin="fire_nmin", sigma_min="sigma_min", r_bond="r_bond", sigma_cap="sigma_cap",
                  skin="skin", k_max="k_max", bond_max="bond_max", gather_lanes="gather_lanes",
                  pair_block="pair_block", quad_rule="quad_rule", force_lanes="force_lanes",
                  gather_stride="gather_stride", relax_chunk="relax_chunk",
                  pair_split="pair_split")


def make_params(params: dict, precision: str = "fp64", **over) -> Params:
    p = default_params()
    for k, v in {**params, **over}.items():
        if k in _PARAM_MAP:
            setattr(p, _PARAM_MAP[k], v)
    p.precision = FP32_MIXED if precision in ("fp32", "fp32_mixed", "mixed") else FP64
    return p


def make_eam(eam: dict) -> Eam:
    e = Eam()
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
    return e


@dataclass
class DeviceState:
    qx: "torch.Tensor"
    qy: "torch.Tensor"
    qz: "torch.Tensor"
    sigma: "torch.Tensor"
    x: "torch.Tensor"
    type: "torch.Tensor"
    reservoir: "torch.Tensor" = None   # int8 kinds (RES_*), optional
    res_value: "torch.Tensor" = None   # held x or mu, FP64, optional
    T_site: "torch.Tensor" = None      # per-site temperature (K), FP64, optional

    def abi(self) -> State:
        opt = lambda t: t.data_ptr() if t is not None else None
        return State(self.qx.data_ptr(), self.qy.data_ptr(), self.qz.data_ptr(),
                     self.sigma.data_ptr(), self.x.data_ptr(), self.type.data_ptr(),
                     opt(self.reservoir), opt(self.res_value), opt(self.T_site))

    def q(self):
        import torch
        return torch.stack([self.qx, self.qy, self.qz], dim=1)


@dataclass
class DeviceOut:
    fx: "torch.Tensor"
    fy: "torch.Tensor"
    fz: "torch.Tensor"
    fsigma: "torch.Tensor"
    mu: "torch.Tensor"
    dxdt: "torch.Tensor"
    rho_bar: "torch.Tensor"
    rho0: "torch.Tensor"
    e_site: "torch.Tensor"
    scalars: "torch.Tensor"

    def abi(self) -> Out:
        return Out(*(getattr(self, n).data_ptr() for n, _ in Out._fields_))

    def force(self):
        import torch
        return torch.stack([self.fx, self.fy, self.fz, self.fsigma], dim=1)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """A plan over one or more systems (sites concatenated in system order)."""

    def __init__(self, systems, eam: dict, params: dict, precision: str = "fp64", **over):
        L = lib()
        arr = (System * len(systems))()
        for k, s in enumerate(systems):
            arr[k].n_sites = int(s.n)
            for a in range(3):
                arr[k].box[a] = float(s.box[a])
                arr[k].periodic[a] = int(bool(s.periodic[a]))
            arr[k].T = float(s.T)
        if "quad_rule" in eam and "quad_rule" not in over:
            over = dict(over, quad_rule=int(eam["quad_rule"]))
        self.params = make_params(params, precision, **over)
        self.eam = make_eam(eam)
        self.n_systems = len(systems)
        self.precision = precision
        h = C.c_void_p()
        _check(L.mxe_plan_create(C.byref(self.params), C.byref(self.eam), len(systems), arr,
                                 C.byref(h)))
        self._h = h
        nb = C.c_size_t()
        _check(L.mxe_workspace_bytes(h, C.byref(nb)))
        self.ws_bytes = int(nb.value)
        self.n_sites = int(L.mxe_plan_sites(h))
        self.offsets = np.array([int(L.mxe_plan_slot_offset(h, k)) for k in range(len(systems) + 1)])

    @staticmethod
    def _system(s) -> System:
        m = System()
        m.n_sites = int(s.n) if s is not None else 0
        for a in range(3):
            m.box[a] = float(s.box[a]) if s is not None else 100.0
            m.periodic[a] = int(bool(s.periodic[a])) if s is not None else 0
        m.T = float(s.T) if s is not None else 300.0
        return m

    def set_system(self, slot: int, s):
        """Rebind a slot to system s (None empties it); applies from the next call."""
        m = self._system(s)
        _check(lib().mxe_plan_set_system(self._h, int(slot), C.byref(m)))

    def check_system(self, slot: int, s) -> bool:
        """Would set_system(slot, s) be accepted? (host-only; raises on a bad box or T)"""
        m = self._system(s)
        code = lib().mxe_plan_check_system(self._h, int(slot), C.byref(m))
        if code == -5:  # MXE_ERANGE: does not fit the slot
            return False
        _check(code)
        return True

    def layout(self, item: int):
        """(byte offset, bytes) of a workspace array (L_NBR, L_NBR_COUNT, L_BOND, L_BOND_COUNT)."""
        off, nb = C.c_size_t(), C.c_size_t()
        _check(lib().mxe_plan_layout(self._h, int(item), C.byref(off), C.byref(nb)))
        return int(off.value), int(nb.value)

    def lists(self, ws):
        """Host copies of the neighbour rows and bonds held in the workspace
        (valid after a call that built them, once the stream has synchronised)."""
        def arr(item, cols):
            off, nb = self.layout(item)
            a = ws[off:off + nb].view(dtype=__import__("torch").int32).cpu().numpy()
            return a.reshape(self.n_sites, cols) if cols else a
        return dict(nbr=arr(L_NBR, self.params.k_max), nbr_count=arr(L_NBR_COUNT, 0),
                    bond=arr(L_BOND, self.params.bond_max), bond_count=arr(L_BOND_COUNT, 0))

    def set_resume(self, on: bool):
        _check(lib().mxe_plan_set_resume(self._h, int(bool(on))))

    def set_steps(self, slot: int, n_steps: int):
        """Budget of free-running diffusion steps for a slot, from the next advance()."""
        _check(lib().mxe_plan_set_steps(self._h, int(slot), int(n_steps)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.mxe_plan_destroy(h)
            self._h = None

    # ---- buffers -------------------------------------------------------
    def workspace(self, device="cuda"):
        import torch
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def state(self, systems, device="cuda") -> DeviceState:
        import torch
        q = np.concatenate([s.q for s in systems], axis=0)
        assert q.shape[0] == self.n_sites, "systems do not match the plan"
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=device)
        return DeviceState(f(q[:, 0]), f(q[:, 1]), f(q[:, 2]),
                           f(np.concatenate([s.sigma for s in systems])),
                           f(np.concatenate([s.x for s in systems])),
                           torch.as_tensor(np.concatenate([s.type for s in systems]).astype(np.int8),
                                           device=device))

    def out(self, device="cuda") -> DeviceOut:
        import torch
        z = lambda: torch.zeros(self.n_sites, dtype=torch.float64, device=device)
        return DeviceOut(z(), z(), z(), z(), z(), z(), z(), z(), z(),
                         torch.zeros(self.n_systems * NSCALARS, dtype=torch.float64, device=device))

    # ---- calls ---------------------------------------------------------
    def evaluate(self, st: DeviceState, out: DeviceOut, ws, stream=None):
        a, o = st.abi(), out.abi()
        _check(lib().mxe_evaluate(self._h, C.byref(a), C.byref(o), C.c_void_p(ws.data_ptr()),
                                  ws.numel(), _stream_ptr(stream)))

    def relax(self, st: DeviceState, out: DeviceOut, ws, stream=None):
        a, o = st.abi(), out.abi()
        _check(lib().mxe_relax(self._h, C.byref(a), C.byref(o), C.c_void_p(ws.data_ptr()),
                               ws.numel(), _stream_ptr(stream)))

    def step(self, st: DeviceState, out: DeviceOut, ws, dt_in: float = 0.0, stream=None):
        a, o = st.abi(), out.abi()
        _check(lib().mxe_step(self._h, C.byref(a), C.byref(o), C.c_double(dt_in),
                              C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))

    def run(self, st: DeviceState, out: DeviceOut, ws, n_steps: int, use_graph: bool = True,
            stream=None):
        a, o = st.abi(), out.abi()
        _check(lib().mxe_run(self._h, C.byref(a), C.byref(o), int(n_steps), int(bool(use_graph)),
                             C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))

    def advance(self, st: DeviceState, out: DeviceOut, ws, max_iters: int, use_graph: bool = True,
                stream=None):
        """Up to max_iters free-running iterations (mxe_advance); stops early once no
        slot has steps left."""
        a, o = st.abi(), out.abi()
        _check(lib().mxe_advance(self._h, C.byref(a), C.byref(o), int(max_iters), int(bool(use_graph)),
                                 C.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)))

    def run_noalloc(self, st: DeviceState, out: DeviceOut, n_steps: int, stream=None):
        """mxe_run on the library's per-device scratch (no workspace argument)."""
        a, o = st.abi(), out.abi()
        _check(lib().mxe_run_noalloc(self._h, C.byref(a), C.byref(o), int(n_steps),
                                     _stream_ptr(stream)))

    def profile(self, on):
        """True: every kernel family bracketed by HIP events; "pair": only the pair
        kernel (the least instrumentation); False: off."""
        mode = PROFILE_PAIR if on == "pair" else (PROFILE_ALL if on else PROFILE_OFF)
        _check(lib().mxe_profile(self._h, mode))

    def profile_read(self):
        """{family: (summed ms, launches)} since the previous read (waits for the events)."""
        ms = (C.c_double * 6)()
        n = (C.c_int64 * 6)()
        _check(lib().mxe_profile_read(self._h, ms, n))
        return {KERNEL_FAMILIES[k]: (ms[k], int(n[k])) for k in range(6)}

    def scalars(self, out: DeviceOut) -> np.ndarray:
        return out.scalars.view(self.n_systems, NSCALARS).cpu().numpy()
