"""FP64 CPU oracle of the Hybrid-VPIC step (arXiv 2305.05600) -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C,
FP64, single-threaded, built from ``hvpic_oracle.c`` by ``oracle/build.py``)
and shares no code with the GPU library.

Arrays are numpy float64 (grid fields component-major, shape (3, ncell));
particles are a dict with keys cell, ox, oy, [oz], ux, uy, uz, w.
"""
from __future__ import annotations

import ctypes
import os
import pathlib

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_LIB = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("ndim", _i32), ("nx", _i32), ("ny", _i32), ("nz", _i32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("nsub", _i32), ("shape", _i32), ("nsmooth", _i32),
        ("qs", ctypes.c_double), ("ms", ctypes.c_double),
        ("te", ctypes.c_double), ("gamma_e", ctypes.c_double), ("n0", ctypes.c_double),
        ("n_floor", ctypes.c_double),
        ("eta", ctypes.c_double), ("eta_h", ctypes.c_double),
        ("energy_eq", _i32), ("kappa0", ctypes.c_double),
        ("open_x", _i32), ("buffer_cells", _i32), ("eta_h_buffer", ctypes.c_double),
    ]


class OrcInflow(ctypes.Structure):
    _fields_ = [("n", ctypes.c_double), ("ux", ctypes.c_double), ("uy", ctypes.c_double),
                ("uz", ctypes.c_double), ("vth", ctypes.c_double), ("ppc", _i32),
                ("faces", _i32)]


class OrcStatus(ctypes.Structure):
    _fields_ = [("moved_gt1", _i64), ("nonfinite", _i64), ("floor_hits", _i64)]


def lib():
    global _LIB
    if _LIB is None:
        path = _HERE / "liboracle.so"
        if not path.exists():
            from . import build as _build

            _build.build()
        L = ctypes.CDLL(str(path))
        P = ctypes.POINTER(OrcParams)
        S = ctypes.POINTER(OrcStatus)
        L.orc_gather.argtypes = [P, _dp, _i32, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _dp]
        L.orc_boris.argtypes = [ctypes.c_double, _dp, _dp, _dp]
        L.orc_push.argtypes = [P, _i64, _ip, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                               _dp, S]
        L.orc_sort.argtypes = [P, _i64, _ip, _lp, _ip]
        L.orc_deposit.argtypes = [P, _i64, _ip, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                  ctypes.c_double, _dp, _dp]
        L.orc_smooth.argtypes = [P, _dp, _i32, _i32]
        L.orc_curl.argtypes = [P, _dp, _dp]
        L.orc_ohm.argtypes = [P, _dp, _dp, _dp, _dp]
        L.orc_field_advance.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _i32, _dp, S]
        L.orc_ohm_pe.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.orc_pe_rate.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.orc_field_advance_pe.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _i32, _dp,
                                           S]
        I = ctypes.POINTER(OrcInflow)
        L.orc_open_fill.argtypes = [P, _dp, _i32]
        L.orc_open_curl.argtypes = [P, _dp, _dp]
        L.orc_open_ohm.argtypes = [P, _dp, _dp, _dp, _dp, _dp]
        L.orc_open_field_advance.argtypes = [P, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _i32,
                                             _dp, S]
        L.orc_open_absorb.argtypes = [P, _i64, _ip]
        L.orc_open_absorb.restype = _i64
        L.orc_inflow_expected.argtypes = [P, I, _i32]
        L.orc_inflow_expected.restype = ctypes.c_double
        L.orc_open_inject.argtypes = [P, I, ctypes.c_uint64, _i64, _i64, _i64, _ip, _dp, _dp,
                                      _dp, _dp, _dp, _dp, _dp]
        L.orc_open_inject.restype = _i64
        L.orc_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_uniform.restype = ctypes.c_double
        for f in ("orc_open_fill", "orc_open_curl", "orc_open_ohm", "orc_open_field_advance"):
            getattr(L, f).restype = None
        for f in ("orc_gather", "orc_boris", "orc_push", "orc_sort", "orc_deposit",
                  "orc_smooth", "orc_curl", "orc_ohm", "orc_field_advance", "orc_ohm_pe",
                  "orc_pe_rate", "orc_field_advance_pe"):
            getattr(L, f).restype = None
        _LIB = L
    return _LIB


def params(cfg) -> OrcParams:
    return OrcParams(cfg.ndim, cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dz, cfg.dt,
                     cfg.nsub, cfg.shape, cfg.nsmooth, cfg.qs, cfg.ms, cfg.te,
                     cfg.gamma_e, cfg.n0, cfg.n_floor, cfg.eta, cfg.eta_h,
                     int(cfg.energy_eq), cfg.kappa0, int(cfg.open_x), int(cfg.buffer_cells),
                     cfg.eta_h_buffer)


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(_dp)


def _i(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


def f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def particles64(parts: dict) -> dict:
    """Copy of a particle dict with FP64 floats (exact for FP32 inputs)."""
    out = {k: (np.ascontiguousarray(v, dtype=np.int32) if k == "cell" else f64(v))
           for k, v in parts.items()}
    return out


def _oz(parts, n):
    oz = parts.get("oz")
    return oz if oz is not None else np.zeros(n, np.float64)


def gather(cfg, F, cell, ox, oy, oz=0.0):
    out = np.zeros(3)
    lib().orc_gather(ctypes.byref(params(cfg)), _d(f64(F).reshape(-1)), int(cell),
                     float(ox), float(oy), float(oz), _d(out))
    return out


def boris(a, E, B, v):
    v = f64(v).copy()
    lib().orc_boris(float(a), _d(f64(E)), _d(f64(B)), _d(v))
    return v


def push(cfg, parts: dict, E, B):
    """In-place leapfrog push of an FP64 particle dict.  Returns (diag[4], status)."""
    n = parts["cell"].size
    oz = _oz(parts, n)
    diag = np.zeros(4)
    st = OrcStatus()
    E = f64(E).reshape(-1)
    B = f64(B).reshape(-1)
    lib().orc_push(ctypes.byref(params(cfg)), n, _i(parts["cell"]), _d(parts["ox"]),
                   _d(parts["oy"]), _d(oz), _d(parts["ux"]), _d(parts["uy"]),
                   _d(parts["uz"]), _d(parts["w"]), _d(E), _d(B), _d(diag),
                   ctypes.byref(st))
    if cfg.ndim == 3:
        parts["oz"] = oz
    return diag, st


def sort(cfg, key):
    """Stable counting sort by cell.  Returns (perm int64[N], cell_start int32[ncell+1])."""
    key = np.ascontiguousarray(key, dtype=np.int32)
    perm = np.zeros(key.size, np.int64)
    cs = np.zeros(cfg.ncell + 1, np.int32)
    lib().orc_sort(ctypes.byref(params(cfg)), key.size, _i(key),
                   perm.ctypes.data_as(_lp), _i(cs))
    return perm, cs


def apply_perm(parts: dict, perm) -> dict:
    return {k: np.ascontiguousarray(v[perm]) for k, v in parts.items()}


def deposit(cfg, parts: dict, half_dt_back: float):
    n = parts["cell"].size
    oz = _oz(parts, n)
    rho = np.zeros(cfg.ncell)
    J = np.zeros((3, cfg.ncell))
    lib().orc_deposit(ctypes.byref(params(cfg)), n, _i(parts["cell"]), _d(parts["ox"]),
                      _d(parts["oy"]), _d(oz), _d(parts["ux"]), _d(parts["uy"]),
                      _d(parts["uz"]), _d(parts["w"]), float(half_dt_back), _d(rho),
                      _d(J))
    return rho, J


def smooth(cfg, F, npasses):
    F = f64(F).copy()
    ncomp = 1 if F.ndim == 1 else F.shape[0]
    lib().orc_smooth(ctypes.byref(params(cfg)), _d(F), ncomp, int(npasses))
    return F


def curl(cfg, A):
    C = np.zeros((3, cfg.ncell))
    lib().orc_curl(ctypes.byref(params(cfg)), _d(f64(A)), _d(C))
    return C


def ohm(cfg, B, n, Ji):
    E = np.zeros((3, cfg.ncell))
    lib().orc_ohm(ctypes.byref(params(cfg)), _d(f64(B)), _d(f64(n)), _d(f64(Ji)), _d(E))
    return E


def ohm_pe(cfg, B, n, Ji, pe):
    E = np.zeros((3, cfg.ncell))
    lib().orc_ohm_pe(ctypes.byref(params(cfg)), _d(f64(B)), _d(f64(n)), _d(f64(Ji)),
                     _d(f64(pe)), _d(E))
    return E


def pe_rate(cfg, B, n, Ji, pe):
    R = np.zeros(cfg.ncell)
    lib().orc_pe_rate(ctypes.byref(params(cfg)), _d(f64(B)), _d(f64(n)), _d(f64(Ji)),
                      _d(f64(pe)), _d(R))
    return R


def eos_pressure(cfg, n):
    """p_e = n0 te (n/n0)^gamma of the floored density (Sec. II.A): the
    starting pressure of a run with the energy equation."""
    ne = np.maximum(f64(n), cfg.n_floor)
    return cfg.n0 * cfg.te * (ne / cfg.n0) ** cfg.gamma_e


def field_advance_pe(cfg, B, pe, n_half, J_half, n_prev=None, J_prev=None, mode=0):
    """Field advance with p_e evolved by the energy equation.  Returns
    (B_new, pe_new, E_out, diag[3], status); B and pe are not modified."""
    if cfg.gamma_e == 1.0:
        raise ValueError("the energy equation needs gamma_e != 1 (W_e = sum p_e V/(gamma-1))")
    B = f64(B).copy()
    pe = f64(pe).copy()
    E = np.zeros((3, cfg.ncell))
    diag = np.zeros(3)
    st = OrcStatus()
    n_prev = f64(n_half if n_prev is None else n_prev)
    J_prev = f64(J_half if J_prev is None else J_prev)
    lib().orc_field_advance_pe(ctypes.byref(params(cfg)), _d(B), _d(pe), _d(f64(n_half)),
                               _d(f64(J_half)), _d(n_prev), _d(J_prev), _d(E), int(mode),
                               _d(diag), ctypes.byref(st))
    return B, pe, E, diag, st


def field_advance(cfg, B, n_half, J_half, n_prev=None, J_prev=None, mode=0):
    """Returns (B_new, E_out, diag[3] = {W_B, W_dB, W_e}, status); B is not modified."""
    B = f64(B).copy()
    E = np.zeros((3, cfg.ncell))
    diag = np.zeros(3)
    st = OrcStatus()
    n_prev = f64(n_half if n_prev is None else n_prev)
    J_prev = f64(J_half if J_prev is None else J_prev)
    lib().orc_field_advance(ctypes.byref(params(cfg)), _d(B), _d(f64(n_half)),
                            _d(f64(J_half)), _d(n_prev), _d(J_prev), _d(E), int(mode),
                            _d(diag), ctypes.byref(st))
    return B, E, diag, st


class OracleSim:
    """The whole step in FP64, in the order the GPU step runs it.

    State at the start of step n: particles sorted by cell at x^n with
    v^{n-1/2}; B^n, E^n; n^{n-1/2}, J^{n-1/2}.  Initialisation (the paper is
    silent on the first half step): v^{-1/2} = v^0 and n^{-1/2}, J^{-1/2} are
    the moments deposited at x^0.
    """

    def __init__(self, cfg, parts: dict, B):
        self.cfg = cfg
        self.p = particles64(parts)
        perm, self.cell_start = sort(cfg, self.p["cell"])
        self.p = apply_perm(self.p, perm)
        self.B = f64(B).copy()
        self.n_prev, self.J_prev = deposit(cfg, self.p, 0.0)
        if cfg.nsmooth:
            self.n_prev = smooth(cfg, self.n_prev, cfg.nsmooth)
            self.J_prev = smooth(cfg, self.J_prev, cfg.nsmooth)
        self.pe = eos_pressure(cfg, self.n_prev) if cfg.energy_eq else None
        self._advance(self.n_prev, self.J_prev, None, None, mode=1)
        self.status = OrcStatus()
        self.push_diag = np.zeros(4)
        self.nstep = 0

    def step(self):
        cfg = self.cfg
        E, B = self.E, self.B
        if cfg.nsmooth:
            E = smooth(cfg, E, cfg.nsmooth)
            B = smooth(cfg, B, cfg.nsmooth)
        self.push_diag, st = push(cfg, self.p, E, B)
        self.status.moved_gt1 += st.moved_gt1
        self.status.nonfinite += st.nonfinite
        perm, self.cell_start = sort(cfg, self.p["cell"])
        self.p = apply_perm(self.p, perm)
        n_half, J_half = deposit(cfg, self.p, 0.5 * cfg.dt)
        if cfg.nsmooth:
            n_half = smooth(cfg, n_half, cfg.nsmooth)
            J_half = smooth(cfg, J_half, cfg.nsmooth)
        self.n_half, self.J_half = n_half, J_half
        st = self._advance(n_half, J_half, self.n_prev, self.J_prev, mode=0)
        self.status.floor_hits += st.floor_hits
        self.n_prev, self.J_prev = n_half, J_half
        self.nstep += 1

    def _advance(self, n_half, J_half, n_prev, J_prev, mode):
        cfg = self.cfg
        if cfg.energy_eq:
            B, self.pe, self.E, self.field_diag, st = field_advance_pe(
                cfg, self.B, self.pe, n_half, J_half, n_prev, J_prev, mode=mode)
        else:
            B, self.E, self.field_diag, st = field_advance(cfg, self.B, n_half, J_half,
                                                           n_prev, J_prev, mode=mode)
        if mode == 0:
            self.B = B
        return st


# ------------------------------------------------------ open boundaries --

def inflow(spec: dict) -> OrcInflow:
    return OrcInflow(spec["n"], spec["ux"], spec["uy"], spec["uz"], spec["vth"], int(spec["ppc"]),
                     int(spec.get("faces", 3)))


def open_fill(cfg, F):
    F = f64(F).copy()
    ncomp = 1 if F.ndim == 1 else F.shape[0]
    lib().orc_open_fill(ctypes.byref(params(cfg)), _d(F), ncomp)
    return F


def open_curl(cfg, A):
    C = np.zeros((3, cfg.ncell))
    lib().orc_open_curl(ctypes.byref(params(cfg)), _d(f64(A)), _d(C))
    return C


def open_ohm(cfg, B0, B1, n, Ji):
    E = np.zeros((3, cfg.ncell))
    lib().orc_open_ohm(ctypes.byref(params(cfg)), _d(f64(B0)), _d(f64(B1)), _d(f64(n)),
                       _d(f64(Ji)), _d(E))
    return E


def open_field_advance(cfg, B0, B1, n_half, J_half, n_prev=None, J_prev=None, mode=0):
    """Returns (B1_new, E_out, Btot, diag[3], status); B1 is not modified."""
    B1 = f64(B1).copy()
    E = np.zeros((3, cfg.ncell))
    Bt = np.zeros((3, cfg.ncell))
    diag = np.zeros(3)
    st = OrcStatus()
    n_prev = f64(n_half if n_prev is None else n_prev)
    J_prev = f64(J_half if J_prev is None else J_prev)
    lib().orc_open_field_advance(ctypes.byref(params(cfg)), _d(f64(B0)), _d(B1), _d(f64(n_half)),
                                 _d(f64(J_half)), _d(n_prev), _d(J_prev), _d(E), _d(Bt),
                                 int(mode), _d(diag), ctypes.byref(st))
    return B1, E, Bt, diag, st


def open_absorb(cfg, parts: dict) -> int:
    return int(lib().orc_open_absorb(ctypes.byref(params(cfg)), parts["cell"].size,
                                     _i(parts["cell"])))


def inflow_expected(cfg, spec: dict, face: int) -> float:
    return float(lib().orc_inflow_expected(ctypes.byref(params(cfg)),
                                           ctypes.byref(inflow(spec)), int(face)))


def uniform(seed: int, ctr: int) -> float:
    return float(lib().orc_uniform(seed, ctr))


def open_inject(cfg, spec: dict, seed: int, step: int, parts: dict, cap_extra: int = 1 << 20):
    """parts with the ions injected this step appended."""
    n = parts["cell"].size
    cap = n + cap_extra
    out = {k: np.concatenate([v, np.zeros(cap_extra, v.dtype)]) for k, v in parts.items()}
    out = {k: np.ascontiguousarray(v) for k, v in out.items()}
    oz = _d(out["oz"]) if "oz" in out else None
    m = lib().orc_open_inject(ctypes.byref(params(cfg)), ctypes.byref(inflow(spec)), seed, step,
                              n, cap, _i(out["cell"]), _d(out["ox"]), _d(out["oy"]), oz,
                              _d(out["ux"]), _d(out["uy"]), _d(out["uz"]), _d(out["w"]))
    return {k: np.ascontiguousarray(v[:m]) for k, v in out.items()}


class OpenOracleSim:
    """The 2D step with open x boundaries (Sec. II.C) in FP64, in the order
    the GPU runs it: push; the mid-point deposit of the pushed store; ions
    in the ghost columns absorbed and fresh ions injected through the faces;
    the stable sort with the absorbed ions last (and dropped); the moments'
    ghost columns filled; the field advance of B1 with B = B0 + B1."""

    def __init__(self, cfg, parts: dict, B0, B1, spec: dict, seed: int):
        self.cfg, self.spec, self.seed = cfg, spec, seed
        self.p = particles64(parts)
        perm, self.cell_start = sort(cfg, self.p["cell"])
        self.p = apply_perm(self.p, perm)
        self.B0 = f64(B0).copy()
        self.B1 = open_fill(cfg, B1)
        n0, J0 = deposit(cfg, self.p, 0.0)
        self.n_prev, self.J_prev = open_fill(cfg, n0), open_fill(cfg, J0)
        self.B1, self.E, self.Btot, self.field_diag, _ = open_field_advance(
            cfg, self.B0, self.B1, self.n_prev, self.J_prev, mode=1)
        self.nstep = 0
        self.absorbed = self.injected = 0

    def step(self):
        cfg = self.cfg
        self.push_diag, _ = push(cfg, self.p, self.E, self.Btot)
        n_half, J_half = deposit(cfg, self.p, 0.5 * cfg.dt)
        self.absorbed += open_absorb(cfg, self.p)
        n_before = self.p["cell"].size
        self.p = open_inject(cfg, self.spec, self.seed, self.nstep, self.p)
        self.injected += self.p["cell"].size - n_before
        key = self.p["cell"]
        order = np.argsort(key, kind="stable")
        alive = int(np.sum(key < cfg.ncell))
        self.p = {k: np.ascontiguousarray(v[order][:alive]) for k, v in self.p.items()}
        self.cell_start = np.concatenate([[0], np.cumsum(np.bincount(self.p["cell"],
                                                                     minlength=cfg.ncell))])
        self.n_half, self.J_half = open_fill(cfg, n_half), open_fill(cfg, J_half)
        self.B1, self.E, self.Btot, self.field_diag, _ = open_field_advance(
            cfg, self.B0, self.B1, self.n_half, self.J_half, self.n_prev, self.J_prev, mode=0)
        self.n_prev, self.J_prev = self.n_half, self.J_half
        self.nstep += 1

