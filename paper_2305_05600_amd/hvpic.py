"""ctypes binding of libhvpic.so (include/hvpic.h).

Argument marshalling only: every function takes torch tensors that live on
the GPU, checks dtype/shape/contiguity, and passes raw device pointers to the
C function of the same name.  No computation happens here.  If the library is
not built the first call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import pathlib

import torch

_PKG = pathlib.Path(__file__).resolve().parent
LIB_PATH = _PKG / "libhvpic.so"
_LIB = None
_NCELL = {}  # context handle -> ncell, for host-side size checks
_NPCAP = {}  # context handle -> np_capacity

HVPIC_OK, HVPIC_EINVAL, HVPIC_ENOMEM, HVPIC_EHIP, HVPIC_ESTATE = 0, -1, -2, -3, -4
HVPIC_SHAPE_NGP, HVPIC_SHAPE_QS = 0, 1
FLAG_MOVE_GT1, FLAG_FLOOR_HIT, FLAG_NONFINITE, FLAG_BAD_INPUT = 1, 2, 4, 8

EXPORTS = ("hvpic_workspace_bytes", "hvpic_init", "hvpic_finalize", "hvpic_set_stream",
           "hvpic_gather_push",
           "hvpic_gather_push_perm", "hvpic_gather_push_select", "hvpic_sort", "hvpic_sort_perm", "hvpic_deposit",
           "hvpic_deposit_noalloc",
           "hvpic_field_advance", "hvpic_field_advance_pe", "hvpic_eos_pressure", "hvpic_smooth",
           "hvpic_sync_status", "hvpic_path_stats", "hvpic_timing_enable", "hvpic_timing_read",
           "hvpic_ensemble_workspace_bytes", "hvpic_tuning_default", "hvpic_ensemble_init",
           "hvpic_ensemble_finalize", "hvpic_ensemble_step", "hvpic_ensemble_steps",
           "hvpic_ensemble_capture", "hvpic_ensemble_get_tuning", "hvpic_ensemble_set_tuning",
           "hvpic_ensemble_autotune", "hvpic_ensemble_time_phases",
           "hvpic_no_params_bytes", "hvpic_no_workspace_bytes", "hvpic_no_load", "hvpic_no_store",
           "hvpic_no_predict", "hvpic_no_train_step", "hvpic_field_advance_no",
           "hvpic_no_conv3x3", "hvpic_no_conv3x3_wgrad",
           "hvpic_open_fill", "hvpic_open_field_advance", "hvpic_open_particles",
           "hvpic_sort_open", "hvpic_open_absorb", "hvpic_open_inject", "hvpic_sort_open_perm",
           "hvpic_strerror")
KERNEL_GATHER_PUSH, KERNEL_DEPOSIT, KERNEL_SORT_SCATTER = 0, 1, 2


class HvpicParams(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("nsub", ctypes.c_int32), ("shape", ctypes.c_int32), ("nsmooth", ctypes.c_int32),
        ("qs", ctypes.c_double), ("ms", ctypes.c_double),
        ("te", ctypes.c_double), ("gamma_e", ctypes.c_double), ("n0", ctypes.c_double),
        ("n_floor", ctypes.c_double),
        ("eta", ctypes.c_double), ("eta_h", ctypes.c_double),
        ("energy_eq", ctypes.c_int32), ("kappa0", ctypes.c_double),
        ("open_x", ctypes.c_int32), ("buffer_cells", ctypes.c_int32),
        ("eta_h_buffer", ctypes.c_double),
        ("np_capacity", ctypes.c_int64),
    ]


class HvpicInflow(ctypes.Structure):
    _fields_ = [("n", ctypes.c_double), ("ux", ctypes.c_double), ("uy", ctypes.c_double),
                ("uz", ctypes.c_double), ("vth", ctypes.c_double), ("ppc", ctypes.c_int32),
                ("faces", ctypes.c_int32)]


class HvpicParticles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cell", ctypes.c_void_p),
                ("ox", ctypes.c_void_p), ("oy", ctypes.c_void_p), ("oz", ctypes.c_void_p),
                ("ux", ctypes.c_void_p), ("uy", ctypes.c_void_p), ("uz", ctypes.c_void_p),
                ("w", ctypes.c_void_p)]


class HvpicRun(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("store", HvpicParticles * 2), ("perm", ctypes.c_void_p),
                ("cell_start", ctypes.c_void_p * 2), ("E", ctypes.c_void_p),
                ("B", ctypes.c_void_p), ("n", ctypes.c_void_p * 2), ("J", ctypes.c_void_p * 2),
                ("push_diag", ctypes.c_void_p), ("field_diag", ctypes.c_void_p)]


class HvpicTuning(ctypes.Structure):
    _fields_ = [("push_chunk", ctypes.c_int32 * 3), ("field_tile", ctypes.c_int32 * 2),
                ("blocks_per_cu", ctypes.c_int32 * 4)]

    def as_dict(self) -> dict:
        return {"push_chunk": list(self.push_chunk), "field_tile": list(self.field_tile),
                "blocks_per_cu": list(self.blocks_per_cu)}


class HvpicError(RuntimeError):
    pass


def lib():
    """Loads libhvpic.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not LIB_PATH.exists():
            raise HvpicError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(str(LIB_PATH))
        vp, i32, P = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER
        L.hvpic_workspace_bytes.argtypes = [P(HvpicParams), P(ctypes.c_size_t)]
        L.hvpic_init.argtypes = [P(HvpicParams), vp, vp, P(vp)]
        L.hvpic_finalize.argtypes = [vp]
        L.hvpic_set_stream.argtypes = [vp, vp]
        L.hvpic_gather_push.argtypes = [vp, P(HvpicParticles), vp, vp, vp, vp, vp, vp]
        L.hvpic_gather_push_perm.argtypes = [vp, P(HvpicParticles), vp, P(HvpicParticles), vp, vp,
                                             vp, vp, vp, vp]
        L.hvpic_gather_push_select.argtypes = [vp, P(HvpicParticles), ctypes.c_int64, vp,
                                               P(HvpicParticles), vp, vp, vp, vp, vp, vp]
        L.hvpic_sort.argtypes = [vp, P(HvpicParticles), P(HvpicParticles), vp, vp, i32]
        L.hvpic_sort_perm.argtypes = [vp, P(HvpicParticles), vp, vp, vp]
        L.hvpic_deposit.argtypes = [vp, P(HvpicParticles), vp, ctypes.c_float, vp, vp]
        L.hvpic_deposit_noalloc.argtypes = [P(HvpicParams), vp, P(HvpicParticles), ctypes.c_float,
                                            vp, vp]
        L.hvpic_field_advance.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32, vp]
        L.hvpic_field_advance_pe.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i32, vp]
        L.hvpic_eos_pressure.argtypes = [vp, vp, vp]
        L.hvpic_smooth.argtypes = [vp, vp, i32, i32]
        L.hvpic_sync_status.argtypes = [vp, P(ctypes.c_uint32), P(ctypes.c_int64)]
        L.hvpic_path_stats.argtypes = [vp, P(ctypes.c_int64)]
        L.hvpic_timing_enable.argtypes = [vp, i32, i32]
        L.hvpic_timing_read.argtypes = [vp, i32, P(ctypes.c_double), P(ctypes.c_int64)]
        RP, TP = P(HvpicRun), P(HvpicTuning)
        L.hvpic_ensemble_workspace_bytes.argtypes = [RP, i32, P(ctypes.c_size_t)]
        L.hvpic_tuning_default.argtypes = [TP]
        L.hvpic_ensemble_init.argtypes = [RP, i32, vp, vp, TP, P(vp)]
        L.hvpic_ensemble_finalize.argtypes = [vp]
        L.hvpic_ensemble_step.argtypes = [vp]
        L.hvpic_ensemble_steps.argtypes = [vp, P(ctypes.c_int64)]
        L.hvpic_ensemble_capture.argtypes = [vp, i32]
        L.hvpic_ensemble_get_tuning.argtypes = [vp, TP]
        L.hvpic_ensemble_set_tuning.argtypes = [vp, TP]
        L.hvpic_ensemble_autotune.argtypes = [vp, i32, TP, P(ctypes.c_double)]
        L.hvpic_ensemble_time_phases.argtypes = [vp, i32, P(ctypes.c_double)]
        L.hvpic_no_params_bytes.argtypes = [P(ctypes.c_size_t)]
        L.hvpic_no_workspace_bytes.argtypes = [i32, i32, i32, P(ctypes.c_size_t)]
        L.hvpic_no_load.argtypes = [vp, vp, vp, vp, vp]
        L.hvpic_no_store.argtypes = [vp, vp, vp, vp]
        L.hvpic_no_predict.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp]
        L.hvpic_no_train_step.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp, i32,
                                          ctypes.c_float, vp, vp]
        L.hvpic_field_advance_no.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                             ctypes.c_float, vp]
        L.hvpic_no_conv3x3.argtypes = [i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        L.hvpic_no_conv3x3_wgrad.argtypes = [i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        L.hvpic_open_fill.argtypes = [vp, vp, i32]
        L.hvpic_open_field_advance.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, vp]
        L.hvpic_open_particles.argtypes = [vp, P(HvpicParticles), P(HvpicInflow), ctypes.c_uint64,
                                           ctypes.c_int64]
        L.hvpic_sort_open.argtypes = [vp, P(HvpicParticles), P(HvpicParticles), vp]
        L.hvpic_open_absorb.argtypes = [vp, P(HvpicParticles)]
        L.hvpic_open_inject.argtypes = [vp, P(HvpicParticles), P(HvpicInflow), ctypes.c_uint64,
                                        ctypes.c_int64]
        L.hvpic_sort_open_perm.argtypes = [vp, P(HvpicParticles), ctypes.c_int64, vp, vp, vp, vp]
        L.hvpic_strerror.argtypes = [ctypes.c_int]
        L.hvpic_strerror.restype = ctypes.c_char_p
        for f in EXPORTS[:-1]:
            getattr(L, f).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(rc: int, what: str):
    if rc != HVPIC_OK:
        raise HvpicError(f"{what}: {lib().hvpic_strerror(rc).decode()} ({rc})")


def _ptr(t, dtype=None, numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise HvpicError("expected a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise HvpicError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise HvpicError(f"expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise HvpicError(f"tensor holds {t.numel()} elements, needs {numel}")
    return t.data_ptr()


def params_from(cfg, np_capacity: int) -> HvpicParams:
    return HvpicParams(cfg.ndim, cfg.nx, cfg.ny, cfg.nz, cfg.dx, cfg.dy, cfg.dz, cfg.dt,
                       cfg.nsub, cfg.shape, cfg.nsmooth, cfg.qs, cfg.ms, cfg.te, cfg.gamma_e,
                       cfg.n0, cfg.n_floor, cfg.eta, cfg.eta_h, int(cfg.energy_eq),
                       cfg.kappa0, int(cfg.open_x), int(cfg.buffer_cells), cfg.eta_h_buffer,
                       int(np_capacity))


class Particles:
    """Structure-of-arrays particle store in device memory."""

    FIELDS = ("cell", "ox", "oy", "oz", "ux", "uy", "uz", "w")

    def __init__(self, ndim: int, capacity: int, device="cuda"):
        self.ndim = ndim
        self.capacity = capacity
        self.n = 0
        self.cell = torch.empty(capacity, dtype=torch.int32, device=device)
        f = lambda: torch.empty(capacity, dtype=torch.float32, device=device)
        self.ox, self.oy = f(), f()
        self.oz = f() if ndim == 3 else None
        self.ux, self.uy, self.uz, self.w = f(), f(), f(), f()

    @classmethod
    def from_numpy(cls, parts: dict, ndim: int, capacity: int | None = None, device="cuda"):
        n = int(parts["cell"].size)
        p = cls(ndim, max(capacity or n, 1), device)
        p.load(parts)
        return p

    def load(self, parts: dict):
        n = int(parts["cell"].size)
        if n > self.capacity:
            raise HvpicError("more particles than capacity")
        self.n = n
        for k in self.FIELDS:
            t = getattr(self, k)
            if t is None:
                continue
            t[:n].copy_(torch.from_numpy(parts[k]))

    def to_numpy(self) -> dict:
        out = {}
        for k in self.FIELDS:
            t = getattr(self, k)
            if t is not None:
                out[k] = t[: self.n].cpu().numpy()
        return out

    def c(self) -> HvpicParticles:
        g = lambda t: None if t is None else t.data_ptr()
        return HvpicParticles(self.n, g(self.cell), g(self.ox), g(self.oy), g(self.oz),
                              g(self.ux), g(self.uy), g(self.uz), g(self.w))


# ---------------------------------------------------------------------------
# One Python function per C entry point (same names).
# ---------------------------------------------------------------------------

def hvpic_workspace_bytes(params: HvpicParams) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().hvpic_workspace_bytes(ctypes.byref(params), ctypes.byref(n)),
           "hvpic_workspace_bytes")
    return n.value


def hvpic_init(params: HvpicParams, stream, workspace: torch.Tensor):
    ctx = ctypes.c_void_p()
    s = None if stream is None else ctypes.c_void_p(stream)
    need = hvpic_workspace_bytes(params)
    _check(lib().hvpic_init(ctypes.byref(params), s, _ptr(workspace, torch.uint8, need),
                            ctypes.byref(ctx)), "hvpic_init")
    _NCELL[ctx.value] = params.nx * params.ny * params.nz
    _NPCAP[ctx.value] = params.np_capacity
    return ctx


def hvpic_finalize(ctx):
    _check(lib().hvpic_finalize(ctx), "hvpic_finalize")
    _NCELL.pop(ctx.value, None)
    _NPCAP.pop(ctx.value, None)


def hvpic_set_stream(ctx, stream):
    # the context keeps its grid: the host-side size checks stay on
    _check(lib().hvpic_set_stream(ctx, None if stream is None else ctypes.c_void_p(stream)),
           "hvpic_set_stream")


def _nc(ctx, k=1):
    return k * _NCELL[ctx.value] if ctx.value in _NCELL else None


def hvpic_gather_push(ctx, p: Particles, cell_start, E, B, n_mid=None, J_mid=None,
                      diag_out=None):
    cp = p.c()
    ncs = None if _nc(ctx) is None else _nc(ctx) + 1
    _check(lib().hvpic_gather_push(ctx, ctypes.byref(cp), _ptr(cell_start, torch.int32, ncs),
                                   _ptr(E, torch.float32, _nc(ctx, 3)),
                                   _ptr(B, torch.float32, _nc(ctx, 3)),
                                   _ptr(n_mid, torch.float32, _nc(ctx)),
                                   _ptr(J_mid, torch.float32, _nc(ctx, 3)),
                                   _ptr(diag_out, torch.float64, 4)),
           "hvpic_gather_push")


def hvpic_gather_push_select(ctx, pin: Particles, n_map: int, perm, pout: Particles, cell_start,
                             E, B, n_mid=None, J_mid=None, diag_out=None):
    ci, co = pin.c(), pout.c()
    if pout.capacity < n_map:
        raise HvpicError("output store too small")
    ncs = None if _nc(ctx) is None else _nc(ctx) + 1
    _check(lib().hvpic_gather_push_select(ctx, ctypes.byref(ci), int(n_map),
                                          _ptr(perm, torch.int32, n_map), ctypes.byref(co),
                                          _ptr(cell_start, torch.int32, ncs),
                                          _ptr(E, torch.float32, _nc(ctx, 3)),
                                          _ptr(B, torch.float32, _nc(ctx, 3)),
                                          _ptr(n_mid, torch.float32, _nc(ctx)),
                                          _ptr(J_mid, torch.float32, _nc(ctx, 3)),
                                          _ptr(diag_out, torch.float64, 4)),
           "hvpic_gather_push_select")
    pout.n = co.n


def hvpic_gather_push_perm(ctx, pin: Particles, perm, pout: Particles, cell_start, E, B,
                           n_mid=None, J_mid=None, diag_out=None):
    ci, co = pin.c(), pout.c()
    if pout.capacity < pin.n:
        raise HvpicError("output store too small")
    ncs = None if _nc(ctx) is None else _nc(ctx) + 1
    _check(lib().hvpic_gather_push_perm(ctx, ctypes.byref(ci), _ptr(perm, torch.int32, pin.n),
                                        ctypes.byref(co), _ptr(cell_start, torch.int32, ncs),
                                        _ptr(E, torch.float32, _nc(ctx, 3)),
                                        _ptr(B, torch.float32, _nc(ctx, 3)),
                                        _ptr(n_mid, torch.float32, _nc(ctx)),
                                        _ptr(J_mid, torch.float32, _nc(ctx, 3)),
                                        _ptr(diag_out, torch.float64, 4)),
           "hvpic_gather_push_perm")
    pout.n = co.n


def hvpic_sort_perm(ctx, pin: Particles, cell_start_prev, perm, cell_start):
    ci = pin.c()
    ncs = None if _nc(ctx) is None else _nc(ctx) + 1
    _check(lib().hvpic_sort_perm(ctx, ctypes.byref(ci), _ptr(cell_start_prev, torch.int32, ncs),
                                 _ptr(perm, torch.int32, pin.n),
                                 _ptr(cell_start, torch.int32, ncs)), "hvpic_sort_perm")


def hvpic_sort(ctx, pin: Particles, pout: Particles, cell_start_prev, cell_start, full=False):
    ci, co = pin.c(), pout.c()
    if pout.capacity < pin.n:
        raise HvpicError("output store too small")
    ncs = None if _nc(ctx) is None else _nc(ctx) + 1
    _check(lib().hvpic_sort(ctx, ctypes.byref(ci), ctypes.byref(co),
                            _ptr(cell_start_prev, torch.int32, ncs),
                            _ptr(cell_start, torch.int32, ncs),
                            1 if full else 0), "hvpic_sort")
    pout.n = co.n


def hvpic_deposit(ctx, p: Particles, cell_start, half_dt_back: float, n, J):
    cp = p.c()
    _check(lib().hvpic_deposit(ctx, ctypes.byref(cp), _ptr(cell_start, torch.int32),
                               ctypes.c_float(half_dt_back), _ptr(n, torch.float32, _nc(ctx)),
                               _ptr(J, torch.float32, _nc(ctx, 3))), "hvpic_deposit")


NOALLOC_MAX_CELLS = 1 << 20  # HVPIC_NOALLOC_MAX_CELLS


def hvpic_deposit_noalloc(params: HvpicParams, stream, p: Particles, half_dt_back: float, n, J):
    """The deposit without a context or workspace (the library's own scratch);
    `stream` is a raw hipStream_t handle (int) or None."""
    nc = params.nx * params.ny * params.nz
    cp = p.c()
    s = None if stream is None else ctypes.c_void_p(stream)
    _check(lib().hvpic_deposit_noalloc(ctypes.byref(params), s, ctypes.byref(cp),
                                       ctypes.c_float(half_dt_back),
                                       _ptr(n, torch.float32, nc), _ptr(J, torch.float32, 3 * nc)),
           "hvpic_deposit_noalloc")


def hvpic_field_advance(ctx, B, n_half, J_half, n_prev, J_prev, E_out, mode=0, diag_out=None):
    v1, v3 = _nc(ctx), _nc(ctx, 3)
    _check(lib().hvpic_field_advance(ctx, _ptr(B, torch.float32, v3),
                                     _ptr(n_half, torch.float32, v1),
                                     _ptr(J_half, torch.float32, v3),
                                     _ptr(n_prev, torch.float32, v1),
                                     _ptr(J_prev, torch.float32, v3),
                                     _ptr(E_out, torch.float32, v3),
                                     int(mode), _ptr(diag_out, torch.float64, 3)),
           "hvpic_field_advance")


def hvpic_field_advance_pe(ctx, B, pe, n_half, J_half, n_prev, J_prev, E_out, mode=0,
                           diag_out=None):
    v1, v3 = _nc(ctx), _nc(ctx, 3)
    _check(lib().hvpic_field_advance_pe(ctx, _ptr(B, torch.float32, v3),
                                        _ptr(pe, torch.float32, v1),
                                        _ptr(n_half, torch.float32, v1),
                                        _ptr(J_half, torch.float32, v3),
                                        _ptr(n_prev, torch.float32, v1),
                                        _ptr(J_prev, torch.float32, v3),
                                        _ptr(E_out, torch.float32, v3),
                                        int(mode), _ptr(diag_out, torch.float64, 3)),
           "hvpic_field_advance_pe")


def hvpic_eos_pressure(ctx, n, pe):
    v1 = _nc(ctx)
    _check(lib().hvpic_eos_pressure(ctx, _ptr(n, torch.float32, v1), _ptr(pe, torch.float32, v1)),
           "hvpic_eos_pressure")


def hvpic_smooth(ctx, F, npasses: int):
    ncomp = 1 if F.dim() == 1 else F.shape[0]
    _check(lib().hvpic_smooth(ctx, _ptr(F, torch.float32, _nc(ctx, ncomp)), int(ncomp),
                              int(npasses)),
           "hvpic_smooth")


def hvpic_sync_status(ctx):
    flags = ctypes.c_uint32(0)
    counts = (ctypes.c_int64 * 3)()
    _check(lib().hvpic_sync_status(ctx, ctypes.byref(flags), counts), "hvpic_sync_status")
    return flags.value, tuple(counts)


def hvpic_path_stats(ctx):
    """(blocks that used the LDS windows, blocks that fell back to global
    accesses) of the particle kernels since the last call."""
    out = (ctypes.c_int64 * 2)()
    _check(lib().hvpic_path_stats(ctx, out), "hvpic_path_stats")
    return out[0], out[1]


def hvpic_timing_enable(ctx, max_launches: int, every: int = 1):
    _check(lib().hvpic_timing_enable(ctx, max_launches, every), "hvpic_timing_enable")


def hvpic_timing_read(ctx, kernel: int):
    """(summed milliseconds, number of timed launches) of kernel id `kernel`."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().hvpic_timing_read(ctx, kernel, ctypes.byref(ms), ctypes.byref(n)),
           "hvpic_timing_read")
    return ms.value, n.value


def hvpic_strerror(code: int) -> str:
    return lib().hvpic_strerror(code).decode()


def hvpic_ensemble_workspace_bytes(runs) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().hvpic_ensemble_workspace_bytes(runs, len(runs), ctypes.byref(n)),
           "hvpic_ensemble_workspace_bytes")
    return n.value


def hvpic_tuning_default() -> HvpicTuning:
    t = HvpicTuning()
    _check(lib().hvpic_tuning_default(ctypes.byref(t)), "hvpic_tuning_default")
    return t


def hvpic_ensemble_init(runs, stream, workspace: torch.Tensor, tuning=None):
    e = ctypes.c_void_p()
    _check(lib().hvpic_ensemble_init(runs, len(runs), stream, _ptr(workspace, torch.uint8),
                                     None if tuning is None else ctypes.byref(tuning),
                                     ctypes.byref(e)),
           "hvpic_ensemble_init")
    return e


def hvpic_ensemble_finalize(e):
    _check(lib().hvpic_ensemble_finalize(e), "hvpic_ensemble_finalize")


def hvpic_ensemble_step(e):
    _check(lib().hvpic_ensemble_step(e), "hvpic_ensemble_step")


def hvpic_ensemble_steps(e) -> int:
    k = ctypes.c_int64(0)
    _check(lib().hvpic_ensemble_steps(e, ctypes.byref(k)), "hvpic_ensemble_steps")
    return k.value


def hvpic_ensemble_capture(e, enable: bool = True):
    _check(lib().hvpic_ensemble_capture(e, int(bool(enable))), "hvpic_ensemble_capture")


def hvpic_ensemble_get_tuning(e) -> HvpicTuning:
    t = HvpicTuning()
    _check(lib().hvpic_ensemble_get_tuning(e, ctypes.byref(t)), "hvpic_ensemble_get_tuning")
    return t


def hvpic_ensemble_set_tuning(e, tuning: HvpicTuning):
    _check(lib().hvpic_ensemble_set_tuning(e, ctypes.byref(tuning)), "hvpic_ensemble_set_tuning")


def hvpic_ensemble_autotune(e, reps: int = 2):
    t = HvpicTuning()
    ms = (ctypes.c_double * 3)()
    _check(lib().hvpic_ensemble_autotune(e, int(reps), ctypes.byref(t), ms),
           "hvpic_ensemble_autotune")
    return t, tuple(ms)


def hvpic_ensemble_time_phases(e, steps: int):
    ms = (ctypes.c_double * 3)()
    _check(lib().hvpic_ensemble_time_phases(e, int(steps), ms), "hvpic_ensemble_time_phases")
    return tuple(ms)


def _stream(stream):
    return (stream if stream is not None else torch.cuda.current_stream()).cuda_stream


def hvpic_no_params_bytes() -> int:
    n = ctypes.c_size_t(0)
    _check(lib().hvpic_no_params_bytes(ctypes.byref(n)), "hvpic_no_params_bytes")
    return n.value


def hvpic_no_workspace_bytes(nx: int, ny: int, batch: int) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().hvpic_no_workspace_bytes(nx, ny, batch, ctypes.byref(n)),
           "hvpic_no_workspace_bytes")
    return n.value


def hvpic_no_load(params, w, b, norm, stream=None):
    _check(lib().hvpic_no_load(_ptr(params, torch.uint8), _ptr(w, torch.float32),
                               _ptr(b, torch.float32), _ptr(norm, torch.float32),
                               _stream(stream)), "hvpic_no_load")


def hvpic_no_store(params, w, b, stream=None):
    _check(lib().hvpic_no_store(_ptr(params, torch.uint8), _ptr(w, torch.float32),
                                _ptr(b, torch.float32), _stream(stream)), "hvpic_no_store")


def hvpic_no_predict(params, workspace, nx, ny, B, n, J, B_out, stream=None):
    P = nx * ny
    _check(lib().hvpic_no_predict(_ptr(params, torch.uint8), _ptr(workspace, torch.uint8), nx, ny,
                                  _ptr(B, torch.float32, 3 * P), _ptr(n, torch.float32, P),
                                  _ptr(J, torch.float32, 3 * P), _ptr(B_out, torch.float32, 3 * P),
                                  _stream(stream)), "hvpic_no_predict")


def hvpic_no_train_step(params, workspace, nx, ny, B, n, J, B_target, idx, lr, loss_out=None,
                        stream=None):
    batch = int(idx.numel())
    _check(lib().hvpic_no_train_step(_ptr(params, torch.uint8), _ptr(workspace, torch.uint8), nx,
                                     ny, _ptr(B, torch.float32), _ptr(n, torch.float32),
                                     _ptr(J, torch.float32), _ptr(B_target, torch.float32),
                                     _ptr(idx, torch.int32), batch, float(lr),
                                     _ptr(loss_out, torch.float64, 1), _stream(stream)),
           "hvpic_no_train_step")


def hvpic_field_advance_no(ctx, params, workspace, B, n_half, J_half, n_prev, J_prev, E_out,
                           tol, diag_out=None, stats=None):
    v1, v3 = _nc(ctx), _nc(ctx, 3)
    _check(lib().hvpic_field_advance_no(ctx, _ptr(params, torch.uint8),
                                        _ptr(workspace, torch.uint8), _ptr(B, torch.float32, v3),
                                        _ptr(n_half, torch.float32, v1),
                                        _ptr(J_half, torch.float32, v3),
                                        _ptr(n_prev, torch.float32, v1),
                                        _ptr(J_prev, torch.float32, v3),
                                        _ptr(E_out, torch.float32, v3),
                                        _ptr(diag_out, torch.float64, 3), float(tol),
                                        _ptr(stats, torch.float64, 2)),
           "hvpic_field_advance_no")


def hvpic_no_conv3x3(nimg, nx, ny, cinp, coutp, mode, x, w, bias, h, out, stream=None):
    _check(lib().hvpic_no_conv3x3(nimg, nx, ny, cinp, coutp, mode, _ptr(x), _ptr(w),
                                  _ptr(bias, torch.float32), _ptr(h), _ptr(out), _stream(stream)),
           "hvpic_no_conv3x3")


def hvpic_no_conv3x3_wgrad(nimg, nx, ny, cinp, coutp, x, dz, dw, db, workspace, stream=None):
    _check(lib().hvpic_no_conv3x3_wgrad(nimg, nx, ny, cinp, coutp, _ptr(x), _ptr(dz),
                                        _ptr(dw, torch.float32), _ptr(db, torch.float32),
                                        _ptr(workspace, torch.uint8), _stream(stream)),
           "hvpic_no_conv3x3_wgrad")


class Context:
    """Owns a context, its workspace and the stream it is bound to."""

    def __init__(self, cfg, np_capacity: int, device="cuda", stream=None):
        self.cfg = cfg
        self.params = params_from(cfg, np_capacity)
        nbytes = hvpic_workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.ctx = hvpic_init(self.params, self.stream.cuda_stream, self.workspace)

    def set_stream(self, stream):
        """Later calls of this context enqueue on `stream` (ordering is the caller's)."""
        hvpic_set_stream(self.ctx, stream.cuda_stream)
        self.stream = stream

    def close(self):
        if self.ctx is not None:
            hvpic_finalize(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Open boundaries in x (Sec. II.C)
# ---------------------------------------------------------------------------

def inflow_from(spec: dict) -> HvpicInflow:
    """The C struct of an inflow spec {n, ux, uy, uz, vth, ppc, faces}."""
    return HvpicInflow(float(spec["n"]), float(spec["ux"]), float(spec["uy"]), float(spec["uz"]),
                       float(spec["vth"]), int(spec["ppc"]), int(spec["faces"]))


def hvpic_open_fill(ctx, F, ncomp: int):
    _check(lib().hvpic_open_fill(ctx, _ptr(F, torch.float32, _nc(ctx, ncomp)), int(ncomp)),
           "hvpic_open_fill")


def hvpic_open_field_advance(ctx, B0, B1, Btot, n_half, J_half, n_prev, J_prev, E_out, mode=0,
                             diag_out=None):
    v1, v3 = _nc(ctx), _nc(ctx, 3)
    _check(lib().hvpic_open_field_advance(ctx, _ptr(B0, torch.float32, v3),
                                          _ptr(B1, torch.float32, v3),
                                          _ptr(Btot, torch.float32, v3),
                                          _ptr(n_half, torch.float32, v1),
                                          _ptr(J_half, torch.float32, v3),
                                          _ptr(n_prev, torch.float32, v1),
                                          _ptr(J_prev, torch.float32, v3),
                                          _ptr(E_out, torch.float32, v3),
                                          int(mode), _ptr(diag_out, torch.float64, 3)),
           "hvpic_open_field_advance")


def hvpic_open_particles(ctx, p: Particles, inflow: HvpicInflow, seed: int, step: int):
    """Absorption and injection; p.n grows by the injected count.  The store
    must hold the context's np_capacity ions (the injection appends up to it)."""
    if ctx.value in _NPCAP and p.capacity < _NPCAP[ctx.value]:
        raise HvpicError("hvpic_open_particles: the store holds fewer ions than np_capacity")
    cp = p.c()
    cp_cap = p.capacity
    _check(lib().hvpic_open_particles(ctx, ctypes.byref(cp), ctypes.byref(inflow),
                                      ctypes.c_uint64(seed & (2**64 - 1)), int(step)),
           "hvpic_open_particles")
    if cp.n > cp_cap:
        raise HvpicError("hvpic_open_particles: store overflow")
    p.n = cp.n


def hvpic_sort_open(ctx, pin: Particles, pout: Particles, cell_start):
    ci, co = pin.c(), pout.c()
    if pout.capacity < pin.n:
        raise HvpicError("output store too small")
    ncs = None if _nc(ctx) is None else _nc(ctx) + 2
    _check(lib().hvpic_sort_open(ctx, ctypes.byref(ci), ctypes.byref(co),
                                 _ptr(cell_start, torch.int32, ncs)), "hvpic_sort_open")
    pout.n = co.n


def hvpic_open_absorb(ctx, p: Particles):
    cp = p.c()
    _check(lib().hvpic_open_absorb(ctx, ctypes.byref(cp)), "hvpic_open_absorb")


def hvpic_open_inject(ctx, p: Particles, inflow: HvpicInflow, seed: int, step: int):
    """Injection alone; p.n grows by the injected count."""
    if ctx.value in _NPCAP and p.capacity < _NPCAP[ctx.value]:
        raise HvpicError("hvpic_open_inject: the store holds fewer ions than np_capacity")
    cp = p.c()
    _check(lib().hvpic_open_inject(ctx, ctypes.byref(cp), ctypes.byref(inflow),
                                   ctypes.c_uint64(seed & (2**64 - 1)), int(step)),
           "hvpic_open_inject")
    p.n = cp.n


def hvpic_sort_open_perm(ctx, pin: Particles, n_pushed: int, cell_start_prev, perm, cell_start,
                         info=None):
    ci = pin.c()
    ncs = None if _nc(ctx) is None else _nc(ctx) + 1
    _check(lib().hvpic_sort_open_perm(ctx, ctypes.byref(ci), int(n_pushed),
                                      _ptr(cell_start_prev, torch.int32, ncs),
                                      _ptr(perm, torch.int32, pin.n),  # live <= in.n entries
                                      _ptr(cell_start, torch.int32, ncs),
                                      _ptr(info, torch.int32, 2)), "hvpic_sort_open_perm")
