"""Sequencing of one hybrid-PIC time step on the GPU (calls into libhvpic.so).

State at the start of step n: particles sorted by cell at x^n carrying
v^{n-1/2}; B^n and E^n; the moments n^{n-1/2}, J^{n-1/2}.  One step:

  1. hvpic_gather_push   E^n, B^n at x^n -> v^{n+1/2}, x^{n+1}; with the fused
                         deposit also n^{n+1/2}, J^{n+1/2} at x^{n+1/2}; given
                         cell_start it also counts the moves for the sort
  2. hvpic_sort          stable sort by the new cells (neighbour-move path)
  3. hvpic_deposit       n^{n+1/2}, J^{n+1/2} (only when not fused)
  4. hvpic_smooth        optional binomial passes on the moments
  5. hvpic_field_advance B^n -> B^{n+1} (subcycled), E^{n+1} from the
                         extrapolated moments (hvpic_field_advance_pe with
                         the electron energy equation: p_e is advanced in
                         the same substeps, starting from the EOS pressure
                         of the first moments)

Step 2 and steps 4-5 touch disjoint data (the particle store, the map and
cell_start versus the moments, B and E), so with `overlap` (fused deposit)
the sort runs on a side stream, ordered by events: it waits for the push,
and the next push waits for it.  The push and the field advance, the step's
critical path, stay in order on the particle stream, with no event between
them; the sort's latency-bound kernels share the GPU with the field
advance's.  The context is rebound to the side stream for the sort call, so
the move counts the push left in its workspace are the ones the sort reads.

With `gather_map` (fused deposit only) the sort leaves the stable order as a
gather map instead of moving the store (hvpic_sort_perm), and the next push
reads the store through it and writes the pushed particles in sorted order
to the other buffer (hvpic_gather_push_perm): the particle data then crosses
HBM once per step instead of twice.  The state is the store `p` plus `perm`;
particles() returns it in sorted order.  Results are bit-identical to the
plain sequence.

Initialisation (the paper leaves the first half step open): v^{-1/2} = v^0,
and n^{-1/2}, J^{-1/2} are the moments deposited at x^0, so E^0 = Ohm(B^0,
n^0, J^0).  This module only orders the calls and swaps buffers.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

from . import hvpic as H

_HIP_EVENT_DISABLE_TIMING = 0x2
_HIP_EVENT_DISABLE_SYSTEM_FENCE = 0x20000000
_hip = None


def _hip_runtime():
    """The HIP runtime already loaded in the process (torch's and the
    library's share it; RTLD_NOLOAD never loads a second copy), or None."""
    global _hip
    if _hip is None:
        _hip = False
        for soname in ("libamdhip64.so.7", "libamdhip64.so.6", "libamdhip64.so"):
            try:
                lib = ctypes.CDLL(soname, mode=os.RTLD_NOLOAD | os.RTLD_LAZY)
            except OSError:
                continue
            for name, args in (("hipEventCreateWithFlags", (ctypes.c_void_p, ctypes.c_uint)),
                               ("hipEventRecord", (ctypes.c_void_p, ctypes.c_void_p)),
                               ("hipStreamWaitEvent",
                                (ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint)),
                               ("hipEventDestroy", (ctypes.c_void_p,))):
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = ctypes.c_int
            _hip = lib
            break
    return _hip or None


class StreamEvent:
    """Orders work between two streams of one device.  No timing and no
    system-scope fence: recording one does not write back and invalidate the
    caches (a few microseconds that a torch event costs on the stream it is
    recorded on).  Kernels of the other stream still see the data, since each
    kernel releases its writes to the device when it ends and acquires at its
    start; host reads go through the runtime's own copies and synchronisation."""

    def __init__(self):
        self._hip = _hip_runtime()
        self.h = ctypes.c_void_p()
        # without the runtime's entry points: a plain torch event (the same
        # ordering, with the system-scope fence)
        self._torch = torch.cuda.Event() if self._hip is None else None
        if self._torch is None:
            self._check(self._hip.hipEventCreateWithFlags(
                ctypes.byref(self.h), _HIP_EVENT_DISABLE_TIMING | _HIP_EVENT_DISABLE_SYSTEM_FENCE))

    @staticmethod
    def _check(rc):
        if rc != 0:
            raise RuntimeError(f"HIP event call failed with error {rc}")

    def record(self, stream: torch.cuda.Stream):
        if self._torch is not None:
            self._torch.record(stream)
            return
        self._check(self._hip.hipEventRecord(self.h, ctypes.c_void_p(stream.cuda_stream)))

    def wait(self, stream: torch.cuda.Stream):
        """Makes later work on `stream` wait for the last record (none: no wait)."""
        if self._torch is not None:
            stream.wait_event(self._torch)
            return
        self._check(self._hip.hipStreamWaitEvent(ctypes.c_void_p(stream.cuda_stream), self.h, 0))

    def __del__(self):
        # (at interpreter exit the module globals may already be gone)
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self._hip.hipEventDestroy(h)
            h.value = None


class GpuSim:
    def __init__(self, cfg, parts: dict, B: np.ndarray, fused: bool = True, device="cuda",
                 diagnostics: bool = True, overlap: bool = True, gather_map: bool = False):
        if gather_map and not fused:
            raise ValueError("gather_map needs the fused deposit")
        self.cfg = cfg
        self.fused = fused
        self.gather_map = gather_map
        self.device = device
        self.overlap = overlap
        n = int(parts["cell"].size)
        self.np = n
        # push and field work on s_p; the sort on s_s (the same stream unless
        # overlapping; the unfused deposit needs the sorted store, so there
        # the sort stays in line)
        self.overlap = overlap and fused
        self.s_p = torch.cuda.Stream(device)
        self.s_s = torch.cuda.Stream(device) if self.overlap else self.s_p
        self.ctx = H.Context(cfg, max(n, 1), device, stream=self.s_p)
        self.ctx_f = self.ctx
        nc = cfg.ncell
        self.p = H.Particles.from_numpy(parts, cfg.ndim, max(n, 1), device)
        self.q = H.Particles(cfg.ndim, max(n, 1), device)
        f32 = dict(dtype=torch.float32, device=device)
        self.cs = torch.zeros(nc + 1, dtype=torch.int32, device=device)
        self.cs_alt = torch.zeros(nc + 1, dtype=torch.int32, device=device)
        self.B = torch.from_numpy(np.ascontiguousarray(B, dtype=np.float32)).to(device)
        self.E = torch.zeros((3, nc), **f32)
        self.n_prev = torch.zeros(nc, **f32)
        self.J_prev = torch.zeros((3, nc), **f32)
        self.n_half = torch.zeros(nc, **f32)
        self.J_half = torch.zeros((3, nc), **f32)
        # electron pressure, state of the energy equation (Sec. II.A eq:dpdt)
        self.pe = torch.zeros(nc, **f32) if cfg.energy_eq else None
        if cfg.nsmooth:
            self.E_s = torch.zeros((3, nc), **f32)
            self.B_s = torch.zeros((3, nc), **f32)
        self.diagnostics = diagnostics
        self.surrogate = None  # (Surrogate, tol): the field advance by the operator
        self.no_stats = None   # per step {residual ratio, accepted} of the surrogate
        self.record = None     # (B, n, J, B_target, k): snapshots of the field advance
        self.push_diag = torch.zeros(4, dtype=torch.float64, device=device)
        self.field_diag = torch.zeros(3, dtype=torch.float64, device=device)
        self.ev_push = StreamEvent()  # the push of the step is done (the sort may start)
        self.ev_sort = StreamEvent()  # the sort of the step is done (the next push may start)
        self.ev_step = StreamEvent()  # the step's work on the particle stream is done
        # the tensors above (and the contexts' workspaces) were filled on the
        # current stream
        torch.cuda.current_stream(device).synchronize()
        c = self.ctx.ctx
        # first sort of an arbitrary order
        H.hvpic_sort(c, self.p, self.q, None, self.cs, full=True)
        self.p, self.q = self.q, self.p
        # the sorted store read through the identity map
        self.perm = None
        if gather_map:
            with torch.cuda.stream(self.s_p):
                self.perm = torch.arange(max(n, 1), dtype=torch.int32, device=device)
        H.hvpic_deposit(c, self.p, self.cs, 0.0, self.n_prev, self.J_prev)
        self._fields(mode=1, n_half=self.n_prev, J_half=self.J_prev)
        self.nstep = 0
        cur = torch.cuda.current_stream(device)
        self.ev_step.record(self.s_p)
        self.ev_step.wait(cur)

    def _fields(self, mode, n_half, J_half):
        """Smoothing of the moments and the field advance (particle stream)."""
        cfg = self.cfg
        cf = self.ctx_f.ctx
        if cfg.nsmooth:
            H.hvpic_smooth(cf, n_half, cfg.nsmooth)
            H.hvpic_smooth(cf, J_half, cfg.nsmooth)
        diag = self.field_diag if self.diagnostics else None
        if mode == 0 and self.record is not None:
            Bs, ns, Js, Bts, k = self.record
            with torch.cuda.stream(self.s_p):
                Bs[k].copy_(self.B)
                ns[k].copy_(n_half)
                Js[k].copy_(J_half)
        if mode == 0 and self.surrogate is not None:
            surr, tol = self.surrogate
            k = self.nstep % self.no_stats.shape[0]
            H.hvpic_field_advance_no(cf, surr.params, surr.ws_one, self.B, n_half, J_half,
                                     self.n_prev, self.J_prev, self.E, tol, diag_out=diag,
                                     stats=self.no_stats[k])
        elif cfg.energy_eq:
            if mode == 1:  # the start: the pressure of the EOS of the first moments
                H.hvpic_eos_pressure(cf, n_half, self.pe)
            H.hvpic_field_advance_pe(cf, self.B, self.pe, n_half, J_half,
                                     None if mode == 1 else self.n_prev,
                                     None if mode == 1 else self.J_prev, self.E, mode=mode,
                                     diag_out=diag)
        elif mode == 1:
            H.hvpic_field_advance(cf, self.B, n_half, J_half, None, None, self.E, mode=1,
                                  diag_out=diag)
        else:
            H.hvpic_field_advance(cf, self.B, n_half, J_half, self.n_prev, self.J_prev, self.E,
                                  mode=0, diag_out=diag)
        if mode == 0 and self.record is not None:
            Bs, ns, Js, Bts, k = self.record
            with torch.cuda.stream(self.s_p):
                Bts[k].copy_(self.B)
            self.record = None

    def _sort(self):
        """The neighbour-move sort of the pushed store: the gather map over q
        (gather map) or the store moved into q; on the side stream once the
        push is done."""
        side = self.s_s is not self.s_p
        if side:
            self.ev_push.record(self.s_p)
            self.ev_push.wait(self.s_s)
            self.ctx.set_stream(self.s_s)
        try:
            c = self.ctx.ctx
            if self.gather_map:
                H.hvpic_sort_perm(c, self.q, self.cs, self.perm, self.cs_alt)
            else:
                H.hvpic_sort(c, self.p, self.q, self.cs, self.cs_alt, full=False)
        finally:
            if side:
                self.ctx.set_stream(self.s_p)
                self.ev_sort.record(self.s_s)
        self.p, self.q = self.q, self.p
        self.cs, self.cs_alt = self.cs_alt, self.cs

    def step(self, order_caller: bool = True):
        """One time step.  With order_caller, later work on the caller's
        stream waits for it (reads of E, B, the moments, the diagnostics).  A
        loop that reads results only after synchronize() can pass False: a
        recorded event holds the particle stream about 5 us per step."""
        cfg = self.cfg
        c = self.ctx.ctx
        cur = torch.cuda.current_stream(self.device)
        # the last sort's map (or store) and cell_start are written, and its
        # workspace counts consumed, before the push.  (Writes into the
        # simulation's tensors by the caller must be finished first: see
        # synchronize().)
        if self.s_s is not self.s_p:
            self.ev_sort.wait(self.s_p)
        E, B = self.E, self.B
        if cfg.nsmooth:
            with torch.cuda.stream(self.s_p):
                self.E_s.copy_(E)
                self.B_s.copy_(B)
            H.hvpic_smooth(c, self.E_s, cfg.nsmooth)
            H.hvpic_smooth(c, self.B_s, cfg.nsmooth)
            E, B = self.E_s, self.B_s
        pd = self.push_diag if self.diagnostics else None
        if self.gather_map:
            # p read through perm -> q in sorted order; then the map of the
            # next order over q
            H.hvpic_gather_push_perm(c, self.p, self.perm, self.q, self.cs, E, B, self.n_half,
                                     self.J_half, pd)
        elif self.fused:
            H.hvpic_gather_push(c, self.p, self.cs, E, B, self.n_half, self.J_half, pd)
        else:
            H.hvpic_gather_push(c, self.p, self.cs, E, B, None, None, pd)
        # enqueued before the field work, so that it starts right after the push
        self._sort()
        if not self.fused:
            H.hvpic_deposit(c, self.p, self.cs, 0.5 * cfg.dt, self.n_half, self.J_half)
        self._fields(mode=0, n_half=self.n_half, J_half=self.J_half)
        self.n_prev, self.n_half = self.n_half, self.n_prev
        self.J_prev, self.J_half = self.J_half, self.J_prev
        self.nstep += 1
        # later work on the caller's stream (reads of E, B, the moments, the
        # store) sees this step; the next step's launches do not wait for it
        if order_caller:
            self.ev_step.record(self.s_p)
            self.ev_step.wait(cur)
            if self.s_s is not self.s_p:
                self.ev_sort.wait(cur)

    def synchronize(self):
        """Waits for all queued work (host and the caller's stream).  Call it
        after writing into the simulation's tensors from another stream."""
        torch.cuda.current_stream(self.device).synchronize()
        self.s_p.synchronize()
        self.s_s.synchronize()

    def status(self):
        """Sticky status bits and counts (waits for both streams)."""
        self.synchronize()
        return H.hvpic_sync_status(self.ctx.ctx)

    def particles(self) -> dict:
        """The particle store in sorted order (host copy)."""
        self.synchronize()
        d = self.p.to_numpy()
        if self.gather_map:
            idx = self.perm[:self.p.n].cpu().numpy()
            d = {k: v[idx] for k, v in d.items()}
        return d


class Ensemble:
    """Independent 2D runs stepped together (hvpic_ensemble_*): every phase of
    the step is one persistent launch over the work items of all runs.

    Takes GpuSim objects set up for the gather-map sequence (their current
    state is the start) and steps them on a stream of its own; their
    tensors hold the state, rotating between the two buffer sets every step
    as GpuSim.step swaps them.  state(r) returns run r's current tensors.
    The GpuSim objects must not be stepped while the ensemble is in use."""

    def __init__(self, sims, tuning=None, device="cuda"):
        for g in sims:
            if not (g.gather_map and g.fused) or g.cfg.nsmooth or g.cfg.ndim != 2:
                raise ValueError("ensemble runs use the fused gather-map sequence in 2D")
            g.synchronize()
        self.sims = list(sims)
        self.stream = torch.cuda.Stream(device)
        recs = (H.HvpicRun * len(self.sims))()
        for r, g in enumerate(self.sims):
            g.q.n = g.p.n
            R = recs[r]
            R.ctx = g.ctx.ctx
            R.store[0] = g.p.c()
            R.store[1] = g.q.c()
            R.perm = g.perm.data_ptr()
            R.cell_start[0], R.cell_start[1] = g.cs.data_ptr(), g.cs_alt.data_ptr()
            R.E, R.B = g.E.data_ptr(), g.B.data_ptr()
            R.n[0], R.n[1] = g.n_prev.data_ptr(), g.n_half.data_ptr()
            R.J[0], R.J[1] = g.J_prev.data_ptr(), g.J_half.data_ptr()
            R.push_diag = g.push_diag.data_ptr() if g.diagnostics else None
            R.field_diag = g.field_diag.data_ptr() if g.diagnostics else None
        self._recs = recs
        # the even state: the sims' tensors as they are now
        self._bufs = [dict(p=(g.p, g.q), cs=(g.cs, g.cs_alt), n=(g.n_prev, g.n_half),
                           J=(g.J_prev, g.J_half)) for g in self.sims]
        nbytes = H.hvpic_ensemble_workspace_bytes(recs)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        self.e = H.hvpic_ensemble_init(recs, self.stream.cuda_stream, self.workspace, tuning)

    @property
    def steps(self) -> int:
        return H.hvpic_ensemble_steps(self.e)

    def step(self):
        H.hvpic_ensemble_step(self.e)

    def capture(self, enable: bool = True):
        H.hvpic_ensemble_capture(self.e, enable)

    def autotune(self, reps: int = 2):
        """Tunes on real steps (they advance the runs); returns (choices, phase ms)."""
        t, ms = H.hvpic_ensemble_autotune(self.e, reps)
        return t.as_dict(), ms

    def time_phases(self, steps: int = 10):
        """Mean ms per step of {push, moments + sort, fields} over `steps`
        real steps launched directly (they advance the runs)."""
        return H.hvpic_ensemble_time_phases(self.e, steps)

    @property
    def tuning(self) -> dict:
        return H.hvpic_ensemble_get_tuning(self.e).as_dict()

    def set_tuning(self, tuning: dict):
        """Changes the given choices (the others stay)."""
        t = H.hvpic_ensemble_get_tuning(self.e)
        for k, v in tuning.items():
            getattr(t, k)[:] = v
        H.hvpic_ensemble_set_tuning(self.e, t)

    def synchronize(self):
        self.stream.synchronize()

    def state(self, r: int) -> dict:
        """Run r's current state (tensors; no copy): store, perm, cell_start,
        E, B, n, J at level n-1/2, and the diagnostics."""
        self.synchronize()
        k = self.steps & 1
        b = self._bufs[r]
        g = self.sims[r]
        return dict(p=b["p"][k], perm=g.perm, cs=b["cs"][k], E=g.E, B=g.B, n_prev=b["n"][k],
                    J_prev=b["J"][k], push_diag=g.push_diag, field_diag=g.field_diag)

    def particles(self, r: int) -> dict:
        """Run r's particle store in sorted order (host copy)."""
        s = self.state(r)
        d = s["p"].to_numpy()
        idx = s["perm"][:s["p"].n].cpu().numpy()
        return {k: v[idx] for k, v in d.items()}

    def status(self, r: int):
        self.synchronize()
        return H.hvpic_sync_status(self.sims[r].ctx.ctx)

    def close(self):
        if getattr(self, "e", None) is not None:
            self.synchronize()
            H.hvpic_ensemble_finalize(self.e)
            self.e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """The convolutional neural operator of the field subcycle on one 2D grid
    (hvpic_no_*): its parameter block, a training workspace for `batch`
    samples and an inference workspace, in device memory.  Weights are lists
    of (W [Cout][9][Cin], b [Cout]) per layer; norm = (mean[7], std[7],
    out_std[3])."""

    LAYERS = ((7, 32), (32, 32), (32, 32), (32, 3))

    def __init__(self, nx: int, ny: int, batch: int = 8, device="cuda"):
        self.nx, self.ny, self.batch = nx, ny, batch
        self.device = device
        self.params = torch.zeros(H.hvpic_no_params_bytes(), dtype=torch.uint8, device=device)
        self.ws_train = torch.empty(H.hvpic_no_workspace_bytes(nx, ny, batch), dtype=torch.uint8,
                                    device=device)
        self.ws_one = torch.empty(H.hvpic_no_workspace_bytes(nx, ny, 1), dtype=torch.uint8,
                                  device=device)

    @classmethod
    def initial_weights(cls, seed: int):
        """Seeded starting weights: uniform in +-sqrt(3/(9 Cin)) per layer
        (unit variance of the pre-activation for unit-variance inputs), zero
        biases."""
        rng = np.random.Generator(np.random.PCG64(seed))
        out = []
        for cin, cout in cls.LAYERS:
            lim = np.sqrt(3.0 / (9 * cin))
            out.append((rng.uniform(-lim, lim, (cout, 9, cin)), np.zeros(cout)))
        return out

    def load(self, weights, norm):
        w = np.concatenate([np.asarray(wl, np.float32).ravel() for wl, _ in weights])
        b = np.concatenate([np.asarray(bl, np.float32).ravel() for _, bl in weights])
        nm = np.concatenate([np.asarray(a, np.float32).ravel() for a in norm])
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.device)
        H.hvpic_no_load(self.params, dev(w), dev(b), dev(nm))
        torch.cuda.current_stream(self.device).synchronize()

    def weights(self):
        nw = sum(o * 9 * i for i, o in self.LAYERS)
        nb = sum(o for _, o in self.LAYERS)
        w = torch.zeros(nw, dtype=torch.float32, device=self.device)
        b = torch.zeros(nb, dtype=torch.float32, device=self.device)
        H.hvpic_no_store(self.params, w, b)
        w, b = w.cpu().numpy(), b.cpu().numpy()
        out, ow, ob = [], 0, 0
        for i, o in self.LAYERS:
            out.append((w[ow:ow + o * 9 * i].reshape(o, 9, i).astype(np.float64),
                        b[ob:ob + o].astype(np.float64)))
            ow += o * 9 * i
            ob += o
        return out

    def predict(self, B, n, J):
        out = torch.empty_like(B)
        H.hvpic_no_predict(self.params, self.ws_one, self.nx, self.ny, B, n, J, out)
        return out

    def train(self, data, steps: int, lr: float, seed: int = 0):
        """`steps` Adam steps on random batches of the snapshots data = (B, n,
        J, B_target) (device tensors [S][...]); returns the loss per step."""
        B, n, J, Bt = data
        S = B.shape[0]
        rng = np.random.Generator(np.random.PCG64(seed))
        idx = torch.from_numpy(np.stack([rng.choice(S, self.batch, replace=False)
                                         for _ in range(steps)]).astype(np.int32)).to(self.device)
        losses = torch.zeros(steps, dtype=torch.float64, device=self.device)
        for k in range(steps):
            H.hvpic_no_train_step(self.params, self.ws_train, self.nx, self.ny, B, n, J, Bt,
                                  idx[k], lr, losses[k:k + 1])
        return losses



class OpenSim:
    """The 2D step with open x boundaries (Sec. II.C) on the GPU.

    The grid carries a ghost column at each x end (the config's open_x); the
    field is B0 + B1 with B0 fixed.  One step, all on one stream, in the
    gather-map form (the default):

      1. hvpic_gather_push_perm    the store read through the map: E^n,
                                   B0 + B1^n at x^n; the pushed ions written
                                   in order to the second store, their moves
                                   counted; fused deposit of n^{n+1/2},
                                   J^{n+1/2}
      2. hvpic_open_inject         fresh ions appended to the second store
      3. hvpic_sort_open_perm      the next map: ions now in a ghost column
                                   left out (absorbed), injected ions last
                                   in their cells
      4. hvpic_open_fill           ghost columns of the moments
      5. hvpic_open_field_advance  B1^n -> B1^{n+1}, E^{n+1}, B0 + B1^{n+1}

    The sort's info (its fallback flag and the live count) is the one
    device-to-host read of a step, taken while the field advance runs.  With
    `overlap` (gather-map form) the sort runs on a side stream beside steps
    4-5, as in GpuSim: they touch disjoint data (the store, the map,
    cell_start and the sort's workspace against the moments, the fields and
    the field scratch).  When
    far movers keep the sort from its neighbour path, hvpic_open_absorb and
    the general hvpic_sort_open order the store instead (the map restarts as
    the identity).  With gather_map=False every step takes that general
    path: push in place, absorb and inject, radix sort with the absorbed
    ions last.  Initialisation as in GpuSim (v^{-1/2} = v^0, moments
    deposited at x^0)."""

    def __init__(self, cfg, parts: dict, B0, B1, spec: dict, seed: int, capacity: int | None = None,
                 device="cuda", diagnostics: bool = True, gather_map: bool = True,
                 overlap: bool = True):
        if not cfg.open_x:
            raise ValueError("OpenSim needs a config with open_x")
        self.cfg, self.spec, self.seed = cfg, spec, int(seed)
        self.device = device
        self.gather_map = gather_map
        n = int(parts["cell"].size)
        # room for the inflow to outrun the outflow for a while
        face = cfg.ny * (cfg.nz if cfg.ndim == 3 else 1)
        cap = int(capacity) if capacity else 2 * n + 4 * face * int(spec["ppc"]) + 4096
        self.capacity = cap
        self.s = torch.cuda.Stream(device)
        self.overlap = overlap and gather_map
        self.s_sort = torch.cuda.Stream(device) if self.overlap else self.s
        self.ev_push = StreamEvent()
        self.ev_sort = StreamEvent()
        self.ctx = H.Context(cfg, cap, device, stream=self.s)
        self.inflow = H.inflow_from(spec)
        nc = cfg.ncell
        f32 = dict(dtype=torch.float32, device=device)
        self.p = H.Particles.from_numpy(parts, cfg.ndim, cap, device)
        self.q = H.Particles(cfg.ndim, cap, device)
        self.cs = torch.zeros(nc + 2, dtype=torch.int32, device=device)
        self.cs_alt = torch.zeros(nc + 2, dtype=torch.int32, device=device)
        self.perm = torch.zeros(cap, dtype=torch.int32, device=device) if gather_map else None
        self.info = torch.zeros(2, dtype=torch.int32, device=device)
        self.B0 = torch.from_numpy(np.ascontiguousarray(B0, dtype=np.float32)).to(device)
        self.B1 = torch.from_numpy(np.ascontiguousarray(B1, dtype=np.float32)).to(device)
        self.Btot = torch.zeros((3, nc), **f32)
        self.E = torch.zeros((3, nc), **f32)
        self.n_prev = torch.zeros(nc, **f32)
        self.J_prev = torch.zeros((3, nc), **f32)
        self.n_half = torch.zeros(nc, **f32)
        self.J_half = torch.zeros((3, nc), **f32)
        self.diagnostics = diagnostics
        self.push_diag = torch.zeros(4, dtype=torch.float64, device=device)
        self.field_diag = torch.zeros(3, dtype=torch.float64, device=device)
        self.h_info = torch.zeros(2, dtype=torch.int32, pin_memory=True)
        self.ev_info = torch.cuda.Event()
        self.fallbacks = 0  # steps that took the general path (gather-map form)
        torch.cuda.current_stream(device).synchronize()
        c = self.ctx.ctx
        self._general_sort(absorb=True)
        H.hvpic_open_fill(c, self.B1, 3)
        H.hvpic_deposit(c, self.p, self.cs[:nc + 1], 0.0, self.n_prev, self.J_prev)
        H.hvpic_open_fill(c, self.n_prev, 1)
        H.hvpic_open_fill(c, self.J_prev, 3)
        H.hvpic_open_field_advance(c, self.B0, self.B1, self.Btot, self.n_prev, self.J_prev, None,
                                   None, self.E, mode=1,
                                   diag_out=self.field_diag if diagnostics else None)
        self.s.synchronize()
        self.nstep = 0
        self.absorbed = self.injected = 0

    def _copy_info(self, src, stream=None):
        """Enqueues the copy of two int32 (the sort's info) to the host."""
        stream = stream or self.s
        with torch.cuda.stream(stream):
            self.h_info.copy_(src, non_blocking=True)
            self.ev_info.record(stream)

    def _general_sort(self, absorb: bool):
        """Orders the current store p (all p.n ions) by the radix path with
        the absorbed ions last, into p; the map restarts as the identity.
        Waits for the live count."""
        c = self.ctx.ctx
        nc = self.cfg.ncell
        if absorb:
            H.hvpic_open_absorb(c, self.p)
        H.hvpic_sort_open(c, self.p, self.q, self.cs)
        self.p, self.q = self.q, self.p
        self._copy_info(self.cs[nc:nc + 2])
        self.ev_info.synchronize()
        self.p.n = int(self.h_info[0])
        self.live = self.p.n
        if self.gather_map:
            with torch.cuda.stream(self.s):
                torch.arange(self.p.n, dtype=torch.int32, device=self.device,
                             out=self.perm[:self.p.n])

    def step(self):
        cfg = self.cfg
        c = self.ctx.ctx
        nc = cfg.ncell
        # writes by the caller's stream come first
        self.s.wait_stream(torch.cuda.current_stream(self.device))
        pd = self.push_diag if self.diagnostics else None
        if self.gather_map:
            # the store p holds p.n ions; the map selects the live ones
            H.hvpic_gather_push_select(c, self.p, self.live, self.perm, self.q, self.cs, self.E,
                                       self.Btot, self.n_half, self.J_half, pd)
            n_pushed = self.q.n
            H.hvpic_open_inject(c, self.q, self.inflow, self.seed, self.nstep)
            self.injected += self.q.n - n_pushed
            total = self.q.n
            if self.overlap:
                # the sort beside the field advance, once the push and the
                # injection are done
                self.ev_push.record(self.s)
                self.ev_push.wait(self.s_sort)
                self.ctx.set_stream(self.s_sort)
            try:
                H.hvpic_sort_open_perm(c, self.q, n_pushed, self.cs, self.perm, self.cs_alt,
                                       self.info)
                self._copy_info(self.info, self.s_sort)
            finally:
                if self.overlap:
                    self.ctx.set_stream(self.s)
                    self.ev_sort.record(self.s_sort)
        else:
            H.hvpic_gather_push(c, self.p, None, self.E, self.Btot, self.n_half, self.J_half, pd)
            n_before = self.p.n
            H.hvpic_open_particles(c, self.p, self.inflow, self.seed, self.nstep)
            self.injected += self.p.n - n_before
            total = self.p.n
            H.hvpic_sort_open(c, self.p, self.q, self.cs)
            self._copy_info(self.cs[nc:nc + 2])
        H.hvpic_open_fill(c, self.n_half, 1)
        H.hvpic_open_fill(c, self.J_half, 3)
        H.hvpic_open_field_advance(c, self.B0, self.B1, self.Btot, self.n_half, self.J_half,
                                   self.n_prev, self.J_prev, self.E, mode=0,
                                   diag_out=self.field_diag if self.diagnostics else None)
        self.n_prev, self.n_half = self.n_half, self.n_prev
        self.J_prev, self.J_half = self.J_half, self.J_prev
        self.ev_info.synchronize()
        if self.overlap:
            self.ev_sort.wait(self.s)  # the next push reads the new map
        if self.gather_map:
            if int(self.h_info[0]) != 0:
                # far movers: the general path on the pushed and injected store
                self.fallbacks += 1
                self.p, self.q = self.q, self.p
                self._general_sort(absorb=True)
                alive = self.p.n
            else:
                alive = int(self.h_info[1])
                self.p, self.q = self.q, self.p
                self.cs, self.cs_alt = self.cs_alt, self.cs
                self.live = alive
        else:
            alive = int(self.h_info[0])
            self.p, self.q = self.q, self.p
            self.p.n = alive
            self.live = alive
        self.absorbed += total - alive
        self.nstep += 1
        torch.cuda.current_stream(self.device).wait_stream(self.s)

    def synchronize(self):
        torch.cuda.current_stream(self.device).synchronize()
        self.s.synchronize()
        self.s_sort.synchronize()

    def status(self):
        self.synchronize()
        return H.hvpic_sync_status(self.ctx.ctx)

    def particles(self) -> dict:
        """The live particle store in sorted order (host copy)."""
        self.synchronize()
        d = self.p.to_numpy()
        if self.gather_map:
            idx = self.perm[:self.live].cpu().numpy()
            d = {k: v[idx] for k, v in d.items()}
        return d
