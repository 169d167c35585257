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
                         extrapolated moments

Initialisation (the paper leaves the first half step open): v^{-1/2} = v^0,
and n^{-1/2}, J^{-1/2} are the moments deposited at x^0, so E^0 = Ohm(B^0,
n^0, J^0).  This module only orders the calls and swaps buffers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hvpic as H


class GpuSim:
    def __init__(self, cfg, parts: dict, B: np.ndarray, fused: bool = True, device="cuda",
                 diagnostics: bool = True):
        self.cfg = cfg
        self.fused = fused
        self.device = device
        n = int(parts["cell"].size)
        self.np = n
        self.ctx = H.Context(cfg, max(n, 1), device)
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
        if cfg.nsmooth:
            self.E_s = torch.zeros((3, nc), **f32)
            self.B_s = torch.zeros((3, nc), **f32)
        self.diagnostics = diagnostics
        self.push_diag = torch.zeros(4, dtype=torch.float64, device=device)
        self.field_diag = torch.zeros(2, dtype=torch.float64, device=device)
        c = self.ctx.ctx
        # first sort of an arbitrary order
        H.hvpic_sort(c, self.p, self.q, None, self.cs, full=True)
        self.p, self.q = self.q, self.p
        H.hvpic_deposit(c, self.p, self.cs, 0.0, self.n_prev, self.J_prev)
        if cfg.nsmooth:
            H.hvpic_smooth(c, self.n_prev, cfg.nsmooth)
            H.hvpic_smooth(c, self.J_prev, cfg.nsmooth)
        H.hvpic_field_advance(c, self.B, self.n_prev, self.J_prev, None, None, self.E, mode=1,
                              diag_out=self.field_diag if diagnostics else None)
        self.nstep = 0

    def step(self):
        cfg = self.cfg
        c = self.ctx.ctx
        E, B = self.E, self.B
        if cfg.nsmooth:
            self.E_s.copy_(E)
            self.B_s.copy_(B)
            H.hvpic_smooth(c, self.E_s, cfg.nsmooth)
            H.hvpic_smooth(c, self.B_s, cfg.nsmooth)
            E, B = self.E_s, self.B_s
        pd = self.push_diag if self.diagnostics else None
        if self.fused:
            H.hvpic_gather_push(c, self.p, self.cs, E, B, self.n_half, self.J_half, pd)
        else:
            H.hvpic_gather_push(c, self.p, self.cs, E, B, None, None, pd)
        H.hvpic_sort(c, self.p, self.q, self.cs, self.cs_alt, full=False)
        self.p, self.q = self.q, self.p
        self.cs, self.cs_alt = self.cs_alt, self.cs
        if not self.fused:
            H.hvpic_deposit(c, self.p, self.cs, 0.5 * cfg.dt, self.n_half, self.J_half)
        if cfg.nsmooth:
            H.hvpic_smooth(c, self.n_half, cfg.nsmooth)
            H.hvpic_smooth(c, self.J_half, cfg.nsmooth)
        H.hvpic_field_advance(c, self.B, self.n_half, self.J_half, self.n_prev, self.J_prev,
                              self.E, mode=0,
                              diag_out=self.field_diag if self.diagnostics else None)
        self.n_prev, self.n_half = self.n_half, self.n_prev
        self.J_prev, self.J_half = self.J_half, self.J_prev
        self.nstep += 1

    def status(self):
        return H.hvpic_sync_status(self.ctx.ctx)

    def particles(self) -> dict:
        return self.p.to_numpy()
