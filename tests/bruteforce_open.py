"""A second, independent FP64 implementation of the open-boundary field
advance (Sec. II.C), in NumPy, to check the C oracle against (it imports
nothing from it).

The fields are held as [component][z][y][x] arrays (nz = 1 in 2D) and
written another way than the oracle's cell loops:
  * the ghost columns x = 0 and x = nx-1 are filled by slicing;
  * x-derivatives are whole-array periodic differences (np.roll) multiplied
    by a column mask that is 0 in the ghost columns, so Ohm's law there has
    no x-gradient; y- and z-derivatives are periodic differences everywhere
    (the z ones only in 3D);
  * the hyper-resistive Laplacian is the forward difference of a backward
    difference, its x part masked the same way, and the buffer's eta_h is a
    per-column array built from the distance to the outermost interior
    column;
  * the RK2 subcycle works on whole arrays, refilling the ghost columns
    after each stage.
Readings are those of the method as the oracle states them: B = B0 + B1
with J = curl B1; the EOS pressure of the floored density; the moments
frozen at n+1/2 in the subcycle; E^{n+1} from the extrapolated moments
3/2 (n+1/2) - 1/2 (n-1/2)."""
from __future__ import annotations

import numpy as np


class OpenGrid:
    def __init__(self, cfg):
        self.cfg = cfg
        self.nx, self.ny, self.nz = cfg.nx, cfg.ny, cfg.nz
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        i = np.arange(cfg.nx)
        self.interior = ((i > 0) & (i < cfg.nx - 1)).astype(float)  # per column
        d = np.maximum(np.minimum(i, cfg.nx - 1 - i) - 1, 0)
        w = cfg.buffer_cells
        ramp = np.where(d < w, cfg.eta_h_buffer * (1.0 - d / max(w, 1)), 0.0) if w > 0 else 0.0 * d
        self.eta_h = cfg.eta_h + ramp  # per column

    def grid(self, F):
        F = np.asarray(F, np.float64)
        return F.reshape((-1,) + self.shape) if F.ndim > 1 else F.reshape(self.shape)

    def flat(self, F):
        return np.asarray(F).reshape(F.shape[0], -1) if F.ndim == 4 else np.asarray(F).ravel()

    def fill(self, F):
        F = F.copy()
        F[..., 0] = F[..., 1]
        F[..., -1] = F[..., -2]
        return F

    def dx(self, Q):
        return (np.roll(Q, -1, -1) - np.roll(Q, 1, -1)) / (2 * self.cfg.dx) * self.interior

    def dy(self, Q):
        return (np.roll(Q, -1, -2) - np.roll(Q, 1, -2)) / (2 * self.cfg.dy)

    def dz(self, Q):
        if self.cfg.ndim == 2:
            return np.zeros_like(Q)
        return (np.roll(Q, -1, -3) - np.roll(Q, 1, -3)) / (2 * self.cfg.dz)

    def lap(self, Q):
        def second(axis, h):
            f = (np.roll(Q, -1, axis) - Q) / h
            return (f - np.roll(f, 1, axis)) / h
        r = second(-2, self.cfg.dy) + second(-1, self.cfg.dx) * self.interior
        if self.cfg.ndim == 3:
            r = r + second(-3, self.cfg.dz)
        return r

    def curl(self, A):
        Ax, Ay, Az = A
        return np.stack([self.dy(Az) - self.dz(Ay), self.dz(Ax) - self.dx(Az),
                         self.dx(Ay) - self.dy(Ax)])

    def ohm(self, B0, B1, n, Ji):
        c = self.cfg
        J = self.curl(B1)
        ne = np.maximum(n, c.n_floor)
        pe = c.n0 * c.te * (ne / c.n0) ** c.gamma_e
        B = B0 + B1
        ui = Ji / ne
        gp = np.stack([self.dx(pe), self.dy(pe), self.dz(pe)])
        E = -gp / ne - np.cross(ui, B, axis=0) + np.cross(J, B, axis=0) / ne + c.eta * J
        hyper = np.stack([self.lap(J[a]) for a in range(3)]) * self.eta_h
        return E - hyper

    def field_advance(self, B0, B1, n_half, J_half, n_prev=None, J_prev=None, mode=0):
        """(B1_new, E_out, B0 + B1_new); the oracle's order of operations."""
        c = self.cfg
        g = self.grid
        B0, B1, nh, Jh = g(B0), g(B1), g(n_half), g(J_half)
        if mode == 0:
            B1 = self.fill(B1)
            h = c.dt / max(c.nsub, 1)
            for _ in range(c.nsub):
                Bs = self.fill(B1 - 0.5 * h * self.curl(self.ohm(B0, B1, nh, Jh)))
                B1 = self.fill(B1 - h * self.curl(self.ohm(B0, Bs, nh, Jh)))
            n1 = 1.5 * nh - 0.5 * g(n_prev)
            J1 = 1.5 * Jh - 0.5 * g(J_prev)
        else:
            n1, J1 = nh, Jh
        E = self.ohm(B0, B1, n1, J1)
        return self.flat(B1), self.flat(E), self.flat(B0 + B1)
