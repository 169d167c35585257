"""A second, independent FP64 implementation of one hybrid-PIC step, in NumPy.

It exists only to check the C oracle against (it imports nothing from it) and
is deliberately written another way wherever the method allows:
  * positions are global coordinates X = (i + 1/2 + o/2) h, moved as
    X + v dt and wrapped modulo the box, then split into cell and offset;
  * the shape weights of App. B eq:quad (QS) and eq:ngp (NGP) are summed over
    EVERY cell of the grid by periodic cell distance, so aliased stencil
    points (an axis of one or two cells) add up by themselves;
  * the gather is the adjoint of that deposit, F(x_p) = sum_c W_c(x_p) F_c
    (the no-self-force form of App. B), not the interpolant form eq:quadF;
  * the Boris update (Sec. II.B eq:vadv) is solved as the linear system of
    the implicit midpoint rule, (I - T) v+ = (I + T) v-, with T v = v x t;
  * the stable sort is numpy's stable argsort;
  * the field solver (Sec. II.A eq:ohm, Ampere, Faraday) uses np.roll
    stencils; the Laplacian of the hyper-resistive and the conduction terms is
    taken as a backward difference of a forward difference;
  * with the electron energy equation (eq:dpdt) the pressure is advanced in
    the same RK2 stages as B, and W_e = sum p_e V / (gamma - 1).
The step order and the readings are those of the oracle: deposit at
x^{n+1/2}; the moments extrapolated as 3/2 (n+1/2) - 1/2 (n-1/2); RK2
subcycle with the moments frozen at n+1/2; v^{-1/2} = v^0 and the level -1/2
moments deposited at x^0.
"""
from __future__ import annotations

import numpy as np


class Grid:
    def __init__(self, cfg):
        self.cfg = cfg
        self.n = np.array([cfg.nx, cfg.ny, cfg.nz])
        self.h = np.array([cfg.dx, cfg.dy, cfg.dz])
        self.L = self.n * self.h
        self.ndim = cfg.ndim
        self.ncell = int(np.prod(self.n))
        c = np.arange(self.ncell)
        self.ijk = np.stack([c % cfg.nx, (c // cfg.nx) % cfg.ny, c // (cfg.nx * cfg.ny)])


def to_global(g: Grid, parts):
    c = parts["cell"].astype(np.int64)
    idx = np.stack([c % g.n[0], (c // g.n[0]) % g.n[1], c // (g.n[0] * g.n[1])])
    offs = [parts["ox"], parts["oy"], parts["oz"] if g.ndim == 3 else np.zeros(c.size)]
    return np.stack([(idx[a] + 0.5 + 0.5 * np.asarray(offs[a], np.float64)) * g.h[a]
                     for a in range(3)])


def to_cell(g: Grid, X):
    """Cell index and offsets in [-1, 1) of global positions (wrapped)."""
    X = np.mod(X, g.L[:, None])
    s = X / g.h[:, None]
    i = np.floor(s)
    o = 2.0 * (s - i) - 1.0
    i = i.astype(np.int64)
    # a position that wraps to exactly L (rounding) belongs to cell 0
    for a in range(3):
        over = i[a] >= g.n[a]
        i[a][over] -= g.n[a]
    cell = i[0] + g.n[0] * (i[1] + g.n[1] * i[2])
    return cell.astype(np.int32), o


def weights_all_cells(g: Grid, cell, o):
    """W[p, c]: the shape weight of every cell c for particle p in `cell`
    with offsets o (3, N) -- eq:quad summed over the stencil points that land
    on c (so an axis of 1 or 2 cells folds its points together), or eq:ngp."""
    N = cell.size
    W = np.zeros((N, g.ncell))
    pc = np.stack([cell % g.n[0], (cell // g.n[0]) % g.n[1], cell // (g.n[0] * g.n[1])])
    x, y = o[0], o[1]
    z = o[2] if g.ndim == 3 else np.zeros(N)
    if g.cfg.shape == 0:
        pts = [((0, 0, 0), np.ones(N))]
    else:
        pts = [((0, 0, 0), (3.0 - x * x - y * y - z * z) / 6.0),
               ((1, 0, 0), (1.0 + x) ** 2 / 12.0), ((-1, 0, 0), (1.0 - x) ** 2 / 12.0),
               ((0, 1, 0), (1.0 + y) ** 2 / 12.0), ((0, -1, 0), (1.0 - y) ** 2 / 12.0),
               ((0, 0, 1), (1.0 + z) ** 2 / 12.0), ((0, 0, -1), (1.0 - z) ** 2 / 12.0)]
    for c in range(g.ncell):
        for (d, wv) in pts:
            hit = np.ones(N, bool)
            for a in range(3):
                hit &= np.mod(pc[a] + d[a] - g.ijk[a, c], g.n[a]) == 0
            W[hit, c] += wv[hit]
    return W


def boris(a, E, B, v):
    """eq:vadv as the implicit midpoint rule: v+ - v- = (v+ + v-) x t."""
    out = np.empty_like(v)
    for p in range(v.shape[1]):
        t = a * B[:, p]
        # T u = u x t
        T = np.array([[0.0, t[2], -t[1]], [-t[2], 0.0, t[0]], [t[1], -t[0], 0.0]])
        vm = v[:, p] + a * E[:, p]
        vp = np.linalg.solve(np.eye(3) - T, (np.eye(3) + T) @ vm)
        out[:, p] = vp + a * E[:, p]
    return out


def deposit(g: Grid, cfg, X, v, w):
    cell, o = to_cell(g, X)
    W = weights_all_cells(g, cell, o)
    qw = cfg.qs * w / (cfg.dx * cfg.dy * cfg.dz)
    n = (qw[:, None] * W).sum(axis=0)
    J = np.stack([((qw * v[a])[:, None] * W).sum(axis=0) for a in range(3)])
    return n, J


def dc(g: Grid, Q, axis):
    """Centred difference along axis (0: x, 1: y, 2: z) of Q[ncell]."""
    shape = (g.n[2], g.n[1], g.n[0])
    q = Q.reshape(shape)
    ax = 2 - axis
    return ((np.roll(q, -1, ax) - np.roll(q, 1, ax)) / (2.0 * g.h[axis])).reshape(-1)


def curl(g: Grid, A):
    return np.stack([dc(g, A[2], 1) - dc(g, A[1], 2), dc(g, A[0], 2) - dc(g, A[2], 0),
                     dc(g, A[1], 0) - dc(g, A[0], 1)])


def lap(g: Grid, Q):
    """Sum over the axes of D-(D+ Q), D+- the one-sided differences."""
    shape = (g.n[2], g.n[1], g.n[0])
    q = Q.reshape(shape)
    out = np.zeros(shape)
    for axis in range(3):
        ax = 2 - axis
        fwd = (np.roll(q, -1, ax) - q) / g.h[axis]
        out += (fwd - np.roll(fwd, 1, ax)) / g.h[axis]
    return out.reshape(-1)


def eos(cfg, n):
    nf = np.maximum(n, cfg.n_floor)
    return cfg.n0 * cfg.te * (nf / cfg.n0) ** cfg.gamma_e


def ohm(g: Grid, cfg, B, n, Ji, pe=None):
    nf = np.maximum(n, cfg.n_floor)
    if pe is None:
        pe = eos(cfg, n)
    J = curl(g, B)
    u = Ji / nf
    gp = np.stack([dc(g, pe, a) for a in range(3)])
    E = -np.cross(u.T, B.T).T + np.cross(J.T, B.T).T / nf - gp / nf + cfg.eta * J
    if cfg.eta_h:
        E -= cfg.eta_h * np.stack([lap(g, J[a]) for a in range(3)])
    return E


def pe_rate(g: Grid, cfg, B, n, Ji, pe):
    """eq:dpdt with H_ei = 0 and Q_e = -kappa0 grad(p_e/n_e)."""
    nf = np.maximum(n, cfg.n_floor)
    ue = (Ji - curl(g, B)) / nf
    gam = cfg.gamma_e
    div = sum(dc(g, pe * ue[a], a) for a in range(3))
    adv = sum(ue[a] * dc(g, pe, a) for a in range(3))
    return -gam * div + (gam - 1.0) * adv + (gam - 1.0) * cfg.kappa0 * lap(g, pe / nf)


def energies(g: Grid, cfg, B, n, pe=None):
    V = cfg.dx * cfg.dy * cfg.dz
    wb = 0.5 * np.sum(B * B) * V
    dB = B - B.mean(axis=1, keepdims=True)
    wdb = 0.5 * np.sum(dB * dB) * V
    nf = np.maximum(n, cfg.n_floor)
    if pe is not None:
        we = np.sum(pe) * V / (cfg.gamma_e - 1.0)
    elif cfg.gamma_e == 1.0:
        we = cfg.te * np.sum(nf * np.log(nf / cfg.n0)) * V
    else:
        we = np.sum(cfg.n0 * cfg.te * (nf / cfg.n0) ** cfg.gamma_e) * V / (cfg.gamma_e - 1.0)
    return np.array([wb, wdb, we])


class BruteSim:
    """State: X (global positions, sorted by cell), v^{n-1/2}, w; B^n, E^n;
    the moments at n-1/2."""

    def __init__(self, cfg, parts):
        self.cfg = cfg
        self.g = Grid(cfg)
        X = to_global(self.g, parts)
        v = np.stack([np.asarray(parts[k], np.float64) for k in ("ux", "uy", "uz")])
        w = np.asarray(parts["w"], np.float64)
        self._set(X, v, w)

    def _set(self, X, v, w):
        cell, _ = to_cell(self.g, X)
        order = np.argsort(cell, kind="stable")
        self.X, self.v, self.w = X[:, order], v[:, order], w[order]

    def init_fields(self, B):
        cfg = self.cfg
        self.B = np.asarray(B, np.float64).copy()
        self.n_prev, self.J_prev = deposit(self.g, cfg, self.X, self.v, self.w)
        self.pe = eos(cfg, self.n_prev) if cfg.energy_eq else None
        self.E = ohm(self.g, cfg, self.B, self.n_prev, self.J_prev, self.pe)

    def particles(self):
        cell, o = to_cell(self.g, self.X)
        d = {"cell": cell, "ox": o[0], "oy": o[1], "ux": self.v[0], "uy": self.v[1],
             "uz": self.v[2], "w": self.w}
        if self.cfg.ndim == 3:
            d["oz"] = o[2]
        return d

    def step(self):
        cfg, g = self.cfg, self.g
        cell, o = to_cell(g, self.X)
        W = weights_all_cells(g, cell, o)
        Ep = (W @ self.E.T).T
        Bp = (W @ self.B.T).T
        a = 0.5 * cfg.qs / cfg.ms * cfg.dt
        v_new = boris(a, Ep, Bp, self.v)
        self.K = 0.5 * cfg.ms * np.sum(self.w * np.sum(self.v * v_new, axis=0))
        self.P = cfg.ms * (0.5 * (self.v + v_new)) @ self.w
        X_new = self.X + cfg.dt * v_new
        if cfg.ndim == 2:
            X_new[2] = self.X[2]
        self._set(X_new, v_new, self.w)
        Xm = self.X - 0.5 * cfg.dt * self.v
        if cfg.ndim == 2:
            Xm[2] = self.X[2]
        n_half, J_half = deposit(g, cfg, Xm, self.v, self.w)
        h = cfg.dt / cfg.nsub
        pe = self.pe
        for _ in range(cfg.nsub):
            Bs = self.B - 0.5 * h * curl(g, ohm(g, cfg, self.B, n_half, J_half, pe))
            if pe is not None:
                ps = pe + 0.5 * h * pe_rate(g, cfg, self.B, n_half, J_half, pe)
                pe = pe + h * pe_rate(g, cfg, Bs, n_half, J_half, ps)
            else:
                ps = None
            self.B = self.B - h * curl(g, ohm(g, cfg, Bs, n_half, J_half, ps))
        self.pe = pe
        n1 = 1.5 * n_half - 0.5 * self.n_prev
        J1 = 1.5 * J_half - 0.5 * self.J_prev
        self.E = ohm(g, cfg, self.B, n1, J1, pe)
        self.field_diag = energies(g, cfg, self.B, n1, pe)
        self.n_prev, self.J_prev = n_half, J_half
