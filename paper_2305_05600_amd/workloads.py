"""Seeded synthetic workloads for the hybrid-PIC step.

This module only *draws inputs*: run parameters, the initial particle store
(cell index, in-cell offsets, velocities, weights) and the initial magnetic
field.  It holds none of the method's arithmetic (no push, no sort, no
deposit, no Ohm's law); both the GPU library and the FP64 oracle start from
what it returns.

All floating-point values are produced in FP64 from ``numpy.random.PCG64`` and
rounded to FP32, so that the FP32 GPU path and the FP64 oracle start from
identical numbers.  Units are the hybrid (Alfvenic) units of Sec. II.A of the
paper: n0 = B0 = m_i = e = mu0 = 1, lengths in d_i, time in 1/Omega_i.

Layout conventions shared with both implementations:
  * cell index I = i + nx*(j + ny*k)
  * offsets ox, oy, oz in [-1, 1): half-cell units about the cell centre
  * grid arrays are component-major, shape (3, ncell)
  * 2D runs have nz = 1, dz = 1 and no oz array
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SHAPE_NGP = 0
SHAPE_QS = 1

_ONE_MINUS = np.nextafter(np.float32(1.0), np.float32(0.0))


@dataclasses.dataclass
class Config:
    """Run parameters.  Field names mirror the C parameter block."""

    name: str
    ndim: int
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    dt: float
    nsub: int
    shape: int = SHAPE_QS
    nsmooth: int = 0
    qs: float = 1.0
    ms: float = 1.0
    te: float = 0.25
    gamma_e: float = 1.0
    n0: float = 1.0
    n_floor: float = 0.05
    eta: float = 1e-3
    eta_h: float = 0.0
    energy_eq: int = 0
    kappa0: float = 0.0
    open_x: int = 0
    buffer_cells: int = 0
    eta_h_buffer: float = 0.0
    steps: int = 1

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    def replace(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


def _f32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def _offsets(raw: np.ndarray) -> np.ndarray:
    """FP32 offsets in [-1, 1) from FP64 draws in [-1, 1)."""
    o = _f32(raw)
    o[o >= np.float32(1.0)] = _ONE_MINUS
    o[o < np.float32(-1.0)] = np.float32(-1.0)
    return o


def _position_to_cell(x: np.ndarray, h: float, n: int):
    """Cell index and half-cell offset of continuous positions in [0, n h)."""
    s = np.mod(x, n * h) / h
    i = np.floor(s).astype(np.int64)
    i = np.clip(i, 0, n - 1)
    return i, _offsets(2.0 * (s - i) - 1.0)


def _particles(cfg: Config, i, j, k, ox, oy, oz, ux, uy, uz, w, order=None):
    cell = (i + cfg.nx * (j + cfg.ny * k)).astype(np.int32)
    out = {
        "cell": cell,
        "ox": ox,
        "oy": oy,
        "ux": _f32(ux),
        "uy": _f32(uy),
        "uz": _f32(uz),
        "w": _f32(w),
    }
    if cfg.ndim == 3:
        out["oz"] = oz
    if order is not None:
        out = {key: v[order] for key, v in out.items()}
    return out


def field_zeros(cfg: Config) -> np.ndarray:
    return np.zeros((3, cfg.ncell), dtype=np.float32)


def cell_centres(cfg: Config):
    """Coordinates (x, y, z) of the cell centres, each of shape (ncell,)."""
    c = np.arange(cfg.ncell)
    i = c % cfg.nx
    j = (c // cfg.nx) % cfg.ny
    k = c // (cfg.nx * cfg.ny)
    return (i + 0.5) * cfg.dx, (j + 0.5) * cfg.dy, (k + 0.5) * cfg.dz


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def periodic_alfven(seed: int = 1, nx: int = 32, ny: int = 32, ppc: int = 64,
                    vth: float = 0.5, amp: float = 0.01, shape: int = SHAPE_QS,
                    steps: int = 100):
    """2D periodic box, uniform B0 = x, a transverse wave dB_y = amp cos(2 pi x/L).

    The small case: 32x32 cells of 0.5 d_i, 64 ions per cell with uniform
    random offsets, Maxwellian velocities of per-component spread vth, isothermal
    electrons with T_e = T_i = vth^2, eta = 1e-3, dt = 0.01, 4 B-subcycles.
    """
    cfg = Config(name=f"2d-periodic-alfven-{nx}x{ny}-ppc{ppc}", ndim=2, nx=nx, ny=ny,
                 nz=1, dx=0.5, dy=0.5, dz=1.0, dt=0.01, nsub=4, shape=shape,
                 te=vth * vth, eta=1e-3, steps=steps)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = cfg.ncell * ppc
    cell = np.repeat(np.arange(cfg.ncell, dtype=np.int64), ppc)
    i = cell % nx
    j = cell // nx
    ox = _offsets(rng.uniform(-1.0, 1.0, n))
    oy = _offsets(rng.uniform(-1.0, 1.0, n))
    u = rng.normal(0.0, vth, (3, n))
    w = np.full(n, cfg.dx * cfg.dy * cfg.dz / ppc)
    parts = _particles(cfg, i, j, 0 * i, ox, oy, None, u[0], u[1], u[2], w,
                       order=rng.permutation(n))
    x, _, _ = cell_centres(cfg)
    B = field_zeros(cfg)
    B[0] = 1.0
    B[1] = _f32(amp * np.cos(2.0 * math.pi * x / (nx * cfg.dx)))
    return cfg, parts, B


def ensemble_specs(seed: int = 4, nruns: int = 64, side=(64, 256), ppc=(32, 200),
                   amp=(0.001, 0.05), te_ratio=(0.1, 1.0), vth: float = 0.5) -> list:
    """Parameters of an ensemble of independent 2D periodic runs of uneven
    size: per run a square grid with side uniform in [side], particles per
    cell uniform in [ppc], a transverse wave of amplitude uniform in [amp]
    (in B0) and T_e/T_i uniform in [te_ratio], otherwise the small periodic
    case (0.5 d_i cells, v_th = 0.5, eta = 1e-3, dt = 0.01, 4 B-subcycles).
    Returns one dict per run for ensemble_run."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.integers(side[0], side[1] + 1, nruns)
    ppcs = rng.integers(ppc[0], ppc[1] + 1, nruns)
    amps = rng.uniform(amp[0], amp[1], nruns)
    ratios = rng.uniform(te_ratio[0], te_ratio[1], nruns)
    return [dict(seed=int(seed * 1000 + r), side=int(sides[r]), ppc=int(ppcs[r]),
                 amp=float(amps[r]), te_ratio=float(ratios[r]), vth=vth) for r in range(nruns)]


def ensemble_run(spec: dict, shape: int = SHAPE_QS):
    """(cfg, parts, B) of one run of ensemble_specs."""
    cfg, parts, B = periodic_alfven(seed=spec["seed"], nx=spec["side"], ny=spec["side"],
                                    ppc=spec["ppc"], vth=spec["vth"], amp=spec["amp"],
                                    shape=shape)
    te = spec["te_ratio"] * spec["vth"] ** 2
    cfg = cfg.replace(te=te, name=f"2d-periodic-{spec['side']}^2-ppc{spec['ppc']}-a{spec['amp']:.3g}"
                                  f"-te{te:.3g}")
    return cfg, parts, B


def open_flow(seed: int = 9, nx: int = 64, ny: int = 32, ppc: int = 32, ux: float = 0.5,
              vth: float = 0.3, b0=(0.0, 1.0, 0.0), amp: float = 0.02, buffer_cells: int = 4,
              eta_h_buffer: float = 0.02, dt: float = 0.02, nsub: int = 4, dx: float = 0.5,
              shape: int = SHAPE_QS, name: str | None = None, nz: int = 1):
    """A plasma drifting along x through a box open in x (Sec. II.C) and
    periodic in y (and z: nz > 1 makes the box 3D), across a fixed external
    field B0 (uniform, curl-free), with a transverse B1 wave of amplitude amp
    in B1_z.

    The grid has nx interior columns plus a ghost column (3D: plane) at each
    x end (i = 0 and nx+1); ions (ppc per cell, density 1, drift ux, thermal
    speed vth per component, T_e = vth^2) fill the interior cells.  The
    same plasma enters through both faces (the inflow spec).  eta = 1e-3
    and a hyper-resistive buffer of buffer_cells cells with eta_h_buffer.
    Returns (cfg, parts, B0, B1, inflow)."""
    ndim = 3 if nz > 1 else 2
    tag = f"{nx}x{ny}" + (f"x{nz}" if ndim == 3 else "")
    cfg = Config(name=name or f"{ndim}d-open-flow-{tag}-ppc{ppc}", ndim=ndim, nx=nx + 2, ny=ny,
                 nz=nz, dx=dx, dy=dx, dz=dx if ndim == 3 else 1.0, dt=dt, nsub=nsub,
                 shape=shape, te=vth * vth, eta=1e-3, open_x=1, buffer_cells=buffer_cells,
                 eta_h_buffer=eta_h_buffer)
    rng = np.random.Generator(np.random.PCG64(seed))
    ncol = nx * ny * nz
    n = ncol * ppc
    col = np.repeat(np.arange(ncol, dtype=np.int64), ppc)
    i = col % nx + 1
    j = (col // nx) % ny
    k = col // (nx * ny)
    ox = _offsets(rng.uniform(-1.0, 1.0, n))
    oy = _offsets(rng.uniform(-1.0, 1.0, n))
    oz = _offsets(rng.uniform(-1.0, 1.0, n)) if ndim == 3 else None
    u = rng.normal(0.0, vth, (3, n))
    u[0] += ux
    w = np.full(n, cfg.dx * cfg.dy * cfg.dz / ppc)
    parts = _particles(cfg, i, j, k, ox, oy, oz, u[0], u[1], u[2], w,
                       order=rng.permutation(n))
    B0 = field_zeros(cfg)
    for a in range(3):
        B0[a] = np.float32(b0[a])
    x, _, _ = cell_centres(cfg)
    B1 = field_zeros(cfg)
    B1[2] = _f32(amp * np.sin(2.0 * math.pi * x / (cfg.nx * cfg.dx)))
    spec = dict(n=1.0, ux=ux, uy=0.0, uz=0.0, vth=vth, ppc=ppc, faces=3)
    return cfg, parts, B0, B1, spec


def solar_wind_box(seed: int = 12, nx: int = 800, ny: int = 1600, ppc: int = 100):
    """The 2D global-magnetosphere run of Sec. III.A without its planet: a
    uniform solar wind through a box open in x (Sec. II.C), periodic in y.
    800 x 1600 cells of 2 d_i, 100 ions per cell (128,000,000 at full
    size), NGP shape, dt = 0.002 / Omega_i with 5 field subcycles,
    isothermal electrons.  The wind flows along +x at Alfven Mach 10 with
    beta_i = beta_e = 0.5 (T = 0.25, thermal speed 0.5 v_A) across a uniform
    interplanetary field B0 = y (in the plane, normal to the flow), with a
    transverse B1 wave of amplitude 0.05; both faces inject the wind, and
    8 buffer cells add eta_h = 1 at each boundary."""
    return open_flow(seed=seed, nx=nx, ny=ny, ppc=ppc, ux=10.0, vth=0.5, b0=(0.0, 1.0, 0.0),
                     amp=0.05, buffer_cells=8, eta_h_buffer=1.0, dt=0.002, nsub=5, dx=2.0,
                     shape=SHAPE_NGP, name=f"2d-open-solar-wind-{nx}x{ny}-ppc{ppc}")


def harris_double(seed: int = 2, nx: int = 512, ny: int = 256, ppc: float = 100.0,
                  steps: int = 1000):
    """Periodic double Harris current sheet (2D, 512x256 cells of 0.125 d_i).

    B_x = tanh((y-Ly/4)/L) - tanh((y-3Ly/4)/L) - 1, L = 0.5 d_i,
    n = sech^2((y-Ly/4)/L) + sech^2((y-3Ly/4)/L) + 0.2, pressure balance
    T_i + T_e = 0.5 with T_e/T_i = 0.2.  Equal particle weights with particles
    per cell proportional to density (average ppc over the box); sheet ions
    drift along z with 2 T_i / L (sign set by the sheet current), background
    ions are at rest.  A 5% perturbation dB = z x grad(psi),
    psi ~ cos(2 pi x/Lx) sin(2 pi y/Ly), max |dB| = 0.05.

    Time step: with 10 B-subcycles, dt = 0.003 keeps the explicit-midpoint
    subcycle stable at the grid scale in the n = 0.2 background, where the
    fastest whistler (k = 1/dx) has omega = k^2/(2n) + k sqrt(1/n + k^2/(4n^2))
    ~ 320 Omega_i, so omega * h ~ 0.1 with h = dt/10; it also satisfies the
    whistler CFL of Sec. II.A with the local ion inertial length.
    """
    L = 0.5
    ti = 0.5 / 1.2
    te = 0.2 * ti
    cfg = Config(name=f"2d-double-harris-{nx}x{ny}-ppc{ppc:g}", ndim=2, nx=nx, ny=ny,
                 nz=1, dx=0.125, dy=0.125, dz=1.0, dt=0.003, nsub=10, shape=SHAPE_QS,
                 te=te, eta=1e-3, steps=steps)
    Lx, Ly = nx * cfg.dx, ny * cfg.dy
    rng = np.random.Generator(np.random.PCG64(seed))
    n_total = int(round(ppc * cfg.ncell))
    # Integrated density: each sheet carries 2 L Lx, the background 0.2 Lx Ly.
    sheet = 2.0 * L * Lx
    back = 0.2 * Lx * Ly
    n_sheet = int(round(n_total * sheet / (2 * sheet + back)))
    n_back = n_total - 2 * n_sheet
    w = (2 * sheet + back) / n_total
    vth = math.sqrt(ti)
    drift = 2.0 * ti / L

    xs, ys, us = [], [], []
    # background: uniform, at rest
    xs.append(rng.uniform(0.0, Lx, n_back))
    ys.append(rng.uniform(0.0, Ly, n_back))
    us.append(rng.normal(0.0, vth, (3, n_back)))
    # sheets: y - y0 = L atanh(2U - 1) samples sech^2((y - y0)/L)
    for y0, sign in ((0.25 * Ly, -1.0), (0.75 * Ly, 1.0)):
        uu = rng.uniform(0.0, 1.0, n_sheet)
        uu = np.clip(uu, 1e-15, 1.0 - 1e-15)
        xs.append(rng.uniform(0.0, Lx, n_sheet))
        ys.append(y0 + L * np.arctanh(2.0 * uu - 1.0))
        v = rng.normal(0.0, vth, (3, n_sheet))
        v[2] += sign * drift
        us.append(v)
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    u = np.concatenate(us, axis=1)
    i, ox = _position_to_cell(x, cfg.dx, nx)
    j, oy = _position_to_cell(y, cfg.dy, ny)
    parts = _particles(cfg, i, j, 0 * i, ox, oy, None, u[0], u[1], u[2],
                       np.full(n_total, w), order=rng.permutation(n_total))

    xc, yc, _ = cell_centres(cfg)
    B = field_zeros(cfg)
    bx = np.tanh((yc - 0.25 * Ly) / L) - np.tanh((yc - 0.75 * Ly) / L) - 1.0
    kx, ky = 2.0 * math.pi / Lx, 2.0 * math.pi / Ly
    # dB = z x grad psi = (-dpsi/dy, dpsi/dx), psi = A cos(kx x) sin(ky y)
    dbx = -ky * np.cos(kx * xc) * np.cos(ky * yc)
    dby = -kx * np.sin(kx * xc) * np.sin(ky * yc)
    scale = 0.05 / np.max(np.sqrt(dbx * dbx + dby * dby))
    B[0] = _f32(bx + scale * dbx)
    B[1] = _f32(scale * dby)
    return cfg, parts, B


def beam_3d(seed: int = 3, n: int = 128, core_ppc: int = 56, beam_ppc: int = 8,
            steps: int = 500):
    """3D periodic box with a core plus a field-aligned ion beam.

    128^3 cells of 1 d_i, B0 = x; core n = 0.95 drifting -0.526 v_A along x
    (zero net current), beam n = 0.05 drifting +10 v_A, both with per-component
    spread 1 v_A; T_e = 1, eta = 1e-4, dt = 0.05, 4 B-subcycles.
    """
    cfg = Config(name=f"3d-beam-{n}^3-ppc{core_ppc + beam_ppc}", ndim=3, nx=n, ny=n,
                 nz=n, dx=1.0, dy=1.0, dz=1.0, dt=0.05, nsub=4, shape=SHAPE_QS,
                 te=1.0, eta=1e-4, steps=steps)
    rng = np.random.Generator(np.random.PCG64(seed))
    ppc = core_ppc + beam_ppc
    nc = cfg.ncell
    total = nc * ppc
    cell = np.repeat(np.arange(nc, dtype=np.int64), ppc)
    slot = np.tile(np.arange(ppc), nc)
    is_beam = slot >= core_ppc
    i = cell % n
    j = (cell // n) % n
    k = cell // (n * n)
    ox = _offsets(rng.uniform(-1.0, 1.0, total))
    oy = _offsets(rng.uniform(-1.0, 1.0, total))
    oz = _offsets(rng.uniform(-1.0, 1.0, total))
    u = rng.normal(0.0, 1.0, (3, total)).astype(np.float32)
    core_drift = -0.05 * 10.0 / 0.95
    u[0] += np.where(is_beam, 10.0, core_drift).astype(np.float32)
    w = np.where(is_beam, 0.05 / beam_ppc, 0.95 / core_ppc)
    parts = _particles(cfg, i, j, k, ox, oy, oz, u[0], u[1], u[2], w,
                       order=rng.permutation(total))
    B = field_zeros(cfg)
    B[0] = 1.0
    return cfg, parts, B


def random_box(seed: int, cfg: Config, ppc: float, vmax_cells: float = 0.9,
               b_amp: float = 0.1, sorted_cells: bool = False):
    """Random particles and a random smooth-ish field on an arbitrary grid.

    Used for parity cases: odd, non-square grids and ragged particle counts.
    Speeds are bounded so a particle moves at most vmax_cells cells per step
    along each axis.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(round(ppc * cfg.ncell))
    cell = rng.integers(0, cfg.ncell, n)
    if sorted_cells:
        cell = np.sort(cell)
    i = cell % cfg.nx
    j = (cell // cfg.nx) % cfg.ny
    k = cell // (cfg.nx * cfg.ny)
    ox = _offsets(rng.uniform(-1.0, 1.0, n))
    oy = _offsets(rng.uniform(-1.0, 1.0, n))
    oz = _offsets(rng.uniform(-1.0, 1.0, n)) if cfg.ndim == 3 else None
    lim = [vmax_cells * h / cfg.dt for h in (cfg.dx, cfg.dy, cfg.dz)]
    u = np.stack([rng.uniform(-lim[a], lim[a], n) for a in range(3)])
    if cfg.ndim == 2:
        u[2] = rng.uniform(-1.0, 1.0, n)
    w = rng.uniform(0.5, 1.5, n) * cfg.dx * cfg.dy * cfg.dz / max(ppc, 1e-9)
    parts = _particles(cfg, i, j, k, ox, oy, oz, u[0], u[1], u[2], w)
    B = field_zeros(cfg)
    B[0] = 1.0
    B += _f32(b_amp * rng.uniform(-1.0, 1.0, (3, cfg.ncell)))
    return cfg, parts, B


def random_field(seed: int, cfg: Config, amp: float = 1.0, offset=(0.0, 0.0, 0.0)):
    rng = np.random.Generator(np.random.PCG64(seed))
    F = _f32(amp * rng.uniform(-1.0, 1.0, (3, cfg.ncell)))
    for a in range(3):
        F[a] += np.float32(offset[a])
    return F


def random_density(seed: int, cfg: Config, lo: float = 0.5, hi: float = 1.5):
    rng = np.random.Generator(np.random.PCG64(seed))
    return _f32(rng.uniform(lo, hi, cfg.ncell))


def quiet_wave(cfg: Config, ppc: int, mode: int, amp: float, du_coeff: float,
               polarization: int, vth: float = 0.0, seed: int = 7):
    """Lattice-loaded uniform plasma carrying one circularly polarised mode.

    dB = amp (0, cos(k x), p sin(k x)) on the grid (p = +-1 is the
    polarization) and ion velocity du = du_coeff * dB evaluated at each
    particle position; k = 2 pi mode / Lx.  Offsets along x sit on a regular
    lattice (ppc per cell), so the initial density is uniform.  The caller
    chooses du_coeff (for an eigenmode it comes from linear theory).
    """
    nc = cfg.ncell
    cell = np.repeat(np.arange(nc, dtype=np.int64), ppc)
    slot = np.tile(np.arange(ppc), nc)
    i = cell % cfg.nx
    j = (cell // cfg.nx) % cfg.ny
    k = cell // (cfg.nx * cfg.ny)
    ox = _offsets(-1.0 + (2.0 * slot + 1.0) / ppc)
    oy = np.zeros(cell.size, np.float32)
    oz = np.zeros(cell.size, np.float32) if cfg.ndim == 3 else None
    Lx = cfg.nx * cfg.dx
    kk = 2.0 * math.pi * mode / Lx
    xp = (i + 0.5 + 0.5 * ox.astype(np.float64)) * cfg.dx
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.normal(0.0, vth, (3, cell.size)) if vth > 0 else np.zeros((3, cell.size))
    u[1] += du_coeff * amp * np.cos(kk * xp)
    u[2] += du_coeff * amp * polarization * np.sin(kk * xp)
    w = np.full(cell.size, cfg.dx * cfg.dy * cfg.dz / ppc)
    parts = _particles(cfg, i, j, k, ox, oy, oz, u[0], u[1], u[2], w)
    x, _, _ = cell_centres(cfg)
    B = field_zeros(cfg)
    B[0] = 1.0
    B[1] = _f32(amp * np.cos(kk * x))
    B[2] = _f32(amp * polarization * np.sin(kk * x))
    return parts, B


WORKLOADS = {
    "small": periodic_alfven,
    "harris": harris_double,
    "beam3d": beam_3d,
}
