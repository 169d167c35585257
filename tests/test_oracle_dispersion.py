"""Whole-step pin of the oracle: parallel ion-cyclotron / whistler dispersion.

Linearising the hybrid equations of Sec. II.A (Ohm's law eq:ohm, Ampere,
Faraday) together with the ion equation of motion for cold ions in a uniform
plasma (n = 1, B0 = xhat, eta = 0, q/m = 1) gives, for a circularly polarised
transverse mode dB = A(0, cos(kx - wt), p sin(kx - wt)) written as
z_B ~ exp(i Omega t) with Omega = p w (derived by hand):

    (Omega + k_e^2)(Omega - 1 + S^2) = k_e^2 S^2,   du = -(p k_e S / (Omega - 1 + S^2)) dB

where k_e = sin(k dx)/dx replaces k in the centred curl and S = S(k) is the
Fourier factor of the particle shape averaged over the particles' offsets:
the deposited current is S times the ion velocity and the gathered field is S
times the grid field.  With S = 1 this is the textbook cold relation
w = -p k^2/2 + k sqrt(1 + k^2/4) (p = +1 ion-cyclotron, p = -1 whistler).

For the QS shape on a grid with one cell along y (both y-neighbours fold onto
the centre, dy = 0) the weights along x are (5 - xi^2)/6 and (1 +- xi)^2/12
(eq:quad), so S = < W0 cos(k dx xi/2) + W+ cos(k dx (1 - xi/2))
+ W- cos(k dx (1 + xi/2)) > over the lattice offsets xi.

The eigenmode is loaded on a quiet (lattice) start with the theory's du; the
measured rotation rate of the mode's complex amplitude must match Omega within
0.3% (the time discretisation error is O((w dt)^2) ~ 1e-5 and the fit over
one period adds ~1e-4).  Dropping the shape factor already moves w by 1-3%;
flipping the Hall term swaps the branches (20-60% apart).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W

PPC = 16


def _shape_factor(k, dx, ppc):
    xi = -1 + (2 * np.arange(ppc) + 1) / ppc
    w0 = (5 - xi**2) / 6
    wp = (1 + xi) ** 2 / 12
    wm = (1 - xi) ** 2 / 12
    th = k * dx
    return float(np.mean(w0 * np.cos(th * xi / 2) + wp * np.cos(th * (1 - xi / 2))
                         + wm * np.cos(th * (1 + xi / 2))))


def _theory(ke, p, S):
    """Root Omega (sign p) of Omega^2 + (k^2 - d) Omega - k^2 = 0, d = 1 - S^2."""
    d = 1 - S * S
    b = ke * ke - d
    om = (-b + p * math.sqrt(b * b + 4 * ke * ke)) / 2
    return om


def _run(p, mode, periods=1.0):
    cfg = W.Config(name="disp", ndim=2, nx=32, ny=1, nz=1, dx=0.5, dy=0.5, dz=1.0,
                   dt=0.01, nsub=4, shape=W.SHAPE_QS, te=0.0, eta=0.0, n_floor=0.05)
    k = 2 * math.pi * mode / (cfg.nx * cfg.dx)
    ke = math.sin(k * cfg.dx) / cfg.dx
    S = _shape_factor(k, cfg.dx, PPC)
    Om = _theory(ke, p, S)
    du = -(p * ke * S) / (Om - 1 + S * S)
    amp = 1e-3
    parts, B = W.quiet_wave(cfg, PPC, mode, amp, du_coeff=du, polarization=p)
    sim = O.OracleSim(cfg, parts, B)
    x, _, _ = W.cell_centres(cfg)
    a = np.stack([np.zeros(cfg.ncell), np.cos(k * x), p * np.sin(k * x)])
    b = np.stack([a[0], a[2], -a[1]])
    nsteps = int(periods * 2 * math.pi / abs(Om) / cfg.dt)
    ts, ph = [], []
    for s in range(nsteps):
        sim.step()
        if s % 10 == 9:
            dB = sim.B.copy()
            dB[0] -= 1.0
            z = (dB * a).sum() / (a * a).sum() + 1j * (dB * b).sum() / (b * b).sum()
            ts.append((s + 1) * cfg.dt)
            ph.append(np.angle(z))
    slope = np.polyfit(np.array(ts), np.unwrap(np.array(ph)), 1)[0]
    # z_B = alpha + i beta rotates as exp(i Omega t)
    return slope, Om, ke


@pytest.mark.parametrize("p,mode", [(1, 1), (-1, 1), (1, 2), (-1, 2), (-1, 3)])
def test_cold_dispersion(p, mode):
    measured, Om, ke = _run(p, mode)
    assert measured == pytest.approx(Om, rel=3e-3), (measured, Om)
    # and the two branches are far apart, so the check discriminates
    other = _theory(ke, -p, 1.0)
    assert abs(abs(other) / abs(Om) - 1) > 0.2
