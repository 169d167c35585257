"""The C oracle against the independent NumPy implementation of
tests/bruteforce_step.py: two whole steps on about 300 ions on small odd
grids, 2D and 3D, QS and NGP, including axes of one and two cells (aliased
stencil points).  They agree to 1e-12 (relative, per array), cell indices and
the sort order exactly.  Any slip in one of them -- an interpolant
coefficient, the 2D fold, a sign of the Boris rotation, the mid-point of the
deposit, the extrapolation, a term of Ohm's law or an energy -- shows up here,
because the two share no code and compute the gather, the push and the move
by different routes."""
import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W
from tests.bruteforce_step import BruteSim


def _cfg(ndim, nx, ny, nz, shape, **kw):
    base = dict(name="bf", ndim=ndim, nx=nx, ny=ny, nz=nz, dx=0.5, dy=0.4,
                dz=(0.7 if ndim == 3 else 1.0), dt=0.05, nsub=3, shape=shape, te=0.3,
                eta=0.02, n_floor=0.05)
    base.update(kw)
    return W.Config(**base)


CASES = [
    ("2d-qs-6x5", _cfg(2, 6, 5, 1, W.SHAPE_QS), 10.0),
    ("2d-ngp-6x5", _cfg(2, 6, 5, 1, W.SHAPE_NGP), 10.0),
    ("3d-qs-4x3x5", _cfg(3, 4, 3, 5, W.SHAPE_QS), 5.0),
    ("3d-ngp-4x3x5", _cfg(3, 4, 3, 5, W.SHAPE_NGP), 5.0),
    ("2d-qs-2x7", _cfg(2, 2, 7, 1, W.SHAPE_QS), 20.0),
    ("2d-qs-1x5-gamma", _cfg(2, 1, 5, 1, W.SHAPE_QS, gamma_e=5.0 / 3.0), 60.0),
    ("2d-qs-6x5-hyper", _cfg(2, 6, 5, 1, W.SHAPE_QS, eta_h=3e-3), 10.0),
    ("2d-qs-6x5-energy", _cfg(2, 6, 5, 1, W.SHAPE_QS, gamma_e=5.0 / 3.0, energy_eq=1,
                              kappa0=0.05, eta_h=1e-3), 10.0),
    ("3d-qs-4x3x5-energy", _cfg(3, 4, 3, 5, W.SHAPE_QS, gamma_e=5.0 / 3.0, energy_eq=1,
                                kappa0=0.05, eta_h=1e-3), 5.0),
    ("2d-qs-2x7-energy", _cfg(2, 2, 7, 1, W.SHAPE_QS, gamma_e=2.0, energy_eq=1,
                              kappa0=0.02), 20.0),
]


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name,cfg,ppc", CASES)
def test_two_steps_match(name, cfg, ppc):
    _, parts, B = W.random_box(17, cfg, ppc, vmax_cells=0.9, b_amp=0.2)
    assert 250 <= parts["cell"].size <= 350
    o = O.OracleSim(cfg, parts, B)
    b = BruteSim(cfg, parts)
    b.init_fields(B)
    assert _rel(b.E, o.E) < 1e-12
    assert _rel(b.n_prev, o.n_prev) < 1e-12 and _rel(b.J_prev, o.J_prev) < 1e-12
    for step in range(2):
        o.step()
        b.step()
        pb = b.particles()
        assert np.array_equal(pb["cell"], o.p["cell"]), (name, step)
        for k in ("ox", "oy", "oz", "ux", "uy", "uz", "w"):
            if k in pb:
                assert np.abs(pb[k] - o.p[k]).max() < 1e-12, (name, step, k)
        for got, ref, what in ((b.n_prev, o.n_prev, "n"), (b.J_prev, o.J_prev, "J"),
                               (b.B, o.B, "B"), (b.E, o.E, "E")):
            assert _rel(got, ref) < 1e-12, (name, step, what, _rel(got, ref))
        assert b.K == pytest.approx(o.push_diag[0], rel=1e-12)
        assert np.allclose(b.P, o.push_diag[1:], rtol=1e-12, atol=1e-12 * np.abs(b.P).max())
        assert np.allclose(b.field_diag, o.field_diag, rtol=1e-12, atol=1e-14)
        if cfg.energy_eq:
            assert _rel(b.pe, o.pe) < 1e-12, (name, step)
