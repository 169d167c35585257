"""Pins of the oracle's Boris push and move (Sec. II.B, eq:vadv) to closed forms.

None of these tests re-types the oracle's Boris arithmetic: each checks a
consequence of eq:vadv that holds exactly (to rounding) for the standard Boris
split -- the implicit-midpoint identities, the exact rotation angle
2 atan(Omega dt / 2), the exact E x B drift of the gyration centre, the exact
parallel kick and free streaming, and the position update x += v dt.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W


def _cfg(**kw):
    base = dict(name="t", ndim=2, nx=64, ny=48, nz=1, dx=0.5, dy=0.25, dz=1.0,
                dt=0.05, nsub=1, shape=W.SHAPE_QS)
    base.update(kw)
    return W.Config(**base)


def _uniform_fields(cfg, E, B):
    Eg = np.zeros((3, cfg.ncell))
    Bg = np.zeros((3, cfg.ncell))
    for a in range(3):
        Eg[a] = E[a]
        Bg[a] = B[a]
    return Eg, Bg


def _one(cfg, cell, ox, oy, u, oz=None):
    p = {"cell": np.array([cell], np.int32), "ox": np.array([ox], float),
         "oy": np.array([oy], float), "ux": np.array([u[0]], float),
         "uy": np.array([u[1]], float), "uz": np.array([u[2]], float),
         "w": np.array([1.0])}
    if cfg.ndim == 3:
        p["oz"] = np.array([0.0 if oz is None else oz])
    return p


def _position(cfg, p):
    c = p["cell"].astype(np.int64)
    i = c % cfg.nx
    j = (c // cfg.nx) % cfg.ny
    return np.stack([(i + 0.5 + 0.5 * p["ox"]) * cfg.dx, (j + 0.5 + 0.5 * p["oy"]) * cfg.dy])


def test_midpoint_identities_random():
    """m dv = q dt (E + vbar x B) and d(v^2/2) = (q/m) dt E.vbar, vbar = mean velocity."""
    rng = np.random.Generator(np.random.PCG64(11))
    for qm, dt in ((1.0, 0.05), (2.5, 0.3), (-1.0, 0.01)):
        a = 0.5 * qm * dt
        for _ in range(200):
            E = rng.normal(0, 1, 3)
            B = rng.normal(0, 3, 3)
            v0 = rng.normal(0, 2, 3)
            v1 = O.boris(a, E, B, v0)
            vbar = 0.5 * (v0 + v1)
            lhs = v1 - v0
            rhs = qm * dt * (E + np.cross(vbar, B))
            assert np.allclose(lhs, rhs, rtol=0, atol=1e-12 * (1 + np.abs(rhs).max()))
            dK = 0.5 * (v1 @ v1 - v0 @ v0)
            assert abs(dK - qm * dt * (E @ vbar)) < 1e-12 * (1 + abs(dK))


def test_gyration_angle_and_sense():
    """Pure B: |v| is kept and v turns by theta = 2 atan(|q/m| B dt / 2), clockwise
    about B for a positive charge."""
    for Bmag, dt in ((1.0, 0.01), (1.0, 0.5), (3.0, 0.7)):
        a = 0.5 * dt
        v = np.array([1.0, 0.0, 0.3])
        theta = 2.0 * math.atan(Bmag * dt / 2.0)
        for n in range(1, 40):
            v = O.boris(a, np.zeros(3), np.array([0.0, 0.0, Bmag]), v)
            expect = np.array([math.cos(n * theta), -math.sin(n * theta), 0.3])
            assert np.allclose(v, expect, atol=1e-12), (n, v, expect)


def test_exb_drift_exact():
    """E perpendicular to B: v - E x B / B^2 rotates rigidly by theta per step."""
    E = np.array([0.0, 0.4, 0.0])
    B = np.array([0.0, 0.0, 2.0])
    dt = 0.2
    vd = np.cross(E, B) / (B @ B)
    theta = 2.0 * math.atan(2.0 * dt / 2.0)
    v0 = np.array([0.3, -0.1, 0.0])
    w0 = v0 - vd
    v = v0.copy()
    for n in range(1, 50):
        v = O.boris(0.5 * dt, E, B, v)
        c, s = math.cos(n * theta), math.sin(n * theta)
        w = np.array([c * w0[0] + s * w0[1], -s * w0[0] + c * w0[1], 0.0])
        assert np.allclose(v, vd + w, atol=1e-12)


def test_parallel_kick_exact():
    E = np.array([0.0, 0.0, 0.7])
    B = np.array([0.0, 0.0, 1.3])
    v = np.array([0.2, 0.1, -0.4])
    dt = 0.1
    vperp = np.hypot(v[0], v[1])
    for n in range(1, 20):
        v = O.boris(0.5 * dt, E, B, v)
        assert abs(v[2] - (-0.4 + n * 0.7 * dt)) < 1e-13
        assert abs(np.hypot(v[0], v[1]) - vperp) < 1e-13


def test_gyro_orbit_circle_through_push():
    """Full push in a uniform B on the grid: positions x^n lie on a circle of
    radius |v_perp| dt / (2 sin(theta/2)); the interpolated field is exact for
    a uniform field, so this also checks gather + move together."""
    cfg = _cfg(nx=64, ny=96, dx=0.5, dy=0.25, dt=0.2)
    Bz = 1.5
    Eg, Bg = _uniform_fields(cfg, (0, 0, 0), (0, 0, Bz))
    vperp = 0.8
    p = _one(cfg, 40 * cfg.nx + 30, 0.1, -0.3, (vperp, 0.0, 0.2))
    theta = 2 * math.atan(Bz * cfg.dt / 2)
    R = vperp * cfg.dt / (2 * math.sin(theta / 2))
    pts = []
    for _ in range(60):
        O.push(cfg, p, Eg, Bg)
        pts.append(_position(cfg, p)[:, 0])
    pts = np.array(pts)
    # centre from the first three points
    (x1, y1), (x2, y2), (x3, y3) = pts[:3]
    A = np.array([[x2 - x1, y2 - y1], [x3 - x1, y3 - y1]])
    b = 0.5 * np.array([x2**2 - x1**2 + y2**2 - y1**2, x3**2 - x1**2 + y3**2 - y1**2])
    cx, cy = np.linalg.solve(A, b)
    r = np.hypot(pts[:, 0] - cx, pts[:, 1] - cy)
    assert np.allclose(r, R, rtol=1e-10), (r[:5], R)


@pytest.mark.parametrize("ndim", [2, 3])
def test_free_streaming_positions(ndim):
    """E = B = 0: v is unchanged and x^{n+1} = x^n + v dt (mod L), including
    exact landings on a face and multi-cell moves (which are counted)."""
    if ndim == 2:
        cfg = _cfg(nx=7, ny=5, dx=0.5, dy=0.25, dt=0.1)
    else:
        cfg = _cfg(ndim=3, nx=5, ny=4, nz=6, dx=0.5, dy=0.25, dz=0.75, dt=0.1)
    rng = np.random.Generator(np.random.PCG64(5))
    n = 4000
    c = rng.integers(0, cfg.ncell, n)
    h = np.array([cfg.dx, cfg.dy, cfg.dz])
    p = {"cell": c.astype(np.int32), "ox": rng.uniform(-1, 1, n), "oy": rng.uniform(-1, 1, n),
         "ux": rng.uniform(-0.95, 0.95, n) * cfg.dx / cfg.dt,
         "uy": rng.uniform(-0.95, 0.95, n) * cfg.dy / cfg.dt,
         "uz": rng.uniform(-0.95, 0.95, n) * cfg.dz / cfg.dt, "w": np.ones(n)}
    if ndim == 3:
        p["oz"] = rng.uniform(-1, 1, n)
    # exact face landings: offset 0.5 moving +0.5 half-cells -> next cell at -1
    p["ox"][:50] = 0.5
    p["ux"][:50] = 0.25 * cfg.dx / cfg.dt
    # multi-cell movers (3 cells in x)
    p["ux"][50:60] = 3.0 * cfg.dx / cfg.dt
    L = np.array([cfg.nx * cfg.dx, cfg.ny * cfg.dy, cfg.nz * cfg.dz])

    def pos(q):
        cc = q["cell"].astype(np.int64)
        ijk = [cc % cfg.nx, (cc // cfg.nx) % cfg.ny, cc // (cfg.nx * cfg.ny)]
        offs = [q["ox"], q["oy"], q.get("oz", np.zeros(n))]
        return np.stack([(ijk[a] + 0.5 + 0.5 * offs[a]) * h[a] for a in range(3)])

    x0 = pos(p)
    v0 = np.stack([p["ux"], p["uy"], p["uz"]]).copy()
    Eg, Bg = _uniform_fields(cfg, (0, 0, 0), (0, 0, 0))
    _, st = O.push(cfg, p, Eg, Bg)
    x1 = pos(p)
    assert np.array_equal(np.stack([p["ux"], p["uy"], p["uz"]]), v0)
    for a in range(ndim):
        d = (x1[a] - x0[a] - v0[a] * cfg.dt) / L[a]
        d -= np.round(d)
        assert np.abs(d).max() < 1e-12
    assert np.all(p["ox"] >= -1) and np.all(p["ox"] < 1)
    assert np.all(p["ox"][:50] == -1.0)
    i0 = (c[:50] % cfg.nx + 1) % cfg.nx
    assert np.array_equal(p["cell"][:50].astype(np.int64) % cfg.nx, i0)
    assert st.moved_gt1 == 10
    assert st.nonfinite == 0


def test_nonfinite_is_counted_and_kept_in_place():
    """A particle whose move is non-finite or runaway (1e6 half-cells or more)
    along any axis stays where it was -- cell and every offset -- and is
    counted once; its neighbours in the store move normally."""
    cfg = _cfg()
    Eg, Bg = _uniform_fields(cfg, (0, 0, 0), (0, 0, 0))
    p = {"cell": np.array([17, 40, 93], np.int32), "ox": np.array([0.2, -0.3, 0.5]),
         "oy": np.array([-0.1, 0.4, 0.0]), "ux": np.array([np.nan, 1.0e9, 0.5]),
         "uy": np.array([0.3, 0.2, 0.0]), "uz": np.zeros(3), "w": np.ones(3)}
    _, st = O.push(cfg, p, Eg, Bg)
    assert st.nonfinite == 2 and st.moved_gt1 == 0
    assert list(p["cell"][:2]) == [17, 40]
    assert list(p["ox"][:2]) == [0.2, -0.3] and list(p["oy"][:2]) == [-0.1, 0.4]
    # the third: 2 v dt / dx = 0.1 half-cells along x
    assert p["cell"][2] == 93 and p["ox"][2] == pytest.approx(0.6, abs=1e-15)
    # the deposit's back step of the NaN particle is kept at x as well
    n, J = O.deposit(cfg, {k: v[:1] for k, v in p.items()}, 0.5 * cfg.dt)
    ref, _ = O.deposit(cfg, {**{k: v[:1] for k, v in p.items()}, "ux": np.zeros(1),
                             "uy": np.zeros(1)}, 0.0)
    assert np.array_equal(n, ref)


def _many(cfg, u, w):
    n = len(w)
    p = {"cell": np.arange(n, dtype=np.int32) * 7 % cfg.ncell, "ox": np.zeros(n),
         "oy": np.zeros(n), "ux": u[:, 0].copy(), "uy": u[:, 1].copy(),
         "uz": u[:, 2].copy(), "w": np.asarray(w, float)}
    if cfg.ndim == 3:
        p["oz"] = np.zeros(n)
    return p


@pytest.mark.parametrize("qs,ms", [(1.0, 1.0), (2.0, 4.0), (-1.0, 0.5)])
def test_push_diagnostics_in_uniform_b(qs, ms):
    """The push's diagnostics K = sum 1/2 m w v^{n-1/2}.v^{n+1/2} and
    P = sum m w vbar against closed forms of a pure gyration (E = 0, B = B zhat):
    v_perp turns by theta = 2 atan(|q|B dt/(2m)) and keeps its length, v_par is
    kept, so v^{n-1/2}.v^{n+1/2} = v_perp^2 cos(theta) + v_par^2 and the mean
    velocity is v_perp cos(theta/2) along the direction half-way round, plus
    v_par."""
    cfg = _cfg(qs=qs, ms=ms, dt=0.1)
    Bz = 2.5
    E, B = _uniform_fields(cfg, (0, 0, 0), (0, 0, Bz))
    rng = np.random.Generator(np.random.PCG64(5))
    u = rng.normal(0, 1.5, (40, 3))
    w = rng.uniform(0.2, 2.0, 40)
    p = _many(cfg, u, w)
    diag, _ = O.push(cfg, p, E, B)
    theta = 2 * math.atan(abs(qs) * Bz * cfg.dt / (2 * ms))
    vperp2 = u[:, 0] ** 2 + u[:, 1] ** 2
    K = 0.5 * ms * np.sum(w * (vperp2 * math.cos(theta) + u[:, 2] ** 2))
    # rotation sense: clockwise about B for q > 0 (angle -theta/2 half-way)
    phi = -math.copysign(theta, qs) / 2
    c, s = math.cos(phi), math.sin(phi)
    vbx = math.cos(theta / 2) * (c * u[:, 0] - s * u[:, 1])
    vby = math.cos(theta / 2) * (s * u[:, 0] + c * u[:, 1])
    P = ms * np.array([np.sum(w * vbx), np.sum(w * vby), np.sum(w * u[:, 2])])
    assert diag[0] == pytest.approx(K, rel=1e-12)
    assert np.allclose(diag[1:], P, rtol=0, atol=1e-12 * np.abs(P).max())


def test_push_diagnostics_under_uniform_e():
    """B = 0: each velocity gets the exact kick (q/m) E dt, so
    K = sum 1/2 m w v.(v + (q/m) E dt) and P = sum m w (v + (q/m) E dt / 2),
    summed with the particle weights."""
    qs, ms = 1.5, 3.0
    cfg = _cfg(qs=qs, ms=ms, dt=0.2)
    Ev = np.array([0.3, -1.1, 0.45])
    E, B = _uniform_fields(cfg, Ev, (0, 0, 0))
    rng = np.random.Generator(np.random.PCG64(6))
    u = rng.normal(0, 1.0, (25, 3))
    w = rng.uniform(0.5, 1.5, 25)
    p = _many(cfg, u, w)
    diag, _ = O.push(cfg, p, E, B)
    kick = qs / ms * cfg.dt * Ev
    K = 0.5 * ms * np.sum(w * np.sum(u * (u + kick), axis=1))
    P = ms * (w @ (u + 0.5 * kick))
    assert diag[0] == pytest.approx(K, rel=1e-12)
    assert np.allclose(diag[1:], P, rtol=1e-12)
