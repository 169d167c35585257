"""Pins of the oracle's open boundaries (Sec. II.C) against what does not
depend on them: the periodic solver where the open rules must agree with it
(x-uniform fields; the B0/B1 split with a uniform B0), exact steady states,
the buffer's closed-form eta_h profile, the injection's count rule and the
closed-form moments of the flux-weighted drifting Maxwellian, and the
absorption count."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W


def _cfg(**kw):
    base = dict(name="open", ndim=2, nx=14, ny=9, nz=1, dx=0.5, dy=0.4, dz=1.0, dt=0.02,
                nsub=4, te=0.09, eta=2e-3, open_x=1)
    base.update(kw)
    return W.Config(**base)


def _y_only(cfg, rng):
    """Fields that vary along y only (the same in every column)."""
    j = np.arange(cfg.ncell) // cfg.nx
    ky = 2 * math.pi / (cfg.ny * cfg.dy)
    y = (j + 0.5) * cfg.dy
    B1 = np.stack([0.1 * np.sin(ky * y), 0.05 * np.cos(2 * ky * y), 0.2 * np.cos(ky * y + 0.3)])
    n = 1.0 + 0.2 * np.sin(ky * y + 1.0)
    Ji = np.stack([0.05 * np.cos(ky * y), 0.1 + 0 * y, 0.02 * np.sin(ky * y)])
    return B1, n, Ji


def test_ghost_fill():
    cfg = _cfg()
    F = np.arange(3 * cfg.ncell, dtype=float).reshape(3, -1)
    G = O.open_fill(cfg, F).reshape(3, cfg.ny, cfg.nx)
    F = F.reshape(3, cfg.ny, cfg.nx)
    assert np.array_equal(G[:, :, 0], F[:, :, 1]) and np.array_equal(G[:, :, -1], F[:, :, -2])
    assert np.array_equal(G[:, :, 1:-1], F[:, :, 1:-1])


@pytest.mark.parametrize("eta_h", [0.0, 1e-3])
def test_x_uniform_fields_agree_with_the_periodic_solver(eta_h):
    """With no variation along x the open rules (no normal gradients in the
    ghost columns, B1 and moments copied) change nothing: the open field
    advance equals the periodic one, ghost columns included."""
    cfg = _cfg(eta_h=eta_h)
    rng = np.random.default_rng(1)
    B1, n, Ji = _y_only(cfg, rng)
    B0 = np.zeros_like(B1)
    B0[0] = 1.0
    per = cfg.replace(open_x=0)
    rB, rE, rd, _ = O.field_advance(per, B0 + B1, n, Ji, n, Ji, mode=0)
    oB1, oE, oBt, od, _ = O.open_field_advance(cfg, B0, B1, n, Ji, n, Ji, mode=0)
    assert np.allclose(oBt, rB, rtol=0, atol=1e-13)
    assert np.allclose(oE, rE, rtol=0, atol=1e-12)


def test_b0_split_is_exact_with_a_uniform_b0():
    """Periodic box, B = B0 + B1 with uniform B0: advancing B1 with J = curl
    B1 gives the periodic solver's B (curl B0 = 0 exactly)."""
    cfg = _cfg(open_x=0)
    rng = np.random.default_rng(2)
    B1 = rng.normal(scale=0.1, size=(3, cfg.ncell))
    n = rng.uniform(0.5, 1.5, cfg.ncell)
    Ji = rng.normal(scale=0.2, size=(3, cfg.ncell))
    B0 = np.zeros_like(B1)
    B0[:] = np.array([[0.4], [1.0], [-0.3]])
    rB, rE, rd, _ = O.field_advance(cfg, B0 + B1, n, Ji, n, Ji, mode=0)
    oB1, oE, oBt, od, _ = O.open_field_advance(cfg, B0, B1, n, Ji, n, Ji, mode=0)
    assert np.allclose(oBt, rB, rtol=0, atol=1e-13)
    assert np.allclose(oE, rE, rtol=0, atol=1e-12)
    assert np.allclose(od, rd, rtol=1e-12)


def test_uniform_flow_is_steady_at_the_open_boundaries():
    """A uniform plasma drifting across a uniform B0 with B1 = 0: E = -u x B0
    everywhere, ghost columns included, so B1 stays exactly zero."""
    cfg = _cfg(te=0.09, eta=0.0)
    B0 = np.zeros((3, cfg.ncell))
    B0[1] = 1.0
    B1 = np.zeros_like(B0)
    n = np.ones(cfg.ncell)
    u = np.array([0.5, 0.0, 0.1])
    Ji = np.tile(u[:, None], (1, cfg.ncell))
    oB1, oE, oBt, od, _ = O.open_field_advance(cfg, B0, B1, n, Ji, n, Ji, mode=0)
    assert np.abs(oB1).max() == 0.0
    want = -np.cross(u, [0.0, 1.0, 0.0])
    assert np.allclose(oE, want[:, None], rtol=0, atol=1e-15)


def test_buffer_raises_eta_h_linearly():
    """With a y-only J the hyper-resistive field is eta_h(i) lap_y J in every
    column: eta_h(i) = eta_h + eta_h_buffer (1 - d/w), d the column's
    distance from the outermost interior column (ghosts take d = 0)."""
    w = 3
    cfg = _cfg(eta=0.0, te=0.0, eta_h=1e-3, buffer_cells=w, eta_h_buffer=0.02)
    rng = np.random.default_rng(3)
    B1, n, Ji = _y_only(cfg, rng)
    B0 = np.zeros_like(B1)
    Ji = np.zeros_like(Ji)
    E = O.open_ohm(cfg, B0, B1, n, Ji).reshape(3, cfg.ny, cfg.nx)
    E0 = O.open_ohm(cfg.replace(eta_h=0.0, eta_h_buffer=0.0), B0, B1, n, Ji).reshape(
        3, cfg.ny, cfg.nx)
    J = O.curl(cfg.replace(open_x=0), B1).reshape(3, cfg.ny, cfg.nx)
    lapJ = (np.roll(J, -1, 1) - 2 * J + np.roll(J, 1, 1)) / cfg.dy ** 2
    for i in range(cfg.nx):
        d = max(min(i, cfg.nx - 1 - i) - 1, 0)
        eh = 1e-3 + (0.02 * (1 - d / w) if d < w else 0.0)
        assert np.allclose(E[:, :, i] - E0[:, :, i], -eh * lapJ[:, :, i], rtol=1e-10, atol=1e-14), i


def test_absorption_takes_the_ghost_columns():
    cfg = _cfg()
    rng = np.random.default_rng(4)
    cell = rng.integers(0, cfg.ncell, 500).astype(np.int32)
    ghosts = np.isin(cell % cfg.nx, [0, cfg.nx - 1])
    parts = {"cell": cell.copy()}
    assert O.open_absorb(cfg, parts) == int(ghosts.sum())
    assert np.all(parts["cell"][ghosts] == cfg.ncell)
    assert np.array_equal(parts["cell"][~ghosts], cell[~ghosts])


def _flux(u, vth):
    a = u / (math.sqrt(2) * vth)
    f1 = vth / math.sqrt(2 * math.pi) * math.exp(-a * a) + 0.5 * u * (1 + math.erf(a))
    f2 = 0.5 * (u * u + vth * vth) * (1 + math.erf(a)) + u * vth / math.sqrt(2 * math.pi) * \
        math.exp(-a * a)
    return f1, f2


@pytest.mark.parametrize("ux", [0.0, 0.5, -0.3])
def test_injection_counts_and_flux_weighted_moments(ux):
    cfg = _cfg(ny=40, dt=0.05)
    spec = dict(n=1.0, ux=ux, uy=0.2, uz=-0.1, vth=0.4, ppc=64, faces=3)
    empty = {k: np.zeros(0, np.int32 if k == "cell" else np.float64)
             for k in ("cell", "ox", "oy", "ux", "uy", "uz", "w")}
    ins = []
    for step in range(60):
        ins.append(O.open_inject(cfg, spec, 99, step, empty))
    allp = {k: np.concatenate([p[k] for p in ins]) for k in empty}
    for f, col in ((0, 1), (1, cfg.nx - 2)):
        un = ux if f == 0 else -ux
        f1, f2 = _flux(un, spec["vth"])
        nexp = spec["ppc"] * cfg.dt / cfg.dx * f1
        assert O.inflow_expected(cfg, spec, f) == pytest.approx(nexp, rel=1e-14)
        side = (allp["cell"] % cfg.nx) == col
        # the count rule: floor(nexp + U) per row and step, U the row's draw
        want = 0
        for step in range(60):
            for j in range(cfg.ny):
                ctr = ((((step * 2 + f) << 16 | j) << 20) << 7) | 127
                want += math.floor(nexp + O.uniform(99, ctr))
        assert int(side.sum()) == want
        vn = allp["ux"][side] * (1 if f == 0 else -1)
        assert np.all(vn > 0)
        k = vn.size
        # flux-weighted normal speed: <v> = F2 / F1 (within 4 sigma)
        sd = math.sqrt(max(np.var(vn), 1e-30) / k)
        assert abs(vn.mean() - f2 / f1) < 4 * sd + 1e-3
        assert abs(allp["uy"][side].mean() - 0.2) < 4 * 0.4 / math.sqrt(k)
        assert abs(allp["uz"][side].std() - 0.4) < 0.05
        o = allp["ox"][side] * (1 if f == 0 else -1)
        assert np.all((allp["ox"][side] >= -1) & (allp["ox"][side] < 1))
        # depth v dt tau, tau uniform: mean offset -1 + dt <v>/dx
        assert abs(o.mean() - (-1 + cfg.dt * vn.mean() / cfg.dx)) < 0.05
    assert np.allclose(allp["w"], np.float32(cfg.dx * cfg.dy * cfg.dz / spec["ppc"]))


def test_open_flow_keeps_its_density():
    """The workload's uniform flow through the open box: over 40 steps the
    ion count stays within a few per cent of the start (the faces inject
    what the opposite faces absorb), and B1 stays small."""
    cfg, parts, B0, B1, spec = W.open_flow(nx=24, ny=8, ppc=16, amp=0.0)
    sim = O.OpenOracleSim(cfg, parts, B0, B1, spec, seed=5)
    n0 = sim.p["cell"].size
    for _ in range(40):
        sim.step()
    n1 = sim.p["cell"].size
    print(f"ions {n0} -> {n1}; absorbed {sim.absorbed}, injected {sim.injected}")
    assert sim.absorbed > 0 and sim.injected > 0
    assert abs(n1 - n0) < 0.05 * n0
    assert np.abs(sim.B1).max() < 0.2


def _splitmix_vectors():
    import pathlib

    state, outs = None, []
    for line in (pathlib.Path(__file__).parent / "golden" / "splitmix64_vectors.txt").read_text().splitlines():
        if line.startswith("state"):
            state = int(line.split()[1])
        elif line.startswith("output"):
            outs.append(int(line.split()[1]))
    return state, outs


def test_draws_follow_the_published_splitmix64_sequence():
    """The injection's uniform is (mix(seed + mix(ctr)) >> 11) 2^-53 with
    mix the splitmix64 finaliser.  Choosing ctr = the published start state
    makes mix(ctr) its first output; the seed that moves that onto the state
    of output k makes the uniform output k's top 53 bits.  So the oracle's
    generator reproduces the published sequence exactly."""
    golden = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1
    state, outs = _splitmix_vectors()
    assert len(outs) >= 3
    for k in range(1, len(outs)):
        # mix(ctr) = outs[0]; want seed + outs[0] = state + k * golden
        seed = (state + k * golden - outs[0]) & M
        assert O.uniform(seed, state) == (outs[k] >> 11) * 2.0 ** -53, k


@pytest.mark.parametrize("nx,ny,nz,nsub,mode,eta_h,buf", [
    (14, 9, 1, 3, 0, 0.0, 3), (14, 9, 1, 3, 0, 2e-3, 4), (5, 6, 1, 2, 0, 1e-3, 1),
    (3, 4, 1, 1, 0, 0.0, 2), (14, 9, 1, 0, 0, 1e-3, 3), (14, 9, 1, 3, 1, 1e-3, 3),
    (30, 7, 1, 4, 0, 0.0, 0), (9, 5, 4, 2, 0, 1e-3, 2), (6, 3, 5, 1, 1, 0.0, 1),
    (4, 4, 2, 3, 0, 2e-3, 3)])
def test_open_field_advance_matches_an_independent_numpy_form(nx, ny, nz, nsub, mode, eta_h, buf):
    """tests/bruteforce_open.py writes the open rules again with whole-array
    NumPy stencils and a column mask for the ghost columns, importing nothing
    from the oracle.  On fields that vary along x and y (so that every ghost
    rule is exercised: the dropped x-derivatives in the ghost columns, the
    refills after each stage, the buffer's per-column eta_h), with densities
    below the floor in some cells, the two agree to rounding."""
    from tests.bruteforce_open import OpenGrid

    cfg = _cfg(nx=nx, ny=ny, nsub=nsub, eta_h=eta_h, buffer_cells=buf, eta_h_buffer=0.03,
               gamma_e=5.0 / 3.0)
    if nz > 1:
        cfg = cfg.replace(ndim=3, nz=nz, dz=0.6)
    rng = np.random.default_rng(nx * 100 + ny + 10 * nz + nsub)
    B0 = np.zeros((3, cfg.ncell))
    B0[:] = np.array([[0.3], [1.0], [-0.2]])
    B1 = rng.normal(scale=0.1, size=(3, cfg.ncell))
    nh = rng.uniform(0.02, 1.5, cfg.ncell)
    nh[cfg.nx + 1] = 0.01  # an interior cell below the floor
    npv = rng.uniform(0.5, 1.5, cfg.ncell)
    Jh = rng.normal(scale=0.2, size=(3, cfg.ncell))
    Jp = rng.normal(scale=0.2, size=(3, cfg.ncell))
    nh, npv, Jh, Jp = (O.open_fill(cfg, a) for a in (nh, npv, Jh, Jp))
    assert np.any(nh < cfg.n_floor)
    rB1, rE, rBt, _, _ = O.open_field_advance(cfg, B0, B1, nh, Jh, npv, Jp, mode=mode)
    bB1, bE, bBt = OpenGrid(cfg).field_advance(B0, B1, nh, Jh, npv, Jp, mode=mode)
    for got, ref in ((bB1, rB1), (bE, rE), (bBt, rBt)):
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    # the ghost rules matter on these inputs: the periodic solver differs
    pE = O.ohm(cfg.replace(open_x=0), B0 + rB1, nh if mode else 1.5 * nh - 0.5 * npv,
               Jh if mode else 1.5 * Jh - 0.5 * Jp)
    assert np.abs(pE - rE).max() > 1e-3 * np.abs(rE).max()


def test_numpy_form_fails_on_a_planted_ghost_mistake():
    """The comparison above is sharp: the NumPy form with the ghost column's
    x-derivative kept (the rule of Sec. II.C dropped) disagrees with the
    oracle."""
    from tests.bruteforce_open import OpenGrid

    cfg = _cfg(nx=14, ny=9, nsub=2)
    rng = np.random.default_rng(5)
    B0 = np.zeros((3, cfg.ncell))
    B0[1] = 1.0
    B1 = rng.normal(scale=0.1, size=(3, cfg.ncell))
    n = O.open_fill(cfg, rng.uniform(0.5, 1.5, cfg.ncell))
    J = O.open_fill(cfg, rng.normal(scale=0.2, size=(3, cfg.ncell)))
    _, rE, _, _, _ = O.open_field_advance(cfg, B0, B1, n, J, n, J, mode=0)
    g = OpenGrid(cfg)
    g.interior = np.ones(cfg.nx)  # keep x-derivatives in the ghost columns
    _, bE, _ = g.field_advance(B0, B1, n, J, n, J, mode=0)
    assert np.abs(bE - rE).max() > 1e-3 * np.abs(rE).max()


@pytest.mark.parametrize("ndim", [2, 3])
def test_injected_values_match_an_independent_inversion(ndim):
    """Each injected ion against values computed another way: the counter
    draws recomputed in Python from the generator's definition (splitmix64's
    finaliser, the counter packing of the injection); the inflow flux F1 and
    the flux-weighted speed distribution by numerical quadrature of
    v f(v) (scipy.integrate.quad) and its inversion by root finding
    (scipy.optimize.brentq), not the closed-form erf expressions; the
    tangential velocities by Box-Muller; the entry depth v dt U.  Values are
    compared after rounding to FP32, as the store holds them."""
    import math

    from scipy import integrate, optimize

    M = (1 << 64) - 1

    def mix(z):
        z = (z + 0x9E3779B97F4A7C15) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    def uni(seed, ctr):
        return (mix((seed + mix(ctr)) & M) >> 11) * 2.0 ** -53

    def ctr(step, f, j, m, d):
        return ((((step * 2 + f) << 16 | j) << 20 | m) << 7 | d) & M

    cfg = _cfg(nx=6, ny=10, dt=0.05)
    if ndim == 3:
        cfg = cfg.replace(ndim=3, ny=4, nz=3, dz=0.6)  # rows r = j + ny k
    spec = dict(n=1.0, ux=0.5, uy=0.2, uz=-0.1, vth=0.4, ppc=128, faces=3)
    seed, step = 77, 9
    keys = ("cell", "ox", "oy") + (("oz",) if ndim == 3 else ()) + ("ux", "uy", "uz", "w")
    empty = {k: np.zeros(0, np.int32 if k == "cell" else np.float64) for k in keys}
    got = O.open_inject(cfg, spec, seed, step, empty)
    vth = spec["vth"]
    q = 0
    for f in (0, 1):
        u = spec["ux"] if f == 0 else -spec["ux"]
        dens = lambda v: v * math.exp(-0.5 * (v - u) ** 2 / vth ** 2) / (math.sqrt(2 * math.pi) * vth)
        F1 = integrate.quad(dens, 0.0, math.inf, epsabs=0, epsrel=1e-13)[0]
        nexp = spec["ppc"] * cfg.dt / cfg.dx * F1
        for r in range(cfg.ny * cfg.nz):
            j, kz = r % cfg.ny, r // cfg.ny
            k = math.floor(nexp + uni(seed, ctr(step, f, r, 0, 127)))
            for m in range(k):
                U = uni(seed, ctr(step, f, r, m, 0))
                cdf = lambda v: integrate.quad(dens, 0.0, v, epsabs=0, epsrel=1e-13)[0] / F1 - U
                v = optimize.brentq(cdf, 0.0, max(u, 0.0) + 10 * vth, xtol=1e-15, rtol=1e-15)

                def normal(d):
                    u1, u2 = uni(seed, ctr(step, f, r, m, d)), uni(seed, ctr(step, f, r, m, d + 1))
                    return math.sqrt(-2.0 * math.log(1.0 - u1)) * math.cos(2 * math.pi * u2)

                s = v * cfg.dt * uni(seed, ctr(step, f, r, m, 100))
                o = -1.0 + 2.0 * s / cfg.dx
                want = {"cell": (1 if f == 0 else cfg.nx - 2) + cfg.nx * (j + cfg.ny * kz),
                        "ox": o if f == 0 else -o,
                        "oy": -1.0 + 2.0 * uni(seed, ctr(step, f, r, m, 101)),
                        "ux": v if f == 0 else -v,
                        "uy": spec["uy"] + vth * normal(96),
                        "uz": spec["uz"] + vth * normal(98)}
                if ndim == 3:
                    want["oz"] = -1.0 + 2.0 * uni(seed, ctr(step, f, r, m, 102))
                assert got["cell"][q] == want["cell"], (f, j, m)
                for key in want:
                    if key == "cell":
                        continue
                    assert abs(got[key][q] - np.float32(want[key])) <= 2e-7 * max(1.0, abs(want[key])), \
                        (key, f, j, m, got[key][q], want[key])
                q += 1
    assert q == got["cell"].size and q > 50


def test_open_flow_3d_keeps_its_density():
    """The 3D form of the open-flow workload (ghost planes at both x ends):
    over 30 steps the faces inject about what the opposite faces absorb."""
    cfg, parts, B0, B1, spec = W.open_flow(nx=12, ny=8, nz=6, ppc=8, amp=0.0)
    sim = O.OpenOracleSim(cfg, parts, B0, B1, spec, seed=5)
    n0 = sim.p["cell"].size
    for _ in range(30):
        sim.step()
    n1 = sim.p["cell"].size
    assert sim.absorbed > 100 and sim.injected > 100
    assert abs(n1 - n0) < 0.05 * n0
    i = sim.p["cell"] % cfg.nx
    assert np.all((i >= 1) & (i <= cfg.nx - 2))  # nothing left in a ghost plane
