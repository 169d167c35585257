"""GPU parity of the open x boundaries (Sec. II.C) against the FP64 oracle:
the ghost fill (bit-exact), the open field advance (B1, E, B0 + B1 within
1e-5 relative L2, ghost columns included; the diagnostics by
check_field_diag; the floor count exact), absorption (bit-exact keys),
injection (the counts and cells exact, the drawn values to FP32 rounding),
the sort with absorbed ions last (bit-exact order and cell_start), and the
whole open step (one step on a straddler-free start compared ion by ion;
ten steps by the injected counts, the absorbed counts and the energy
history)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W
from tests.helpers import announce, check_field_diag, compare_particles, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_05600_amd import hvpic

    hvpic.lib()
    return hvpic


def dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _cfg(nx, ny, **kw):
    base = dict(name="open", ndim=2, nx=nx, ny=ny, nz=1, dx=0.5, dy=0.4, dz=1.0, dt=0.05,
                nsub=3, te=0.2, eta=1e-3, open_x=1, buffer_cells=3, eta_h_buffer=0.02)
    base.update(kw)
    return W.Config(**base)


GRIDS = [("37x23", _cfg(37, 23)), ("3x5", _cfg(3, 5)), ("6x2", _cfg(6, 2)),
         ("70x9-wide-buffer", _cfg(70, 9, buffer_cells=12))]


def _inputs(cfg, seed):
    B0 = np.zeros((3, cfg.ncell))
    B0[:] = np.array([[0.3], [1.0], [-0.2]])
    B1 = W.random_field(seed, cfg, 0.2)
    nh = O.open_fill(cfg, W.random_density(seed + 1, cfg, 0.02, 1.5))  # some below the floor
    npv = O.open_fill(cfg, W.random_density(seed + 2, cfg, 0.5, 1.5))
    Jh = O.open_fill(cfg, W.random_field(seed + 3, cfg, 0.2))
    Jp = O.open_fill(cfg, W.random_field(seed + 4, cfg, 0.2))
    return B0, B1, nh, npv, Jh, Jp


def test_open_fill(H):
    announce("open_fill")
    cfg = _cfg(37, 23)
    ctx = H.Context(cfg, 1)
    F = np.random.default_rng(3).normal(size=(5, cfg.ncell)).astype(np.float32)
    Fd = dev(F)
    H.hvpic_open_fill(ctx.ctx, Fd, 5)
    assert np.array_equal(Fd.cpu().numpy(), O.open_fill(cfg, F).astype(np.float32))


@pytest.mark.parametrize("name,cfg", GRIDS)
@pytest.mark.parametrize("mode,nsub", [(0, 0), (0, 1), (0, 3), (1, 3)])
@pytest.mark.parametrize("eta_h", [0.0, 2e-3])
def test_open_field_advance(H, name, cfg, mode, nsub, eta_h):
    announce("open_field_advance", name, mode, nsub, eta_h)
    cfg = cfg.replace(nsub=nsub, eta_h=eta_h)
    B0, B1, nh, npv, Jh, Jp = _inputs(cfg, 601)
    ctx = H.Context(cfg, 1)
    B0d, B1d = dev(B0), dev(B1)
    Btd = torch.zeros((3, cfg.ncell), device="cuda")
    Ed = torch.zeros((3, cfg.ncell), device="cuda")
    diag = torch.zeros(3, dtype=torch.float64, device="cuda")
    rB1, rE, rBt, rd, st = O.open_field_advance(cfg, B0, B1, nh, Jh, npv, Jp, mode=mode)
    for _ in range(2):  # twice: scratch and partials are reused
        B1d.copy_(dev(B1))
        H.hvpic_open_field_advance(ctx.ctx, B0d, B1d, Btd, dev(nh), dev(Jh), dev(npv), dev(Jp),
                                   Ed, mode, diag)
        flags, counts = H.hvpic_sync_status(ctx.ctx)
        assert rel_l2(B1d.cpu().numpy(), rB1) < 1e-5
        assert rel_l2(Btd.cpu().numpy(), rBt) < 1e-5
        assert rel_l2(Ed.cpu().numpy(), rE) < 1e-5
        # the ghost columns on their own
        g = np.zeros((cfg.ny, cfg.nx), bool)
        g[:, [0, -1]] = True
        g = g.ravel()
        assert rel_l2(Ed.cpu().numpy()[:, g], rE[:, g]) < 1e-5
        check_field_diag(diag.cpu().numpy(), rd)
        assert counts[2] == st.floor_hits
    if mode == 0 and nsub > 0:
        assert rel_l2(rB1, B1) > 1e-4  # B1 did evolve


def test_open_rules_matter(H):
    """The open path differs from the periodic one on these inputs (the
    comparison above is not vacuous): the ghost rules and the buffer change E."""
    announce("open_rules_matter")
    cfg = _cfg(37, 23)
    B0, B1, nh, npv, Jh, Jp = _inputs(cfg, 611)
    _, rE, rBt, _, _ = O.open_field_advance(cfg, B0, B1, nh, Jh, npv, Jp, mode=0)
    per = cfg.replace(open_x=0)
    _, pE, _, _ = O.field_advance(per, B0 + B1, nh, Jh, npv, Jp, mode=0)
    assert rel_l2(pE, rE) > 1e-2


def test_entry_points_check_the_open_flag(H):
    announce("open_flags")
    cfg = _cfg(8, 4)
    z3 = torch.zeros((3, cfg.ncell), device="cuda")
    z1 = torch.ones(cfg.ncell, device="cuda")
    a = H.Context(cfg, 1)
    with pytest.raises(H.HvpicError):
        H.hvpic_field_advance(a.ctx, z3, z1, z3, z1, z3, z3.clone(), 0)
    b = H.Context(cfg.replace(open_x=0), 1)
    with pytest.raises(H.HvpicError):
        H.hvpic_open_field_advance(b.ctx, z3, z3.clone(), z3.clone(), z1, z3, z1, z3, z3.clone(), 0)
    with pytest.raises(H.HvpicError):
        H.hvpic_open_fill(b.ctx, z3, 3)
    with pytest.raises(H.HvpicError):
        H.Context(cfg.replace(ndim=3, nz=2), 1)


def _store(cfg, n, seed, dead_frac=0.0, ghost_frac=0.0):
    """A random store; cells uniform over the grid, a fraction moved into
    the ghost columns (ghost_frac) or marked absorbed (dead_frac)."""
    rng = np.random.default_rng(seed)
    i = rng.integers(1, cfg.nx - 1, n)
    j = rng.integers(0, cfg.ny, n)
    g = rng.random(n) < ghost_frac
    i[g] = np.where(rng.random(g.sum()) < 0.5, 0, cfg.nx - 1)
    cell = (i + cfg.nx * j).astype(np.int32)
    cell[rng.random(n) < dead_frac] = cfg.ncell
    f = lambda: rng.uniform(-1, 1, n).astype(np.float32)
    return dict(cell=cell, ox=f(), oy=f(), ux=f(), uy=f(), uz=f(),
                w=rng.uniform(0.5, 1.5, n).astype(np.float32))


@pytest.mark.parametrize("nx,ny,n,dead", [(37, 23, 50000, 0.1), (6, 5, 257, 0.5), (6, 5, 0, 0.0),
                                          (66, 40, 100000, 0.0), (12, 7, 300, 1.0)])
def test_sort_open(H, nx, ny, n, dead):
    announce("sort_open", nx, ny, n, dead)
    cfg = _cfg(nx, ny)
    ctx = H.Context(cfg, max(n, 1))
    parts = _store(cfg, n, 7, dead_frac=dead)
    p = H.Particles.from_numpy(parts, 2, max(n, 1))
    q = H.Particles(2, max(n, 1))
    cs = torch.full((cfg.ncell + 2,), -7, dtype=torch.int32, device="cuda")
    H.hvpic_sort_open(ctx.ctx, p, q, cs)
    got = q.to_numpy()
    order = np.argsort(parts["cell"], kind="stable")
    for k in got:
        assert np.array_equal(got[k], parts[k][order]), k
    ref_cs = np.concatenate([[0], np.cumsum(np.bincount(parts["cell"], minlength=cfg.ncell + 1))])
    csh = cs.cpu().numpy()
    assert np.array_equal(csh, ref_cs)
    assert csh[cfg.ncell] == int(np.sum(parts["cell"] < cfg.ncell))


def _spec(**kw):
    s = dict(n=1.0, ux=0.5, uy=0.1, uz=-0.2, vth=0.3, ppc=32, faces=3)
    s.update(kw)
    return s


@pytest.mark.parametrize("nx,ny,n,spec,step", [
    (37, 23, 20000, _spec(), 0),
    (37, 23, 20000, _spec(ux=-0.8, faces=1), 17),
    (10, 700, 3000, _spec(ppc=8, vth=1.0), 5),          # rows in more than one chunk
    (5, 3, 0, _spec(ux=0.0, ppc=200, faces=2), 123456),
    (8, 4, 100, _spec(ux=3.0, vth=0.1, ppc=50), 1),     # a cold fast beam: N > 1 per row
])
def test_absorb_and_inject(H, nx, ny, n, spec, step):
    announce("absorb_inject", nx, ny, n, spec, step)
    cfg = _cfg(nx, ny)
    cap = n + 4 * ny * spec["ppc"] + 64
    ctx = H.Context(cfg, cap)
    parts = _store(cfg, n, 11, ghost_frac=0.05)
    p = H.Particles.from_numpy(parts, 2, cap)
    seed = 0x9E3779B97F4A7C15 ^ step
    H.hvpic_open_particles(ctx.ctx, p, H.inflow_from(spec), seed, step)
    got = p.to_numpy()
    ref = O.particles64(parts)
    k_abs = O.open_absorb(cfg, ref)
    assert np.array_equal(got["cell"][:n], ref["cell"])
    assert int(np.sum(got["cell"][:n] == cfg.ncell)) == k_abs
    new = O.open_inject(cfg, spec, seed, step, ref)
    m = new["cell"].size
    assert p.n == m, (p.n, m)
    print(f"absorbed {k_abs}, injected {m - n}", flush=True)
    if m > n:
        sl = slice(n, m)
        assert np.array_equal(got["cell"][sl], new["cell"][sl])
        assert np.array_equal(got["w"][sl].astype(np.float64), new["w"][sl])
        for k in ("ox", "oy", "ux", "uy", "uz"):
            a = got[k][sl].astype(np.float64)
            b = new[k][sl]
            assert np.all(np.abs(a - b) <= 2e-7 * np.maximum(1.0, np.abs(b))), k
        assert np.all(got["ox"][sl] >= -1) and np.all(got["ox"][sl] < 1)
        assert np.all(got["oy"][sl] >= -1) and np.all(got["oy"][sl] < 1)


def test_inject_capacity_and_step_range(H):
    announce("inject_limits")
    cfg = _cfg(8, 64)
    ctx = H.Context(cfg, 16)
    p = H.Particles(2, 16)
    with pytest.raises(H.HvpicError):  # 2 x 64 rows at ~1 ion each do not fit in 16
        H.hvpic_open_particles(ctx.ctx, p, H.inflow_from(_spec(ux=3.0, ppc=50)), 1, 0)
    assert p.n == 0
    with pytest.raises(H.HvpicError):
        H.hvpic_open_particles(ctx.ctx, p, H.inflow_from(_spec()), 1, 1 << 20)
    with pytest.raises(H.HvpicError):
        H.hvpic_open_particles(ctx.ctx, p, H.inflow_from(_spec(vth=0.0)), 1, 0)


def _clean_start(cfg, parts, B0, B1, spec, seed, band=1e-5):
    """The open-flow ions minus those the FP64 oracle's first step puts
    within band half-cells of a face, or whose mid-point deposit point lands
    there (FP32 and FP64 may decide such cells differently)."""
    from tests.helpers import deposit_point_straddlers, _near_face

    keep = np.ones(parts["cell"].size, bool)
    for _ in range(4):
        sub = {k: v[keep] for k, v in parts.items()}
        sim = O.OpenOracleSim(cfg, sub, B0, B1, spec, seed)
        ids = np.nonzero(keep)[0]
        # the oracle's initial sort permutes; recover each ion's id
        sub_ids = {**sub, "id": ids.astype(np.float64)}
        p = O.particles64(sub_ids)
        perm, _ = O.sort(cfg, p["cell"])
        p = O.apply_perm(p, perm)
        O.push(cfg, p, sim.E, sim.Btot)
        near = _near_face(p["ox"], band) | _near_face(p["oy"], band)
        near |= deposit_point_straddlers(cfg, p, 0.5 * cfg.dt, band)
        if not near.any():
            print(f"straddlers removed: {int((~keep).sum())} of {keep.size}", flush=True)
            return sub
        keep[p["id"].astype(np.int64)[near]] = False
    raise AssertionError("straddler removal did not converge")


def test_open_step_matches_oracle(H):
    announce("open_step", "one step")
    from paper_2305_05600_amd.sim import OpenSim

    cfg, parts, B0, B1, spec = W.open_flow(nx=32, ny=16, ppc=16)
    seed = 21
    parts = _clean_start(cfg, parts, B0, B1, spec, seed)
    ref = O.OpenOracleSim(cfg, parts, B0, B1, spec, seed)
    sim = OpenSim(cfg, parts, B0, B1, spec, seed)
    assert rel_l2(sim.E.cpu().numpy(), ref.E) < 1e-5
    ref.step()
    sim.step()
    assert sim.injected == ref.injected and sim.absorbed == ref.absorbed
    got = sim.particles()
    assert got["cell"].size == ref.p["cell"].size
    compare_particles(cfg, got, ref.p)
    assert rel_l2(sim.B1.cpu().numpy(), ref.B1) < 1e-5
    assert rel_l2(sim.E.cpu().numpy(), ref.E) < 1e-5
    assert rel_l2(sim.Btot.cpu().numpy(), ref.Btot) < 1e-5
    check_field_diag(sim.field_diag.cpu().numpy(), ref.field_diag)
    assert np.allclose(sim.push_diag.cpu().numpy(), ref.push_diag, rtol=1e-5, atol=1e-9)
    flags, counts = sim.status()
    assert flags & (H.FLAG_BAD_INPUT | H.FLAG_NONFINITE) == 0, flags


def test_open_steps_history(H):
    """Ten steps: the injected count of every step equals the oracle's (it
    does not depend on the ions), the absorbed totals agree up to ions whose
    FP32 and FP64 cells differ, and the energy history agrees to 1e-3."""
    announce("open_step", "ten steps")
    from paper_2305_05600_amd.sim import OpenSim

    cfg, parts, B0, B1, spec = W.open_flow(nx=32, ny=16, ppc=16)
    seed = 22
    ref = O.OpenOracleSim(cfg, parts, B0, B1, spec, seed)
    sim = OpenSim(cfg, parts, B0, B1, spec, seed)
    for s in range(10):
        ref.step()
        sim.step()
        assert sim.injected == ref.injected, s
        assert abs(sim.absorbed - ref.absorbed) <= 2, (s, sim.absorbed, ref.absorbed)
        fd = sim.field_diag.cpu().numpy()
        assert abs(fd[0] - ref.field_diag[0]) <= 1e-3 * abs(ref.field_diag[0])
        assert abs(fd[2] - ref.field_diag[2]) <= 1e-3 * abs(ref.field_diag[2])
        pd = sim.push_diag.cpu().numpy()
        assert abs(pd[0] - ref.push_diag[0]) <= 1e-3 * abs(ref.push_diag[0])
    print(f"absorbed {sim.absorbed} (oracle {ref.absorbed}), injected {sim.injected}", flush=True)
    assert sim.absorbed > 0 and sim.injected > 0
    assert rel_l2(sim.B1.cpu().numpy(), ref.B1) < 1e-3
