"""GPU parity on the paths the production runs take and on the edge cases of
the move, against the FP64 oracle.

* Dense sorted boxes (>= 72 ions per cell) so that every block of the push
  and of the deposit works through its LDS windows (asserted with the
  library's path counters): 2D/3D x QS/NGP, with and without the move counts
  for the sort, fused and stand-alone deposit; far movers and an
  inconsistent cell_start inside a window.
* Exact face landings with dyadic offsets, velocities and steps: FP32 and
  FP64 then compute the same numbers, so every cell index must agree with no
  straddler band.
* Non-finite input: NaN velocities and a non-finite B cell.
* The 3D whole step after one step at 1e-5, particles included; a 3D grid
  above 512^2 cells through the neighbour sort and its far-mover fallback;
  whole steps with smoothing passes.

Tolerances as elsewhere: sort order, cell_start and cell indices bit-exact;
moments and fields 1e-5 relative L2; velocities FP32 rounding."""
import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W
from tests.helpers import (announce, check_field_diag, compare_particles,
                           drop_push_straddlers, drop_straddlers, rel_l2)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_05600_amd import hvpic

    hvpic.lib()
    return hvpic


def cfg2(nx=37, ny=23, shape=W.SHAPE_QS, **kw):
    base = dict(name="p2", ndim=2, nx=nx, ny=ny, nz=1, dx=0.5, dy=0.3, dz=1.0, dt=0.05,
                nsub=3, shape=shape, te=0.2, eta=1e-3)
    base.update(kw)
    return W.Config(**base)


def cfg3(nx=13, ny=11, nz=9, shape=W.SHAPE_QS, **kw):
    base = dict(name="p3", ndim=3, nx=nx, ny=ny, nz=nz, dx=0.5, dy=0.4, dz=0.7, dt=0.05,
                nsub=3, shape=shape, te=0.2, eta=1e-3)
    base.update(kw)
    return W.Config(**base)


CASES = [("2d-qs", cfg2()), ("2d-ngp", cfg2(shape=W.SHAPE_NGP)), ("3d-qs", cfg3()),
         ("3d-ngp", cfg3(shape=W.SHAPE_NGP))]


def dev(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _sorted(cfg, parts):
    perm, cs = O.sort(cfg, parts["cell"])
    return {k: np.ascontiguousarray(v[perm]) for k, v in parts.items()}, cs


def _dense(cfg):
    """Ions per cell at which every chunk of the push spans few enough cells
    for its windows (3072 ions over at most 59 cells in 2D, 1024 over 19 in
    3D)."""
    return 72.0 if cfg.ndim == 2 else 96.0


def _check_sorted(cfg, src: dict, out: dict, cs):
    perm, rcs = O.sort(cfg, src["cell"])
    assert np.array_equal(cs, rcs)
    for k in src:
        assert np.array_equal(out[k], src[k][perm]), k


def _assert_windows(H, ctx, min_frac=1.0):
    win, glob = H.hvpic_path_stats(ctx.ctx)
    print(f"blocks through the LDS windows: {win}, global: {glob}", flush=True)
    assert win > 0 and win >= min_frac * (win + glob), (win, glob)


@pytest.mark.parametrize("name,cfg", CASES)
@pytest.mark.parametrize("counted", [False, True])
@pytest.mark.parametrize("fused", [False, True])
def test_window_path_dense(H, name, cfg, counted, fused):
    """Every block takes the window path; particles, moments and (counted)
    the next neighbour sort match the oracle."""
    announce("window_dense", name, counted, fused)
    _, parts, B = W.random_box(201, cfg, _dense(cfg), vmax_cells=0.9)
    E = W.random_field(202, cfg, 0.3)
    parts = drop_push_straddlers(cfg, parts, E, B, back=0.5 * cfg.dt)
    parts, cs0 = _sorted(cfg, parts)
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    H.hvpic_path_stats(ctx.ctx)  # clear
    p = H.Particles.from_numpy(parts, cfg.ndim)
    nd = torch.full((cfg.ncell,), 7.0, device="cuda")
    Jd = torch.full((3, cfg.ncell), 7.0, device="cuda")
    diag = torch.zeros(4, dtype=torch.float64, device="cuda")
    cs_prev = dev(cs0, np.int32)
    H.hvpic_gather_push(ctx.ctx, p, cs_prev if counted else None, dev(E), dev(B),
                        nd if fused else None, Jd if fused else None, diag)
    _assert_windows(H, ctx)
    pushed = p.to_numpy()
    q = H.Particles(cfg.ndim, n)
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
    if not fused:
        # the stand-alone deposit of the sorted store, as the unfused step
        # runs it: its blocks work through their windows too
        H.hvpic_deposit(ctx.ctx, q, cs, 0.5 * cfg.dt, nd, Jd)
        _assert_windows(H, ctx)
    flags, counts = H.hvpic_sync_status(ctx.ctx)
    ref = O.particles64(parts)
    rd, st = O.push(cfg, ref, E, B)
    assert flags == 0 and counts[0] == st.moved_gt1 == 0
    compare_particles(cfg, pushed, ref, band=0.0)
    _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())
    rn, rJ = O.deposit(cfg, ref, 0.5 * cfg.dt)
    assert rel_l2(nd.cpu().numpy(), rn) < 1e-5
    assert rel_l2(Jd.cpu().numpy(), rJ) < 1e-5
    assert np.allclose(diag.cpu().numpy(), rd, rtol=1e-5, atol=1e-6 * abs(rd[0]))


@pytest.mark.parametrize("name,cfg", CASES)
def test_window_path_far_movers(H, name, cfg):
    """A few particles inside windowed chunks move 2.5 cells: they are pushed
    and deposited like the oracle (their mid-points leave the window), counted,
    flagged, and the next sort completes with the general path."""
    announce("window_far", name)
    _, parts, B = W.random_box(211, cfg, _dense(cfg), vmax_cells=0.9)
    parts, _ = _sorted(cfg, parts)
    n0 = parts["cell"].size
    far = np.array([n0 // 7, n0 // 2, (5 * n0) // 6])
    parts["ux"][far] = np.float32(2.5 * cfg.dx / cfg.dt)
    parts["uy"][far[1]] = np.float32(-2.5 * cfg.dy / cfg.dt)
    E = W.random_field(212, cfg, 0.01)
    parts = drop_push_straddlers(cfg, parts, E, B, back=0.5 * cfg.dt)
    parts, cs0 = _sorted(cfg, parts)
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    H.hvpic_path_stats(ctx.ctx)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    q = H.Particles(cfg.ndim, n)
    nd = torch.zeros(cfg.ncell, device="cuda")
    Jd = torch.zeros((3, cfg.ncell), device="cuda")
    cs_prev = dev(cs0, np.int32)
    H.hvpic_gather_push(ctx.ctx, p, cs_prev, dev(E), dev(B), nd, Jd)
    _assert_windows(H, ctx)
    pushed = p.to_numpy()
    ref = O.particles64(parts)
    _, st = O.push(cfg, ref, E, B)
    assert st.moved_gt1 >= 3
    compare_particles(cfg, pushed, ref, band=0.0)
    rn, rJ = O.deposit(cfg, ref, 0.5 * cfg.dt)
    assert rel_l2(nd.cpu().numpy(), rn) < 1e-5 and rel_l2(Jd.cpu().numpy(), rJ) < 1e-5
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
    flags, counts = H.hvpic_sync_status(ctx.ctx)
    assert flags & H.FLAG_MOVE_GT1 and counts[0] == st.moved_gt1
    _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())


@pytest.mark.parametrize("name,cfg", [CASES[0], CASES[2]])
def test_window_path_bad_cell_start(H, name, cfg):
    """cell_start inconsistent at a cell inside a windowed chunk: the push
    flags bad input, pushes and deposits every particle from its own cell,
    and the next neighbour sort completes with the general path."""
    announce("window_bad_cs", name)
    _, parts, B = W.random_box(221, cfg, _dense(cfg), vmax_cells=0.9)
    E = W.random_field(222, cfg, 0.1)
    parts = drop_push_straddlers(cfg, parts, E, B, back=0.5 * cfg.dt)
    parts, cs0 = _sorted(cfg, parts)
    bad = cs0.copy()
    mid = cfg.ncell // 3
    bad[mid] = bad[mid + 1]  # cell mid-1 claims cell mid's particles
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    H.hvpic_path_stats(ctx.ctx)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    q = H.Particles(cfg.ndim, n)
    nd = torch.zeros(cfg.ncell, device="cuda")
    Jd = torch.zeros((3, cfg.ncell), device="cuda")
    cs_bad = dev(bad, np.int32)
    H.hvpic_gather_push(ctx.ctx, p, cs_bad, dev(E), dev(B), nd, Jd)
    _assert_windows(H, ctx)
    pushed = p.to_numpy()
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_sort(ctx.ctx, p, q, cs_bad, cs, full=False)
    flags, _ = H.hvpic_sync_status(ctx.ctx)
    assert flags & H.FLAG_BAD_INPUT
    ref = O.particles64(parts)
    O.push(cfg, ref, E, B)
    compare_particles(cfg, pushed, ref, band=0.0)
    rn, rJ = O.deposit(cfg, ref, 0.5 * cfg.dt)
    assert rel_l2(nd.cpu().numpy(), rn) < 1e-5 and rel_l2(Jd.cpu().numpy(), rJ) < 1e-5
    _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())


def _dyadic_box(cfg, seed, ppc):
    """Offsets on the grid of quarter half-cells, velocities such that every
    displacement (and its half, the deposit's mid-point) is a multiple of
    1/8 half-cell: all exact in FP32, many landing exactly on faces."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(ppc * cfg.ncell)
    cell = np.sort(rng.integers(0, cfg.ncell, n)).astype(np.int32)
    off = lambda: (rng.integers(-4, 4, n) / 4.0).astype(np.float32)
    # displacement per unit speed 2 dt / h; a speed of m * h / (8 dt) moves
    # m/4 half-cells, m in [-8, 8] keeps every move within one cell
    vel = lambda h: (rng.integers(-8, 9, n) * h / (8.0 * cfg.dt)).astype(np.float32)
    parts = {"cell": cell, "ox": off(), "oy": off(), "ux": vel(cfg.dx), "uy": vel(cfg.dy),
             "uz": vel(cfg.dz) if cfg.ndim == 3 else rng.uniform(-1, 1, n).astype(np.float32),
             "w": np.full(n, 0.01, np.float32)}
    if cfg.ndim == 3:
        parts["oz"] = off()
    return parts


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("shape", [W.SHAPE_QS, W.SHAPE_NGP])
def test_exact_face_landings(H, ndim, shape):
    """E = B = 0 and dyadic numbers: every landing exactly on a face (x' = +1
    goes to the next cell at -1; x' = -3 one cell back at -1) must give the
    oracle's cell and offset exactly, with no straddler band; so must the
    deposit cells of the mid-points."""
    announce("exact_faces", ndim, shape)
    cfg = (cfg2 if ndim == 2 else cfg3)(shape=shape, dx=0.5, dy=0.25, dz=1.0, dt=0.125)
    parts = _dyadic_box(cfg, 231 + ndim, 40.0 if ndim == 2 else 60.0)
    ox = parts["ox"].astype(np.float64) + 2 * cfg.dt / cfg.dx * parts["ux"].astype(np.float64)
    assert np.sum(np.abs(ox) == 1.0) > 100  # many exact face landings
    zero = np.zeros((3, cfg.ncell), np.float32)
    n = parts["cell"].size
    cs0 = O.sort(cfg, parts["cell"])[1]
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    nd = torch.zeros(cfg.ncell, device="cuda")
    Jd = torch.zeros((3, cfg.ncell), device="cuda")
    cs_prev = dev(cs0, np.int32)
    H.hvpic_gather_push(ctx.ctx, p, cs_prev, dev(zero), dev(zero), nd, Jd)
    got = p.to_numpy()
    ref = O.particles64(parts)
    O.push(cfg, ref, zero, zero)
    assert np.array_equal(got["cell"], ref["cell"])
    for k in ["ox", "oy"] + (["oz"] if ndim == 3 else []):
        assert np.array_equal(got[k].astype(np.float64), ref[k]), k
    rn, rJ = O.deposit(cfg, ref, 0.5 * cfg.dt)
    assert rel_l2(nd.cpu().numpy(), rn) < 1e-5 and rel_l2(Jd.cpu().numpy(), rJ) < 1e-5
    q = H.Particles(cfg.ndim, n)
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
    flags, _ = H.hvpic_sync_status(ctx.ctx)
    assert flags == 0
    _check_sorted(cfg, got, q.to_numpy(), cs.cpu().numpy())


@pytest.mark.parametrize("name,cfg", [CASES[0], CASES[2], CASES[1]])
@pytest.mark.parametrize("counted", [False, True])
def test_nonfinite_inputs(H, name, cfg, counted):
    """NaN velocities and a non-finite B cell: the particles whose move is
    non-finite stay where they were, are counted once each (the oracle's count
    exactly) and raise the flag; every other particle moves as the oracle's;
    the sort stays on its neighbour path."""
    announce("nonfinite", name, counted)
    _, parts, B = W.random_box(241, cfg, _dense(cfg), vmax_cells=0.9)
    E = W.random_field(242, cfg, 0.1)
    B[1, cfg.ncell // 2] = np.inf
    parts = drop_push_straddlers(cfg, parts, E, B)
    parts, cs0 = _sorted(cfg, parts)
    n = parts["cell"].size
    nan_at = np.array([3, n // 3, n - 2])
    parts["ux"][nan_at] = np.nan
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    cs_prev = dev(cs0, np.int32)
    H.hvpic_gather_push(ctx.ctx, p, cs_prev if counted else None, dev(E), dev(B))
    flags, counts = H.hvpic_sync_status(ctx.ctx)
    got = p.to_numpy()
    ref = O.particles64(parts)
    _, st = O.push(cfg, ref, E, B)
    assert st.nonfinite >= 3
    assert flags & H.FLAG_NONFINITE and counts[1] == st.nonfinite and counts[0] == 0
    assert np.array_equal(got["cell"], ref["cell"])
    bad = ~np.isfinite(ref["ux"]) | ~np.isfinite(ref["uy"]) | ~np.isfinite(ref["uz"])
    for k in ["ox", "oy"] + (["oz"] if cfg.ndim == 3 else []):
        # the non-finite particles keep their offsets bit for bit
        assert np.array_equal(got[k][bad], parts[k][bad]), k
        assert np.abs(got[k][~bad] - ref[k][~bad]).max() < 1e-5, k
    for k in ("ux", "uy", "uz"):
        assert np.array_equal(np.isfinite(got[k]), np.isfinite(ref[k])), k
    if counted:
        q = H.Particles(cfg.ndim, n)
        cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
        H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
        flags, _ = H.hvpic_sync_status(ctx.ctx)
        assert not flags & (H.FLAG_MOVE_GT1 | H.FLAG_BAD_INPUT)
        perm, rcs = O.sort(cfg, got["cell"])
        assert np.array_equal(cs.cpu().numpy(), rcs)
        assert np.array_equal(q.to_numpy()["cell"], got["cell"][perm])


def test_3d_beam_one_step(H):
    """The 3D beam case (16^3) after one whole step: moments and fields at
    1e-5, sort and cell indices exact, diagnostics at 1e-5."""
    from paper_2305_05600_amd import sim as S

    announce("beam3d_one_step")
    cfg, parts, B = W.beam_3d(n=16)
    parts = drop_straddlers(cfg, parts, B)
    g = S.GpuSim(cfg, parts, B, fused=True, gather_map=True)
    o = O.OracleSim(cfg, parts, B)
    g.step()
    o.step()
    for got, ref in ((g.E, o.E), (g.B, o.B), (g.n_prev, o.n_prev), (g.J_prev, o.J_prev)):
        assert rel_l2(got.cpu().numpy(), ref) < 1e-5
    assert np.array_equal(g.cs.cpu().numpy(), o.cell_start)
    assert compare_particles(cfg, g.particles(), o.p, band=0.0) == 0
    assert np.allclose(g.push_diag.cpu().numpy(), o.push_diag, rtol=1e-5, atol=1e-9)
    check_field_diag(g.field_diag.cpu().numpy(), o.field_diag)


@pytest.mark.parametrize("far", [False, True])
@pytest.mark.parametrize("perm_form", [False, True])
def test_neighbour_sort_large_grid_3d(H, far, perm_form):
    """A 3D grid above 512^2 cells (67 x 65 x 61) takes the sort's large-tile
    scan path; with far movers the neighbour path hands over to the general
    sort on the device."""
    cfg = cfg3(nx=67, ny=65, nz=61)
    announce("nb_sort_large_3d", cfg.ncell, far, perm_form)
    _, parts, B = W.random_box(251, cfg, 0.5, vmax_cells=0.9)
    parts, cs0 = _sorted(cfg, parts)
    if far:
        n0 = parts["cell"].size
        parts["uz"][[n0 // 5, n0 // 2]] = np.float32(2.5 * cfg.dz / cfg.dt)
    E = W.random_field(252, cfg, 0.01)
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    cs_prev = dev(cs0, np.int32)
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_gather_push(ctx.ctx, p, cs_prev, dev(E), dev(B))
    pushed = p.to_numpy()
    if perm_form:
        perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        H.hvpic_sort_perm(ctx.ctx, p, cs_prev, perm, cs)
        flags, _ = H.hvpic_sync_status(ctx.ctx)
        rperm, rcs = O.sort(cfg, pushed["cell"])
        assert np.array_equal(perm.cpu().numpy(), rperm)
        assert np.array_equal(cs.cpu().numpy(), rcs)
    else:
        q = H.Particles(cfg.ndim, n)
        H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
        flags, _ = H.hvpic_sync_status(ctx.ctx)
        _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())
    assert bool(flags & H.FLAG_MOVE_GT1) == far


@pytest.mark.parametrize("case", ["alfven", "beam3d"])
def test_whole_step_with_smoothing(H, case):
    """Two binomial passes on the moments after the deposit and on the copies
    of E and B the gather reads: one whole step at 1e-5, sort and cells exact."""
    from paper_2305_05600_amd import sim as S

    announce("smoothing_step", case)
    if case == "alfven":
        cfg, parts, B = W.periodic_alfven()
    else:
        cfg, parts, B = W.beam_3d(n=16)
    cfg = cfg.replace(nsmooth=2)
    parts = drop_straddlers(cfg, parts, B)
    g = S.GpuSim(cfg, parts, B, fused=True, gather_map=True)
    o = O.OracleSim(cfg, parts, B)
    for got, ref in ((g.E, o.E), (g.n_prev, o.n_prev), (g.J_prev, o.J_prev)):
        assert rel_l2(got.cpu().numpy(), ref) < 1e-5
    g.step()
    o.step()
    for got, ref in ((g.E, o.E), (g.B, o.B), (g.n_prev, o.n_prev), (g.J_prev, o.J_prev)):
        assert rel_l2(got.cpu().numpy(), ref) < 1e-5
    assert np.array_equal(g.cs.cpu().numpy(), o.cell_start)
    compare_particles(cfg, g.particles(), o.p, band=0.0)


def test_set_stream_keeps_size_checks(H):
    """After rebinding a context to another stream the binding still checks
    tensor sizes against the grid."""
    cfg = cfg2()
    ctx = H.Context(cfg, 16)
    s = torch.cuda.Stream()
    ctx.set_stream(s)
    small = torch.zeros((3, cfg.ncell - 1), device="cuda")
    B = torch.zeros((3, cfg.ncell), device="cuda")
    n = torch.ones(cfg.ncell, device="cuda")
    with pytest.raises(H.HvpicError):
        H.hvpic_field_advance(ctx.ctx, B, n, small, n, B, B, 0)
