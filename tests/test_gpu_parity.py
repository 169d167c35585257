"""GPU parity: every entry point of libhvpic.so against the FP64 oracle.

Tolerances: sort order, cell_start and cell indices bit-exact (cell indices
outside the 1e-5 face band); moments and fields within 1e-5 relative L2 after
one step; FP64 diagnostics within 1e-5.  All inputs are seeded synthetic
workloads from paper_2305_05600_amd.workloads.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W
from tests.helpers import (_near_face, announce, check_field_diag, compare_particles,
                           deposit_point_straddlers, rel_l2)

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


def dev(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


CASES = [("2d-qs", cfg2()), ("2d-ngp", cfg2(shape=W.SHAPE_NGP)), ("3d-qs", cfg3()),
         ("3d-ngp", cfg3(shape=W.SHAPE_NGP))]


def _sorted(cfg, parts):
    perm, cs = O.sort(cfg, parts["cell"])
    return {k: np.ascontiguousarray(v[perm]) for k, v in parts.items()}, cs


@pytest.mark.parametrize("name,cfg", CASES)
@pytest.mark.parametrize("ppc", [3.7, 40.2])
@pytest.mark.parametrize("counted", [False, True])
def test_gather_push(H, name, cfg, ppc, counted):
    announce("gather_push", name, ppc, counted)
    _, parts, B = W.random_box(21, cfg, ppc)
    parts, cs0 = _sorted(cfg, parts)
    E = W.random_field(22, cfg, 0.3)
    ctx = H.Context(cfg, parts["cell"].size)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    diag = torch.zeros(4, dtype=torch.float64, device="cuda")
    cs = dev(cs0, np.int32) if counted else None
    H.hvpic_gather_push(ctx.ctx, p, cs, dev(E), dev(B), None, None, diag)
    flags, counts = H.hvpic_sync_status(ctx.ctx)
    got = p.to_numpy()
    ref = O.particles64(parts)
    rd, st = O.push(cfg, ref, E, B)
    compare_particles(cfg, got, ref)
    assert np.allclose(diag.cpu().numpy(), rd, rtol=1e-5, atol=1e-6 * abs(rd[0]))
    assert counts[0] == st.moved_gt1 and counts[1] == st.nonfinite
    assert not flags & H.FLAG_BAD_INPUT


@pytest.mark.parametrize("name,cfg", CASES)
@pytest.mark.parametrize("ppc,sorted_", [(0.9, True), (37.0, True), (12.0, False)])
@pytest.mark.parametrize("back", [0.0, 0.025])
def test_deposit(H, name, cfg, ppc, sorted_, back):
    announce("deposit", name, ppc, sorted_, back)
    _, parts, _ = W.random_box(31, cfg, ppc)
    # FP32 and FP64 may disagree on the cell of a deposit point within rounding
    # of a face; such points are kept out of the input
    keep = ~deposit_point_straddlers(cfg, parts, back)
    parts = {k: v[keep] for k, v in parts.items()}
    cs = None
    if sorted_:
        parts, cs0 = _sorted(cfg, parts)
        cs = dev(cs0, np.int32)
    ctx = H.Context(cfg, parts["cell"].size)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    n = torch.full((cfg.ncell,), 7.0, device="cuda")   # overwritten
    J = torch.full((3, cfg.ncell), 7.0, device="cuda")
    H.hvpic_deposit(ctx.ctx, p, cs, back, n, J)
    rn, rJ = O.deposit(cfg, O.particles64(parts), back)
    assert rel_l2(n.cpu().numpy(), rn) < 1e-5
    assert rel_l2(J.cpu().numpy(), rJ) < 1e-5


@pytest.mark.parametrize("name,cfg", CASES)
@pytest.mark.parametrize("counted", [False, True])
def test_fused_push_deposit(H, name, cfg, counted):
    """Push with the mid-point deposit fused in == oracle push, then deposit at
    x^{n+1} - (dt/2) v^{n+1/2}."""
    announce("fused", name, counted)
    _, parts, B = W.random_box(41, cfg, 33.3)
    E = W.random_field(42, cfg, 0.3)
    ref = O.particles64(parts)
    O.push(cfg, ref, E, B)
    offs = ["ox", "oy"] + (["oz"] if cfg.ndim == 3 else [])
    near = deposit_point_straddlers(cfg, ref, 0.5 * cfg.dt)
    for k in offs:
        near |= (np.abs(ref[k] + 1) < 1e-5) | (np.abs(ref[k] - 1) < 1e-5)
    parts = {k: v[~near] for k, v in parts.items()}
    parts, cs0 = _sorted(cfg, parts)
    ctx = H.Context(cfg, parts["cell"].size)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    n = torch.zeros(cfg.ncell, device="cuda")
    J = torch.zeros((3, cfg.ncell), device="cuda")
    H.hvpic_gather_push(ctx.ctx, p, dev(cs0, np.int32) if counted else None, dev(E), dev(B), n, J,
                        None)
    ref = O.particles64(parts)
    O.push(cfg, ref, E, B)
    rn, rJ = O.deposit(cfg, ref, 0.5 * cfg.dt)
    compare_particles(cfg, p.to_numpy(), ref)
    assert rel_l2(n.cpu().numpy(), rn) < 1e-5
    assert rel_l2(J.cpu().numpy(), rJ) < 1e-5


def _check_sorted(cfg, src: dict, out: dict, cs):
    perm, rcs = O.sort(cfg, src["cell"])
    assert np.array_equal(cs, rcs)
    for k in src:
        assert np.array_equal(out[k], src[k][perm]), k


@pytest.mark.parametrize("name,cfg", CASES)
@pytest.mark.parametrize("ppc", [0.3, 5.0, 70.0])
def test_full_sort(H, name, cfg, ppc):
    announce("full_sort", name, ppc)
    _, parts, _ = W.random_box(51, cfg, ppc)
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    q = H.Particles(cfg.ndim, max(n, 1))
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_sort(ctx.ctx, p, q, None, cs, full=True)
    _check_sorted(cfg, parts, q.to_numpy(), cs.cpu().numpy())


@pytest.mark.parametrize("name,cfg", CASES)
@pytest.mark.parametrize("far", [False, True])
@pytest.mark.parametrize("counted", [False, True])
def test_neighbour_sort_after_push(H, name, cfg, far, counted):
    """Sorted store -> push -> neighbour-move sort gives the stable order; with
    a particle moved two cells the call falls back to the general sort.  With
    cell_start given to the push, the sort uses the push's move counts."""
    announce("nb_sort", name, far, counted)
    _, parts, B = W.random_box(61, cfg, 20.0, vmax_cells=0.95)
    parts, cs0 = _sorted(cfg, parts)
    if far:
        parts["ux"][len(parts["ux"]) // 2] = np.float32(2.5 * cfg.dx / cfg.dt)
    E = W.random_field(62, cfg, 0.01)
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    q = H.Particles(cfg.ndim, n)
    cs_prev = dev(cs0, np.int32)
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_gather_push(ctx.ctx, p, cs_prev if counted else None, dev(E), dev(B))
    pushed = p.to_numpy()
    H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
    flags, counts = H.hvpic_sync_status(ctx.ctx)
    _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())
    assert bool(flags & H.FLAG_MOVE_GT1) == far
    # repeated call with a new generation tag behaves the same
    H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
    _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())


@pytest.mark.parametrize("name,cfg", CASES)
@pytest.mark.parametrize("path", ["neighbour", "neighbour-counted", "far", "general"])
def test_sort_perm(H, name, cfg, path):
    """The gather-map form of the sort is the oracle's stable order itself
    (the permutation of a stable sort is unique) with the same cell_start, on
    the neighbour path (with or without the push's counts), on the fallback
    for a far mover, and on the general path."""
    announce("sort_perm", name, path)
    _, parts, B = W.random_box(63, cfg, 20.0, vmax_cells=0.95)
    parts, cs0 = _sorted(cfg, parts)
    if path == "far":
        parts["ux"][len(parts["ux"]) // 3] = np.float32(2.5 * cfg.dx / cfg.dt)
    E = W.random_field(64, cfg, 0.01)
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    cs_prev = dev(cs0, np.int32)
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    H.hvpic_gather_push(ctx.ctx, p, cs_prev if path == "neighbour-counted" else None, dev(E),
                        dev(B))
    pushed = p.to_numpy()
    H.hvpic_sort_perm(ctx.ctx, p, None if path == "general" else cs_prev, perm, cs)
    flags, _ = H.hvpic_sync_status(ctx.ctx)
    rperm, rcs = O.sort(cfg, pushed["cell"])
    assert np.array_equal(perm.cpu().numpy(), rperm)
    assert np.array_equal(cs.cpu().numpy(), rcs)
    assert bool(flags & H.FLAG_MOVE_GT1) == (path == "far")
    # nothing but the map and cell_start was written
    for k, v in p.to_numpy().items():
        assert np.array_equal(v, pushed[k]), k


@pytest.mark.parametrize("name,cfg", CASES)
@pytest.mark.parametrize("fused", [False, True])
def test_gather_push_perm(H, name, cfg, fused):
    """The push through a gather map equals the sort into a store followed by
    the push of that store, bit for bit: particles, moments, diagnostics, and
    the move counts (through the next sort of each)."""
    announce("gather_push_perm", name, fused)
    _, parts, B = W.random_box(65, cfg, 9.0, vmax_cells=0.9)
    E = W.random_field(66, cfg, 0.05)
    n = parts["cell"].size
    Ed, Bd = dev(E), dev(B)
    z = lambda *shape: torch.zeros(*shape, dtype=torch.float32, device="cuda")
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    runs = {}
    for mode in ("plain", "perm"):
        ctx = H.Context(cfg, n)
        p = H.Particles.from_numpy(parts, cfg.ndim)
        q = H.Particles(cfg.ndim, n)
        r = H.Particles(cfg.ndim, n)
        diag = torch.zeros(4, dtype=torch.float64, device="cuda")
        nm, Jm = (z(cfg.ncell), z(3, cfg.ncell)) if fused else (None, None)
        cs1 = torch.zeros_like(cs)
        if mode == "plain":
            H.hvpic_sort(ctx.ctx, p, q, None, cs, full=True)
            H.hvpic_gather_push(ctx.ctx, q, cs, Ed, Bd, nm, Jm, diag)
            H.hvpic_sort(ctx.ctx, q, r, cs, cs1, full=False)
            out = q.to_numpy()
            nxt = r.to_numpy()
        else:
            perm = torch.empty(n, dtype=torch.int32, device="cuda")
            H.hvpic_sort_perm(ctx.ctx, p, None, perm, cs)
            H.hvpic_gather_push_perm(ctx.ctx, p, perm, q, cs, Ed, Bd, nm, Jm, diag)
            perm1 = torch.empty(n, dtype=torch.int32, device="cuda")
            H.hvpic_sort_perm(ctx.ctx, q, cs, perm1, cs1)
            out = q.to_numpy()
            idx = perm1.cpu().numpy()
            nxt = {k: v[idx] for k, v in out.items()}
        flags, _ = H.hvpic_sync_status(ctx.ctx)
        runs[mode] = (out, nxt, cs1.cpu().numpy(), diag.cpu().numpy(),
                      None if nm is None else (nm.cpu().numpy(), Jm.cpu().numpy()), flags)
    a, b = runs["plain"], runs["perm"]
    for k in a[0]:
        assert np.array_equal(a[0][k], b[0][k]), k
        assert np.array_equal(a[1][k], b[1][k]), k
    assert np.array_equal(a[2], b[2])
    assert np.array_equal(a[3], b[3])
    if fused:
        assert np.array_equal(a[4][0], b[4][0]) and np.array_equal(a[4][1], b[4][1])
    assert a[5] == b[5] == 0


@pytest.mark.parametrize("name,cfg", [CASES[0], CASES[2]])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("gamma", [1.0, 5.0 / 3.0])
@pytest.mark.parametrize("nsub", [0, 1, 3, 4])
def test_field_advance(H, name, cfg, mode, gamma, nsub):
    """2D tiles take two substeps per launch (one for an odd last one)."""
    if mode == 1 and nsub != 3:
        pytest.skip("mode 1 has no subcycle")
    announce("field", name, mode, gamma, nsub)
    cfg = cfg.replace(gamma_e=gamma, nsub=nsub)
    B = W.random_field(71, cfg, 0.2, (1.0, 0.3, -0.2))
    nh = W.random_density(72, cfg, 0.02, 1.5)  # some cells below the floor
    npv = W.random_density(73, cfg, 0.5, 1.5)
    Jh = W.random_field(74, cfg, 0.2)
    Jp = W.random_field(75, cfg, 0.2)
    ctx = H.Context(cfg, 1)
    Bd = dev(B)
    Ed = torch.zeros((3, cfg.ncell), device="cuda")
    diag = torch.zeros(3, dtype=torch.float64, device="cuda")
    H.hvpic_field_advance(ctx.ctx, Bd, dev(nh), dev(Jh), dev(npv), dev(Jp), Ed, mode, diag)
    flags, counts = H.hvpic_sync_status(ctx.ctx)
    rB, rE, rd, st = O.field_advance(cfg, B, nh, Jh, npv, Jp, mode=mode)
    assert rel_l2(Bd.cpu().numpy(), rB) < 1e-5
    assert rel_l2(Ed.cpu().numpy(), rE) < 1e-5
    check_field_diag(diag.cpu().numpy(), rd)
    assert counts[2] == st.floor_hits and bool(flags & H.FLAG_FLOOR_HIT) == (st.floor_hits > 0)


@pytest.mark.parametrize("nx,ny", [(5, 3), (70, 19)])
@pytest.mark.parametrize("nsub", [2, 5])
def test_field_advance_2d_tiles(H, nx, ny, nsub):
    """Grids smaller than one tile (the halo wraps more than once) and grids
    of several tiles with ragged edges."""
    announce("field-tiles", nx, ny, nsub)
    cfg = cfg2(nx=nx, ny=ny, nsub=nsub)
    B = W.random_field(171, cfg, 0.2, (1.0, 0.3, -0.2))
    nh = W.random_density(172, cfg, 0.5, 1.5)
    npv = W.random_density(173, cfg, 0.5, 1.5)
    Jh = W.random_field(174, cfg, 0.2)
    Jp = W.random_field(175, cfg, 0.2)
    ctx = H.Context(cfg, 1)
    Bd = dev(B)
    Ed = torch.zeros((3, cfg.ncell), device="cuda")
    diag = torch.zeros(3, dtype=torch.float64, device="cuda")
    for _ in range(2):  # twice: the diagnostics' ticket is reset by its last block
        Bd.copy_(dev(B))
        H.hvpic_field_advance(ctx.ctx, Bd, dev(nh), dev(Jh), dev(npv), dev(Jp), Ed, 0, diag)
        rB, rE, rd, st = O.field_advance(cfg, B, nh, Jh, npv, Jp, mode=0)
        assert rel_l2(Bd.cpu().numpy(), rB) < 1e-5
        assert rel_l2(Ed.cpu().numpy(), rE) < 1e-5
        check_field_diag(diag.cpu().numpy(), rd)


@pytest.mark.parametrize("name,cfg", [CASES[0], CASES[2], ("2d-3x2", cfg2(nx=3, ny=2)),
                                      ("3d-1x5x2", cfg3(nx=1, ny=5, nz=2)),
                                      ("2d-70x19", cfg2(nx=70, ny=19))])
@pytest.mark.parametrize("npasses,ncomp", [(1, 3), (3, 3), (5, 1), (9, 3)])
def test_smooth(H, name, cfg, npasses, ncomp):
    """Binomial passes on LDS tiles (up to four per launch, so 5 and 9 take
    several launches), grids with ragged tiles and axes shorter than the
    halo, one or three components."""
    announce("smooth", name, npasses, ncomp)
    F = W.random_field(81, cfg, 1.0)[:ncomp].copy()
    if ncomp == 1:
        F = F[0].copy()
    ctx = H.Context(cfg, 1)
    Fd = dev(F)
    H.hvpic_smooth(ctx.ctx, Fd, npasses)
    assert rel_l2(Fd.cpu().numpy(), O.smooth(cfg, F, npasses)) < 1e-6


def test_empty_and_single(H):
    cfg = cfg2()
    announce("empty")
    empty = {k: np.zeros(0, np.int32 if k == "cell" else np.float32)
             for k in ("cell", "ox", "oy", "ux", "uy", "uz", "w")}
    ctx = H.Context(cfg, 4)
    p = H.Particles.from_numpy(empty, 2, capacity=4)
    q = H.Particles(2, 4)
    cs = torch.full((cfg.ncell + 1,), -1, dtype=torch.int32, device="cuda")
    diag = torch.full((4,), 9.0, dtype=torch.float64, device="cuda")
    E = torch.zeros((3, cfg.ncell), device="cuda")
    n = torch.ones(cfg.ncell, device="cuda")
    J = torch.ones((3, cfg.ncell), device="cuda")
    H.hvpic_gather_push(ctx.ctx, p, None, E, E, n, J, diag)
    H.hvpic_sort(ctx.ctx, p, q, None, cs, full=True)
    assert np.all(diag.cpu().numpy() == 0) and np.all(cs.cpu().numpy() == 0)
    assert float(n.abs().sum()) == 0 and float(J.abs().sum()) == 0
    # the same with cell_start (all zero for an empty store) and a
    # neighbour sort that takes the push's (zero) move counts
    diag.fill_(9.0)
    n.fill_(1.0)
    cs2 = torch.full((cfg.ncell + 1,), -1, dtype=torch.int32, device="cuda")
    H.hvpic_gather_push(ctx.ctx, p, cs, E, E, n, J, diag)
    H.hvpic_sort(ctx.ctx, p, q, cs, cs2, full=False)
    flags, _ = H.hvpic_sync_status(ctx.ctx)
    assert flags == 0
    assert np.all(diag.cpu().numpy() == 0) and np.all(cs2.cpu().numpy() == 0)
    assert float(n.abs().sum()) == 0 and float(J.abs().sum()) == 0
    # the gather-map forms on the empty store
    perm = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    cs3 = torch.full((cfg.ncell + 1,), -1, dtype=torch.int32, device="cuda")
    H.hvpic_sort_perm(ctx.ctx, p, None, perm, cs3)
    diag.fill_(9.0)
    n.fill_(1.0)
    H.hvpic_gather_push_perm(ctx.ctx, p, perm, q, cs3, E, E, n, J, diag)
    flags, _ = H.hvpic_sync_status(ctx.ctx)
    assert flags == 0 and q.n == 0
    assert np.all(diag.cpu().numpy() == 0) and np.all(cs3.cpu().numpy() == 0)
    assert float(n.abs().sum()) == 0 and float(J.abs().sum()) == 0
    announce("single")
    one = {k: v[:1] for k, v in W.random_box(3, cfg, 1.0)[1].items()}
    p = H.Particles.from_numpy(one, 2, capacity=4)
    H.hvpic_sort(ctx.ctx, p, q, None, cs, full=True)
    got = cs.cpu().numpy()
    assert got[0] == 0 and got[-1] == 1 and np.all(np.diff(got) >= 0)
    # one particle through the map equals the in-place push of the sorted copy
    H.hvpic_sort_perm(ctx.ctx, p, None, perm, cs3)
    assert perm.cpu().numpy()[0] == 0 and np.array_equal(cs3.cpu().numpy(), got)
    r = H.Particles(2, 4)
    Bf = dev(W.random_field(4, cfg, 0.3, (0.2, 0.1, 1.0)))
    Ef = dev(W.random_field(5, cfg, 0.1))
    H.hvpic_gather_push_perm(ctx.ctx, p, perm, r, cs3, Ef, Bf)
    H.hvpic_gather_push(ctx.ctx, q, cs, Ef, Bf)
    a, b = q.to_numpy(), r.to_numpy()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("nx,ny", [(1, 5), (2, 3), (3, 1)])
@pytest.mark.parametrize("counted", [False, True])
def test_tiny_grids(H, nx, ny, counted):
    """Degenerate grids (periodic axes of 1-3 cells): push, sort, deposit."""
    cfg = cfg2(nx=nx, ny=ny)
    announce("tiny", nx, ny, counted)
    _, parts, B = W.random_box(91, cfg, 50.0, vmax_cells=0.9)
    parts, cs0 = _sorted(cfg, parts)
    E = W.random_field(92, cfg, 0.1)
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, 2)
    q = H.Particles(2, n)
    nd = torch.zeros(cfg.ncell, device="cuda")
    Jd = torch.zeros((3, cfg.ncell), device="cuda")
    cs_prev = dev(cs0, np.int32)
    H.hvpic_gather_push(ctx.ctx, p, cs_prev if counted else None, dev(E), dev(B), nd, Jd)
    pushed = p.to_numpy()
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
    ref = O.particles64(parts)
    O.push(cfg, ref, E, B)
    compare_particles(cfg, pushed, ref)
    _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())
    rn, rJ = O.deposit(cfg, ref, 0.5 * cfg.dt)
    assert rel_l2(nd.cpu().numpy(), rn) < 1e-5 and rel_l2(Jd.cpu().numpy(), rJ) < 1e-5


@pytest.mark.parametrize("counted", [False, True])
def test_dense_single_cell(H, counted):
    """All particles in one cell: the neighbour sort's one-wavefront-per-cell
    loop and the deposit window see one long segment."""
    cfg = cfg2(nx=9, ny=8)
    announce("dense", counted)
    rng = np.random.Generator(np.random.PCG64(5))
    n = 20000
    parts = {"cell": np.full(n, 40, np.int32),
             "ox": W._offsets(rng.uniform(-1, 1, n)),
             "oy": W._offsets(rng.uniform(-1, 1, n)),
             "ux": rng.uniform(-4, 4, n).astype(np.float32),
             "uy": rng.uniform(-2, 2, n).astype(np.float32),
             "uz": rng.uniform(-1, 1, n).astype(np.float32),
             "w": np.full(n, 1e-3, np.float32)}
    _, _, B = W.random_box(6, cfg, 1.0)
    E = W.random_field(7, cfg, 0.1)
    cs0 = np.zeros(cfg.ncell + 1, np.int32)
    cs0[41:] = n
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, 2)
    q = H.Particles(2, n)
    nd = torch.zeros(cfg.ncell, device="cuda")
    Jd = torch.zeros((3, cfg.ncell), device="cuda")
    cs_prev = dev(cs0)
    H.hvpic_gather_push(ctx.ctx, p, cs_prev if counted else None, dev(E), dev(B), nd, Jd)
    pushed = p.to_numpy()
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
    _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())
    ref = O.particles64(parts)
    O.push(cfg, ref, E, B)
    rn, rJ = O.deposit(cfg, ref, 0.5 * cfg.dt)
    assert rel_l2(nd.cpu().numpy(), rn) < 1e-5 and rel_l2(Jd.cpu().numpy(), rJ) < 1e-5


@pytest.mark.parametrize("kind", ["claim", "decreasing"])
@pytest.mark.parametrize("name,cfg", [CASES[0], CASES[2]])
def test_push_inconsistent_cell_start(H, name, cfg, kind):
    """A cell_start that disagrees with the store: the push flags bad input,
    still pushes every particle from its own cell and deposits it, and the
    next neighbour sort completes with the general sort.  claim: a cell
    claims its neighbour's particles (still monotone); decreasing: a row's
    start exceeds the next row's (in 3D the push's chunk order then falls
    back to the store order, so that no chunk is pushed twice or skipped)."""
    announce("push_bad_cs", name, kind)
    _, parts, B = W.random_box(95, cfg, 6.0, vmax_cells=0.9)
    parts, cs0 = _sorted(cfg, parts)
    E = W.random_field(96, cfg, 0.1)
    ref = O.particles64(parts)
    O.push(cfg, ref, E, B)
    near = deposit_point_straddlers(cfg, ref, 0.5 * cfg.dt)
    for k in ["ox", "oy"] + (["oz"] if cfg.ndim == 3 else []):
        near |= (np.abs(ref[k] + 1) < 1e-5) | (np.abs(ref[k] - 1) < 1e-5)
    parts = {k: v[~near] for k, v in parts.items()}
    parts, cs0 = _sorted(cfg, parts)
    bad = cs0.copy()
    if kind == "claim":
        mid = cfg.ncell // 2
        bad[mid] = bad[mid + 1]  # cell mid-1 claims cell mid's particles
    else:
        mid = cfg.nx * (cfg.ncell // cfg.nx // 2)  # a row start
        bad[mid] = bad[-1]
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    q = H.Particles(cfg.ndim, n)
    nd = torch.zeros(cfg.ncell, device="cuda")
    Jd = torch.zeros((3, cfg.ncell), device="cuda")
    cs_bad = dev(bad, np.int32)
    H.hvpic_gather_push(ctx.ctx, p, cs_bad, dev(E), dev(B), nd, Jd)
    pushed = p.to_numpy()
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_sort(ctx.ctx, p, q, cs_bad, cs, full=False)
    flags, _ = H.hvpic_sync_status(ctx.ctx)
    assert flags & H.FLAG_BAD_INPUT
    ref = O.particles64(parts)
    O.push(cfg, ref, E, B)
    compare_particles(cfg, pushed, ref)
    rn, rJ = O.deposit(cfg, ref, 0.5 * cfg.dt)
    assert rel_l2(nd.cpu().numpy(), rn) < 1e-5 and rel_l2(Jd.cpu().numpy(), rJ) < 1e-5
    _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())


@pytest.mark.parametrize("nx,ny", [(1031, 517), (2053, 2049)])
def test_neighbour_sort_large_grid(H, nx, ny):
    """Grids above 512*512 cells take the sort's large-tile scan path
    (261 and 2054 tiles of 2048 cells)."""
    cfg = cfg2(nx=nx, ny=ny)
    announce("nb_sort_large", cfg.ncell)
    _, parts, B = W.random_box(97, cfg, 0.7, vmax_cells=0.9)
    parts, cs0 = _sorted(cfg, parts)
    E = W.random_field(98, cfg, 0.01)
    n = parts["cell"].size
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    q = H.Particles(cfg.ndim, n)
    cs_prev = dev(cs0, np.int32)
    cs = torch.zeros(cfg.ncell + 1, dtype=torch.int32, device="cuda")
    H.hvpic_gather_push(ctx.ctx, p, cs_prev, dev(E), dev(B))
    pushed = p.to_numpy()
    H.hvpic_sort(ctx.ctx, p, q, cs_prev, cs, full=False)
    flags, _ = H.hvpic_sync_status(ctx.ctx)
    assert flags == 0
    _check_sorted(cfg, pushed, q.to_numpy(), cs.cpu().numpy())


@pytest.mark.parametrize("name,cfg", CASES)
def test_gather_push_select(H, name, cfg):
    """The push of the ions a gather map selects from a larger store (the
    open step's form): the map takes a sorted subset of a sorted store, so
    the source arrays hold ions the map leaves out, and its entries reach
    past the number pushed.  The pushed store, its moments and diagnostics
    equal the oracle's push of the same subset in map order; a map longer
    than the store is rejected."""
    announce("gather_push_select", name)
    _, parts, B = W.random_box(71, cfg, 20.0, vmax_cells=0.9)
    parts, _ = _sorted(cfg, parts)
    E = W.random_field(72, cfg, 0.1)
    n = parts["cell"].size
    rng = np.random.default_rng(73)
    sel = np.sort(rng.choice(n, size=(3 * n) // 4, replace=False))
    # without the ions that the FP64 push puts within 1e-5 half-cells of a
    # face, or whose mid-point deposit point lands there (exact cells)
    probe = O.particles64({k: v[sel] for k, v in parts.items()})
    O.push(cfg, probe, E, B)
    near = np.zeros(sel.size, bool)
    for k in ["ox", "oy"] + (["oz"] if cfg.ndim == 3 else []):
        near |= _near_face(probe[k], 1e-5)
    near |= deposit_point_straddlers(cfg, probe, 0.5 * cfg.dt)
    print(f"straddlers removed: {int(near.sum())} of {sel.size}", flush=True)
    sel = sel[~near]
    sub = {k: v[sel] for k, v in parts.items()}
    m = sel.size
    ctx = H.Context(cfg, n)
    p = H.Particles.from_numpy(parts, cfg.ndim)
    q = H.Particles(cfg.ndim, n)
    perm = dev(sel, np.int32)
    nd = torch.zeros(cfg.ncell, dtype=torch.float32, device="cuda")
    Jd = torch.zeros((3, cfg.ncell), dtype=torch.float32, device="cuda")
    diag = torch.zeros(4, dtype=torch.float64, device="cuda")
    H.hvpic_gather_push_select(ctx.ctx, p, m, perm, q, None, dev(E), dev(B), nd, Jd, diag)
    flags, _ = H.hvpic_sync_status(ctx.ctx)
    assert not flags & H.FLAG_BAD_INPUT
    assert q.n == m
    ref = O.particles64(sub)
    rd, _ = O.push(cfg, ref, E, B)
    compare_particles(cfg, q.to_numpy(), ref)
    rn, rJ = O.deposit(cfg, ref, 0.5 * cfg.dt)
    assert rel_l2(nd.cpu().numpy(), rn) < 1e-5 and rel_l2(Jd.cpu().numpy(), rJ) < 1e-5
    assert np.allclose(diag.cpu().numpy(), rd, rtol=1e-5, atol=1e-6 * abs(rd[0]))
    with pytest.raises(H.HvpicError):
        H.hvpic_gather_push_select(ctx.ctx, p, n + 1, torch.zeros(n + 1, dtype=torch.int32,
                                                                  device="cuda"), q, None,
                                   dev(E), dev(B))
