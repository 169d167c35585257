"""GPU tests of the ensemble (hvpic_ensemble_*): independent 2D runs of
uneven size stepped together by persistent launches over their work items.

Each run of an ensemble must give what the same run gives stepped on its own
by the plain gather-map sequence: the sort order, cell_start and cells
exactly, moments and fields to FP32 rounding (the push chunk length changes
which particles share a lane's running sums, so with a chunk other than the
plain one the last bits may differ: relative L2 <= 1e-6), and the oracle
within the parity bound.  The step captured in a hipGraph replays to the
same bits as eager steps.
"""
import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W
from tests.helpers import announce, drop_straddlers, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_05600_amd import hvpic, sim

    hvpic.lib()
    return hvpic, sim


# small, uneven runs spanning the three classes of particles per cell and both
# grid classes (the largest is 130^2 cells)
SPECS = [dict(seed=11, side=9, ppc=20, amp=0.03, te_ratio=0.5, vth=0.5),
         dict(seed=12, side=17, ppc=70, amp=0.01, te_ratio=0.2, vth=0.5),
         dict(seed=13, side=24, ppc=150, amp=0.05, te_ratio=1.0, vth=0.5),
         dict(seed=14, side=13, ppc=40, amp=0.002, te_ratio=0.1, vth=0.5),
         dict(seed=15, side=130, ppc=33, amp=0.02, te_ratio=0.7, vth=0.5)]


def _runs(specs=SPECS, clean=False, shape=W.SHAPE_QS):
    out = []
    for s in specs:
        cfg, parts, B = W.ensemble_run(s, shape=shape)
        if clean:
            parts = drop_straddlers(cfg, parts, B, steps=2)
        out.append((cfg, parts, B))
    return out


def _sims(S, runs):
    return [S.GpuSim(cfg, parts, B, fused=True, gather_map=True) for cfg, parts, B in runs]


def _same_state(ens, r, g, exact=True, tol=1e-6):
    s = ens.state(r)
    g.synchronize()
    assert torch.equal(s["cs"], g.cs), r
    pa, pb = ens.particles(r), g.particles()
    assert np.array_equal(pa["cell"], pb["cell"]), r
    for name, a, b in (("E", s["E"], g.E), ("B", s["B"], g.B), ("n", s["n_prev"], g.n_prev),
                       ("J", s["J_prev"], g.J_prev)):
        if exact:
            assert torch.equal(a, b), (r, name)
        else:
            assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) <= tol, (r, name)
    for k in ("ox", "oy", "ux", "uy", "uz", "w"):
        if exact:
            assert np.array_equal(pa[k], pb[k]), (r, k)
        else:
            assert np.allclose(pa[k], pb[k], rtol=1e-6, atol=1e-6), (r, k)


@pytest.mark.parametrize("shape", [W.SHAPE_QS, W.SHAPE_NGP])
def test_ensemble_matches_separate_runs(mods, shape):
    H, S = mods
    announce("ensemble_vs_plain", shape)
    runs = _runs(shape=shape)
    ens = S.Ensemble(_sims(S, runs))  # default choices: the plain path's chunk and tile
    plain = _sims(S, runs)
    assert ens.tuning == H.hvpic_tuning_default().as_dict()
    for step in range(3):
        ens.step()
        for g in plain:
            g.step()
        for r, g in enumerate(plain):
            _same_state(ens, r, g, exact=True)
            assert torch.equal(ens.state(r)["push_diag"], g.push_diag), (step, r)
            assert torch.equal(ens.state(r)["field_diag"], g.field_diag), (step, r)
    for r in range(len(runs)):
        flags, counts = ens.status(r)
        assert flags & H.FLAG_BAD_INPUT == 0


@pytest.mark.parametrize("chunk", [0, 1, 2])
@pytest.mark.parametrize("tile", [0, 1, 2])
def test_ensemble_choices_compute_the_same_step(mods, chunk, tile):
    H, S = mods
    announce("ensemble_choices", chunk, tile)
    runs = _runs()
    ens = S.Ensemble(_sims(S, runs))
    ens.set_tuning({"push_chunk": [chunk] * 3, "field_tile": [tile] * 2,
                    "blocks_per_cu": [2, 1, 2, 1]})
    plain = _sims(S, runs)
    for _ in range(3):
        ens.step()
        for g in plain:
            g.step()
    for r, g in enumerate(plain):
        _same_state(ens, r, g, exact=(chunk == 2), tol=1e-6)


def test_ensemble_against_the_oracle(mods):
    H, S = mods
    announce("ensemble_vs_oracle")
    runs = _runs(SPECS[:4], clean=True)
    ens = S.Ensemble(_sims(S, runs), tuning=None)
    ens.set_tuning({"push_chunk": [0, 1, 2], "field_tile": [1, 2], "blocks_per_cu": [4, 2, 4, 2]})
    orc = [O.OracleSim(cfg, parts, B) for cfg, parts, B in runs]
    for _ in range(2):
        ens.step()
        for o in orc:
            o.step()
    for r, o in enumerate(orc):
        s = ens.state(r)
        assert np.array_equal(s["cs"].cpu().numpy(), o.cell_start), r
        for name, got, ref in (("E", s["E"], o.E), ("B", s["B"], o.B),
                               ("n", s["n_prev"], o.n_prev), ("J", s["J_prev"], o.J_prev)):
            err = rel_l2(got.cpu().numpy(), ref)
            assert err < 2e-5, (r, name, err)


def test_ensemble_graph_replays_match_eager(mods):
    H, S = mods
    announce("ensemble_graph")
    runs = _runs()
    eager = S.Ensemble(_sims(S, runs))
    graph = S.Ensemble(_sims(S, runs))
    graph.capture(True)
    scratch = torch.zeros(1 << 20, device="cuda")
    for step in range(5):
        eager.step()
        graph.step()
        # the program's own work between replays
        scratch.add_(1.0)
        torch.cuda.synchronize()
        for r in range(len(runs)):
            a, b = eager.state(r), graph.state(r)
            for k in ("cs", "E", "B", "n_prev", "J_prev", "push_diag", "field_diag"):
                assert torch.equal(a[k], b[k]), (step, r, k)
    assert graph.steps == eager.steps == 5
    # switching capture off and on again keeps the sequence
    graph.capture(False)
    graph.step()
    graph.capture(True)
    graph.step()
    eager.step()
    eager.step()
    for r in range(len(runs)):
        pa, pb = eager.particles(r), graph.particles(r)
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), (r, k)


def test_autotune_steps_are_real_steps(mods):
    H, S = mods
    announce("ensemble_autotune")
    runs = _runs()
    ens = S.Ensemble(_sims(S, runs))
    choices, ms = ens.autotune(reps=1)
    k = ens.steps
    assert k > 0 and all(m > 0.0 for m in ms)
    assert all(c in (0, 1, 2) for c in choices["push_chunk"])
    assert all(t in (0, 1, 2) for t in choices["field_tile"])
    assert all(1 <= b <= 64 for b in choices["blocks_per_cu"])
    assert ens.tuning == choices
    print(f"autotune: {choices}, phase ms {ms}, {k} steps", flush=True)
    phases = ens.time_phases(3)
    assert all(m > 0.0 for m in phases) and ens.steps == k + 3
    k = ens.steps
    plain = _sims(S, runs)
    for _ in range(k):
        for g in plain:
            g.step()
    for r, g in enumerate(plain):
        _same_state(ens, r, g, exact=False, tol=1e-6)


def test_far_movers_take_the_fallback(mods):
    """A run whose ions move more than one cell per step: its sort falls back
    to the general stable sort inside the batched scatter; the other runs
    are unaffected."""
    H, S = mods
    announce("ensemble_far")
    runs = _runs(SPECS[:3])
    cfg = W.Config(name="far", ndim=2, nx=19, ny=11, nz=1, dx=0.5, dy=0.5, dz=1.0, dt=0.05,
                   nsub=4, te=0.1, eta=1e-3)
    _, parts, B = W.random_box(77, cfg, 30.0, vmax_cells=2.5)
    runs.append((cfg, parts, B))
    ens = S.Ensemble(_sims(S, runs))
    plain = _sims(S, runs)
    for _ in range(2):
        ens.step()
        for g in plain:
            g.step()
    flags, counts = ens.status(3)
    assert flags & H.FLAG_MOVE_GT1 and counts[0] > 0
    for r, g in enumerate(plain):
        _same_state(ens, r, g, exact=True)


def test_ensemble_rejects_what_it_does_not_batch(mods):
    H, S = mods
    announce("ensemble_rejects")
    runs = _runs(SPECS[:2])
    sims = _sims(S, runs)
    cfg, parts, B = W.periodic_alfven(nx=8, ny=8, ppc=8)
    few = S.GpuSim(cfg.replace(nsub=2), parts, B, fused=True, gather_map=True)
    with pytest.raises(H.HvpicError):
        S.Ensemble(sims + [few])
    with pytest.raises(ValueError):
        S.Ensemble(sims + [S.GpuSim(cfg, parts, B, fused=True, gather_map=False)])
    ens = S.Ensemble(sims)
    with pytest.raises(H.HvpicError):
        ens.set_tuning({"push_chunk": [3, 0, 0]})
    with pytest.raises(H.HvpicError):
        ens.set_tuning({"blocks_per_cu": [0, 1, 1, 1]})


def test_ensemble_full_size(mods):
    """The benchmarked ensemble at full size (64 runs, sides 64-256, 32-200
    ions per cell: about 247M ions and 2.1M cells), with the default choices
    (the plain path's chunk and tile) and the step replayed from its
    hipGraph as the benchmark runs it: after three steps every run's
    cell_start, E, B and moments equal those of the same run stepped on its
    own, bit for bit, and so do the stores of the smallest and largest runs."""
    H, S = mods
    announce("ensemble_full_size")
    specs = W.ensemble_specs()
    runs = [W.ensemble_run(s) for s in specs]
    n_total = sum(int(p["cell"].size) for _, p, _ in runs)
    ens = S.Ensemble(_sims(S, runs))
    plain = _sims(S, runs)
    del runs
    assert ens.tuning == H.hvpic_tuning_default().as_dict()
    ens.capture(True)
    for _ in range(3):
        ens.step()
        for g in plain:
            g.step()
    sizes = [s["side"] ** 2 * s["ppc"] for s in specs]
    check = {int(np.argmin(sizes)), int(np.argmax(sizes))}
    for r, g in enumerate(plain):
        s = ens.state(r)
        g.synchronize()
        assert torch.equal(s["cs"], g.cs), r
        for name, a, b in (("E", s["E"], g.E), ("B", s["B"], g.B), ("n", s["n_prev"], g.n_prev),
                           ("J", s["J_prev"], g.J_prev)):
            assert torch.equal(a, b), (r, name)
        if r in check:
            _same_state(ens, r, g, exact=True)
        flags, _ = ens.status(r)
        assert flags & (H.FLAG_BAD_INPUT | H.FLAG_NONFINITE) == 0, (r, flags)
    print(f"ensemble: {len(specs)} runs, {n_total} ions, equal to the plain runs after "
          f"3 graph-replayed steps", flush=True)
