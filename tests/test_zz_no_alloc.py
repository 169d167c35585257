"""hvpic_deposit_noalloc (the deposit with the library's own scratch, for
callers that cannot allocate) against hvpic_deposit with a context and
workspace, and against the FP64 oracle: two calls in a row on one stream, the
second on a smaller grid with fewer particles, plus a 3D call and the size
limit.  Tolerance: 1e-5 relative L2 on n and J (the atomics' order differs)."""
import numpy as np
import pytest

import oracle as O
from paper_2305_05600_amd import workloads as W
from tests.helpers import announce, deposit_point_straddlers, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_05600_amd import hvpic

    hvpic.lib()
    return hvpic


def _cfg(ndim, nx, ny, nz, shape=W.SHAPE_QS):
    return W.Config(name="na", ndim=ndim, nx=nx, ny=ny, nz=nz, dx=0.5, dy=0.3,
                    dz=(0.7 if ndim == 3 else 1.0), dt=0.05, nsub=2, shape=shape, te=0.2)


def _case(cfg, seed, ppc, sort):
    _, parts, _ = W.random_box(seed, cfg, ppc, vmax_cells=0.9)
    keep = ~deposit_point_straddlers(cfg, parts, 0.5 * cfg.dt)
    parts = {k: v[keep] for k, v in parts.items()}
    if sort:
        perm, _ = O.sort(cfg, parts["cell"])
        parts = {k: np.ascontiguousarray(v[perm]) for k, v in parts.items()}
    return parts


def test_noalloc_deposit_matches_context_deposit(H):
    stream = torch.cuda.Stream()
    cases = [(_cfg(2, 37, 23, 1), 301, 40.0, True),      # first call: larger
             (_cfg(2, 19, 11, 1), 302, 9.0, False),       # second: smaller grid and store
             (_cfg(3, 9, 7, 5, W.SHAPE_NGP), 303, 12.0, True)]
    for cfg, seed, ppc, sort in cases:
        announce("noalloc_deposit", cfg.ndim, cfg.nx, cfg.ny, cfg.nz, ppc, sort)
        parts = _case(cfg, seed, ppc, sort)
        back = 0.5 * cfg.dt
        with torch.cuda.stream(stream):
            p = H.Particles.from_numpy(parts, cfg.ndim)
            n_a = torch.full((cfg.ncell,), 7.0, device="cuda")
            J_a = torch.full((3, cfg.ncell), 7.0, device="cuda")
            n_b = torch.full((cfg.ncell,), -7.0, device="cuda")
            J_b = torch.full((3, cfg.ncell), -7.0, device="cuda")
        stream.synchronize()
        params = H.params_from(cfg, parts["cell"].size)
        H.hvpic_deposit_noalloc(params, stream.cuda_stream, p, back, n_a, J_a)
        ctx = H.Context(cfg, parts["cell"].size, stream=stream)
        H.hvpic_deposit(ctx.ctx, p, None, back, n_b, J_b)
        stream.synchronize()
        rn, rJ = O.deposit(cfg, O.particles64(parts), back)
        na, Ja = n_a.cpu().numpy(), J_a.cpu().numpy()
        assert rel_l2(na, n_b.cpu().numpy()) < 1e-5 and rel_l2(Ja, J_b.cpu().numpy()) < 1e-5
        assert rel_l2(na, rn) < 1e-5 and rel_l2(Ja, rJ) < 1e-5


def test_noalloc_deposit_limits(H):
    """A grid above the scratch's cell limit is refused before any launch;
    bad arguments are refused as for the other entry points; an empty store
    gives zero moments."""
    big = _cfg(2, 1025, 1024, 1)
    assert big.ncell > H.NOALLOC_MAX_CELLS
    p = H.Particles(2, 4)
    n = torch.full((big.ncell,), 3.0, device="cuda")
    J = torch.full((3, big.ncell), 3.0, device="cuda")
    with pytest.raises(H.HvpicError, match="out of memory"):
        H.hvpic_deposit_noalloc(H.params_from(big, 4), None, p, 0.0, n, J)
    torch.cuda.synchronize()
    assert float(n.min()) == 3.0  # nothing was launched
    small = _cfg(2, 5, 4, 1)
    bad = H.params_from(small, 4)
    bad.dx = -1.0
    n = torch.full((small.ncell,), 3.0, device="cuda")
    J = torch.full((3, small.ncell), 3.0, device="cuda")
    with pytest.raises(H.HvpicError, match="invalid"):
        H.hvpic_deposit_noalloc(bad, None, p, 0.0, n, J)
    H.hvpic_deposit_noalloc(H.params_from(small, 4), None, p, 0.0, n, J)
    torch.cuda.synchronize()
    assert float(n.abs().max()) == 0.0 and float(J.abs().max()) == 0.0
