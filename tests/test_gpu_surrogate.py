"""GPU tests of the neural-operator surrogate (hvpic_no_*, hvpic_field_advance_no)
against the FP64 oracle of oracle/no_oracle.py.

Layer kernels take BF16 inputs and weights and accumulate in FP32, so they
are compared element by element with the FP64 convolution of the same
BF16 values: an FP32 output within 1e-5 of the output's scale, a BF16
output within one BF16 rounding (2^-8 relative) plus that.  The whole
network is compared with the FP64 network that rounds its inputs, weights
and activations to BF16 at the same points: only a rounding that falls the
other way of a BF16 tie can differ, so the bound is 1e-3 relative L2 on the
increment (measured 4e-6; a wrong layout or tap gives O(1)).
"""
import numpy as np
import pytest

import oracle as O
from oracle import no_oracle as NO
from paper_2305_05600_amd import workloads as W
from tests.helpers import announce, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_05600_amd import hvpic, sim

    hvpic.lib()
    return hvpic, sim


def _bf16_bits(a):
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def _from_bits(h):
    return (np.asarray(h, np.uint32) << 16).view(np.float32).astype(np.float64)


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).cuda()


def _to_chw(x, nimg, ny, nx):
    """[N][C] pixel-major -> [nimg][C][ny][nx]"""
    C = x.shape[1]
    return x.reshape(nimg, ny, nx, C).transpose(0, 3, 1, 2)


GRIDS = [(2, 13, 21), (1, 1, 6), (3, 2, 5), (1, 33, 17)]


@pytest.mark.parametrize("nimg,ny,nx", GRIDS)
@pytest.mark.parametrize("cinp,coutp,mode", [(16, 32, 0), (32, 32, 0), (32, 16, 1), (16, 32, 2),
                                             (32, 32, 2)])
def test_conv_layer(mods, nimg, ny, nx, cinp, coutp, mode):
    H, S = mods
    announce("no_conv", nimg, ny, nx, cinp, coutp, mode)
    rng = np.random.default_rng(cinp * 7 + coutp + mode + nx)
    N = nimg * ny * nx
    xb = _bf16_bits(rng.normal(size=(N, cinp)))
    wb = _bf16_bits(rng.normal(scale=0.3, size=(coutp, 9, cinp)))
    bias = rng.normal(scale=0.1, size=coutp).astype(np.float32)
    hb = _bf16_bits(rng.uniform(-0.9, 0.9, size=(N, coutp)))
    out = torch.zeros((N, coutp), dtype=torch.float32 if mode == 1 else torch.int16,
                      device="cuda")
    H.hvpic_no_conv3x3(nimg, nx, ny, cinp, coutp, mode, _dev(xb.view(np.int16), np.int16),
                       _dev(wb.view(np.int16), np.int16), _dev(bias, np.float32),
                       _dev(hb.view(np.int16), np.int16), out)
    torch.cuda.synchronize()
    x = _to_chw(_from_bits(xb), nimg, ny, nx)
    w = _from_bits(wb)
    ref = np.stack([NO.conv3x3(x[i], w, np.zeros(coutp) if mode == 2 else bias)
                    for i in range(nimg)])                      # [nimg][O][ny][nx]
    ref = ref.transpose(0, 2, 3, 1).reshape(N, coutp)
    if mode == 0:
        ref = np.tanh(ref)
    elif mode == 2:
        h = _from_bits(hb)
        ref = ref * (1.0 - h * h)
    if mode == 1:
        got = out.cpu().numpy().astype(np.float64)
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-5 * scale
    else:
        got = _from_bits(out.cpu().numpy().view(np.uint16))
        scale = np.abs(ref).max()
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * scale)


@pytest.mark.parametrize("nimg,ny,nx", GRIDS)
@pytest.mark.parametrize("cinp,coutp", [(32, 16), (32, 32), (16, 32)])
def test_weight_gradient(mods, nimg, ny, nx, cinp, coutp):
    H, S = mods
    announce("no_wgrad", nimg, ny, nx, cinp, coutp)
    rng = np.random.default_rng(cinp + 3 * coutp + nx)
    N = nimg * ny * nx
    xb = _bf16_bits(rng.normal(size=(N, cinp)))
    zb = _bf16_bits(rng.normal(size=(N, coutp)))
    dw = torch.full((coutp, 9, cinp), 0.5, dtype=torch.float32, device="cuda")  # added to
    db = torch.full((coutp,), 0.25, dtype=torch.float32, device="cuda")
    ws = torch.empty(H.hvpic_no_workspace_bytes(nx, ny, nimg), dtype=torch.uint8, device="cuda")
    H.hvpic_no_conv3x3_wgrad(nimg, nx, ny, cinp, coutp, _dev(xb.view(np.int16), np.int16),
                             _dev(zb.view(np.int16), np.int16), dw, db, ws)
    torch.cuda.synchronize()
    x = _to_chw(_from_bits(xb), nimg, ny, nx)
    z = _to_chw(_from_bits(zb), nimg, ny, nx)
    ref = np.zeros((coutp, 9, cinp))
    for i in range(nimg):
        for t in range(9):
            dy, dx = t // 3 - 1, t % 3 - 1
            xs = np.roll(np.roll(x[i], -dy, axis=1), -dx, axis=2)
            ref[:, t, :] += np.einsum("ohw,chw->oc", z[i], xs)
    assert rel_l2(dw.cpu().numpy() - 0.5, ref) < 1e-5
    assert np.allclose(db.cpu().numpy() - 0.25, z.sum(axis=(0, 2, 3)), rtol=1e-5, atol=1e-4)


def _random_state(rng, ny, nx):
    P = ny * nx
    B = rng.normal(size=(3, P)) * 0.2 + np.array([[1.0], [0.0], [0.0]])
    n = rng.uniform(0.5, 1.5, P)
    J = rng.normal(scale=0.3, size=(3, P))
    return B.astype(np.float32), n.astype(np.float32), J.astype(np.float32)


def _norm(rng):
    return (rng.normal(scale=0.1, size=7), rng.uniform(0.5, 2.0, 7), rng.uniform(0.005, 0.02, 3))


def test_network_forward(mods):
    H, S = mods
    announce("no_forward")
    rng = np.random.default_rng(11)
    ny, nx = 24, 40
    surr = S.Surrogate(nx, ny, batch=2)
    params = NO.init_params(3)
    params = [(w, rng.normal(scale=0.05, size=b.shape)) for w, b in params]
    norm = _norm(rng)
    surr.load(params, norm)
    back = surr.weights()
    for (w0, b0), (w1, b1) in zip(params, back):  # FP32 master copies
        assert np.allclose(w1, w0.astype(np.float32)) and np.allclose(b1, b0.astype(np.float32))
    B, n, J = _random_state(rng, ny, nx)
    got = surr.predict(_dev(B, np.float32), _dev(n, np.float32), _dev(J, np.float32))
    torch.cuda.synchronize()
    ref = NO.predict(params, norm, B, n, J, (ny, nx), round_bf16=True).reshape(3, -1)
    inc_g = (got.cpu().numpy() - B) / norm[2][:, None]
    inc_r = (ref - B) / norm[2][:, None]
    err = rel_l2(inc_g, inc_r)
    print(f"network forward: increment rel L2 {err:.2e}", flush=True)
    assert err < 1e-3


def test_train_step_against_oracle_gradients(mods):
    """One Adam step from zero moments moves every weight by -lr * sign(g)
    (|g| >> eps): the signs of the GPU's gradients against the oracle's, and
    the loss."""
    H, S = mods
    announce("no_train_grad")
    rng = np.random.default_rng(12)
    ny, nx, K = 16, 20, 3
    surr = S.Surrogate(nx, ny, batch=K)
    params = NO.init_params(5)
    params = [(w, rng.normal(scale=0.05, size=b.shape)) for w, b in params]
    norm = _norm(rng)
    surr.load(params, norm)
    data = [_random_state(rng, ny, nx) for _ in range(K)]
    Bt = [d[0] + (0.01 * rng.normal(size=d[0].shape)).astype(np.float32) for d in data]
    dB = _dev(np.stack([d[0] for d in data]), np.float32)
    dn = _dev(np.stack([d[1] for d in data]), np.float32)
    dJ = _dev(np.stack([d[2] for d in data]), np.float32)
    dBt = _dev(np.stack(Bt), np.float32)
    idx = torch.arange(K, dtype=torch.int32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    lr = 1e-3
    H.hvpic_no_train_step(surr.params, surr.ws_train, nx, ny, dB, dn, dJ, dBt, idx, lr, loss)
    torch.cuda.synchronize()
    new = surr.weights()
    ref_loss, grads = NO.loss_and_grads(params, norm, [(d[0], d[1], d[2], t) for d, t in
                                                        zip(data, Bt)], (ny, nx))
    print(f"loss gpu {float(loss[0]):.6e} oracle {ref_loss:.6e}", flush=True)
    assert float(loss[0]) == pytest.approx(ref_loss, rel=2e-2)
    agree = total = 0
    for (w0, b0), (w1, b1), (gw, gb) in zip(params, new, grads):
        for p0, p1, g in ((w0, w1, gw), (b0, b1, gb)):
            big = np.abs(g) > 1e-2 * np.abs(g).max()
            step = (p1 - p0.astype(np.float32))[big]
            agree += int(np.sum(np.sign(step) == -np.sign(g[big])))
            total += int(big.sum())
            assert np.all(np.abs(step) <= 1.01 * lr + 1e-7)
    print(f"gradient signs: {agree} of {total} agree", flush=True)
    assert agree >= 0.98 * total


def test_training_reduces_the_loss(mods):
    H, S = mods
    announce("no_training")
    rng = np.random.default_rng(13)
    ny, nx, K = 16, 16, 12
    surr = S.Surrogate(nx, ny, batch=4)
    surr.load(NO.init_params(9), _norm(rng))
    data = [_random_state(rng, ny, nx) for _ in range(K)]
    # a target the network can represent: a smooth function of the input
    Bt = [d[0] + 0.01 * np.tanh(d[2]).astype(np.float32) for d in data]
    tens = tuple(_dev(np.stack(a), np.float32) for a in
                 ([d[0] for d in data], [d[1] for d in data], [d[2] for d in data], Bt))
    losses = surr.train(tens, steps=150, lr=3e-3, seed=1).cpu().numpy()
    print(f"loss {losses[:3]} ... {losses[-3:]}", flush=True)
    assert losses[-10:].mean() < 0.3 * losses[:10].mean()


def _field_case():
    cfg = W.Config(name="no", ndim=2, nx=37, ny=23, nz=1, dx=0.5, dy=0.3, dz=1.0, dt=0.02,
                   nsub=5, te=0.2, eta=1e-3)
    B = W.random_field(81, cfg, 0.05, (1.0, 0.3, -0.2))
    nh = W.random_density(82, cfg, 0.5, 1.5)
    npv = W.random_density(83, cfg, 0.5, 1.5)
    Jh = W.random_field(84, cfg, 0.2)
    Jp = W.random_field(85, cfg, 0.2)
    return cfg, B, nh, npv, Jh, Jp


@pytest.mark.parametrize("tol", [0.0, 1e30])
def test_field_advance_no_branches(mods, tol):
    """tol = 0: every proposal is rejected and the plain subcycle runs (the
    oracle's field advance); tol = huge: the proposal is taken (B^{n+1} is
    the operator's prediction and E^{n+1} is Ohm's law of it).  The residual
    ratio is the oracle's for the same proposal."""
    H, S = mods
    announce("no_field", tol)
    cfg, B, nh, npv, Jh, Jp = _field_case()
    rng = np.random.default_rng(14)
    surr = S.Surrogate(cfg.nx, cfg.ny, batch=1)
    params = [(w, rng.normal(scale=0.05, size=b.shape)) for w, b in NO.init_params(2)]
    surr.load(params, _norm(rng))
    ctx = H.Context(cfg, 1)
    Bd = _dev(B, np.float32)
    Ed = torch.zeros((3, cfg.ncell), device="cuda")
    diag = torch.zeros(3, dtype=torch.float64, device="cuda")
    stats = torch.zeros(2, dtype=torch.float64, device="cuda")
    prop = surr.predict(Bd.clone(), _dev(nh, np.float32), _dev(Jh, np.float32))
    H.hvpic_field_advance_no(ctx.ctx, surr.params, surr.ws_one, Bd, _dev(nh, np.float32),
                             _dev(Jh, np.float32), _dev(npv, np.float32), _dev(Jp, np.float32),
                             Ed, tol, diag_out=diag, stats=stats)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    ratio = NO.residual(cfg, B, prop.cpu().numpy(), nh, Jh)
    assert st[0] == pytest.approx(ratio, rel=1e-3)
    if tol == 0.0:
        assert st[1] == 0.0
        rB, rE, rd, _ = O.field_advance(cfg, B, nh, Jh, npv, Jp, mode=0)
    else:
        assert st[1] == 1.0
        assert torch.equal(Bd, prop)
        rB = prop.cpu().numpy().astype(np.float64)
        n1 = 1.5 * nh.astype(np.float64) - 0.5 * npv
        J1 = 1.5 * Jh.astype(np.float64) - 0.5 * Jp
        rE = O.ohm(cfg, rB, n1, J1)
    assert rel_l2(Bd.cpu().numpy(), rB) < 1e-5
    assert rel_l2(Ed.cpu().numpy(), rE) < 1e-5


@pytest.mark.parametrize("tol", [0.0, 1e30])
def test_field_advance_no_full_size(mods, tol):
    """The benchmarked grid (the double Harris sheet, 512x256 cells, 10
    subcycles, its B): the operator's forward there against the oracle's
    network on the same BF16-rounded values, and both branches of the
    surrogate's field advance against the oracle (tol = 0: the plain
    subcycle; tol = huge: the proposal and Ohm's law of it)."""
    H, S = mods
    announce("no_field_full", tol)
    cfg, _, B = W.harris_double(ppc=0.01)  # the grid and the field
    B = np.asarray(B, np.float32)
    nh = W.random_density(82, cfg, 0.5, 1.5)
    npv = W.random_density(83, cfg, 0.5, 1.5)
    Jh = W.random_field(84, cfg, 0.2)
    Jp = W.random_field(85, cfg, 0.2)
    rng = np.random.default_rng(21)
    surr = S.Surrogate(cfg.nx, cfg.ny, batch=1)
    params = [(w, rng.normal(scale=0.05, size=b.shape)) for w, b in NO.init_params(4)]
    norm = _norm(rng)
    surr.load(params, norm)
    ctx = H.Context(cfg, 1)
    Bd = _dev(B, np.float32)
    Ed = torch.zeros((3, cfg.ncell), device="cuda")
    diag = torch.zeros(3, dtype=torch.float64, device="cuda")
    stats = torch.zeros(2, dtype=torch.float64, device="cuda")
    prop = surr.predict(Bd.clone(), _dev(nh, np.float32), _dev(Jh, np.float32))
    torch.cuda.synchronize()
    ref = NO.predict(params, norm, B, nh, Jh, (cfg.ny, cfg.nx), round_bf16=True).reshape(3, -1)
    inc_g = (prop.cpu().numpy() - B) / norm[2][:, None]
    inc_r = (ref - B) / norm[2][:, None]
    err = rel_l2(inc_g, inc_r)
    print(f"network forward at {cfg.nx}x{cfg.ny}: increment rel L2 {err:.2e}", flush=True)
    assert err < 1e-3
    H.hvpic_field_advance_no(ctx.ctx, surr.params, surr.ws_one, Bd, _dev(nh, np.float32),
                             _dev(Jh, np.float32), _dev(npv, np.float32), _dev(Jp, np.float32),
                             Ed, tol, diag_out=diag, stats=stats)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    assert st[0] == pytest.approx(NO.residual(cfg, B, prop.cpu().numpy(), nh, Jh), rel=1e-3)
    if tol == 0.0:
        assert st[1] == 0.0
        rB, rE, rd, _ = O.field_advance(cfg, B, nh, Jh, npv, Jp, mode=0)
    else:
        assert st[1] == 1.0
        assert torch.equal(Bd, prop)
        rB = prop.cpu().numpy().astype(np.float64)
        rE = O.ohm(cfg, rB, 1.5 * nh.astype(np.float64) - 0.5 * npv,
                   1.5 * Jh.astype(np.float64) - 0.5 * Jp)
    eB, eE = rel_l2(Bd.cpu().numpy(), rB), rel_l2(Ed.cpu().numpy(), rE)
    print(f"field advance (tol {tol:g}): rel L2 B {eB:.2e}, E {eE:.2e}", flush=True)
    assert eB < 1e-5 and eE < 1e-5
