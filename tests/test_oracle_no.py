"""Pins of the neural-operator oracle (oracle/no_oracle.py) against what
does not depend on it: a brute-force loop convolution, the library's circular
convolution, a delta input (the output is the stencil itself), finite
differences of the loss, the bfloat16 rounding rule on hand-picked values,
and the Adam update's first step (|update| = lr for every nonzero gradient)."""
import numpy as np
import pytest

from oracle import no_oracle as NO


def _brute(x, w, b):
    C, H, W = x.shape
    O = w.shape[0]
    y = np.zeros((O, H, W))
    for o in range(O):
        for j in range(H):
            for i in range(W):
                s = b[o]
                for c in range(C):
                    for t in range(9):
                        dy, dx = t // 3 - 1, t % 3 - 1
                        s += w[o, t, c] * x[c, (j + dy) % H, (i + dx) % W]
                y[o, j, i] = s
    return y


def test_conv_matches_brute_force_on_odd_grids():
    rng = np.random.default_rng(1)
    for H, W in ((5, 4), (3, 7), (1, 6), (2, 2)):
        x = rng.normal(size=(3, H, W))
        w = rng.normal(size=(4, 9, 3))
        b = rng.normal(size=4)
        assert np.allclose(NO.conv3x3(x, w, b), _brute(x, w, b), rtol=1e-13, atol=1e-13)


def test_conv_matches_the_library_circular_convolution():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    x = rng.normal(size=(5, 9, 11))
    w = rng.normal(size=(6, 9, 5))
    b = rng.normal(size=6)
    # torch's conv2d is a cross-correlation: weight [O][C][ky][kx] with
    # tap t = 3 ky + kx reading x[j + ky - 1][i + kx - 1]
    wt = torch.tensor(w.reshape(6, 3, 3, 5).transpose(0, 3, 1, 2))
    xp = torch.nn.functional.pad(torch.tensor(x)[None], (1, 1, 1, 1), mode="circular")
    ref = torch.nn.functional.conv2d(xp, wt, torch.tensor(b))[0].numpy()
    assert np.allclose(NO.conv3x3(x, w, b), ref, rtol=1e-12, atol=1e-12)


def test_delta_input_reproduces_the_stencil():
    """x = delta at (j0, i0): y[o][j0-dy][i0-dx] = W[o][t][c] for tap (dy, dx)."""
    H, W = 6, 7
    rng = np.random.default_rng(3)
    w = rng.normal(size=(2, 9, 1))
    x = np.zeros((1, H, W))
    j0, i0 = 2, 0
    x[0, j0, i0] = 1.0
    y = NO.conv3x3(x, w, np.zeros(2))
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        assert np.allclose(y[:, (j0 - dy) % H, (i0 - dx) % W], w[:, t, 0])
    assert np.count_nonzero(np.abs(y) > 0) == 2 * 9


def test_bf16_rounding_rule():
    one = 1.0
    ulp = 2.0 ** -7  # bf16 spacing in [1, 2)
    vals = np.array([one, one + ulp / 2, one + 1.5 * ulp, one + ulp / 4, -3.0, 0.0])
    got = NO.bf16(vals)
    # ties go to the even neighbour: 1 + ulp/2 -> 1, 1 + 1.5 ulp -> 1 + 2 ulp
    assert got.tolist() == [1.0, 1.0, one + 2 * ulp, 1.0, -3.0, 0.0]
    assert np.all(np.abs(NO.bf16(np.linspace(-5, 5, 101)) - np.linspace(-5, 5, 101))
                  <= 2.0 ** -8 * np.abs(np.linspace(-5, 5, 101)) + 1e-30)


def _batch(rng, H, W, k=2):
    out = []
    for _ in range(k):
        B = rng.normal(size=(3, H * W))
        n = rng.uniform(0.5, 1.5, H * W)
        J = rng.normal(size=(3, H * W))
        Bt = B + 0.01 * rng.normal(size=(3, H * W))
        out.append((B, n, J, Bt))
    return out


def test_loss_gradients_match_finite_differences():
    pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    H, W = 4, 5
    params = NO.init_params(7)
    params = [(w, rng.normal(scale=0.1, size=b.shape)) for w, b in params]
    norm = (rng.normal(size=7), rng.uniform(0.5, 2.0, 7), rng.uniform(0.01, 0.1, 3))
    batch = _batch(rng, H, W)
    loss, grads = NO.loss_and_grads(params, norm, batch, (H, W))

    def loss_of(ps):
        tot, cnt = 0.0, 0
        mean, std, out_std = norm
        for B, n, J, Bt in batch:
            x0 = (NO.pack_input(B, n, J, (H, W)) - mean[:, None, None]) / std[:, None, None]
            d, _ = NO.forward(ps, x0)
            tgt = (Bt - B).reshape(3, H, W) / out_std[:, None, None]
            tot += ((d - tgt) ** 2).sum()
            cnt += 3 * H * W
        return tot / cnt

    assert loss == pytest.approx(loss_of(params), rel=1e-12)
    h = 1e-6
    for li, idx in ((0, (3, 4, 2)), (1, (10, 0, 31)), (2, (5, 8, 7)), (3, (2, 4, 16))):
        ps = [(w.copy(), b.copy()) for w, b in params]
        ps[li][0][idx] += h
        up = loss_of(ps)
        ps[li][0][idx] -= 2 * h
        dn = loss_of(ps)
        assert grads[li][0][idx] == pytest.approx((up - dn) / (2 * h), rel=1e-5, abs=1e-10)
    for li, o in ((0, 5), (3, 1)):
        ps = [(w.copy(), b.copy()) for w, b in params]
        ps[li][1][o] += h
        up = loss_of(ps)
        ps[li][1][o] -= 2 * h
        dn = loss_of(ps)
        assert grads[li][1][o] == pytest.approx((up - dn) / (2 * h), rel=1e-5, abs=1e-10)


def test_adam_first_step_moves_each_weight_by_lr():
    rng = np.random.default_rng(5)
    params = NO.init_params(1)
    grads = [(rng.normal(size=w.shape), rng.normal(size=b.shape)) for w, b in params]
    zeros = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    new, m, v = NO.adam(params, grads, zeros, zeros, step=1, lr=1e-3, eps=0.0)
    for (w0, b0), (w1, b1), (gw, gb) in zip(params, new, grads):
        assert np.allclose(w1 - w0, -1e-3 * np.sign(gw), rtol=1e-12, atol=1e-15)
        assert np.allclose(b1 - b0, -1e-3 * np.sign(gb), rtol=1e-12, atol=1e-15)
