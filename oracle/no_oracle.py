"""FP64 CPU oracle of the convolutional neural operator that stands in for the
magnetic-field subcycle -- TEST INFRASTRUCTURE (tests, smoke() and the
bench's CPU leg only; shares no code with the GPU library).

The operator maps the state a field advance starts from -- B^n (3 channels),
n^{n+1/2} (1) and J_i^{n+1/2} (3) on the 2D periodic grid -- to B^{n+1}, the
result of the subcycled Faraday/Ohm advance of Sec. II.A:

    x0 = (input - mean) / std                 7 channels, per-channel scales
    h1 = tanh(conv(x0; W1, b1))               7 -> 32
    h2 = tanh(conv(h1; W2, b2))               32 -> 32
    h3 = tanh(conv(h2; W3, b3))               32 -> 32
    d  = conv(h3; W4, b4)                     32 -> 3
    B^{n+1} ~ B^n + out_std * d

conv is the 3x3 cross-correlation with periodic wrap (the grid is a periodic
box): y[o][j][i] = b[o] + sum_{c,t} W[o][t][c] x[c][j+dy(t)][i+dx(t)], with
tap t = 3*(dy+1) + (dx+1).  Weights are stored [out][tap][in], the layout of
the GPU kernels' records.  Training minimises the mean over the batch, the
3 output channels and the cells of (d - (B^{n+1} - B^n)/out_std)^2.

The residual of a proposal B' (the acceptance test of the surrogate step):
    r = (B' - B^n)/dt + curl E(B_mid),  B_mid = (B^n + B')/2,
with E from Ohm's law at the frozen moments n^{n+1/2}, J_i^{n+1/2};
accepted when ||r|| <= tol ||(B' - B^n)/dt||.
"""
from __future__ import annotations

import numpy as np

CIN, HID, COUT = 7, 32, 3
LAYERS = ((CIN, HID), (HID, HID), (HID, HID), (HID, COUT))


def conv3x3(x, w, b):
    """Periodic 3x3 cross-correlation. x [C][H][W], w [O][9][C], b [O] -> [O][H][W]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    out = np.zeros((w.shape[0],) + x.shape[1:])
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        # x shifted so that [j][i] holds x[j+dy][i+dx] (periodic)
        xs = np.roll(np.roll(x, -dy, axis=1), -dx, axis=2)
        out += np.einsum("oc,chw->ohw", w[:, t, :], xs)
    return out + np.asarray(b, np.float64)[:, None, None]


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64: the
    upper 16 bits of the FP32 value after round-to-nearest-even of the lower 16."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def init_params(seed: int):
    """Seeded weights of the four layers (uniform, fan-in scaled) and zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ps = []
    for cin, cout in LAYERS:
        lim = np.sqrt(3.0 / (9 * cin))
        ps.append((rng.uniform(-lim, lim, (cout, 9, cin)), np.zeros(cout)))
    return ps


def pack_input(B, n, J, shape2d):
    """The 7 input channels [7][H][W] from component-major fields."""
    H, W = shape2d
    return np.concatenate([np.asarray(B, np.float64).reshape(3, H, W),
                           np.asarray(n, np.float64).reshape(1, H, W),
                           np.asarray(J, np.float64).reshape(3, H, W)])


def forward(params, x0, round_bf16=False):
    """The network on normalised input x0 [7][H][W]; returns (d, activations).
    round_bf16: round the inputs of every layer and the weights to bfloat16,
    as the GPU stores them (the accumulation stays FP64)."""
    r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    acts = [r(x0)]
    h = acts[0]
    for li, (w, b) in enumerate(params):
        z = conv3x3(h, r(w), b)
        h = z if li == len(params) - 1 else np.tanh(z)
        if li < len(params) - 1:
            h = r(h)
            acts.append(h)
    return h, acts


def predict(params, norm, B, n, J, shape2d, round_bf16=False):
    """B^{n+1} proposed by the operator; norm = (mean[7], std[7], out_std[3])."""
    mean, std, out_std = (np.asarray(a, np.float64) for a in norm)
    x = pack_input(B, n, J, shape2d)
    x0 = (x - mean[:, None, None]) / std[:, None, None]
    d, _ = forward(params, x0, round_bf16)
    H, W = shape2d
    return np.asarray(B, np.float64).reshape(3, H, W) + out_std[:, None, None] * d


def loss_and_grads(params, norm, batch, shape2d):
    """Mean-square loss of the normalised increment over a batch of
    (B, n, J, B_target) and its gradients (FP64, by reverse-mode automatic
    differentiation of the forward written above with torch ops)."""
    import torch

    mean, std, out_std = (torch.tensor(np.asarray(a, np.float64)) for a in norm)
    ws = [torch.tensor(w, requires_grad=True) for w, _ in params]
    bs = [torch.tensor(b, requires_grad=True) for _, b in params]
    H, W = shape2d
    total = 0.0
    count = 0
    for B, n, J, Bt in batch:
        x = torch.tensor(pack_input(B, n, J, shape2d))
        h = (x - mean[:, None, None]) / std[:, None, None]
        for li in range(len(ws)):
            out = bs[li][:, None, None].clone().expand(-1, H, W).clone()
            for t in range(9):
                dy, dx = t // 3 - 1, t % 3 - 1
                xs = torch.roll(h, shifts=(-dy, -dx), dims=(1, 2))
                out = out + torch.einsum("oc,chw->ohw", ws[li][:, t, :], xs)
            h = out if li == len(ws) - 1 else torch.tanh(out)
        tgt = (torch.tensor(np.asarray(Bt, np.float64).reshape(3, H, W)) -
               torch.tensor(np.asarray(B, np.float64).reshape(3, H, W))) / out_std[:, None, None]
        total = total + ((h - tgt) ** 2).sum()
        count += 3 * H * W
    loss = total / count
    loss.backward()
    return float(loss.detach()), [(w.grad.numpy(), b.grad.numpy()) for w, b in zip(ws, bs)]


def adam(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected; returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for (w, b), (gw, gb), (mw, mb), (vw, vb) in zip(params, grads, m, v):
        new = []
        for p, g, mm, vv in ((w, gw, mw, vw), (b, gb, mb, vb)):
            mm = beta1 * mm + (1 - beta1) * g
            vv = beta2 * vv + (1 - beta2) * g * g
            mh = mm / (1 - beta1 ** step)
            vh = vv / (1 - beta2 ** step)
            new.append((p - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        out_p.append((new[0][0], new[1][0]))
        out_m.append((new[0][1], new[1][1]))
        out_v.append((new[0][2], new[1][2]))
    return out_p, out_m, out_v


def residual(cfg, B0, B1, n_half, J_half):
    """||r|| / ||(B1 - B0)/dt|| of a proposal B1 (the surrogate's acceptance
    test), r = (B1 - B0)/dt + curl E(B_mid) with E from Ohm's law at the
    frozen moments; uses the step oracle's Ohm's law and curl."""
    import oracle as O

    B0 = np.asarray(B0, np.float64)
    B1 = np.asarray(B1, np.float64)
    rate = (B1 - B0) / cfg.dt
    E = O.ohm(cfg, 0.5 * (B0 + B1), n_half, J_half)
    r = rate + O.curl(cfg, E)
    return float(np.linalg.norm(r) / max(np.linalg.norm(rate), 1e-300))
