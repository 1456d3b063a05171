"""Learned k-space completion network (oracle): the network's arithmetic in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Nothing here is used by the product
path; the tests feed the same inputs and weights to both sides.

One temporal-frequency bin k of the Eq. 3 decomposition gives a complex grid over
(transmit angle theta_i, receive angle theta_o) pairs: every pair is one k-space sample
(Sec. II-B: k_x = nu (sin th_o - sin th_i) / c).  Compressive sampling observes only some
receive columns of a uniform receive bank; the network predicts the rest.

Grids are channel-last: x[b][h][w][c] with b the sample (one bin of one frame), h the
transmit angle, w the receive angle of the bank, c the channel.

  sample input   c = 0, 1: Re, Im of the observed pairs divided by the bin's scale, 0 where
                 unobserved; c = 2: 1 where observed.  scale = root mean square of the
                 observed pairs' moduli.  Target: Re, Im of the full grid / scale.
  conv3x3        y[b][h][w][o] = bias[o] + sum_{t, c} W[t][o][c] x[b][h+dy*eh][w+dx*ew][c], with
                 t = 3 (dy + 1) + (dx + 1), dy, dx in {-1, 0, 1}, dilation (eh, ew) >= 1,
                 x = 0 outside the grid
  network        a_0 = input; a_l = relu(conv_l(a_{l-1})), l = 1..L-1; out = conv_L(a_{L-1})
  loss           mean over unobserved positions and both components of (out - target)^2
  completion     observed pairs keep their values; unobserved take out * scale
  Adam           m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
                 p = p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shifted(x: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """s[b][h][w][c] = x[b][h+dy][w+dx][c], zero outside the grid."""
    B, H, W, C = x.shape
    out = np.zeros_like(x)
    h0, h1 = max(0, -dy), min(H, H - dy)
    w0, w1 = max(0, -dx), min(W, W - dx)
    out[:, h0:h1, w0:w1, :] = x[:, h0 + dy:h1 + dy, w0 + dx:w1 + dx, :]
    return out


def conv3x3(x: np.ndarray, W: np.ndarray, bias: np.ndarray, dil=(1, 1)) -> np.ndarray:
    """x [B][H][W][Ci], W [9][Co][Ci], bias [Co], dilation (eh, ew) -> y [B][H][W][Co] (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros(x.shape[:3] + (W.shape[1],), dtype=np.float64)
    for t, (dy, dx) in enumerate(TAPS):
        y += _shifted(x, dy * dil[0], dx * dil[1]) @ np.asarray(W[t], dtype=np.float64).T
    return y + np.asarray(bias, dtype=np.float64)


def conv3x3_backward(x: np.ndarray, W: np.ndarray, gy: np.ndarray, dil=(1, 1)):
    """Gradients of sum(gy * conv3x3(x, W, b, dil)): (gx [B][H][W][Ci], gW [9][Co][Ci], gb [Co])."""
    x = np.asarray(x, dtype=np.float64)
    gy = np.asarray(gy, dtype=np.float64)
    gW = np.zeros(W.shape, dtype=np.float64)
    gx = np.zeros(x.shape, dtype=np.float64)
    for t, (dy, dx) in enumerate(TAPS):
        sy, sx = dy * dil[0], dx * dil[1]
        xs = _shifted(x, sy, sx)
        gW[t] = np.einsum("bhwo,bhwc->oc", gy, xs)
        # y[h][w] took x[h+sy][w+sx]: its gradient flows back to that position
        gx += _shifted(gy @ np.asarray(W[t], dtype=np.float64), -sy, -sx)
    return gx, gW, gy.sum(axis=(0, 1, 2))


def forward(x: np.ndarray, params, dils=None):
    """params: list of (W, bias) per layer, dils: (eh, ew) per layer (default 1).  Returns
    (out, activations a_0..a_{L-1})."""
    dils = dils or [(1, 1)] * len(params)
    acts = [np.asarray(x, dtype=np.float64)]
    a = acts[0]
    for l, (W, b) in enumerate(params):
        z = conv3x3(a, W, b, dils[l])
        if l < len(params) - 1:
            a = np.maximum(z, 0.0)
            acts.append(a)
        else:
            return z, acts
    raise ValueError("empty network")


def backward(params, acts, gout, dils=None):
    """Gradients [(gW, gb)] per layer of sum(gout * out), from forward's activations."""
    dils = dils or [(1, 1)] * len(params)
    grads = [None] * len(params)
    g = np.asarray(gout, dtype=np.float64)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        if l < len(params) - 1:
            g = g * (acts[l + 1] > 0)          # relu: a_{l+1} = relu(z_{l+1}) > 0 exactly where z > 0
        gx, gW, gb = conv3x3_backward(acts[l], W, g, dils[l])
        grads[l] = (gW, gb)
        g = gx
    return grads


def masked_mse(out: np.ndarray, target: np.ndarray, observed: np.ndarray):
    """out, target [B][H][W][2]; observed [B][H][W] (1/0).  Returns (loss, d loss / d out)."""
    u = (1.0 - np.asarray(observed, dtype=np.float64))[..., None]
    n = 2.0 * float(u.sum())
    d = np.asarray(out, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    if n == 0:
        return 0.0, np.zeros_like(d)
    return float((u * d * d).sum() / n), 2.0 * u * d / n


def adam(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step count t >= 1).  Returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def prepare(grid: np.ndarray, cols) -> tuple:
    """grid complex [H][W] (one bin, fully sampled), cols: observed receive columns.
    Returns (input [H][W][3], target [H][W][2], observed [H][W], scale)."""
    H, W = grid.shape
    obs = np.zeros((H, W))
    obs[:, list(cols)] = 1.0
    vals = grid[:, list(cols)]
    scale = float(np.sqrt(np.mean(np.abs(vals) ** 2)))
    if scale == 0.0:
        scale = 1.0
    g = grid / scale
    inp = np.zeros((H, W, 3))
    inp[..., 0] = g.real * obs
    inp[..., 1] = g.imag * obs
    inp[..., 2] = obs
    tgt = np.stack([g.real, g.imag], axis=-1)
    return inp, tgt, obs, scale


def merge(observed_grid: np.ndarray, out: np.ndarray, observed: np.ndarray, scale: float) -> np.ndarray:
    """Completed complex grid: observed pairs as given, the rest out * scale."""
    pred = (out[..., 0] + 1j * out[..., 1]) * scale
    return np.where(observed > 0, observed_grid, pred)
