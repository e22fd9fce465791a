"""CPU FP64 oracle of the warm-start network (test infrastructure only).

The learned warm start maps the two marginals of a grid problem to dual
potentials; their c-transform then selects the initial support (the
initial-support rule of Section 3.2, end, fed with predicted duals instead of
the costs alone).  The network is small and fixed:

    layer  in -> out  kernel  dilation  activation
      1     2 ->  32   3x3       1        ReLU
      2    32 ->  32   3x3       2        ReLU
      3    32 ->  32   3x3       4        ReLU
      4    32 ->   2   3x3       8        none

with zero padding equal to the dilation (output size = input size).  Flat
parameter layout: for each layer, W[out][in][ky][kx] then b[out].

Everything here is a plain definition: a convolution written as a sum over
its nine taps, its gradient written from that sum, the mean-squared error, and
Adam (Kingma & Ba, 2015).  Pins (tests/test_cnn_oracle.py): single-channel
convolutions against scipy.signal.correlate2d with the dilated kernel, every
analytic gradient against central finite differences, mass preservation and
identities of the resampling maps.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(2, 32, 1, True), (32, 32, 2, True), (32, 32, 4, True), (32, 2, 8, False)]
GRID = 32   # side of the grid the network is trained on


def param_count() -> int:
    return sum(co * ci * 9 + co for ci, co, _, _ in LAYERS)


def unpack(theta: np.ndarray):
    """Split the flat parameter vector into [(W, b), ...]."""
    out, off = [], 0
    for ci, co, _, _ in LAYERS:
        W = theta[off:off + co * ci * 9].reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = theta[off:off + co]
        off += co
        out.append((W, b))
    assert off == theta.size
    return out


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights (fan-in = 9 * in channels), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co, _, _ in LAYERS:
        lim = np.sqrt(6.0 / (9 * ci))
        parts.append(rng.uniform(-lim, lim, co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def _shifted(x: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """s[..., y, x] = x[..., y + dy, x + dx], zero outside the image."""
    H, W = x.shape[-2:]
    s = np.zeros_like(x)
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    if ys < ye and xs < xe:
        s[..., ys:ye, xs:xe] = x[..., ys + dy:ye + dy, xs + dx:xe + dx]
    return s


def conv2d(x: np.ndarray, W: np.ndarray, b: np.ndarray, dil: int) -> np.ndarray:
    """out[n,o,y,x] = b[o] + sum_{c,ky,kx} W[o,c,ky,kx] x[n,c,y+(ky-1)dil,x+(kx-1)dil]."""
    out = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:])
    for ky in range(3):
        for kx in range(3):
            s = _shifted(x, (ky - 1) * dil, (kx - 1) * dil)
            out += np.einsum("nchw,oc->nohw", s, W[:, :, ky, kx])
    return out + b[None, :, None, None]


def forward(theta: np.ndarray, x: np.ndarray):
    """Activations [x, a1, a2, a3, out] (post-ReLU for the hidden layers)."""
    acts = [np.asarray(x, np.float64)]
    for (W, b), (_, _, dil, relu) in zip(unpack(theta), LAYERS):
        z = conv2d(acts[-1], W, b, dil)
        acts.append(np.maximum(z, 0.0) if relu else z)
    return acts


def mse(out: np.ndarray, target: np.ndarray) -> float:
    return float(np.mean((out - target) ** 2))


def grad(theta: np.ndarray, x: np.ndarray, target: np.ndarray):
    """(loss, d loss / d theta) of the mean-squared error, by the chain rule
    through each convolution's tap sum."""
    acts = forward(theta, x)
    out = acts[-1]
    loss = mse(out, target)
    g = 2.0 * (out - target) / out.size            # d loss / d out
    grads = []
    params = unpack(theta)
    for li in range(len(LAYERS) - 1, -1, -1):
        W, b = params[li]
        dil = LAYERS[li][2]
        xin = acts[li]
        gW = np.zeros_like(W)
        gx = np.zeros_like(xin)
        for ky in range(3):
            for kx in range(3):
                dy, dx = (ky - 1) * dil, (kx - 1) * dil
                s = _shifted(xin, dy, dx)
                gW[:, :, ky, kx] = np.einsum("nohw,nchw->oc", g, s)
                # x[n,c,y+dy,x+dx] received W[o,c,ky,kx] g[n,o,y,x]
                gx += _shifted(np.einsum("nohw,oc->nchw", g, W[:, :, ky, kx]), -dy, -dx)
        gb = g.sum(axis=(0, 2, 3))
        grads.append((gW, gb))
        if li > 0:
            g = gx * (xin > 0.0)                  # through the ReLU that produced xin
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])
    return loss, flat


def adam(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- grid maps
def _overlap(side: int, grid: int):
    """R[t, u] = |cell t of the grid-cell partition of [0,1] intersected with
    cell u of the side-cell partition| / |cell t|."""
    R = np.zeros((grid, side))
    for t in range(grid):
        t0, t1 = t / grid, (t + 1) / grid
        for u in range(side):
            u0, u1 = u / side, (u + 1) / side
            R[t, u] = max(0.0, min(t1, u1) - max(t0, u0)) * grid
    return R


def network_input(a: np.ndarray, b: np.ndarray, side: int, grid: int = GRID) -> np.ndarray:
    """(2, grid, grid) input: each marginal as a density (mass * side^2 per
    pixel), averaged over the cells of a grid x grid partition of the square."""
    R = _overlap(side, grid)
    out = []
    for h in (a, b):
        d = np.asarray(h, np.float64).reshape(side, side) * side * side
        out.append(R @ d @ R.T)
    return np.stack(out)


def upsample_duals(out2: np.ndarray, side: int, grid: int = GRID):
    """Duals on the side x side grid in cost units of pixel coordinates: the
    network's (normalised-coordinate) output bilinearly interpolated at pixel
    centres, clamped at the border, times side^2."""
    t = (np.arange(side) + 0.5) * grid / side - 0.5
    t = np.clip(t, 0.0, grid - 1.0)
    i0 = np.floor(t).astype(int)
    i1 = np.minimum(i0 + 1, grid - 1)
    f = t - i0
    res = []
    for ch in range(2):
        P = np.asarray(out2[ch], np.float64)
        rows = P[i0, :] * (1 - f)[:, None] + P[i1, :] * f[:, None]
        full = rows[:, i0] * (1 - f)[None, :] + rows[:, i1] * f[None, :]
        res.append(full.reshape(-1) * side * side)
    return res[0], res[1]


def predict_duals(theta: np.ndarray, a, b, side: int):
    x = network_input(a, b, side)[None]
    out = forward(theta, x)[-1][0]
    return upsample_duals(out, side)


def dual_targets(y: np.ndarray, z: np.ndarray, side: int) -> np.ndarray:
    """Training target of optimal duals (pixel cost units): shift to the gauge
    mean(y) = mean(z) and divide by side^2 (normalised coordinates)."""
    t = 0.5 * (np.mean(z) - np.mean(y))
    return np.stack([(y + t).reshape(side, side), (z - t).reshape(side, side)]) / (side * side)
