"""Float64 oracle of the learned preconditioner (an extension of the method:
the paper solves the Gauss-Newton systems with plain CG, Sec. 2.3.1).

TEST INFRASTRUCTURE ONLY (see the package header).

Definitions computed here, written out plainly:

* 3x3x3 convolution with zero padding on a node grid, channels last:
  y[z, y, x, o] = b[o] + sum_t sum_c W[t, c, o] x[z + dz_t, y + dy_t, x + dx_t, c]
  with the 27 taps t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1), x = 0 outside.
  Its derivatives follow from the chain rule: db = sum_n dy[n],
  dW[t, c, o] = sum_n x[n + off_t, c] dy[n, o],
  dx[m, c] = sum_t sum_o W[t, c, o] dy[m - off_t, o].
* The network: four such layers, ReLU after the first three.
* The preconditioner: y = D^-1 r (Jacobi), z = y + rms(y) * CNN(features)[:3],
  features = RMS-normalised (y, r, diag, |grad R| on the nodes), zero-padded
  to 16 channels.
* The training loss: the A-norm energy of the residual equation at the best
  step along z, relative to the same quantity for the Jacobi direction:
  L(z) = -((z.r)^2 / (z.Az)) / ((y.r)^2 / (y.Ay));  -1 for z = y.
* bfloat16 rounding (round to nearest, ties to even) for modelling the
  network's 16-bit activations.
"""
from __future__ import annotations

import numpy as np

CH = 16          # channels of every layer (inputs and outputs zero-padded)
LAYERS = 4
IN_USED = 10     # y (3), r (3), diag (3), |grad R| (1)
OUT_USED = 3

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shifted(a, dz, dy, dx):
    """b[z, y, x] = a[z + dz, y + dy, x + dx], zero outside (leading 3 axes)."""
    nz, ny, nx = a.shape[:3]
    out = np.zeros_like(a)
    zs, ys, xs = (slice(max(0, -d), n - max(0, d)) for d, n in ((dz, nz), (dy, ny), (dx, nx)))
    zt, yt, xt = (slice(max(0, d), n - max(0, -d)) for d, n in ((dz, nz), (dy, ny), (dx, nx)))
    out[zs, ys, xs] = a[zt, yt, xt]
    return out


def conv3d(x, W, b):
    """x [nz, ny, nx, Cin], W [27, Cin, Cout], b [Cout] -> y [nz, ny, nx, Cout]."""
    x = np.asarray(x, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    y = np.zeros(x.shape[:3] + (W.shape[2],)) + np.asarray(b, dtype=np.float64)
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += _shifted(x, dz, dy, dx) @ W[t]
    return y


def conv3d_backward(x, W, dy):
    """(dx, dW, db) of sum(dy * conv3d(x, W, b)) with respect to x, W, b."""
    x = np.asarray(x, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    db = dy.reshape(-1, dy.shape[-1]).sum(axis=0)
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    flat = lambda a: a.reshape(-1, a.shape[-1])
    for t, (dz, dyy, dxx) in enumerate(TAPS):
        dW[t] = flat(_shifted(x, dz, dyy, dxx)).T @ flat(dy)
        dx += _shifted(dy, -dz, -dyy, -dxx) @ W[t].T
    return dx, dW, db


def relu(a):
    return np.maximum(a, 0.0)


def bf16_round(a):
    """Nearest bfloat16 value of each float32 (ties to even), as float64."""
    f = np.atleast_1d(np.asarray(a, dtype=np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    out[np.isnan(f)] = np.nan
    return out.reshape(np.shape(a))


def forward(params, h0, round_hidden=False):
    """params: list of LAYERS (W [27, 16, 16], b [16]).  Returns the list of
    activations [h0, h1, h2, h3, o]; hidden activations optionally rounded to
    bfloat16 (as the device network stores them)."""
    acts = [np.asarray(h0, dtype=np.float64)]
    for l, (W, b) in enumerate(params):
        a = conv3d(acts[-1], W, b)
        if l < LAYERS - 1:
            a = relu(a)
            if round_hidden:
                a = bf16_round(a)
        acts.append(a)
    return acts


def backward(params, acts, do):
    """Weight and bias gradients of sum(do * o) through the network."""
    grads = [None] * LAYERS
    g = np.asarray(do, dtype=np.float64)
    for l in range(LAYERS - 1, -1, -1):
        W, _ = params[l]
        dx, dW, db = conv3d_backward(acts[l], W, g)
        grads[l] = (dW, db)
        if l > 0:
            g = dx * (acts[l] > 0.0)   # ReLU of the layer below
    return grads


def rms(a):
    a = np.asarray(a, dtype=np.float64)
    return float(np.sqrt(np.mean(a * a)))


def _safe_scale(a):
    s = rms(a)
    return a / s if s > 0.0 else np.zeros_like(a)


def features(r, diag, gR):
    """Network input [nz, ny, nx, 16] from node vectors r, diag [3, nz, ny, nx]
    and the node field gR [nz, ny, nx]."""
    r = np.asarray(r, dtype=np.float64)
    diag = np.asarray(diag, dtype=np.float64)
    y = r / diag
    f = np.zeros(r.shape[1:] + (CH,))
    ys, rs, ds = _safe_scale(y), _safe_scale(r), _safe_scale(diag)
    for d in range(3):
        f[..., d] = ys[d]
        f[..., 3 + d] = rs[d]
        f[..., 6 + d] = ds[d]
    f[..., 9] = _safe_scale(gR)
    return f


def apply(params, r, diag, gR, round_hidden=False):
    """z = D^-1 r + rms(D^-1 r) * CNN(features)[:3] (node vector [3, nz, ny, nx]).
    round_hidden: the input features and hidden activations are rounded to
    bfloat16, as the device network stores them."""
    y = np.asarray(r, dtype=np.float64) / np.asarray(diag, dtype=np.float64)
    h0 = features(r, diag, gR)
    if round_hidden:
        h0 = bf16_round(h0)
    o = forward(params, h0, round_hidden)[-1]
    return y + rms(y) * np.moveaxis(o[..., :OUT_USED], -1, 0)


def loss_and_grad(z, r, Az, y, Ay):
    """L(z) = -((z.r)^2 / z.Az) / ((y.r)^2 / y.Ay) and dL/dz."""
    z, r, Az, y, Ay = (np.asarray(a, dtype=np.float64).ravel() for a in (z, r, Az, y, Ay))
    zr, zAz = float(z @ r), float(z @ Az)
    EJ = float(y @ r) ** 2 / float(y @ Ay)
    s = zr / zAz
    return -(zr * zr / zAz) / EJ, 2.0 * s * (s * Az - r) / EJ


def grad_magnitude(grid, R):
    """|grad R| per voxel from the short differences of the NGF norm
    (eq. NGF_discretized), without the edge parameter:
    sqrt(1/2 sum_k ((R_{i+k} - R_i)^2 + (R_{i-k} - R_i)^2) / h_k^2), neighbours clamped."""
    R = np.asarray(R, dtype=np.float64)
    acc = np.zeros_like(R)
    for ax, hk in ((2, grid.h[0]), (1, grid.h[1]), (0, grid.h[2])):
        n = R.shape[ax]
        idx = np.arange(n)
        up = np.take(R, np.minimum(idx + 1, n - 1), axis=ax) - R
        dn = np.take(R, np.maximum(idx - 1, 0), axis=ax) - R
        acc += 0.5 * (up * up + dn * dn) / hk ** 2
    return np.sqrt(acc)


def node_average(grid, v):
    """(P^T v) / (P^T 1): the interpolation-weighted mean of a voxel field
    around each node (P of eq. grid_conversion), shape [nz, ny, nx]."""
    P = grid.P_matrix()
    v = np.asarray(v, dtype=np.float64).ravel()
    num = P.T @ v
    den = P.T @ np.ones(v.size)
    return (num / den).reshape(grid.my[2], grid.my[1], grid.my[0])
