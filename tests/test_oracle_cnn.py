"""Pins of the learned-preconditioner oracle (oracle.cnn, oracle.solver.fpcg)
against things other than itself: library correlation routines, shifted
identities, finite differences, adjoint identities, closed-form optima, CG
theory and torch's bfloat16 conversion."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from oracle import Grid, cnn, solver

RNG = np.random.default_rng(7)


def rand(*shape, scale=1.0):
    return scale * RNG.standard_normal(shape)


def test_delta_kernel_reproduces_input_and_shift_kernel_shifts():
    x = rand(4, 5, 6, 3)
    W = np.zeros((27, 3, 3))
    W[13] = np.eye(3)                      # centre tap (0, 0, 0)
    assert np.array_equal(cnn.conv3d(x, W, np.zeros(3)), x)
    W = np.zeros((27, 3, 3))
    W[14] = np.eye(3)                      # tap (0, 0, +1): y[..., x] = x[..., x + 1]
    y = cnn.conv3d(x, W, np.zeros(3))
    assert np.array_equal(y[:, :, :-1], x[:, :, 1:])
    assert np.all(y[:, :, -1] == 0.0)
    W = np.zeros((27, 3, 3))
    W[0] = np.eye(3)                       # tap (-1, -1, -1)
    y = cnn.conv3d(x, W, np.zeros(3))
    assert np.array_equal(y[1:, 1:, 1:], x[:-1, :-1, :-1])
    assert np.all(y[0] == 0.0) and np.all(y[:, 0] == 0.0) and np.all(y[:, :, 0] == 0.0)


def test_conv_matches_scipy_correlate_per_channel_pair():
    x = rand(5, 6, 7, 4)
    W = rand(27, 4, 3)
    b = rand(3)
    y = cnn.conv3d(x, W, b)
    for o in range(3):
        ref = np.full(x.shape[:3], b[o])
        for c in range(4):
            k = W[:, c, o].reshape(3, 3, 3)     # taps ordered (dz, dy, dx)
            ref += ndi.correlate(x[..., c], k, mode="constant", cval=0.0)
        assert np.allclose(y[..., o], ref, rtol=1e-12, atol=1e-12)


def test_conv_backward_adjoint_identity():
    x = rand(4, 5, 6, 5)
    W = rand(27, 5, 4)
    g = rand(4, 5, 6, 4)
    y = cnn.conv3d(x, W, np.zeros(4))
    dx, _, _ = cnn.conv3d_backward(x, W, g)
    assert np.isclose(np.sum(y * g), np.sum(x * dx), rtol=1e-12)


def test_conv_backward_finite_differences():
    x = rand(3, 4, 5, 2)
    W = rand(27, 2, 3)
    b = rand(3)
    c = rand(3, 4, 5, 3)
    f = lambda x_, W_, b_: float(np.sum(c * cnn.conv3d(x_, W_, b_)))
    dx, dW, db = cnn.conv3d_backward(x, W, c)
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (2, 3, 4, 1), (1, 2, 0, 1)]:
        e = np.zeros_like(x); e[idx] = eps
        assert np.isclose((f(x + e, W, b) - f(x - e, W, b)) / (2 * eps), dx[idx], rtol=1e-6, atol=1e-8)
    for idx in [(0, 0, 0), (13, 1, 2), (26, 1, 0), (5, 0, 1)]:
        e = np.zeros_like(W); e[idx] = eps
        assert np.isclose((f(x, W + e, b) - f(x, W - e, b)) / (2 * eps), dW[idx], rtol=1e-6, atol=1e-8)
    for o in range(3):
        e = np.zeros(3); e[o] = eps
        assert np.isclose((f(x, W, b + e) - f(x, W, b - e)) / (2 * eps), db[o], rtol=1e-6)


def _params(scale=0.3):
    return [(rand(27, 16, 16, scale=scale), rand(16, scale=0.1)) for _ in range(cnn.LAYERS)]


def test_network_backward_finite_differences():
    params = _params()
    h0 = rand(3, 4, 5, 16)
    c = rand(3, 4, 5, 16)
    acts = cnn.forward(params, h0)
    grads = cnn.backward(params, acts, c)
    f = lambda P: float(np.sum(c * cnn.forward(P, h0)[-1]))
    eps = 1e-6
    for l, idx in [(0, (13, 2, 5)), (1, (4, 7, 1)), (2, (20, 15, 0)), (3, (13, 3, 2))]:
        Pp = [(W.copy(), b.copy()) for W, b in params]
        Pm = [(W.copy(), b.copy()) for W, b in params]
        Pp[l][0][idx] += eps
        Pm[l][0][idx] -= eps
        fd = (f(Pp) - f(Pm)) / (2 * eps)
        assert np.isclose(fd, grads[l][0][idx], rtol=1e-5, atol=1e-7), (l, idx, fd, grads[l][0][idx])
    for l in range(cnn.LAYERS):
        Pp = [(W.copy(), b.copy()) for W, b in params]
        Pm = [(W.copy(), b.copy()) for W, b in params]
        Pp[l][1][3] += eps
        Pm[l][1][3] -= eps
        assert np.isclose((f(Pp) - f(Pm)) / (2 * eps), grads[l][1][3], rtol=1e-5, atol=1e-7)


def test_relu_layers_zero_negative_parts():
    params = _params()
    acts = cnn.forward(params, rand(2, 3, 4, 16))
    for a in acts[1:-1]:
        assert np.all(a >= 0.0)
    assert np.any(acts[-1] < 0.0)          # no ReLU on the output layer


def test_bf16_round_matches_torch_conversion():
    vals = np.concatenate([rand(10000, scale=100.0), [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -0.0, 0.0,
                                                     1.0 + 2.0 ** -9 * 1.5, 3.0e38, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cnn.bf16_round(vals), ref)
    assert cnn.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0             # tie -> even
    assert cnn.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6  # tie -> even (up)


def test_zero_network_is_jacobi():
    r = rand(3, 4, 5, 6)
    diag = np.abs(rand(3, 4, 5, 6)) + 0.5
    gR = np.abs(rand(4, 5, 6))
    params = [(np.zeros((27, 16, 16)), np.zeros(16)) for _ in range(cnn.LAYERS)]
    assert np.array_equal(cnn.apply(params, r, diag, gR), r / diag)


def test_features_are_rms_normalised_and_padded():
    r = rand(3, 4, 5, 6)
    diag = np.abs(rand(3, 4, 5, 6)) + 0.5
    gR = np.abs(rand(4, 5, 6))
    f = cnn.features(r, diag, gR)
    for ch in (slice(0, 3), slice(3, 6), slice(6, 9), slice(9, 10)):
        assert np.isclose(np.sqrt(np.mean(f[..., ch] ** 2)), 1.0)
    assert np.all(f[..., cnn.IN_USED:] == 0.0)
    assert np.allclose(f[..., 0] * cnn.rms(r / diag), (r / diag)[0])


def _spd(n):
    Q = rand(n, n)
    return Q @ Q.T + n * np.eye(n)


def test_loss_closed_forms_and_gradient():
    n = 30
    A = _spd(n)
    r = rand(n)
    d = np.diag(A).copy()
    y = r / d
    L, _ = cnn.loss_and_grad(y, r, A @ y, y, A @ y)
    assert np.isclose(L, -1.0)
    zs = np.linalg.solve(A, r)               # exact solve: the best possible direction
    L, g = cnn.loss_and_grad(zs, r, A @ zs, y, A @ y)
    EJ = (y @ r) ** 2 / (y @ A @ y)
    assert np.isclose(L, -(r @ zs) / EJ)
    assert L <= -1.0 + 1e-12
    assert np.allclose(g, 0.0, atol=1e-12)
    L3, _ = cnn.loss_and_grad(3.0 * zs, r, A @ (3.0 * zs), y, A @ y)   # scale invariant
    assert np.isclose(L3, L)
    z = rand(n)
    _, g = cnn.loss_and_grad(z, r, A @ z, y, A @ y)
    eps = 1e-6
    for i in (0, 7, 29):
        e = np.zeros(n); e[i] = eps
        fd = (cnn.loss_and_grad(z + e, r, A @ (z + e), y, A @ y)[0]
              - cnn.loss_and_grad(z - e, r, A @ (z - e), y, A @ y)[0]) / (2 * eps)
        assert np.isclose(fd, g[i], rtol=1e-5, atol=1e-9)


def test_fpcg_equals_pcg_for_a_fixed_linear_preconditioner():
    n = 40
    A = _spd(n)
    b = rand(n)
    d = np.diag(A).copy()
    for it in (1, 3, 10):
        s1, i1 = solver.pcg(lambda p: A @ p, b, diag=d, max_iter=it, rtol=0.0)
        s2, i2 = solver.fpcg(lambda p: A @ p, b, lambda r: r / d, max_iter=it, rtol=0.0)
        assert np.allclose(s1, s2, rtol=1e-9, atol=1e-12)
        assert i1["iters"] == i2["iters"]


def test_fpcg_plain_cg_exact_in_n_steps_and_fallback():
    # inputs drawn here, not from the module's shared generator, so they do not depend
    # on which tests ran before in the same process
    rng = np.random.default_rng(12)
    n = 12
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.standard_normal(n)
    s, info = solver.fpcg(lambda p: A @ p, b, lambda r: r, max_iter=n, rtol=1e-10)
    assert info["flag"] == 0 and info["iters"] <= n
    assert np.allclose(A @ s, b, rtol=1e-8)
    # a poor preconditioner (random positive scales over six decades) has not converged after
    # 3 steps; the solve then continues with Jacobi and converges
    d = np.diag(A).copy()
    w = 10.0 ** rng.uniform(-3.0, 3.0, n)
    s, info = solver.fpcg(lambda p: A @ p, b, lambda r: w * r, max_iter=60,
                          rtol=1e-8, fallback=lambda r: r / d, fallback_iters=3)
    assert info["used_fallback"] == 1 and info["flag"] == 0
    assert np.allclose(A @ s, b, rtol=1e-6, atol=1e-8)


def test_grad_magnitude_ramp_and_node_average():
    g = Grid((12, 10, 8), (1.0, 2.0, 0.5), (4, 4, 3), 1.0, 1.0, 1.0)
    z, y, x = np.meshgrid(np.arange(8), np.arange(10), np.arange(12), indexing="ij")
    R = 3.0 * x + 4.0 * y * 2.0      # gradient (3, 4) in physical units (h_y = 2)
    gm = cnn.grad_magnitude(g, R)
    inner = gm[:, 1:-1, 1:-1]
    assert np.allclose(inner, 5.0)
    # at the x boundary one of the two x differences vanishes: sqrt(9/2 + 16)
    assert np.allclose(gm[:, 1:-1, 0], np.sqrt(4.5 + 16.0))
    # node average of a constant field is that constant; of the ramp it is a weighted mean in range
    assert np.allclose(cnn.node_average(g, np.full(R.shape, 2.5)), 2.5)
    na = cnn.node_average(g, x.astype(float))
    assert np.all(na >= 0.0) and np.all(na <= 11.0)
    assert np.all(np.diff(na, axis=2) > 0.0)   # increasing along x
