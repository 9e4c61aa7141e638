"""Pins of the 2D oracle (oracle.plane, the d = 2 case of Sec. 2-4) against
what the mathematics and the paper fix: pure-Python loops, finite differences,
symmetry and positive semi-definiteness, the d = 2 structure of
Table hessian_indices, exact reproduction properties of P and of the template,
closed forms of the curvature term, and the 3D oracle on a problem extruded
along z (which reduces the 3D discretisation to the 2D one exactly)."""
import os

import numpy as np
import pytest

import bruteforce
from oracle import Grid, curvature, multilevel, ngf, plane, solver

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def problem(seed=0, m=(7, 6), my=(4, 4), h=(1.0, 1.3), tau=0.3, rho=0.2, alpha=0.7, amp=0.4):
    rng = np.random.default_rng(seed)
    g = plane.Grid2(m, h, my, tau, rho, alpha)
    R = rng.standard_normal((m[1], m[0]))
    T = rng.standard_normal((m[1], m[0]))
    u = amp * rng.standard_normal((2, my[1], my[0]))
    return g, R, T, u, rng


def test_distance_and_curvature_against_loops():
    g, R, T, u, _ = problem(1)
    D = plane.distance(g, R, T, u)
    Db = bruteforce.objective_D_2d(g.m, g.h, g.my, g.tau, g.rho, R.tolist(), T.tolist(), u.tolist())
    assert abs(D - Db) <= 1e-12 * abs(Db)
    S = plane.curvature_energy(g, u)
    Sb = bruteforce.curvature_S_2d(g.my, g.hy, u.tolist())
    assert abs(S - Sb) <= 1e-12 * abs(Sb)


def test_distance_against_loops_separate_template_grid():
    rng = np.random.default_rng(2)
    g = plane.Grid2((6, 5), (1.0, 1.0), (4, 3), 0.4, 0.3, 1.0, mT=(4, 7), hT=(1.6, 0.75))
    R = rng.standard_normal((5, 6))
    T = rng.standard_normal((7, 4))
    u = 0.6 * rng.standard_normal((2, 3, 4))
    D = plane.distance(g, R, T, u)
    Db = bruteforce.objective_D_2d(g.m, g.h, g.my, g.tau, g.rho, R.tolist(), T.tolist(), u.tolist(), g.mT, g.hT)
    assert abs(D - Db) <= 1e-12 * abs(Db)


def _fd(f, u, d, eps=1e-6):
    return (f(u + eps * d) - f(u - eps * d)) / (2 * eps)


def test_gradient_against_finite_differences():
    g, R, T, u, rng = problem(3)
    prob = plane.Problem2(g, R, T)
    _, grad = prob.gradient(u)
    for _ in range(4):
        d = rng.standard_normal(u.shape)
        fd = _fd(lambda v: prob.objective(v)[0], u, d)
        assert abs(np.sum(grad * d) - fd) <= 1e-6 * max(abs(fd), 1e-8), (np.sum(grad * d), fd)
    # every component of the boundary nodes
    for idx in [(0, 0, 0), (1, 0, 0), (0, g.my[1] - 1, g.my[0] - 1), (1, g.my[1] - 1, 0), (1, 2, g.my[0] - 1)]:
        e = np.zeros_like(u)
        e[idx] = 1.0
        fd = _fd(lambda v: prob.objective(v)[0], u, e)
        assert abs(grad[idx] - fd) <= 1e-6 * max(abs(fd), 1e-6), (idx, grad[idx], fd)


def test_jacobian_against_finite_differences_of_the_residual():
    g, R, T, u, rng = problem(4)
    J, _ = plane.jacobian(g, R, T, u)
    p = rng.standard_normal(u.shape)
    res = lambda v: plane.residual_parts(g, R, T, v, np.arange(g.mbar))["r"]
    fd = _fd(res, u, p)
    np.testing.assert_allclose(J @ p.ravel(), fd, rtol=1e-6, atol=1e-8)


def test_hessian_symmetric_psd_and_diagonal():
    g, R, T, u, rng = problem(5)
    prob = plane.Problem2(g, R, T)
    Jac = prob.jacobian(u)
    n = 2 * g.nbar
    H = np.column_stack([prob.hess_vec(u, e.reshape(u.shape), Jac).ravel() for e in np.eye(n)])
    np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() >= -1e-10 * np.abs(H).max()
    np.testing.assert_allclose(prob.jacobi_diag(u, Jac).ravel(), np.diag(H), rtol=1e-12, atol=1e-14)
    p = rng.standard_normal(u.shape)
    Jp = Jac @ p.ravel()
    Hd = plane.hess_vec_D(g, R, T, u, p, Jac)
    assert abs(np.sum(p * Hd) - 2 * g.hbar * Jp @ Jp) <= 1e-12 * abs(2 * g.hbar * Jp @ Jp)


def test_dr_interior_rows_have_the_13_offsets_of_the_d2_table():
    rng = np.random.default_rng(6)
    g = plane.Grid2((9, 9), (1.0, 1.0), (5, 5), 0.5, 0.5, 0.0)
    R, T = rng.standard_normal((9, 9)), rng.standard_normal((9, 9))
    dr, _ = plane.dr_rows(g, R, T, np.zeros((2, 5, 5)), np.arange(g.mbar))
    i = g.voxel_id(4, 4)
    # a row of dr: the voxel and its four neighbours
    assert set(dr[i].indices) == {i, i - 1, i + 1, i - 9, i + 9}
    # (dr^T dr)_{i, i+o}: the offsets and, per offset, the number of rows l contributing
    want = {}
    for line in open(os.path.join(GOLDEN, "hessian_offsets_2d.txt")):
        if line.strip() and not line.startswith("#"):
            dx, dy, mult = (int(v) for v in line.split())
            want[(dx, dy)] = mult
    S5 = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    counted = {}
    for s in S5:   # brute-force count of the stencil overlaps
        for t in S5:
            o = (t[0] - s[0], t[1] - s[1])
            counted[o] = counted.get(o, 0) + 1
    assert counted == want
    rows_of = {o: 0 for o in want}
    for l in dr[:, [i]].nonzero()[0]:
        for j in dr[l].indices:
            o = ((j % 9) - 4, (j // 9) - 4)
            rows_of[o] += 1
    assert rows_of == want
    M = (dr.T @ dr).tocsr()
    offs = {((j % 9) - 4, (j // 9) - 4) for j in M[i].indices}
    assert offs == set(want)


def test_conversion_reproduces_affine_fields_and_is_a_partition_of_unity():
    g = plane.Grid2((10, 7), (1.0, 2.0), (6, 3), 1.0, 1.0, 1.0)
    P = g.P_matrix()
    X = g.node_positions()
    centres = g.voxel_centres(np.arange(g.mbar))
    np.testing.assert_allclose(P @ X[0].ravel(), centres[:, 0], atol=1e-12)
    np.testing.assert_allclose(P @ X[1].ravel(), centres[:, 1], atol=1e-12)
    np.testing.assert_allclose(P @ np.ones(g.nbar), 1.0, atol=1e-14)
    rng = np.random.default_rng(7)
    a, b = rng.standard_normal(g.nbar), rng.standard_normal(g.mbar)
    assert abs((P @ a) @ b - a @ (P.T @ b)) < 1e-12


def test_template_exact_at_samples_zero_outside_linear_inside_and_derivative():
    rng = np.random.default_rng(8)
    g = plane.Grid2((6, 5), (1.0, 1.0), (3, 3), 1.0, 1.0, 1.0, mT=(6, 5), hT=(1.5, 0.8))
    T = rng.standard_normal((5, 6))
    iy, ix = np.meshgrid(np.arange(5), np.arange(6), indexing="ij")
    pts = np.stack([(ix.ravel() + 0.5) * 1.5, (iy.ravel() + 0.5) * 0.8], axis=-1)
    v, _ = plane.template_sample(g, T, pts)
    np.testing.assert_allclose(v, T.ravel(), atol=1e-14)
    far = np.array([[-1.6, 1.0], [10.0, 1.0], [2.0, -0.9], [2.0, 5.0]])
    v, gr = plane.template_sample(g, T, far)
    assert np.all(v == 0) and np.all(gr == 0)
    lin = 0.7 * (ix + 0.5) * 1.5 - 0.3 * (iy + 0.5) * 0.8 + 2.0
    q = np.array([[2.1, 1.7], [5.9, 2.6], [3.3, 0.9]])
    v, gr = plane.template_sample(g, lin, q)
    np.testing.assert_allclose(v, 0.7 * q[:, 0] - 0.3 * q[:, 1] + 2.0, atol=1e-12)
    np.testing.assert_allclose(gr, np.tile([0.7, -0.3], (3, 1)), atol=1e-12)
    q = rng.uniform(0.9, 7.5, size=(20, 2)) * np.array([1.0, 0.5])
    _, gr = plane.template_sample(g, T, q)
    for d in range(2):
        e = np.zeros(2)
        e[d] = 1e-7
        fd = (plane.template_sample(g, T, q + e)[0] - plane.template_sample(g, T, q - e)[0]) / 2e-7
        np.testing.assert_allclose(gr[:, d], fd, rtol=1e-6, atol=1e-6)


def test_identical_images_give_unit_residual_and_zero_derivatives():
    rng = np.random.default_rng(9)
    g = plane.Grid2((8, 6), (1.0, 1.0), (5, 4), 0.5, 0.5, 0.0)
    R = rng.standard_normal((6, 8))
    u = np.zeros((2, 4, 5))
    r = plane.residual_parts(g, R, R, u, np.arange(g.mbar))["r"]
    np.testing.assert_allclose(r, 1.0, atol=1e-14)
    assert abs(plane.distance(g, R, R, u)) < 1e-12
    np.testing.assert_allclose(plane.gradient_D(g, R, R, u), 0.0, atol=1e-12)
    np.testing.assert_allclose(plane.hess_vec_D(g, R, R, u, rng.standard_normal(u.shape)), 0.0, atol=1e-12)


def test_curvature_closed_forms():
    g = plane.Grid2((12, 10), (1.0, 1.0), (7, 6), 1.0, 1.0, 1.0)
    L = plane.laplacian(g)
    X = g.node_positions()
    t = np.stack([np.full(X[0].shape, 0.3), np.full(X[0].shape, -1.2)])
    assert plane.curvature_energy(g, t) <= 1e-28   # rounding of the summed clamped entries only
    # u_x = a x: interior Laplacian 0; at the first / last node column the clamped
    # difference gives +-a / hy_x, so S = hbar^y * 2 ny (a / hy_x)^2
    a = 0.4
    lin = np.stack([a * X[0], np.zeros_like(X[0])])
    want = g.hybar * 2 * g.my[1] * (a / g.hy[0]) ** 2
    assert abs(plane.curvature_energy(g, lin) - want) <= 1e-12 * want
    # interior diag(L^2) = (sum_k 2/hy_k^2)^2 + sum_k 2/hy_k^4
    d = np.asarray(L.multiply(L).sum(axis=0)).ravel()
    i = g.node_id(3, 3)
    want = (2 / g.hy[0] ** 2 + 2 / g.hy[1] ** 2) ** 2 + 2 / g.hy[0] ** 4 + 2 / g.hy[1] ** 4
    assert abs(d[i] - want) <= 1e-12 * want
    np.testing.assert_allclose((L - L.T).toarray(), 0.0, atol=1e-14)


def test_extruded_3d_problem_reduces_to_the_2d_one():
    # z-constant images on 2 voxel planes with 2 node planes, z displacement 0 and the
    # same 2D field on both node planes: the 3D discretisation collapses to the 2D one
    # (z differences vanish, the z conversion weights of a node plane sum to 1), so
    # D3 = 2 h_z D2 and the x, y parts of the 3D derivatives equal h_z times the 2D ones;
    # the curvature term: S3 = 2 hy_z S2 and grad S3 = hy_z grad S2 (x, y components).
    rng = np.random.default_rng(10)
    m2, my2, h2 = (7, 6), (4, 4), (1.0, 1.3)
    hz = 0.9
    g2 = plane.Grid2(m2, h2, my2, 0.3, 0.2, 0.7)
    g3 = Grid(m2 + (2,), h2 + (hz,), my2 + (2,), 0.3, 0.2, 0.7)
    R2, T2 = rng.standard_normal((6, 7)), rng.standard_normal((6, 7))
    u2 = 0.4 * rng.standard_normal((2, 4, 4))
    p2 = rng.standard_normal((2, 4, 4))
    R3, T3 = np.stack([R2, R2]), np.stack([T2, T2])
    u3 = np.zeros((3, 2, 4, 4))
    u3[:2] = u2[:, None]
    p3 = np.zeros((3, 2, 4, 4))
    p3[:2] = p2[:, None]
    D2, D3 = plane.distance(g2, R2, T2, u2), ngf.distance(g3, R3, T3, u3)
    assert abs(D3 - 2 * hz * D2) <= 1e-12 * abs(D3)
    gD2, gD3 = plane.gradient_D(g2, R2, T2, u2), ngf.gradient_D(g3, R3, T3, u3)
    hD2, hD3 = plane.hess_vec_D(g2, R2, T2, u2, p2), ngf.hess_vec_D(g3, R3, T3, u3, p3)
    for k in range(2):
        np.testing.assert_allclose(gD3[:2, k], hz * gD2, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(hD3[:2, k], hz * hD2, rtol=1e-12, atol=1e-12)
    hyz = g3.hy[2]
    S2, S3 = plane.curvature_energy(g2, u2), curvature.energy(g3, u3)
    assert abs(S3 - 2 * hyz * S2) <= 1e-12 * abs(S3)
    gS2, gS3 = plane.curvature_gradient(g2, u2), curvature.gradient(g3, u3)
    for k in range(2):
        np.testing.assert_allclose(gS3[:2, k], hyz * gS2, rtol=1e-12, atol=1e-10)


def test_gauss_newton_decreases_and_pcg_solves_small_systems():
    g, R, T, u, _ = problem(11, m=(10, 9), my=(6, 5), amp=0.0)
    prob = plane.Problem2(g, R, T)
    u1, hist = solver.gauss_newton(prob, u, iters=3)
    assert prob.objective(u1)[0] < prob.objective(u)[0]
    assert all(h["J_new"] <= h["J"] for h in hist if "J_new" in h)
    # CG on the assembled system converges to the dense solution
    Jac = prob.jacobian(u1)
    n = 2 * g.nbar
    A = np.column_stack([prob.hess_vec(u1, e.reshape(u.shape), Jac).ravel() for e in np.eye(n)])
    b = -prob.gradient(u1)[1]
    s, info = solver.pcg(lambda p: prob.hess_vec(u1, p, Jac), b, prob.jacobi_diag(u1, Jac), max_iter=n, rtol=1e-10)
    np.testing.assert_allclose(s.ravel(), np.linalg.solve(A, b.ravel()), rtol=1e-6, atol=1e-9)


def test_pyramid_restriction_and_prolongation_2d():
    rng = np.random.default_rng(12)
    for shape in [(6, 8), (5, 7), (1, 3)]:
        I = rng.standard_normal(shape)
        out = plane.restrict_image(I)
        ref = np.zeros(((shape[0] + 1) // 2, (shape[1] + 1) // 2))
        for b in range(ref.shape[0]):
            for a in range(ref.shape[1]):
                ref[b, a] = sum(I[min(2 * b + j, shape[0] - 1), min(2 * a + i, shape[1] - 1)]
                                for j in (0, 1) for i in (0, 1)) / 4.0
        np.testing.assert_allclose(out, ref, atol=1e-14)
    # linear fields at fine centres restrict to the same field at coarse centres
    y, x = np.meshgrid(np.arange(8) + 0.5, np.arange(10) + 0.5, indexing="ij")
    yc, xc = np.meshgrid(2 * (np.arange(4) + 0.5), 2 * (np.arange(5) + 0.5), indexing="ij")
    np.testing.assert_allclose(plane.restrict_image(0.3 * x - 0.8 * y), 0.3 * xc - 0.8 * yc, atol=1e-13)
    z, yy = np.meshgrid(np.arange(4), np.arange(6), indexing="ij")
    np.testing.assert_allclose(plane.restrict_image((-1.0) ** (z + yy)), 0.0, atol=1e-15)
    g = plane.Grid2((16, 12), (1, 1), (9, 7), 1, 1, 1)
    gc = plane.coarse_grid(g)
    assert gc.m == (8, 6) and gc.my == (5, 4)
    uc = rng.standard_normal((2, 4, 5))
    uf = plane.prolong(uc, gc, g)
    np.testing.assert_allclose(uf[:, ::2, ::2], uc, atol=1e-14)
    Xc, Xf = gc.node_positions(), g.node_positions()
    np.testing.assert_allclose(plane.prolong(np.stack([0.2 * Xc[0] - Xc[1], 0.5 * Xc[1]]), gc, g),
                               np.stack([0.2 * Xf[0] - Xf[1], 0.5 * Xf[1]]), atol=1e-12)


def test_node_outputs_match_full_evaluation():
    g, R, T, u, rng = problem(13, m=(12, 10), my=(7, 6))
    p = rng.standard_normal(u.shape)
    grad = plane.gradient_D(g, R, T, u).reshape(2, -1)
    hv = plane.hess_vec_D(g, R, T, u, p).reshape(2, -1)
    dg = plane.hessian_diag_D(g, R, T, u).reshape(2, -1)
    for node in [0, g.nbar - 1, g.node_id(3, 2), g.node_id(6, 0), g.node_id(0, 5)]:
        a, b, c = plane.node_outputs(g, R, T, u, p, node)
        np.testing.assert_allclose(a, grad[:, node], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(b, hv[:, node], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(c, dg[:, node], rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("my,gamma", [((7, 5), 0.3), ((2, 9), 2.0), ((11, 11), 0.05)])
def test_h0_solver_two_dimensional_on_cosine_eigenvectors(my, gamma):
    """L-BFGS initial matrix (Sec. 2.3.2) on a two-dimensional grid: the 5-point
    Neumann Laplacian's eigenvectors are products of DCT-II cosines
    cos(pi k (i + 1/2) / n), eigenvalue -4 sin^2(pi k / 2n) / hy^2 per axis, so
    H_0 = 2 alpha hbar^y L^T L + gamma I scales them by 2 alpha hbar^y lam^2 + gamma."""
    from oracle import lbfgs

    g = plane.Grid2((13, 10), (1.0, 1.3), my, 1.0, 1.0, 0.7)
    h0 = lbfgs.H0Solver(g, gamma, plane.laplacian(g))
    for ks in [(0, 0), (1, 2), (my[0] - 1, my[1] - 1), (2, 1)]:
        ks = tuple(min(k, n - 1) for k, n in zip(ks, my))
        ax = [np.cos(np.pi * ks[d] * (np.arange(my[d]) + 0.5) / my[d]) for d in range(2)]
        v = np.outer(ax[1], ax[0])
        lam = -sum(4.0 * np.sin(np.pi * ks[d] / (2 * my[d])) ** 2 / g.hy[d] ** 2 for d in range(2))
        mu = 2.0 * g.alpha * g.hybar * lam * lam + gamma
        V = np.stack([v, -3.0 * v])
        np.testing.assert_allclose(h0.apply(V), V / mu, rtol=1e-9, atol=1e-12)


def test_lbfgs_two_dimensional_first_step_is_the_regularised_newton_step():
    """With T = R = 0, D = 0 and J = alpha S is quadratic with Hessian
    A = 2 alpha hbar^y L^T L: the first L-BFGS step from u0 is
    -(A + gamma I)^{-1} A u0 and eta = 1 passes the Armijo test."""
    from oracle import lbfgs

    g = plane.Grid2((11, 9), (1.0, 1.0), (6, 5), 0.3, 0.3, 0.6)
    Z = np.zeros((9, 11))
    prob = plane.Problem2(g, Z, Z)
    u0 = np.random.default_rng(4).standard_normal((2, 5, 6))
    gamma = 0.05
    u1, hist = lbfgs.lbfgs(prob, u0, iters=1, gamma=gamma)
    L = plane.laplacian(g).toarray()
    A = 2.0 * g.alpha * g.hybar * (L.T @ L)
    M = A + gamma * np.eye(g.nbar)
    want = np.stack([u0[d].ravel() - np.linalg.solve(M, A @ u0[d].ravel()) for d in range(2)]).reshape(u0.shape)
    assert hist[0]["eta"] == 1.0
    np.testing.assert_allclose(u1, want, rtol=1e-9, atol=1e-11)
