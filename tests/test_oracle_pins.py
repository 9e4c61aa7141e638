"""Pins of the float64 oracle against facts fixed by the paper and by the
mathematics -- not against the oracle itself.

Each check is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, a transposed operand, a wrong boundary rule) fails it:
brute-force loop evaluation of the objective, finite differences of the
objective and of the residual vector, affine reproduction of the grid
conversion, closed forms of the curvature term, exact structural facts stated
in Sec. 4 (7 non-zeros per row of dr, 25 offsets of dr^T dr per
Table hessian_indices), symmetry / positive semi-definiteness of the
Gauss-Newton matrix, and dense solves for PCG.
"""
import os

import numpy as np
import pytest

import bruteforce
from oracle import Grid, curvature, diffusive, elastic, interp, lbfgs, multilevel, ngf, solver, ssd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_problem(seed=0, m=(6, 5, 4), my=(4, 3, 3), h=(1.0, 1.2, 0.9), tau=0.3, rho=0.2, alpha=0.7,
                 amp=0.4):
    rng = np.random.default_rng(seed)
    g = Grid(m, h, my, tau, rho, alpha)
    R = rng.standard_normal((m[2], m[1], m[0]))
    T = rng.standard_normal((m[2], m[1], m[0]))
    u = amp * rng.standard_normal((3, my[2], my[1], my[0]))
    return g, R, T, u, rng


GRIDS = [
    ((6, 5, 4), (4, 3, 3), (1.0, 1.2, 0.9)),      # non-integer ratios
    ((8, 8, 8), (5, 5, 5), (1.0, 1.0, 1.0)),      # ratio 2
    ((8, 4, 6), (9, 5, 7), (0.5, 1.0, 2.0)),      # ratio 1 (nodes = cells + 1)
    ((12, 9, 7), (4, 4, 3), (1.0, 1.0, 1.0)),     # ratios 4, 3, 3.5
]


# ---------------------------------------------------------------------------
# Grid conversion P (Sec. 4.3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,my,h", GRIDS)
def test_P_reproduces_identity_and_affine_fields(m, my, h):
    # P x^y = x pins the node count (my nodes), c(a) = (a+1/2)(my-1)/m and
    # the node spacing m h/(my-1): any other reading breaks affine reproduction.
    g = Grid(m, h, my, 1.0, 1.0, 1.0)
    xy = g.node_positions()
    Px = g.apply_P(xy)
    cen = g.voxel_centres(np.arange(g.mbar)).T.reshape(3, m[2], m[1], m[0])
    np.testing.assert_allclose(Px, cen, rtol=0, atol=1e-12)
    A = np.array([[0.3, -1.1, 0.2], [0.5, 0.1, -0.7], [1.3, 0.4, 0.9]])
    b = np.array([0.2, -0.4, 1.5])
    aff = np.einsum("ij,jzyx->izyx", A, xy) + b[:, None, None, None]
    want = np.einsum("ij,jzyx->izyx", A, cen) + b[:, None, None, None]
    np.testing.assert_allclose(g.apply_P(aff), want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("m,my,h", GRIDS)
def test_P_structure_and_adjoint(m, my, h):
    g = Grid(m, h, my, 1.0, 1.0, 1.0)
    P = g.P_matrix().toarray()
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-14)         # partition of unity
    assert (P >= 0).all()
    assert ((P > 0).sum(axis=1) <= 8).all()                              # 8 coefficients per row
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3,) + (my[2], my[1], my[0]))
    bvox = rng.standard_normal((3,) + (m[2], m[1], m[0]))
    lhs = np.sum(g.apply_P(a) * bvox)
    rhs = np.sum(a * g.apply_PT(bvox))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_P_dense_bruteforce_against_equation():
    # Entry-by-entry: (P)_{i,n} = prod_k w_k where node n_k in {lo_k, lo_k+1}.
    m, my = (6, 5, 4), (4, 3, 3)
    g = Grid(m, (1, 1, 1), my, 1, 1, 1)
    P = g.P_matrix().toarray()
    for c in range(m[2]):
        for b in range(m[1]):
            for a in range(m[0]):
                i = a + m[0] * (b + m[1] * c)
                row = np.zeros(g.nbar)
                for (ii, wi) in bruteforce._node_weights_1d(a, m[0], my[0]):
                    for (jj, wj) in bruteforce._node_weights_1d(b, m[1], my[1]):
                        for (kk, wk) in bruteforce._node_weights_1d(c, m[2], my[2]):
                            row[ii + my[0] * (jj + my[1] * kk)] += wi * wj * wk
                np.testing.assert_allclose(P[i], row, atol=1e-15)


def test_PT_ones_closed_form_integer_ratio():
    # ratio s = 2: interior node collects s^3 = 8 (weights sum to s per axis),
    # boundary node along one axis collects s/2 along that axis.
    g = Grid((8, 8, 8), (1, 1, 1), (5, 5, 5), 1, 1, 1)
    ones = np.ones((3, 8, 8, 8))
    pt = g.apply_PT(ones)[0]
    per_axis = np.array([1.0, 2.0, 2.0, 2.0, 1.0])
    want = per_axis[:, None, None] * per_axis[None, :, None] * per_axis[None, None, :]
    np.testing.assert_allclose(pt, want, atol=1e-12)


# ---------------------------------------------------------------------------
# Template interpolation (Sec. 2.2, eq. dT)
# ---------------------------------------------------------------------------

def test_template_exact_at_centres_and_zero_outside():
    rng = np.random.default_rng(0)
    g = Grid((5, 4, 3), (1.0, 2.0, 0.5), (3, 3, 2), 1, 1, 1)
    T = rng.standard_normal((3, 4, 5))
    vox = np.arange(g.mbar)
    val, _ = interp.template_sample(g, T, g.voxel_centres(vox))
    np.testing.assert_allclose(val, T.ravel(), atol=1e-14)
    far = np.array([[-1.1 * 1.0 - 0.5, 1.0, 0.5], [5.0 * 1.0 + 0.6, 2.0, 0.5], [2.0, 4 * 2.0 + 1.3, 0.5]])
    v, gr = interp.template_sample(g, T, far)
    np.testing.assert_array_equal(v, 0.0)
    np.testing.assert_array_equal(gr, 0.0)


def test_zero_displacement_puts_voxels_exactly_on_template_samples():
    # with the template on the reference grid, u = 0 samples the template exactly at
    # its own samples, where the derivative is the forward difference (floor cell)
    g = Grid(m=(7, 6, 5), h=(1.0, 1.0, 1.0), my=(4, 3, 4), tau=0.1, rho=0.1, alpha=0.1)
    vox = np.arange(g.mbar)
    pts = interp.deformed_points(g, np.zeros((3, 4, 3, 4)), vox)
    assert np.array_equal(pts, g.voxel_centres(vox))
    T = np.zeros((5, 6, 7))
    T[:, :, 3:] = 1.0                                    # a step in x between samples 2 and 3
    _, grad = interp.template_sample(g, T, pts)
    a = g.voxel_abc(vox)[0]
    expect = np.where(a == 2, 1.0, np.where(a == 6, -1.0, 0.0))   # forward differences (zero outside)
    np.testing.assert_array_equal(grad[:, 0], expect)


def test_template_linear_inside_and_derivative_fd():
    g = Grid((6, 5, 4), (1.0, 1.5, 0.7), (3, 3, 3), 1, 1, 1)
    cen = g.voxel_centres(np.arange(g.mbar))
    coef = np.array([0.7, -1.3, 2.1])
    T = (cen @ coef + 0.4).reshape(4, 5, 6)
    rng = np.random.default_rng(5)
    lo = np.array([0.5 * g.h[k] for k in range(3)])
    hi = np.array([(g.m[k] - 0.5) * g.h[k] for k in range(3)])
    pts = lo + (hi - lo) * rng.uniform(0.02, 0.98, size=(50, 3))
    val, gr = interp.template_sample(g, T, pts)
    np.testing.assert_allclose(val, pts @ coef + 0.4, atol=1e-12)
    np.testing.assert_allclose(gr, np.broadcast_to(coef, gr.shape), atol=1e-12)
    # derivative of a generic template against central differences (off kinks)
    T2 = rng.standard_normal((4, 5, 6))
    pts = rng.uniform(-1.0, 7.0, size=(200, 3)) * np.array([1.0, 1.5, 0.7])
    s = pts / np.array(g.hT) - 0.5
    frac = s - np.floor(s)
    ok = np.all((frac > 1e-3) & (frac < 1 - 1e-3), axis=1)
    pts = pts[ok]
    _, gr = interp.template_sample(g, T2, pts)
    e = 1e-7
    for d in range(3):
        dp = np.zeros(3)
        dp[d] = e
        fd = (interp.template_sample(g, T2, pts + dp)[0] - interp.template_sample(g, T2, pts - dp)[0]) / (2 * e)
        np.testing.assert_allclose(gr[:, d], fd, rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------------------
# Residual and distance (eq. NGF_discretized, eq. residual)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_distance_matches_bruteforce_loops(seed):
    g, R, T, u, _ = tiny_problem(seed)
    D = ngf.distance(g, R, T, u)
    Db = bruteforce.objective_D(g.m, g.h, g.my, g.tau, g.rho, R.tolist(), T.tolist(), u.tolist())
    assert abs(D - Db) <= 1e-12 * abs(Db)


def test_distance_bruteforce_separate_template_grid():
    rng = np.random.default_rng(11)
    m, my = (5, 4, 4), (3, 3, 3)
    mT, hT = (7, 5, 6), (0.8, 1.1, 0.7)
    g = Grid(m, (1.0, 1.0, 1.0), my, 0.3, 0.5, 1.0, mT, hT)
    R = rng.standard_normal((4, 4, 5))
    T = rng.standard_normal((6, 5, 7))
    u = 0.3 * rng.standard_normal((3, 3, 3, 3))
    D = ngf.distance(g, R, T, u)
    Db = bruteforce.objective_D(m, (1.0, 1.0, 1.0), my, 0.3, 0.5, R.tolist(), T.tolist(), u.tolist(), mT, hT)
    assert abs(D - Db) <= 1e-12 * abs(Db)


def test_identical_images_give_zero_distance_and_derivatives():
    # T = R sampled at the cell centres (u = 0) and tau = rho: r = 1, D = 0,
    # grad D = 0 and the Gauss-Newton matrix vanishes (eq. residual).
    rng = np.random.default_rng(4)
    g = Grid((6, 5, 4), (1, 1, 1), (4, 3, 3), 0.2, 0.2, 1.0)
    R = rng.standard_normal((4, 5, 6))
    u = np.zeros((3, 3, 3, 4))
    r = ngf.residual(g, R, R, u)
    np.testing.assert_allclose(r, 1.0, atol=1e-14)
    assert abs(ngf.distance(g, R, R, u)) < 1e-12
    np.testing.assert_allclose(ngf.gradient_D(g, R, R, u), 0.0, atol=1e-12)
    p = rng.standard_normal(u.shape)
    np.testing.assert_allclose(ngf.hess_vec_D(g, R, R, u, p), 0.0, atol=1e-12)


def test_residual_bounds_and_invariances():
    g, R, T, u, rng = tiny_problem(7, amp=0.2)
    r = ngf.residual(g, R, T, u)
    assert np.all(np.abs(r) <= 1.0 + 1e-14)                       # Cauchy-Schwarz
    D = ngf.distance(g, R, T, u)
    assert 0.0 <= D <= g.hbar * g.mbar
    # scale covariance: D(cT, c'R; c tau, c' rho) = D(T, R; tau, rho)
    c1, c2 = 3.7, 0.21
    g2 = Grid(g.m, g.h, g.my, g.tau * c1, g.rho * c2, g.alpha)
    assert abs(ngf.distance(g2, c2 * R, c1 * T, u) - D) <= 1e-12 * D
    # offset invariance of R (no Dirichlet effect for the reference)
    assert abs(ngf.distance(g, R + 5.0, T, u) - D) <= 1e-12 * D


def test_one_voxel_pair_by_hand():
    # Two voxels along x, u = 0: differences of T and R are +-(T1-T0) etc.
    g = Grid((2, 1, 1), (1, 1, 1), (2, 2, 2), 0.5, 0.25, 1.0)
    R = np.array([[[1.0, 3.0]]])
    T = np.array([[[2.0, -1.0]]])
    u = np.zeros((3, 2, 2, 2))
    # voxel 0: backward x clamped -> 0, forward x: T: -3, R: 2
    num = 0.5 * (-3.0 * 2.0) + 0.5 * 0.25
    nT = np.sqrt(0.5 * 9.0 + 0.25)
    nR = np.sqrt(0.5 * 4.0 + 0.0625)
    r0 = num / (nT * nR)
    # voxel 1 has the same single non-zero difference (backward x)
    want = 2.0 * (1.0 - r0 * r0)
    assert abs(ngf.distance(g, R, T, u) - want) < 1e-14


# ---------------------------------------------------------------------------
# Derivatives (eq. NGF_discretized_gradient / _hessian)
# ---------------------------------------------------------------------------

def _fd_dir(f, u, d, e=1e-6):
    return (f(u + e * d) - f(u - e * d)) / (2 * e)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_against_fd_of_bruteforce(seed):
    g, R, T, u, rng = tiny_problem(seed)
    grad = ngf.gradient_D(g, R, T, u)

    def Db(uu):
        return bruteforce.objective_D(g.m, g.h, g.my, g.tau, g.rho, R.tolist(), T.tolist(), uu.tolist())

    for _ in range(3):
        d = rng.standard_normal(u.shape)
        fd = _fd_dir(Db, u, d)
        assert abs(fd - np.sum(grad * d)) <= 1e-6 * max(1.0, abs(fd))


def test_gradient_each_component_fd_including_boundary_nodes():
    # every node / component, catches boundary-only slips (clamped columns)
    g, R, T, u, _ = tiny_problem(3, m=(5, 4, 3), my=(3, 3, 2))
    grad = ngf.gradient_D(g, R, T, u).ravel()
    f = lambda uu: ngf.distance(g, R, T, uu)
    for j in range(grad.size):
        d = np.zeros(grad.size)
        d[j] = 1.0
        fd = _fd_dir(f, u, d.reshape(u.shape))
        assert abs(fd - grad[j]) <= 1e-6 * max(1.0, abs(fd)), j


@pytest.mark.parametrize("seed", [0, 5])
def test_jacobian_against_fd_of_residual_vector(seed):
    g, R, T, u, rng = tiny_problem(seed)
    J, _ = ngf.jacobian(g, R, T, u)
    for _ in range(3):
        p = rng.standard_normal(u.shape)
        fd = _fd_dir(lambda uu: ngf.residual(g, R, T, uu).ravel(), u, p)
        np.testing.assert_allclose(J @ p.ravel(), fd, rtol=1e-6, atol=1e-8)


def test_hessian_symmetric_psd_and_gauss_newton_form():
    g, R, T, u, rng = tiny_problem(2)
    J, _ = ngf.jacobian(g, R, T, u)
    n = 3 * g.nbar
    H = np.stack([ngf.hess_vec_D(g, R, T, u, e.reshape(u.shape), J).ravel() for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > -1e-10 * np.abs(H).max()
    # <p, H p> = 2 hbar ||J p||^2 with J p pinned by finite differences
    p = rng.standard_normal(u.shape)
    jp = _fd_dir(lambda uu: ngf.residual(g, R, T, uu).ravel(), u, p)
    php = float(np.sum(p * ngf.hess_vec_D(g, R, T, u, p, J)))
    assert abs(php - 2 * g.hbar * float(jp @ jp)) <= 1e-6 * php
    # diagonal = e_j^T H e_j
    np.testing.assert_allclose(ngf.hessian_diag_D(g, R, T, u, J).ravel(), np.diag(H), rtol=1e-12, atol=1e-14)


def test_dr_structure_seven_nonzeros_and_25_offsets_of_drTdr():
    # eq. dr: 7 non-zeros per interior row; Table hessian_indices: interior
    # rows of dr^T dr have exactly the 25 listed offsets.
    rng = np.random.default_rng(9)
    m = (9, 8, 7)
    g = Grid(m, (1, 1, 1), (4, 4, 4), 0.3, 0.3, 1)
    R = rng.standard_normal((m[2], m[1], m[0]))
    T = rng.standard_normal((m[2], m[1], m[0]))
    u = 0.3 * rng.standard_normal((3, 4, 4, 4))
    dr, _ = ngf.dr_rows(g, R, T, u, np.arange(g.mbar))
    i0 = g.voxel_id(4, 4, 3)
    assert dr[i0].nnz == 7
    M = (dr.T @ dr).tocsr()
    cols = M[i0].indices
    a, b, c = g.voxel_abc(cols)
    got = sorted(zip((c - 3).tolist(), (b - 4).tolist(), (a - 4).tolist()))
    table = np.loadtxt(os.path.join(GOLDEN, "hessian_offsets.txt"), dtype=int)
    offs = {tuple(r[:3]) for r in table} | {tuple(-r[:3]) for r in table}
    assert len(offs) == 25
    assert got == sorted(offs)
    # multiplicities of Table hessian_indices = |N^{-1}(kappa)| over M x M
    Mset = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    for r in table:
        k = tuple(r[:3])
        cnt = sum(1 for p in Mset for q in Mset if tuple(np.subtract(q, p)) == k)
        assert cnt == r[3]
    mult = {tuple(r[:3]): int(r[3]) for r in table}
    mult.update({tuple(-r[:3]): int(r[3]) for r in table})
    assert sum(mult.values()) == 49 == len(Mset) ** 2


def test_residual_one_where_translation_aligns_exactly():
    # T is R shifted by whole cells; the displacement u = (0, -1, +1) cells
    # samples T exactly at cell centres, so T(P y) = R wherever the sample and
    # its neighbours stay inside the template, and there r = 1 (tau = rho).
    rng = np.random.default_rng(12)
    m = (8, 6, 5)
    g = Grid(m, (1, 1, 1), (5, 4, 3), 0.4, 0.4, 1)
    big = rng.standard_normal((m[2] + 4, m[1] + 4, m[0] + 4))
    R = big[2:-2, 2:-2, 2:-2]
    T = big[1:-3, 3:-1, 2:-2]          # T[c, b, a] = R[c - 1, b + 1, a]
    u = np.zeros((3, 3, 4, 5))
    u[1] = -1.0
    u[2] = 1.0
    r = ngf.residual(g, R, T, u)
    np.testing.assert_allclose(r[0:m[2] - 2, 2:, :], 1.0, atol=1e-13)
    assert np.abs(r[:, 0, :] - 1.0).max() > 1e-3      # the Dirichlet edge does not align


# ---------------------------------------------------------------------------
# Curvature (eq. CURV_discretized, eq. curvatureMF, eq. curv_hessMult)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("my,hy_cells", [((5, 4, 3), (8, 6, 4)), ((7, 7, 7), (6, 6, 6))])
def test_curvature_against_bruteforce_and_closed_forms(my, hy_cells):
    g = Grid(hy_cells, (1.0, 1.0, 1.0), my, 1, 1, 1)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((3, my[2], my[1], my[0]))
    S = curvature.energy(g, u)
    Sb = bruteforce.curvature_S(my, g.hy, u.tolist())
    assert abs(S - Sb) <= 1e-12 * Sb
    L = curvature.laplacian(g)
    assert abs(L - L.T).max() < 1e-14                                  # symmetric with clamping
    # translations: S = 0, grad S = 0
    t = np.broadcast_to(np.array([1.5, -2.0, 0.3])[:, None, None, None], u.shape).copy()
    assert curvature.energy(g, t) < 1e-28
    np.testing.assert_allclose(curvature.gradient(g, t), 0.0, atol=1e-13)
    # linear u: zero Laplacian inside; boundary nodes see the one-sided term
    xy = g.node_positions()
    lin = np.stack([0.5 * xy[0], np.zeros_like(xy[0]), np.zeros_like(xy[0])])
    lap = (L @ lin[0].ravel()).reshape(my[2], my[1], my[0])
    a = 0.5
    want = np.zeros_like(lap)
    want[:, :, 0] = a / g.hy[0]
    want[:, :, -1] = -a / g.hy[0]
    np.testing.assert_allclose(lap, want, atol=1e-13)
    assert abs(curvature.energy(g, lin) - g.hybar * np.sum(want ** 2)) < 1e-12
    # gradient by FD (quadratic: central differences are exact up to rounding)
    d = rng.standard_normal(u.shape)
    fd = _fd_dir(lambda uu: curvature.energy(g, uu, L), u, d, 1e-3)
    gr = curvature.gradient(g, u, L)
    assert abs(fd - np.sum(gr * d)) <= 1e-8 * abs(fd)
    # Hessian quadratic form and diagonal
    php = np.sum(d * curvature.hess_vec(g, d, L))
    Lp = np.stack([L @ d[k].ravel() for k in range(3)])
    assert abs(php - 2 * g.hybar * np.sum(Lp ** 2)) <= 1e-12 * php
    diag = curvature.hessian_diag(g, L)[0]
    hy = g.hy
    interior = (sum(2 / hy[k] ** 2 for k in range(3))) ** 2 + sum(2 / hy[k] ** 4 for k in range(3))
    assert abs(diag[1, 1, 1] - 2 * g.hybar * interior) < 1e-12 * diag[1, 1, 1]


# ---------------------------------------------------------------------------
# Exact single-node evaluation (used for sampled parity on large problems)
# ---------------------------------------------------------------------------

def test_node_outputs_match_full_evaluation():
    g, R, T, u, rng = tiny_problem(8, m=(10, 9, 8), my=(5, 4, 4))
    p = rng.standard_normal(u.shape)
    grad = ngf.gradient_D(g, R, T, u)
    hv = ngf.hess_vec_D(g, R, T, u, p)
    diag = ngf.hessian_diag_D(g, R, T, u)
    for node in [0, g.nbar - 1, g.node_id(2, 1, 2), g.node_id(4, 3, 0), g.node_id(1, 2, 3)]:
        gn, hn, dn = ngf.node_outputs(g, R, T, u, p, node)
        a, b, c = g.node_abc(node)
        np.testing.assert_allclose(gn, grad[:, c, b, a], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(hn, hv[:, c, b, a], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(dn, diag[:, c, b, a], rtol=1e-12, atol=1e-13)


def test_curvature_node_outputs_match_full_evaluation():
    g, R, T, u, rng = tiny_problem(9, m=(10, 9, 8), my=(5, 4, 6))
    p = rng.standard_normal(u.shape)
    grad = curvature.gradient(g, u)
    hv = curvature.hess_vec(g, p)
    diag = curvature.hessian_diag(g)
    for node in [0, g.nbar - 1, g.node_id(2, 1, 2), g.node_id(4, 3, 0), g.node_id(1, 2, 5), g.node_id(4, 0, 3)]:
        gn, hn, dn = curvature.node_outputs(g, u, p, node)
        a, b, c = g.node_abc(node)
        np.testing.assert_allclose(gn, grad[:, c, b, a], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(hn, hv[:, c, b, a], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(dn, diag[:, c, b, a], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Solvers (Sec. 2.3)
# ---------------------------------------------------------------------------

def test_pcg_matches_dense_solve_and_monotone_energy_error():
    rng = np.random.default_rng(0)
    n = 40
    B = rng.standard_normal((n, n))
    A = B @ B.T + 0.5 * np.eye(n)
    b = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)
    errs = []

    def apply(p):
        return A @ p

    x, info = solver.pcg(apply, b, np.diag(A), max_iter=200, rtol=1e-12)
    assert info["flag"] == 0
    np.testing.assert_allclose(x, xs, rtol=1e-8, atol=1e-10)
    for k in range(1, 15):
        xk, _ = solver.pcg(apply, b, np.diag(A), max_iter=k, rtol=0.0)
        e = xk - xs
        errs.append(float(e @ A @ e))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))


def test_pcg_breakdown_flag():
    A = np.diag([1.0, -1.0])
    _, info = solver.pcg(lambda p: A @ p, np.array([0.0, 1.0]), None, 10, 1e-10)
    assert info["flag"] == 2


def test_pcg_zero_diagonal_entries_left_unscaled():
    # a block-diagonal system with a zero block: Jacobi with zero entries acts as 1
    # there, so the iterates equal those of the solve on the non-zero block alone
    rng = np.random.default_rng(2)
    B = rng.standard_normal((6, 6))
    A1 = B @ B.T + 0.5 * np.eye(6)
    A = np.zeros((9, 9))
    A[:6, :6] = A1
    b = np.concatenate([rng.standard_normal(6), np.zeros(3)])
    d = np.concatenate([np.diag(A1), np.zeros(3)])
    for k in (1, 3, 6):
        s, info = solver.pcg(lambda p: A @ p, b, d, k, 0.0)
        s1, info1 = solver.pcg(lambda p: A1 @ p, b[:6], np.diag(A1), k, 0.0)
        assert np.all(np.isfinite(s)) and np.all(s[6:] == 0.0)
        np.testing.assert_allclose(s[:6], s1, rtol=1e-12, atol=1e-14)
        assert info["iters"] == info1["iters"]


def test_gauss_newton_monotone_on_tiny_problem():
    g, R, T, u, rng = tiny_problem(1, m=(8, 7, 6), my=(5, 4, 4), amp=0.0)
    T = R + 0.1 * rng.standard_normal(R.shape)
    prob = solver.Problem(g, R, T)
    _, hist = solver.gauss_newton(prob, u, iters=3, pcg_max=20, pcg_rtol=1e-3)
    Js = [h["J"] for h in hist] + [hist[-1].get("J_new", hist[-1]["J"])]
    assert all(Js[i + 1] <= Js[i] for i in range(len(Js) - 1))


def test_prolongation_exact_for_linear_fields_and_restriction_of_constants():
    g = Grid((16, 12, 8), (1, 1, 1), (9, 7, 5), 1, 1, 1)
    gc = multilevel.coarse_grid(g)
    assert gc.m == (8, 6, 4) and gc.my == (5, 4, 3)
    xc = gc.node_positions()
    uc = np.stack([0.3 * xc[0] - 0.1 * xc[2], 0.2 * xc[1], -0.4 * xc[0] + 1.0])
    uf = multilevel.prolong(uc, gc, g)
    xf = g.node_positions()
    want = np.stack([0.3 * xf[0] - 0.1 * xf[2], 0.2 * xf[1], -0.4 * xf[0] + 1.0])
    np.testing.assert_allclose(uf, want, atol=1e-12)
    I = np.full((7, 5, 9), 2.5)
    Ic = multilevel.restrict_image(I)
    assert Ic.shape == (4, 3, 5)
    np.testing.assert_allclose(Ic, 2.5)


def _restrict_loops(I):
    """The 2x2x2 mean by explicit loops over coarse voxels and their (up to 8)
    fine children, an index past the end replaced by the last one."""
    mz, my, mx = I.shape
    out = np.zeros(((mz + 1) // 2, (my + 1) // 2, (mx + 1) // 2))
    for c in range(out.shape[0]):
        for b in range(out.shape[1]):
            for a in range(out.shape[2]):
                acc = 0.0
                for k in (0, 1):
                    for j in (0, 1):
                        for i in (0, 1):
                            acc += I[min(2 * c + k, mz - 1), min(2 * b + j, my - 1), min(2 * a + i, mx - 1)]
                out[c, b, a] = acc / 8.0
    return out


@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 7, 3), (1, 2, 3), (3, 1, 1), (9, 4, 6)])
def test_restriction_brute_force_loops_odd_and_even(shape):
    # Sec. 2.3 (coarse-to-fine): one pyramid level of random images of odd and even sizes
    I = np.random.default_rng(sum(shape)).standard_normal(shape)
    np.testing.assert_allclose(multilevel.restrict_image(I), _restrict_loops(I), rtol=0, atol=1e-14)


def test_restriction_reproduces_linear_fields_at_coarse_centres():
    # a field linear in the position, sampled at fine cell centres (a + 1/2) h, restricts to
    # the same field at the coarse cell centres (a' + 1/2) 2h: this fixes the voxel pairing
    # (a shifted pairing moves it by h, subsampling by h/2); with odd sizes the last coarse
    # cell is the mean of the last fine cell with itself, i.e. that cell's value
    mz, my, mx = 6, 8, 10
    z, y, x = np.meshgrid(np.arange(mz) + 0.5, np.arange(my) + 0.5, np.arange(mx) + 0.5, indexing="ij")
    I = 0.7 * x - 1.3 * y + 0.4 * z + 2.0
    zc, yc, xc = np.meshgrid(2 * (np.arange(3) + 0.5), 2 * (np.arange(4) + 0.5), 2 * (np.arange(5) + 0.5),
                             indexing="ij")
    np.testing.assert_allclose(multilevel.restrict_image(I), 0.7 * xc - 1.3 * yc + 0.4 * zc + 2.0, atol=1e-13)
    I2 = (0.5 * (np.arange(7) + 0.5))[None, None, :] * np.ones((2, 2, 7))   # odd x: 7 cells
    Ic = multilevel.restrict_image(I2)[0, 0]
    np.testing.assert_allclose(Ic[:3], 0.5 * 2 * (np.arange(3) + 0.5), atol=1e-14)
    assert Ic[3] == I2[0, 0, 6]


def test_restriction_preserves_the_mean_and_annihilates_the_checkerboard():
    rng = np.random.default_rng(11)
    I = rng.standard_normal((6, 4, 8))
    assert abs(multilevel.restrict_image(I).mean() - I.mean()) < 1e-14
    z, y, x = np.meshgrid(np.arange(6), np.arange(4), np.arange(8), indexing="ij")
    np.testing.assert_allclose(multilevel.restrict_image((-1.0) ** (x + y + z)), 0.0, atol=1e-15)
    np.testing.assert_allclose(multilevel.restrict_image((-1.0) ** x), 0.0, atol=1e-15)


def test_prolongation_exact_at_coincident_nodes_and_partition_of_unity():
    # every other fine node sits on a coarse node (ceil((my - 1)/2) coarse cells of twice
    # the spacing): the prolongated field takes the coarse value there exactly; constants stay
    g = Grid((16, 12, 8), (1, 1, 1), (9, 7, 5), 1, 1, 1)
    gc = multilevel.coarse_grid(g)
    uc = np.random.default_rng(3).standard_normal((3, gc.my[2], gc.my[1], gc.my[0]))
    uf = multilevel.prolong(uc, gc, g)
    np.testing.assert_allclose(uf[:, ::2, ::2, ::2], uc, atol=1e-14)
    np.testing.assert_allclose(multilevel.prolong(np.full_like(uc, 1.5), gc, g), 1.5, atol=1e-14)
    # odd deformation-cell counts (5 fine cells -> 3 coarse ones of spacing 10/3): fine
    # nodes no longer coincide with coarse ones, linear fields are still reproduced
    g2 = Grid((10, 9, 7), (1, 1, 1), (6, 4, 4), 1, 1, 1)
    gc2 = multilevel.coarse_grid(g2)
    assert gc2.my == (4, 3, 3)
    xc = gc2.node_positions()
    xf = g2.node_positions()
    lin = lambda X: np.stack([0.2 * X[0] + 0.1 * X[1], -0.3 * X[2] + 0.5, 0.05 * X[0] - 0.2 * X[1]])
    inside = (xf[1] <= xc[1].max() + 1e-12) & (xf[2] <= xc[2].max() + 1e-12)
    uf2 = multilevel.prolong(lin(xc), gc2, g2)
    np.testing.assert_allclose(uf2[:, inside], lin(xf)[:, inside], atol=1e-12)


# ---------------------------------------------------------------------------
# Sum-of-squared-differences distance (Sec. 4.4: dr/dT = identity)
# ---------------------------------------------------------------------------

def ssd_problem(seed=0, m=(6, 5, 4), my=(4, 3, 3), h=(1.0, 1.2, 0.9), alpha=0.7, amp=0.4):
    rng = np.random.default_rng(seed)
    g = Grid(m, h, my, 1.0, 1.0, alpha, distance="ssd")
    R = rng.standard_normal((m[2], m[1], m[0]))
    T = rng.standard_normal((m[2], m[1], m[0]))
    u = amp * rng.standard_normal((3, my[2], my[1], my[0]))
    return g, R, T, u, rng


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ssd_distance_matches_bruteforce_loops(seed):
    g, R, T, u, _ = ssd_problem(seed)
    ref = bruteforce.objective_ssd(g.m, g.h, g.my, R.tolist(), T.tolist(), u.tolist())
    assert abs(ssd.distance(g, R, T, u) - ref) <= 1e-12 * abs(ref)


def test_ssd_closed_forms_at_zero_displacement():
    # u = 0 puts every voxel on its template sample (up to the rounding of
    # (a + 1/2) h / h - 1/2 for spacings such as 0.9): T = R + c gives
    # D = hbar/2 mbar c^2; T = R gives D = 0 and a zero gradient
    g, R, _, _, _ = ssd_problem(3)
    u0 = np.zeros((3, g.my[2], g.my[1], g.my[0]))
    c = 0.37
    assert abs(ssd.distance(g, R, R + c, u0) - 0.5 * g.hbar * g.mbar * c * c) <= 1e-12
    assert ssd.distance(g, R, R, u0) <= 1e-24
    assert np.abs(ssd.gradient_D(g, R, R, u0)).max() <= 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_ssd_gradient_against_fd_of_bruteforce(seed):
    g, R, T, u, rng = ssd_problem(seed)
    grad = ssd.gradient_D(g, R, T, u)

    def Db(uu):
        return bruteforce.objective_ssd(g.m, g.h, g.my, R.tolist(), T.tolist(), uu.tolist())

    for _ in range(3):
        d = rng.standard_normal(u.shape)
        fd = _fd_dir(Db, u, d)
        assert abs(fd - np.sum(grad * d)) <= 1e-6 * max(1.0, abs(fd))


def test_ssd_gradient_each_component_fd_including_boundary_nodes():
    g, R, T, u, _ = ssd_problem(4, m=(5, 4, 3), my=(3, 3, 2))
    grad = ssd.gradient_D(g, R, T, u).ravel()
    f = lambda uu: ssd.distance(g, R, T, uu)
    for j in range(grad.size):
        d = np.zeros(grad.size)
        d[j] = 1.0
        fd = _fd_dir(f, u, d.reshape(u.shape))
        assert abs(fd - grad[j]) <= 1e-6 * max(1.0, abs(fd)), j


def test_ssd_hessian_is_the_true_hessian_where_the_residual_vanishes():
    # With R = T(P y) (from the brute-force loops) the residual is 0 at u, so the
    # dropped second-derivative term vanishes and the Gauss-Newton product equals
    # the derivative of the gradient (centred differences along p).
    g, _, T, u, rng = ssd_problem(5)
    R = np.array(bruteforce.warped_template(g.m, g.h, g.my, T.tolist(), u.tolist()))
    assert np.abs(ssd.residual(g, R, T, u)).max() <= 1e-13
    J, _ = ssd.jacobian(g, R, T, u)
    for _ in range(3):
        p = rng.standard_normal(u.shape)
        fd = _fd_dir(lambda uu: ssd.gradient_D(g, R, T, uu), u, p)
        hp = ssd.hess_vec_D(g, R, T, u, p, J)
        np.testing.assert_allclose(hp, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def test_ssd_hessian_symmetric_psd_diagonal_and_node_outputs():
    g, R, T, u, rng = ssd_problem(6, m=(7, 6, 5), my=(4, 4, 3))
    J, _ = ssd.jacobian(g, R, T, u)
    n = 3 * g.nbar
    H = np.stack([ssd.hess_vec_D(g, R, T, u, e.reshape(u.shape), J).ravel() for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > -1e-10 * np.abs(H).max()
    # <p, H p> = hbar ||J p||^2 with J p from differences of the residual vector
    p = rng.standard_normal(u.shape)
    jp = _fd_dir(lambda uu: ssd.residual(g, R, T, uu).ravel(), u, p)
    php = float(np.sum(p * ssd.hess_vec_D(g, R, T, u, p, J)))
    assert abs(php - g.hbar * float(jp @ jp)) <= 1e-6 * php
    np.testing.assert_allclose(ssd.hessian_diag_D(g, R, T, u, J).ravel(), np.diag(H), rtol=1e-12, atol=1e-14)
    grad = ssd.gradient_D(g, R, T, u)
    hv = ssd.hess_vec_D(g, R, T, u, p, J)
    diag = ssd.hessian_diag_D(g, R, T, u, J)
    for node in [0, g.nbar - 1, g.node_id(2, 1, 2), g.node_id(3, 3, 0), g.node_id(1, 2, 1)]:
        gn, hn, dn = ssd.node_outputs(g, R, T, u, p, node)
        a, b, c = g.node_abc(node)
        np.testing.assert_allclose(gn, grad[:, c, b, a], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(hn, hv[:, c, b, a], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(dn, diag[:, c, b, a], rtol=1e-12, atol=1e-13)


def test_ssd_gauss_newton_reduces_objective_and_multilevel_keeps_distance():
    g, R, T, u, _ = ssd_problem(7, m=(8, 7, 6), my=(5, 4, 4), amp=0.0)
    prob = solver.Problem(g, R, T)
    J0 = prob.objective(u)[0]
    u1, hist = solver.gauss_newton(prob, u, iters=3)
    assert prob.objective(u1)[0] < J0
    assert all(h["J_new"] <= h["J"] for h in hist if "J_new" in h)
    assert multilevel.coarse_grid(g).distance == "ssd"


# ---------------------------------------------------------------------------
# L-BFGS with H_0 = alpha nabla^2 S + gamma I (Sec. 2.3.2)
# ---------------------------------------------------------------------------

def test_lbfgs_two_loop_equals_dense_bfgs_inverse_update():
    # the recursion against the textbook product form of the inverse update,
    # H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T from H = H_0^{-1}
    rng = np.random.default_rng(11)
    n = 12
    B = rng.standard_normal((n, n))
    H0 = B @ B.T + n * np.eye(n)
    H0inv = np.linalg.inv(H0)
    A = rng.standard_normal((n, n))
    A = A @ A.T + np.eye(n)
    pairs = []
    H = H0inv.copy()
    for _ in range(4):
        s = rng.standard_normal(n)
        y = A @ s
        rho = 1.0 / float(s @ y)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
        pairs.append((s, y))
    g = rng.standard_normal(n)
    d = lbfgs.two_loop(g, pairs, lambda v: H0inv @ v)
    np.testing.assert_allclose(d, -H @ g, rtol=1e-10, atol=1e-12)
    # secant condition of the newest pair
    s, y = pairs[-1]
    np.testing.assert_allclose(-lbfgs.two_loop(y, pairs, lambda v: H0inv @ v), s, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("my,gamma", [((5, 4, 3), 0.3), ((6, 2, 4), 2.0)])
def test_h0_solver_on_cosine_eigenvectors(my, gamma):
    # the Neumann Laplacian's eigenvectors are the DCT-II cosines
    # cos(pi k (i + 1/2) / n) with eigenvalue -4 sin^2(pi k / 2n) / hy^2 per axis
    g = Grid((12, 9, 8), (1.0, 1.3, 0.8), my, 1.0, 1.0, 0.7)
    h0 = lbfgs.H0Solver(g, gamma)
    for ks in [(0, 0, 0), (1, 0, 2), (my[0] - 1, my[1] - 1, my[2] - 1), (2, 1, 1)]:
        ks = tuple(min(k, n - 1) for k, n in zip(ks, my))
        axes = [np.cos(np.pi * ks[d] * (np.arange(my[d]) + 0.5) / my[d]) for d in range(3)]
        v = np.einsum("k,j,i->kji", axes[2], axes[1], axes[0])
        lam = -sum(4.0 * np.sin(np.pi * ks[d] / (2 * my[d])) ** 2 / g.hy[d] ** 2 for d in range(3))
        mu = 2.0 * g.alpha * g.hybar * lam * lam + gamma
        V = np.stack([v, 2.0 * v, -v])
        np.testing.assert_allclose(h0.apply(V), V / mu, rtol=1e-9, atol=1e-12)


def test_lbfgs_first_step_is_the_regularised_newton_step():
    # zero images (SSD): D = 0 and J = alpha S is quadratic with Hessian A = alpha nabla^2 S,
    # so the first step is -(A + gamma I)^{-1} A u0 and eta = 1 passes the Armijo test
    g = Grid((10, 8, 7), (1.0, 1.0, 1.0), (5, 4, 4), 1.0, 1.0, 0.6, distance="ssd")
    rng = np.random.default_rng(4)
    Z = np.zeros((7, 8, 10))
    prob = solver.Problem(g, Z, Z)
    u0 = rng.standard_normal((3, 4, 4, 5))
    gamma = 0.05
    u1, hist = lbfgs.lbfgs(prob, u0, iters=1, gamma=gamma)
    L = curvature.laplacian(g)
    A = 2.0 * g.alpha * g.hybar * (L.T @ L).toarray()
    M = A + gamma * np.eye(g.nbar)
    want = np.stack([u0[d].ravel() - np.linalg.solve(M, A @ u0[d].ravel()) for d in range(3)]).reshape(u0.shape)
    assert hist[0]["eta"] == 1.0
    np.testing.assert_allclose(u1, want, rtol=1e-9, atol=1e-11)


def test_lbfgs_monotone_armijo_and_curvature_pairs_on_tiny_problem():
    g, R, T, u, rng = tiny_problem(12, m=(9, 8, 7), my=(5, 4, 4), amp=0.0)
    T = R + 0.2 * rng.standard_normal(R.shape)
    prob = solver.Problem(g, R, T)
    recs = []
    u1, hist = lbfgs.lbfgs(prob, u, iters=6, mem=3, gamma=0.5, callback=lambda rec, uu, d: recs.append(
        (rec["J"], float(np.sum(prob.gradient(uu)[1] * d)))))
    assert len(hist) >= 3
    for h, (J0, slope) in zip(hist, recs):
        assert slope < 0
        if "J_new" in h:
            assert h["J_new"] <= h["J"] + 1e-4 * h["eta"] * slope + 1e-14
    assert prob.objective(u1)[0] < prob.objective(u)[0]


# ---------------------------------------------------------------------------
# Diffusive regulariser (Sec. 4.4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("my,h", [((4, 3, 5), (1.0, 1.2, 0.9)), ((2, 6, 3), (0.5, 1.0, 2.0))])
def test_diffusive_energy_bruteforce_closed_forms_and_laplacian(my, h):
    rng = np.random.default_rng(21)
    m = tuple(2 * (n - 1) for n in my)
    g = Grid(m, h, my, 1.0, 1.0, 0.7, regulariser="diffusive")
    u = rng.standard_normal((3, my[2], my[1], my[0]))
    ref = bruteforce.diffusive_S(g.my, g.hy, u.tolist())
    assert abs(diffusive.energy(g, u) - ref) <= 1e-12 * abs(ref)
    # constants cost nothing; a linear field a.x in component d costs
    # hbar^y/2 sum_k a_k^2 (edges along k)
    X = g.node_positions()
    assert diffusive.energy(g, np.ones_like(u) * 3.0) == 0.0
    a = (0.3, -0.2, 0.5)
    lin = np.zeros_like(u)
    lin[1] = a[0] * X[0] + a[1] * X[1] + a[2] * X[2]
    edges = [(my[0] - 1) * my[1] * my[2], my[0] * (my[1] - 1) * my[2], my[0] * my[1] * (my[2] - 1)]
    want = 0.5 * g.hybar * sum(a[k] ** 2 * edges[k] for k in range(3))
    assert abs(diffusive.energy(g, lin) - want) <= 1e-12 * want
    # the operator is minus the clamped 7-point Laplacian of the curvature term
    np.testing.assert_allclose(diffusive.operator(g).toarray(), -curvature.laplacian(g).toarray(), atol=1e-12)


def test_diffusive_gradient_fd_hessian_diag_and_node_outputs():
    rng = np.random.default_rng(22)
    my = (5, 4, 3)
    g = Grid((8, 6, 4), (1.0, 1.3, 0.8), my, 1.0, 1.0, 0.5, regulariser="diffusive")
    u = rng.standard_normal((3, my[2], my[1], my[0]))
    grad = diffusive.gradient(g, u).ravel()
    f = lambda uu: diffusive.energy(g, uu)
    for j in range(grad.size):
        d = np.zeros(grad.size)
        d[j] = 1.0
        fd = _fd_dir(f, u, d.reshape(u.shape))
        assert abs(fd - grad[j]) <= 1e-6 * max(1.0, abs(fd)), j
    p = rng.standard_normal(u.shape)
    # quadratic: the Hessian product equals the gradient's directional derivative exactly
    np.testing.assert_allclose(diffusive.hess_vec(g, p).ravel(), _fd_dir(lambda uu: diffusive.gradient(g, uu), u, p).ravel(),
                               rtol=1e-7, atol=1e-9)
    H = diffusive.hessian_matrix(g).toarray()
    np.testing.assert_allclose(diffusive.hessian_diag(g)[0].ravel(), np.diag(H), rtol=1e-12)
    gr, hv, dg = diffusive.gradient(g, u), diffusive.hess_vec(g, p), diffusive.hessian_diag(g)
    for node in [0, g.nbar - 1, g.node_id(2, 1, 1), g.node_id(4, 0, 2)]:
        gn, hn, dn = diffusive.node_outputs(g, u, p, node)
        a, b, c = g.node_abc(node)
        np.testing.assert_allclose(gn, gr[:, c, b, a], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(hn, hv[:, c, b, a], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(dn, dg[:, c, b, a], rtol=1e-12, atol=1e-12)


def test_problem_and_h0_use_the_diffusive_regulariser():
    g, R, T, u, rng = tiny_problem(23, m=(8, 7, 6), my=(5, 4, 4))
    gd = Grid(g.m, g.h, g.my, g.tau, g.rho, g.alpha, regulariser="diffusive")
    prob = solver.Problem(gd, R, T)
    Jv, D, S = prob.objective(u)
    assert abs(S - diffusive.energy(gd, u)) <= 1e-12 * S and abs(Jv - (D + gd.alpha * S)) <= 1e-12 * abs(Jv)
    h0 = lbfgs.H0Solver(gd, 0.3)
    v = rng.standard_normal(u.shape)
    np.testing.assert_allclose(h0.matvec(h0.apply(v)), v, rtol=1e-9, atol=1e-11)
    A = gd.alpha * diffusive.hessian_matrix(gd).toarray() + 0.3 * np.eye(gd.nbar)
    np.testing.assert_allclose(h0.apply(v)[0].ravel(), np.linalg.solve(A, v[0].ravel()), rtol=1e-9, atol=1e-11)
    assert multilevel.coarse_grid(gd).regulariser == "diffusive"


# ---------------------------------------------------------------------------
# Linear-elastic regulariser (Sec. 4.4)
# ---------------------------------------------------------------------------

def test_elastic_energy_bruteforce_divergence_of_linear_fields_and_limits():
    rng = np.random.default_rng(31)
    my, h = (4, 3, 5), (1.0, 1.2, 0.9)
    g = Grid(tuple(2 * (n - 1) for n in my), h, my, 1.0, 1.0, 0.7, regulariser="elastic", lame_mu=0.8,
             lame_lambda=1.7)
    u = rng.standard_normal((3, my[2], my[1], my[0]))
    ref = bruteforce.elastic_S(g.my, g.hy, u.tolist(), 0.8, 1.7)
    assert abs(elastic.energy(g, u) - ref) <= 1e-12 * abs(ref)
    # the cell divergence of a linear field A x is trace(A) in every cell
    A = rng.standard_normal((3, 3))
    X = g.node_positions()
    lin = np.stack([sum(A[d, k] * X[k] for k in range(3)) for d in range(3)])
    div = elastic.divergence(g) @ lin.ravel()
    np.testing.assert_allclose(div, np.trace(A), rtol=1e-12, atol=1e-12)
    # lambda = -mu leaves mu times the diffusive energy; constants cost nothing
    g2 = Grid(g.m, g.h, g.my, 1.0, 1.0, 0.7, regulariser="elastic", lame_mu=0.8, lame_lambda=-0.8)
    assert abs(elastic.energy(g2, u) - 0.8 * diffusive.energy(g2, u)) <= 1e-12 * elastic.energy(g2, u)
    assert elastic.energy(g, np.full_like(u, 2.0)) == 0.0


def test_elastic_gradient_fd_hessian_symmetric_psd_and_diagonal():
    rng = np.random.default_rng(32)
    my = (4, 4, 3)
    g = Grid((6, 6, 4), (1.0, 1.3, 0.8), my, 1.0, 1.0, 0.5, regulariser="elastic", lame_mu=1.3, lame_lambda=0.6)
    u = rng.standard_normal((3, my[2], my[1], my[0]))
    grad = elastic.gradient(g, u)
    for _ in range(4):
        d = rng.standard_normal(u.shape)
        fd = _fd_dir(lambda uu: elastic.energy(g, uu), u, d)
        assert abs(fd - float(np.sum(grad * d))) <= 1e-6 * max(1.0, abs(fd))
    H = elastic.hessian_matrix(g).toarray()
    np.testing.assert_allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.linalg.eigvalsh(H).min() > -1e-10 * np.abs(H).max()
    np.testing.assert_allclose(elastic.hessian_diag(g).ravel(), np.diag(H), rtol=1e-12)
    prob = solver.Problem(g, np.zeros((4, 6, 6)), np.zeros((4, 6, 6)))
    assert abs(prob.objective(u)[2] - elastic.energy(g, u)) <= 1e-12 * elastic.energy(g, u)


def test_elastic_node_outputs_match_full_evaluation():
    rng = np.random.default_rng(33)
    my = (5, 4, 4)
    g = Grid((8, 6, 6), (1.0, 1.2, 0.9), my, 1.0, 1.0, 0.5, regulariser="elastic", lame_mu=0.7, lame_lambda=1.4)
    u = rng.standard_normal((3, my[2], my[1], my[0]))
    p = rng.standard_normal(u.shape)
    gr, hv, dg = elastic.gradient(g, u), elastic.hess_vec(g, p), elastic.hessian_diag(g)
    for node in [0, g.nbar - 1, g.node_id(2, 1, 2), g.node_id(4, 3, 0), g.node_id(1, 2, 3)]:
        gn, hn, dn = elastic.node_outputs(g, u, p, node)
        a, b, c = g.node_abc(node)
        np.testing.assert_allclose(gn, gr[:, c, b, a], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(hn, hv[:, c, b, a], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(dn, dg[:, c, b, a], rtol=1e-12, atol=1e-12)


def test_multilevel_registration_recovers_the_aligning_displacement_where_ngf_sees_edges():
    """Sec. 2.3 on a synthetic warp: the float64 multilevel Gauss-Newton
    registration of a 32 x 32 x 24 CT-like pair moves the displacement towards
    the one that aligns the pair (T is the phantom at x - u*(x), so the aligning
    field solves v = u*(x + v)) along the edge normals (3x smaller RMS error) and
    inside the body.  Over all voxels no such bound holds: where both images are
    constant (the air around the body) NGF carries no information."""
    from oracle import Grid, multilevel
    from synth import GridSpec, alignment_errors, ct_pair

    m = (32, 32, 24)
    spec = GridSpec(m=m, h=(1.0, 1.0, 1.0), my=(17, 17, 13), tau=50.0, rho=50.0, alpha=0.1)
    R, T, _, _ = ct_pair(0, m)
    R = R.numpy().astype(np.float64)
    g = Grid.from_spec(spec)
    u, hists = multilevel.register(g, R, T.numpy().astype(np.float64), levels=3, gn_iters=10, pcg_max=50,
                                   pcg_rtol=1e-3)
    assert all(h[-1]["J_new"] < h[0]["J"] for h in hists)
    uf = u.reshape(3, -1)
    err = alignment_errors(0, m, R, lambda idx: g.P_rows(idx) @ uf.T)
    (n0, n1, _), (b0, b1, _) = err["edges"], err["body"]
    assert n1 <= n0 / 3.0, (n0, n1)
    assert b1 <= 0.5 * b0, (b0, b1)
