"""The two-dimensional case (d = 2) of the whole path: grids, grid conversion,
template, NGF distance and curvature regulariser with their derivatives, the
Gauss-Newton system, and the coarse-to-fine pyramid.

Test infrastructure: a float64 CPU reference, never called by the library.

The paper states its discretisation for general d (Sec. 2.2: cell-centred
image grid, nodal deformation grid spanning the domain, lexicographic x-fastest
ordering, component-major vectors; eq. NGF_discretized with the short
differences of eq. gradient_discretized and clamped neighbours of
eq. boundary_conditions; eq. CURV_discretized with the clamped Laplacian of
eq. laplace_discretized; the chain of eq. function_chain) and runs its GPU
experiments in 2D (Sec. 6.3).  With d = 2:

* P interpolates bilinearly between the 4 nodes around a voxel centre
  (eq. grid_conversion with c_k(a) = (a + 1/2)(my_k - 1)/m_k, the same reading
  as in 3D); u has two components [2][n_y][n_x].
* The template is bilinear with zero extension; its derivative is the exact
  derivative of the interpolant (floor cell at cell faces).
* ||grad I_i||_eps^2 = 1/2 sum_{k in x, y} (Delta_{+k}^2 + Delta_{-k}^2)/h_k^2
  + eps^2: four short differences per voxel, so a row of dr has 5 entries and
  an interior row of dr^T dr has 13 (the d = 2 case of Table hessian_indices).
* L is the 5-point Laplacian with clamped (Neumann) neighbours.

Everything here is written for d = 2 only and shares no code with the 3D
modules of this package (it reuses only the generic CG / Gauss-Newton drivers
of ``solver``, which see the problem through objective / gradient / Hv calls).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .solver import gauss_newton

_DIRS = ("-x", "-y", "+x", "+y")
_AXIS = {"-x": 0, "-y": 1, "+x": 0, "+y": 1}


class Grid2:
    """Image grid (m cells, spacing h), deformation grid (my nodes), template
    grid (mT cells, spacing hT; default the image grid), tau, rho, alpha.
    Sizes are (x, y)."""

    def __init__(self, m, h, my, tau, rho, alpha, mT=None, hT=None):
        self.m = tuple(int(k) for k in m)
        self.h = tuple(float(k) for k in h)
        self.my = tuple(int(k) for k in my)
        self.mT = tuple(int(k) for k in (mT if mT is not None else m))
        self.hT = tuple(float(k) for k in (hT if hT is not None else h))
        self.tau, self.rho, self.alpha = float(tau), float(rho), float(alpha)
        for k in range(2):
            if not (2 <= self.my[k] and self.my[k] - 1 <= self.m[k]):
                raise ValueError("need 2 <= my <= m + 1 in every dimension")

    @classmethod
    def from_spec(cls, spec):
        """From a spec whose m, h, my (and mT, hT) have 2 entries or 3 with a
        trailing 1 (the library's encoding of a 2D problem)."""
        t = lambda a: None if a is None else tuple(a)[:2]
        return cls(t(spec.m), t(spec.h), t(spec.my), spec.tau, spec.rho, spec.alpha,
                   t(getattr(spec, "mT", None)), t(getattr(spec, "hT", None)))

    mbar = property(lambda s: s.m[0] * s.m[1])
    nbar = property(lambda s: s.my[0] * s.my[1])
    hbar = property(lambda s: s.h[0] * s.h[1])
    hy = property(lambda s: tuple(s.m[k] * s.h[k] / (s.my[k] - 1) for k in range(2)))
    hybar = property(lambda s: s.hy[0] * s.hy[1])

    def node_shape(self):
        return (2, self.my[1], self.my[0])

    # indexing -----------------------------------------------------------------
    def voxel_ab(self, vox):
        vox = np.asarray(vox, dtype=np.int64)
        return vox % self.m[0], vox // self.m[0]

    def voxel_id(self, a, b):
        return a + self.m[0] * b

    def node_ab(self, node):
        node = np.asarray(node, dtype=np.int64)
        return node % self.my[0], node // self.my[0]

    def node_id(self, a, b):
        return a + self.my[0] * b

    def voxel_centres(self, vox):
        a, b = self.voxel_ab(vox)
        return np.stack([(a + 0.5) * self.h[0], (b + 0.5) * self.h[1]], axis=-1)

    def node_positions(self):
        """x^y: (2, ny, nx)."""
        Y, X = np.meshgrid(np.arange(self.my[1]) * self.hy[1], np.arange(self.my[0]) * self.hy[0], indexing="ij")
        return np.stack([X, Y])

    def neighbours(self, vox):
        """Clamped neighbours (eq. boundary_conditions, 0-based)."""
        a, b = self.voxel_ab(vox)
        return {"-x": self.voxel_id(np.maximum(a - 1, 0), b), "+x": self.voxel_id(np.minimum(a + 1, self.m[0] - 1), b),
                "-y": self.voxel_id(a, np.maximum(b - 1, 0)), "+y": self.voxel_id(a, np.minimum(b + 1, self.m[1] - 1))}

    # grid conversion ----------------------------------------------------------
    def lower_node(self, k, a):
        """Lower node and fraction along axis k of voxel index a:
        c = (a + 1/2)(my_k - 1)/m_k, lower node min(floor(c), my_k - 2)."""
        c = (np.asarray(a, dtype=np.float64) + 0.5) * (self.my[k] - 1) / self.m[k]
        n0 = np.minimum(np.floor(c), self.my[k] - 2).astype(np.int64)
        return n0, c - n0

    def P_rows(self, vox):
        """Rows of one component block of P: bilinear weights of the 4 nodes."""
        vox = np.asarray(vox, dtype=np.int64)
        a, b = self.voxel_ab(vox)
        i0, fx = self.lower_node(0, a)
        j0, fy = self.lower_node(1, b)
        rows, cols, vals = [], [], []
        loc = np.arange(len(vox))
        for oy in (0, 1):
            for ox in (0, 1):
                rows.append(loc)
                cols.append(self.node_id(i0 + ox, j0 + oy))
                vals.append((fx if ox else 1.0 - fx) * (fy if oy else 1.0 - fy))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(len(vox), self.nbar))

    def P_matrix(self):
        return self.P_rows(np.arange(self.mbar))


# ---------------------------------------------------------------------------
# template and residual
# ---------------------------------------------------------------------------

def template_sample(grid, T, pos):
    """Bilinear template value and gradient at physical points pos (N, 2) with
    zero extension; the gradient is the interpolant's (floor cell at faces)."""
    T = np.asarray(T, dtype=np.float64)
    pos = np.asarray(pos, dtype=np.float64)
    s = pos / np.asarray(grid.hT) - 0.5
    k0 = np.floor(s).astype(np.int64)
    f = s - k0
    val = np.zeros(len(pos))
    grad = np.zeros((len(pos), 2))
    for oy in (0, 1):
        for ox in (0, 1):
            ix, iy = k0[:, 0] + ox, k0[:, 1] + oy
            ok = (ix >= 0) & (ix < grid.mT[0]) & (iy >= 0) & (iy < grid.mT[1])
            t = np.where(ok, T.ravel()[np.where(ok, ix + grid.mT[0] * iy, 0)], 0.0)
            wx = f[:, 0] if ox else 1.0 - f[:, 0]
            wy = f[:, 1] if oy else 1.0 - f[:, 1]
            val += wx * wy * t
            grad[:, 0] += (1.0 if ox else -1.0) / grid.hT[0] * wy * t
            grad[:, 1] += wx * (1.0 if oy else -1.0) / grid.hT[1] * t
    return val, grad


def warped_template(grid, T, u, vox):
    """T(x_i + (P u)_i) and its gradient at the voxels vox (P x^y = x)."""
    vox = np.asarray(vox, dtype=np.int64)
    Pr = grid.P_rows(vox)
    uc = np.asarray(u, dtype=np.float64).reshape(2, grid.nbar)
    pos = grid.voxel_centres(vox) + np.stack([Pr @ uc[0], Pr @ uc[1]], axis=-1)
    return template_sample(grid, T, pos)


def residual_parts(grid, R, T, u, vox):
    """r1, nT, nR, the 4 short differences of T(P y) and R, r = r1/(nT nR)."""
    vox = np.asarray(vox, dtype=np.int64)
    nb = grid.neighbours(vox)
    need = np.unique(np.concatenate([vox] + [nb[d] for d in _DIRS]))
    tw, _ = warped_template(grid, T, u, need)
    Tat = lambda ids: tw[np.searchsorted(need, ids)]
    Rf = np.asarray(R, dtype=np.float64).ravel()
    Rat = lambda ids: Rf[ids]
    dT = np.empty((len(vox), 4))
    dR = np.empty((len(vox), 4))
    for j, d in enumerate(_DIRS):
        hk = grid.h[_AXIS[d]]
        sgn = -1.0 if d[0] == "-" else 1.0   # backward (I_i - I_{i-k}), forward (I_{i+k} - I_i)
        dT[:, j] = sgn * (Tat(nb[d]) - Tat(vox)) / hk
        dR[:, j] = sgn * (Rat(nb[d]) - Rat(vox)) / hk
    r1 = 0.5 * np.sum(dT * dR, axis=1) + grid.tau * grid.rho
    nT = np.sqrt(0.5 * np.sum(dT * dT, axis=1) + grid.tau ** 2)
    nR = np.sqrt(0.5 * np.sum(dR * dR, axis=1) + grid.rho ** 2)
    return dict(r=r1 / (nT * nR), r1=r1, nT=nT, nR=nR, dT=dT, dR=dR)


def distance(grid, R, T, u):
    """D = hbar sum_i (1 - r_i^2) (eq. NGF_discretized_ri)."""
    r = residual_parts(grid, R, T, u, np.arange(grid.mbar))["r"]
    return grid.hbar * float(np.sum(1.0 - r * r))


def dr_rows(grid, R, T, u, rows):
    """Rows of dr/dT (quotient rule, eq. ritcomp) through the 4 x mbar
    Jacobian of the short differences, coinciding (clamped) columns summed."""
    rows = np.asarray(rows, dtype=np.int64)
    p = residual_parts(grid, R, T, u, rows)
    coef = 0.5 * (p["dR"] / (p["nT"] * p["nR"])[:, None] - (p["r1"] / (p["nT"] ** 3 * p["nR"]))[:, None] * p["dT"])
    nb = grid.neighbours(rows)
    loc = np.arange(len(rows))
    ri, ci, vi = [], [], []
    for j, d in enumerate(_DIRS):
        c = coef[:, j] / grid.h[_AXIS[d]]
        lo, hi = (nb[d], rows) if d[0] == "-" else (rows, nb[d])   # difference = (I_hi - I_lo)/h
        ri += [loc, loc]
        ci += [hi, lo]
        vi += [c, -c]
    M = sp.coo_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci))),
                      shape=(len(rows), grid.mbar)).tocsr()
    M.sum_duplicates()
    return M, p["r"]


def jacobian_rows(grid, R, T, u, rows):
    """Rows of J = dr/dT dT/dP P (len(rows) x 2 nbar) and r at those rows."""
    dr, r = dr_rows(grid, R, T, u, rows)
    used = np.unique(dr.indices)
    _, g = warped_template(grid, T, u, used)
    Pr = grid.P_rows(used)
    dtp = sp.hstack([sp.diags(g[:, 0]) @ Pr, sp.diags(g[:, 1]) @ Pr]).tocsr()
    return (dr[:, used] @ dtp).tocsr(), r


def jacobian(grid, R, T, u):
    return jacobian_rows(grid, R, T, u, np.arange(grid.mbar))


def gradient_D(grid, R, T, u):
    """grad D = -2 hbar J^T r (eq. dPsi, eq. NGF_discretized_gradient)."""
    J, r = jacobian(grid, R, T, u)
    return (-2.0 * grid.hbar * (J.T @ r)).reshape(grid.node_shape())


def hess_vec_D(grid, R, T, u, p, J=None):
    """H p = 2 hbar J^T J p (eq. NGF_discretized_hessian, positive semi-definite)."""
    if J is None:
        J, _ = jacobian(grid, R, T, u)
    pv = np.asarray(p, dtype=np.float64).ravel()
    return (2.0 * grid.hbar * (J.T @ (J @ pv))).reshape(grid.node_shape())


def hessian_diag_D(grid, R, T, u, J=None):
    if J is None:
        J, _ = jacobian(grid, R, T, u)
    return (2.0 * grid.hbar * np.asarray(J.multiply(J).sum(axis=0)).ravel()).reshape(grid.node_shape())


def rows_touching_node(grid, node):
    """Residual rows whose Jacobian row reaches node ``node``: voxels of the
    node's 4-node stencil support, dilated by one voxel (the 5-point dr)."""
    na, nb_ = grid.node_ab(node)
    rng = []
    for k, n in enumerate((int(na), int(nb_))):
        a = np.arange(grid.m[k])
        n0, _ = grid.lower_node(k, a)
        sup = a[(n0 == n) | (n0 + 1 == n)]
        rng.append(np.arange(max(0, int(sup.min()) - 1), min(grid.m[k] - 1, int(sup.max()) + 1) + 1))
    B, A = np.meshgrid(rng[1], rng[0], indexing="ij")
    return grid.voxel_id(A.ravel(), B.ravel())


def node_outputs(grid, R, T, u, p, node):
    """Exact (grad D, H p, diag H) at one node (both components) of a problem
    of any size, from the rows of J that touch it."""
    rows = rows_touching_node(grid, node)
    J, r = jacobian_rows(grid, R, T, u, rows)
    Jn = J[:, [node, grid.nbar + node]].toarray()
    grad = -2.0 * grid.hbar * (Jn.T @ r)
    hv = 2.0 * grid.hbar * (Jn.T @ (J @ np.asarray(p, dtype=np.float64).ravel()))
    diag = 2.0 * grid.hbar * np.sum(Jn * Jn, axis=0)
    return grad, hv, diag


# ---------------------------------------------------------------------------
# curvature regulariser
# ---------------------------------------------------------------------------

def laplacian(grid):
    """5-point L (nbar x nbar), rows sum_{k in x, y} (u_{n-k} - 2 u_n + u_{n+k})/hy_k^2,
    clamped neighbours (coinciding columns summed)."""
    n = np.arange(grid.nbar)
    a, b = grid.node_ab(n)
    hy = grid.hy
    ri, ci, vi = [], [], []
    pairs = ((grid.node_id(np.maximum(a - 1, 0), b), grid.node_id(np.minimum(a + 1, grid.my[0] - 1), b)),
             (grid.node_id(a, np.maximum(b - 1, 0)), grid.node_id(a, np.minimum(b + 1, grid.my[1] - 1))))
    for k, (lo, hi) in enumerate(pairs):
        w = 1.0 / hy[k] ** 2
        ri += [n, n, n]
        ci += [lo, n, hi]
        vi += [np.full(len(n), w), np.full(len(n), -2.0 * w), np.full(len(n), w)]
    L = sp.coo_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci))),
                      shape=(grid.nbar, grid.nbar)).tocsr()
    L.sum_duplicates()
    L.eliminate_zeros()
    return L


def curvature_energy(grid, u, L=None):
    """S = hbar^y sum_n sum_d (L u_d)_n^2 (eq. CURV_discretized)."""
    L = laplacian(grid) if L is None else L
    uc = np.asarray(u, dtype=np.float64).reshape(2, grid.nbar)
    return grid.hybar * float(np.sum((L @ uc[0]) ** 2) + np.sum((L @ uc[1]) ** 2))


def curvature_gradient(grid, u, L=None):
    """grad S = 2 hbar^y L^T L u (eq. curvatureMF); also the Hessian product."""
    L = laplacian(grid) if L is None else L
    uc = np.asarray(u, dtype=np.float64).reshape(2, grid.nbar)
    return np.stack([2.0 * grid.hybar * (L.T @ (L @ uc[d])) for d in range(2)]).reshape(grid.node_shape())


def curvature_diag(grid, L=None):
    L = laplacian(grid) if L is None else L
    d = 2.0 * grid.hybar * np.asarray(L.multiply(L).sum(axis=0)).ravel()
    return np.stack([d, d]).reshape(grid.node_shape())


class Problem2:
    """One 2D registration level: J = D + alpha S and its Gauss-Newton system,
    with the interface of solver.Problem (objective, gradient, jacobian,
    hess_vec, jacobi_diag) so that solver.pcg and solver.gauss_newton drive it."""

    def __init__(self, grid, R, T):
        self.grid = grid
        self.R = np.asarray(R, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.float64)
        self.L = laplacian(grid)

    def objective(self, u):
        D = distance(self.grid, self.R, self.T, u)
        S = curvature_energy(self.grid, u, self.L)
        return D + self.grid.alpha * S, D, S

    def gradient(self, u):
        Jv = self.objective(u)[0]
        return Jv, (gradient_D(self.grid, self.R, self.T, u)
                    + self.grid.alpha * curvature_gradient(self.grid, u, self.L))

    def jacobian(self, u):
        return jacobian(self.grid, self.R, self.T, u)[0]

    def hess_vec(self, u, p, Jac=None):
        return (hess_vec_D(self.grid, self.R, self.T, u, p, Jac)
                + self.grid.alpha * curvature_gradient(self.grid, p, self.L))

    def jacobi_diag(self, u, Jac=None):
        return hessian_diag_D(self.grid, self.R, self.T, u, Jac) + self.grid.alpha * curvature_diag(self.grid, self.L)


# ---------------------------------------------------------------------------
# coarse-to-fine (Sec. 2.3), with the readings of the 3D pyramid
# ---------------------------------------------------------------------------

def restrict_image(I):
    """2 x 2 means, ceil(m/2) cells (array order y, x), a missing odd row or
    column replaced by the last one."""
    I = np.asarray(I, dtype=np.float64)
    my, mx = I.shape
    ys = np.arange((my + 1) // 2)
    xs = np.arange((mx + 1) // 2)
    y0, y1 = 2 * ys, np.minimum(2 * ys + 1, my - 1)
    x0, x1 = 2 * xs, np.minimum(2 * xs + 1, mx - 1)
    return 0.25 * ((I[y0][:, x0] + I[y0][:, x1]) + (I[y1][:, x0] + I[y1][:, x1]))


def coarse_grid(g):
    return Grid2(tuple((k + 1) // 2 for k in g.m), tuple(2.0 * k for k in g.h),
                 tuple(int(math.ceil((k - 1) / 2)) + 1 for k in g.my), g.tau, g.rho, g.alpha,
                 tuple((k + 1) // 2 for k in g.mT), tuple(2.0 * k for k in g.hT))


def prolong(u_c, g_c, g_f):
    """Linear interpolation of the coarse node values at the fine node
    positions, per axis, clamped to the coarse extent."""
    mats = []
    for k in range(2):
        t = np.clip(np.arange(g_f.my[k]) * g_f.hy[k] / g_c.hy[k], 0.0, g_c.my[k] - 1)
        k0 = np.minimum(np.floor(t).astype(np.int64), g_c.my[k] - 2)
        f = t - k0
        M = np.zeros((g_f.my[k], g_c.my[k]))
        M[np.arange(g_f.my[k]), k0] += 1.0 - f
        M[np.arange(g_f.my[k]), k0 + 1] += f
        mats.append(M)
    return np.einsum("dji,yj,xi->dyx", np.asarray(u_c, dtype=np.float64), mats[1], mats[0])


def register(grid, R, T, levels=3, gn_iters=10, pcg_max=50, pcg_rtol=1e-3, u0=None, **kw):
    """Multilevel Gauss-Newton; u0 (coarsest grid) or 0.  Returns (u, histories)."""
    pyr = [(grid, np.asarray(R, dtype=np.float64), np.asarray(T, dtype=np.float64))]
    for _ in range(levels - 1):
        g, r, t = pyr[-1]
        pyr.append((coarse_grid(g), restrict_image(r), restrict_image(t)))
    pyr = pyr[::-1]
    u, hists = None, []
    for li, (g, r, t) in enumerate(pyr):
        if u is None:
            u = np.zeros(g.node_shape()) if u0 is None else np.asarray(u0, dtype=np.float64)
        else:
            u = prolong(u, pyr[li - 1][0], g)
        u, h = gauss_newton(Problem2(g, r, t), u, gn_iters, pcg_max, pcg_rtol, **kw)
        hists.append(h)
    return u, hists
