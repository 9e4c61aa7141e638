"""Discretised curvature regulariser (Sec. 2.2, eq. CURV_discretized and
eq. laplace_discretized) and its derivatives (Sec. 3.1, eq. curvatureMF;
Sec. 4.2, eq. curv_hessMult).

L is the 7-point Laplacian on the nodal grid with homogeneous Neumann
boundary conditions realised by clamped neighbours (entries of coinciding
columns summed); it acts on each displacement component separately.
S(u) = hbar^y sum_d ||L u_d||^2, grad S = 2 hbar^y L^T L u, and the
(constant) Hessian is 2 hbar^y L^T L.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def laplacian(grid):
    """L (nbar x nbar) with rows sum_k (u_{n-k} - 2 u_n + u_{n+k}) / hy_k^2."""
    n = np.arange(grid.nbar)
    a, b, c = grid.node_abc(n)
    hy = grid.hy
    ri, ci, vi = [], [], []
    for k, (lo, hi) in enumerate((
        (grid.node_id(np.maximum(a - 1, 0), b, c), grid.node_id(np.minimum(a + 1, grid.my[0] - 1), b, c)),
        (grid.node_id(a, np.maximum(b - 1, 0), c), grid.node_id(a, np.minimum(b + 1, grid.my[1] - 1), c)),
        (grid.node_id(a, b, np.maximum(c - 1, 0)), grid.node_id(a, b, np.minimum(c + 1, grid.my[2] - 1))),
    )):
        w = 1.0 / hy[k] ** 2
        ri += [n, n, n]
        ci += [lo, n, hi]
        vi += [np.full(len(n), w), np.full(len(n), -2.0 * w), np.full(len(n), w)]
    L = sp.coo_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci))),
                      shape=(grid.nbar, grid.nbar)).tocsr()
    L.sum_duplicates()
    L.eliminate_zeros()
    return L


def _comps(grid, u):
    return np.asarray(u, dtype=np.float64).reshape(3, grid.nbar)


def energy(grid, u, L=None):
    """S(u) = hbar^y sum_n sum_d (L u_d)_n^2."""
    L = laplacian(grid) if L is None else L
    uc = _comps(grid, u)
    return grid.hybar * float(sum(np.sum((L @ uc[d]) ** 2) for d in range(3)))


def gradient(grid, u, L=None):
    """grad S = 2 hbar^y L^T L u, shaped (3, nz, ny, nx)."""
    L = laplacian(grid) if L is None else L
    uc = _comps(grid, u)
    g = np.stack([2.0 * grid.hybar * (L.T @ (L @ uc[d])) for d in range(3)])
    return g.reshape(3, grid.my[2], grid.my[1], grid.my[0])


def hess_vec(grid, p, L=None):
    """(nabla^2 S) p = 2 hbar^y L^T L p."""
    return gradient(grid, p, L)


def hessian_diag(grid, L=None):
    """diag(2 hbar^y L^T L) = 2 hbar^y (column sums of L o L), per component."""
    L = laplacian(grid) if L is None else L
    d = 2.0 * grid.hybar * np.asarray(L.multiply(L).sum(axis=0)).ravel()
    return np.stack([d, d, d]).reshape(3, grid.my[2], grid.my[1], grid.my[0])


def hessian_matrix(grid, L=None):
    """The per-component Hessian 2 hbar^y L^T L."""
    L = laplacian(grid) if L is None else L
    return 2.0 * grid.hybar * (L.T @ L)


def _row_entries(grid, m):
    """Column -> coefficient of row ``m`` of L (coinciding clamped columns summed)."""
    abc = [int(x) for x in grid.node_abc(m)]
    out = {}
    for k in range(3):
        w = 1.0 / grid.hy[k] ** 2
        lo, hi = list(abc), list(abc)
        lo[k] = max(abc[k] - 1, 0)
        hi[k] = min(abc[k] + 1, grid.my[k] - 1)
        for idx, c in ((lo, w), (abc, -2.0 * w), (hi, w)):
            col = int(grid.node_id(*idx))
            out[col] = out.get(col, 0.0) + c
    return out


def node_outputs(grid, u, p, node):
    """Exact (grad S, (nabla^2 S) p, diag nabla^2 S) at one node (all three
    components) of a grid of any size: (L^T L f)_n = sum over the rows m of L
    with a non-zero in column n (the node and its neighbours) of
    L[m, n] (L f)_m, every row evaluated from its own stencil."""
    abc = [int(x) for x in grid.node_abc(node)]
    rows = {int(node)}
    for k in range(3):
        for s in (-1, 1):
            q = list(abc)
            q[k] += s
            if 0 <= q[k] < grid.my[k]:
                rows.add(int(grid.node_id(*q)))
    uc = _comps(grid, u)
    pc = _comps(grid, p) if p is not None else None
    grad, hv, dg = np.zeros(3), np.zeros(3), 0.0
    for m in sorted(rows):
        e = _row_entries(grid, m)
        lmn = e.get(int(node), 0.0)
        if lmn == 0.0:
            continue
        dg += lmn * lmn
        for d in range(3):
            grad[d] += lmn * sum(c * uc[d][col] for col, c in e.items())
            if pc is not None:
                hv[d] += lmn * sum(c * pc[d][col] for col, c in e.items())
    s = 2.0 * grid.hybar
    return s * grad, (s * hv if pc is not None else None), np.full(3, s * dg)
