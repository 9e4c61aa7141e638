"""Linear-elastic regulariser on the nodal grid (Sec. 4.4 names it, with the
diffusive one, as a regulariser built from finite differences of the
deformation).

The paper gives no formula; the oracle takes the Navier-Lame energy
S(y) = 1/2 int mu sum_d |grad (y_d - x_d)|^2 + (lambda + mu) (div (y - x))^2
discretised on the nodal grid as

    S(u) = hbar^y / 2 [ mu sum_d sum_k ||D_k u_d||^2 / hy_k^2 + (lambda + mu) ||B u||^2 ],

with D_k the forward node differences of the diffusive regulariser and B the
divergence at the cell centres of the nodal grid: per cell, sum over d of the
mean of its four edge differences along d divided by hy_d.  Gradient and (constant)
Hessian: hbar^y [ mu A u_d (each component) + (lambda + mu) B^T B u ].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import diffusive


def cells(grid):
    return tuple(n - 1 for n in grid.my)


def divergence(grid):
    """B ((nx-1)(ny-1)(nz-1) x 3 nbar): cell-centred divergence, entry by entry."""
    cx, cy, cz = cells(grid)
    nc = cx * cy * cz
    c = np.arange(nc)
    a, b, k = c % cx, (c // cx) % cy, c // (cx * cy)
    rows, cols, vals = [], [], []
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                node = grid.node_id(a + ox, b + oy, k + oz)
                off = (ox, oy, oz)
                for d in range(3):
                    sgn = 1.0 if off[d] else -1.0
                    rows.append(c)
                    cols.append(d * grid.nbar + node)
                    vals.append(np.full(nc, sgn / (4.0 * grid.hy[d])))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nc, 3 * grid.nbar)).tocsr()


def hessian_matrix(grid):
    """The full (3 nbar x 3 nbar) Hessian hbar^y [mu blockdiag(A) + (lambda + mu) B^T B]."""
    A = diffusive.operator(grid)
    B = divergence(grid)
    blk = sp.block_diag([A, A, A])
    return grid.hybar * (grid.lame_mu * blk + (grid.lame_lambda + grid.lame_mu) * (B.T @ B))


def energy(grid, u, H=None):
    uv = np.asarray(u, dtype=np.float64).ravel()
    B = divergence(grid)
    div = B @ uv
    return grid.lame_mu * diffusive.energy(grid, u) + 0.5 * grid.hybar * (grid.lame_lambda + grid.lame_mu) * float(div @ div)


def gradient(grid, u, H=None):
    H = hessian_matrix(grid) if H is None else H
    return (H @ np.asarray(u, dtype=np.float64).ravel()).reshape(3, grid.my[2], grid.my[1], grid.my[0])


def hess_vec(grid, p, H=None):
    return gradient(grid, p, H)


def hessian_diag(grid, H=None):
    H = hessian_matrix(grid) if H is None else H
    return H.diagonal().reshape(3, grid.my[2], grid.my[1], grid.my[0])


def _cell_div(grid, f, a, b, c):
    """Divergence of the node field f (3, nz, ny, nx) at cell (a, b, c)."""
    tot = 0.0
    for d in range(3):
        s = 0.0
        for oz in (0, 1):
            for oy in (0, 1):
                for ox in (0, 1):
                    off = (ox, oy, oz)
                    s += (1.0 if off[d] else -1.0) * f[d][c + oz][b + oy][a + ox]
        tot += s / (4.0 * grid.hy[d])
    return tot


def node_outputs(grid, u, p, node):
    """Exact (grad S, (nabla^2 S) p, diag nabla^2 S) at one node: mu times the
    diffusive node outputs plus (lambda + mu) hbar^y sum over the (up to eight)
    cells at the node of (d div_c / d f_d(node)) div_c."""
    from . import diffusive as _dif
    gd, hd, dd = _dif.node_outputs(grid, u, p, node)
    mu, kap = grid.lame_mu, grid.lame_lambda + grid.lame_mu
    shp = (3, grid.my[2], grid.my[1], grid.my[0])
    uf = np.asarray(u, dtype=np.float64).reshape(shp)
    pf = np.asarray(p, dtype=np.float64).reshape(shp) if p is not None else None
    i, j, k = (int(x) for x in grid.node_abc(node))
    g2, h2, d2 = np.zeros(3), np.zeros(3), np.zeros(3)
    for c in range(max(k - 1, 0), min(k, grid.my[2] - 2) + 1):
        for b in range(max(j - 1, 0), min(j, grid.my[1] - 2) + 1):
            for a in range(max(i - 1, 0), min(i, grid.my[0] - 2) + 1):
                du = _cell_div(grid, uf, a, b, c)
                dp = _cell_div(grid, pf, a, b, c) if pf is not None else 0.0
                cell = (a, b, c)
                nd = (i, j, k)
                for d in range(3):
                    w = (1.0 if cell[d] == nd[d] - 1 else -1.0) / (4.0 * grid.hy[d])
                    g2[d] += w * du
                    h2[d] += w * dp
                    d2[d] += w * w
    s = grid.hybar * kap
    return mu * gd + s * g2, (mu * hd + s * h2 if p is not None else None), mu * dd + s * d2
