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
