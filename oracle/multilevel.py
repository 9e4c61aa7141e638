"""Coarse-to-fine multilevel driver (Sec. 2.3: the problem is solved on
consecutively finer image and deformation grids).

Readings where the paper gives no formula:
* Image pyramid: coarse cells ceil(m/2) per dimension, spacing doubled; a
  coarse voxel is the mean of its 2 x 2 x 2 fine voxels, a missing trailing
  fine plane (odd m) replaced by the last existing one.
* Deformation grid: ceil((my - 1)/2) cells per dimension on the coarse level.
* Prolongation of the displacement: linear interpolation, per dimension, of
  the coarse node values at the physical positions of the fine nodes (clamped
  to the coarse grid's extent).
* The coarsest level starts from u = 0 unless an initial field is given.
"""
from __future__ import annotations

import math

import numpy as np

from .grid import Grid
from .solver import Problem, gauss_newton


def restrict_image(I):
    """2 x 2 x 2 mean with ceil(m/2) output cells (array order z, y, x)."""
    I = np.asarray(I, dtype=np.float64)
    for ax in range(3):
        n = I.shape[ax]
        nc = (n + 1) // 2
        lo = np.take(I, 2 * np.arange(nc), axis=ax)
        hi = np.take(I, np.minimum(2 * np.arange(nc) + 1, n - 1), axis=ax)
        I = 0.5 * (lo + hi)
    return I


def coarse_grid(g):
    m = tuple((k + 1) // 2 for k in g.m)
    h = tuple(2.0 * k for k in g.h)
    my = tuple(int(math.ceil((k - 1) / 2)) + 1 for k in g.my)
    mT = tuple((k + 1) // 2 for k in g.mT)
    hT = tuple(2.0 * k for k in g.hT)
    return Grid(m, h, my, g.tau, g.rho, g.alpha, mT, hT, g.distance, g.regulariser, g.lame_mu, g.lame_lambda)


def _interp_matrix_1d(n_f, hy_f, n_c, hy_c):
    """(n_f x n_c) linear interpolation of coarse node values at fine node positions."""
    x = np.arange(n_f) * hy_f
    t = np.clip(x / hy_c, 0.0, n_c - 1)
    k0 = np.minimum(np.floor(t).astype(np.int64), n_c - 2)
    f = t - k0
    M = np.zeros((n_f, n_c))
    M[np.arange(n_f), k0] += 1.0 - f
    M[np.arange(n_f), k0 + 1] += f
    return M


def prolong(u_c, g_c, g_f):
    """Coarse node field (3, nz, ny, nx) on g_c -> fine node field on g_f."""
    Mx = _interp_matrix_1d(g_f.my[0], g_f.hy[0], g_c.my[0], g_c.hy[0])
    My = _interp_matrix_1d(g_f.my[1], g_f.hy[1], g_c.my[1], g_c.hy[1])
    Mz = _interp_matrix_1d(g_f.my[2], g_f.hy[2], g_c.my[2], g_c.hy[2])
    return np.einsum("dkji,zk,yj,xi->dzyx", np.asarray(u_c, dtype=np.float64), Mz, My, Mx)


def pyramid(grid, R, T, levels):
    """[(grid, R, T)] from coarsest to finest."""
    out = [(grid, np.asarray(R, dtype=np.float64), np.asarray(T, dtype=np.float64))]
    for _ in range(levels - 1):
        g, r, t = out[-1]
        out.append((coarse_grid(g), restrict_image(r), restrict_image(t)))
    return out[::-1]


def register(grid, R, T, levels=3, gn_iters=10, pcg_max=50, pcg_rtol=1e-3, u0=None, **kw):
    """Multilevel Gauss-Newton registration.  Returns (u_finest, per-level histories)."""
    pyr = pyramid(grid, R, T, levels)
    u = None
    hists = []
    for li, (g, r, t) in enumerate(pyr):
        if u is None:
            u = np.zeros((3, g.my[2], g.my[1], g.my[0])) if u0 is None else np.asarray(u0, dtype=np.float64)
        else:
            u = prolong(u, pyr[li - 1][0], g)
        u, h = gauss_newton(Problem(g, r, t), u, gn_iters, pcg_max, pcg_rtol, **kw)
        hists.append(h)
    return u, hists
