"""Template evaluation: trilinear interpolation with zero (Dirichlet) extension
and the derivative of that interpolant (Sec. 2.2; eq. dT in Sec. 4.1.1).

The template ``T`` holds samples at the cell centres of its own grid
(``mT`` cells of spacing ``hT``).  A physical point ``y`` has continuous index
``s = y / hT - 1/2``; the interpolant is the weighted sum over the 8 corners
``floor(s) + {0,1}^3`` with samples outside the grid taken as zero.  The
derivative is the exact derivative of that piecewise-trilinear function, with
the floor cell used at cell faces (right-continuous).
"""
from __future__ import annotations

import numpy as np


def template_sample(grid, T, pos):
    """Interpolated template values and gradients at physical points.

    ``T``: array (mTz, mTy, mTx); ``pos``: (N, 3) points (x, y, z).
    Returns (value (N,), grad (N, 3)) in float64."""
    T = np.asarray(T, dtype=np.float64)
    pos = np.asarray(pos, dtype=np.float64)
    mT, hT = grid.mT, grid.hT
    s = pos / np.asarray(hT) - 0.5
    k0 = np.floor(s).astype(np.int64)
    f = s - k0
    val = np.zeros(len(pos))
    grad = np.zeros((len(pos), 3))
    flat = T.ravel()
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                o = (ox, oy, oz)
                idx = [k0[:, d] + o[d] for d in range(3)]
                inside = np.ones(len(pos), dtype=bool)
                for d in range(3):
                    inside &= (idx[d] >= 0) & (idx[d] < mT[d])
                lin = np.where(inside, idx[0] + mT[0] * (idx[1] + mT[1] * idx[2]), 0)
                t = np.where(inside, flat[lin], 0.0)
                w1 = [f[:, d] if o[d] else 1.0 - f[:, d] for d in range(3)]   # 1-D weights
                dw = [(1.0 if o[d] else -1.0) / hT[d] for d in range(3)]      # their derivatives
                val += w1[0] * w1[1] * w1[2] * t
                grad[:, 0] += dw[0] * w1[1] * w1[2] * t
                grad[:, 1] += w1[0] * dw[1] * w1[2] * t
                grad[:, 2] += w1[0] * w1[1] * dw[2] * t
    return val, grad


def deformed_points(grid, u, vox):
    """hat-y_i = (P y)_i at the voxels ``vox`` for the deformation
    y = x^y + u (Sec. 2.2: u is the displacement on the nodal grid), evaluated
    as x_i + (P u)_i: P reproduces the node positions exactly (P x^y = x, the
    node-count reading of m^y), and forming x_i directly keeps voxel centres
    that coincide with template samples exactly on them, where the derivative
    takes the floor cell (no rounding of P x^y to either side).
    u: (3, nz, ny, nx).  Returns (N, 3)."""
    vox = np.asarray(vox, dtype=np.int64)
    Pr = grid.P_rows(vox)
    uc = np.asarray(u, dtype=np.float64).reshape(3, grid.nbar)
    return grid.voxel_centres(vox) + np.stack([Pr @ uc[d] for d in range(3)], axis=-1)


def warped_template(grid, T, u, vox):
    """T_i = T(hat-y_i) and dT_i/d hat-y_i at voxels ``vox``."""
    return template_sample(grid, T, deformed_points(grid, u, vox))
