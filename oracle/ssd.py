"""Sum-of-squared-differences distance, its gradient and its Gauss-Newton
Hessian as products of assembled sparse Jacobians.

Sec. 4.4 (extension to related models): of the chain D = psi(r(T(P y))) only
the residual and its Jacobian dr/dT depend on the distance measure; the grid
conversion P and the template derivative dT are the same as for NGF, and for
SSD the residual Jacobian is the identity.  The paper gives no SSD formula;
the oracle takes the common discretisation

    D(y) = hbar / 2 sum_i (T(P y)_i - R_i)^2,

i.e. psi(r) = hbar/2 r^T r with r = T(P y) - R, so that with J = dT P
(eq. dT, eq. grid_conversion):

    grad D = hbar J^T r,   H = hbar J^T J  (Gauss-Newton: the second
    derivative of the interpolant is dropped, as for NGF in Sec. 3.2),
    diag H = hbar (column sums of J o J).

Everything is float64; J is assembled row by row from P and the template
derivative, with the same helpers the NGF oracle uses for dT P.
"""
from __future__ import annotations

import numpy as np

from .interp import warped_template
from .ngf import dTP_rows


def residual(grid, R, T, u):
    """r = T(P y) - R over all voxels, shaped (mz, my, mx)."""
    vox = np.arange(grid.mbar)
    tw, _ = warped_template(grid, T, u, vox)
    return (tw - np.asarray(R, dtype=np.float64).ravel()).reshape(grid.m[2], grid.m[1], grid.m[0])


def distance(grid, R, T, u):
    """D(y) = hbar/2 sum_i r_i^2."""
    r = residual(grid, R, T, u).ravel()
    return 0.5 * grid.hbar * float(r @ r)


def jacobian_rows(grid, R, T, u, rows):
    """Rows ``rows`` of J = dr/dy = dT P (dr/dT = identity) and r at them."""
    rows = np.asarray(rows, dtype=np.int64)
    J = dTP_rows(grid, T, u, rows)
    tw, _ = warped_template(grid, T, u, rows)
    r = tw - np.asarray(R, dtype=np.float64).ravel()[rows]
    return J, r


def jacobian(grid, R, T, u):
    return jacobian_rows(grid, R, T, u, np.arange(grid.mbar))


def gradient_D(grid, R, T, u):
    """grad D = hbar J^T r, shaped (3, nz, ny, nx)."""
    J, r = jacobian(grid, R, T, u)
    return (grid.hbar * (J.T @ r)).reshape(3, grid.my[2], grid.my[1], grid.my[0])


def hess_vec_D(grid, R, T, u, p, J=None):
    """H p = hbar J^T (J p)."""
    if J is None:
        J, _ = jacobian(grid, R, T, u)
    pv = np.asarray(p, dtype=np.float64).ravel()
    return (grid.hbar * (J.T @ (J @ pv))).reshape(3, grid.my[2], grid.my[1], grid.my[0])


def hessian_diag_D(grid, R, T, u, J=None):
    """diag(H) = hbar (column sums of J o J)."""
    if J is None:
        J, _ = jacobian(grid, R, T, u)
    d = grid.hbar * np.asarray(J.multiply(J).sum(axis=0)).ravel()
    return d.reshape(3, grid.my[2], grid.my[1], grid.my[0])


def rows_touching_node(grid, node):
    """Voxels whose 8-node conversion stencil contains ``node`` (the rows of J
    with a non-zero in that node's columns: dr/dT is the identity)."""
    na, nb_, nc = grid.node_abc(node)
    ranges = []
    for k, n in enumerate((int(na), int(nb_), int(nc))):
        a = np.arange(grid.m[k])
        n0, _ = grid.conversion_1d(k, a)
        ranges.append(a[(n0 == n) | (n0 + 1 == n)])
    C, B, A = np.meshgrid(ranges[2], ranges[1], ranges[0], indexing="ij")
    return grid.voxel_id(A.ravel(), B.ravel(), C.ravel())


def node_outputs(grid, R, T, u, p, node):
    """Exact (grad D, H p, diag H) at one node (all 3 components) of a problem
    of any size, from the rows of J that touch the node."""
    rows = rows_touching_node(grid, node)
    J, r = jacobian_rows(grid, R, T, u, rows)
    cols = np.array([d * grid.nbar + node for d in range(3)])
    Jn = J[:, cols].toarray()
    grad = grid.hbar * (Jn.T @ r)
    hv = grid.hbar * (Jn.T @ (J @ np.asarray(p, dtype=np.float64).ravel())) if p is not None else None
    diag = grid.hbar * np.sum(Jn * Jn, axis=0)
    return grad, hv, diag
