"""Discretised NGF distance, its residual, and its derivatives as products of
assembled sparse Jacobians.

* Residual and distance: eq. NGF_discretized, eq. residual and
  eq. NGF_discretized_ri (Sec. 2.2, Sec. 3.2), with the short differences of
  eq. gradient_discretized and the clamped neighbours of
  eq. boundary_conditions.  ||v||_eps = sqrt(1/2 <v, v> + eps^2).
* Derivatives: the chain y -> P -> T -> r -> psi (eq. function_chain).
  dpsi/dr = -2 hbar r (eq. dPsi); dr/dT row i from the quotient rule applied
  to the definition (eq. ri_quotient and eq. ritcomp), written with the 6 x m
  difference Jacobian; dT/dP = [diag(g_x) diag(g_y) diag(g_z)] (eq. dT);
  dP/dy = P (Sec. 4.3).
* Gradient: grad D = (dpsi/dr dr/dT dT/dP dP/dy)^T (eq. NGF_discretized_gradient).
* Gauss-Newton Hessian: H = 2 hbar P^T dT^T dr^T dr dT P with the sign
  flipped to the positive semi-definite form (eq. NGF_discretized_hessian).

Everything is float64; matrices are assembled entry by entry (COO, duplicate
entries summed) and multiplied with scipy.sparse.  The functions accept a set
of residual ROWS so that a few outputs of a very large problem can be
evaluated exactly with global boundary semantics.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .interp import warped_template

_DIRS = ("-x", "-y", "-z", "+x", "+y", "+z")   # backward x,y,z then forward x,y,z
_AXIS = {"-x": 0, "-y": 1, "-z": 2, "+x": 0, "+y": 1, "+z": 2}


def _flat(I):
    return np.asarray(I, dtype=np.float64).ravel()


def short_differences(grid, values_at, vox):
    """The 6 short differences of eq. gradient_discretized at voxels ``vox``:
    backward (I_i - I_{i-k})/h_k and forward (I_{i+k} - I_i)/h_k for k = x, y, z,
    with clamped neighbours.  ``values_at(ids)`` returns image values."""
    nb = grid.voxel_neighbours(vox)
    Ii = values_at(vox)
    out = np.empty((len(vox), 6))
    for j, d in enumerate(_DIRS):
        hk = grid.h[_AXIS[d]]
        In = values_at(nb[d])
        out[:, j] = (Ii - In) / hk if d[0] == "-" else (In - Ii) / hk
    return out


def _warped_lookup(grid, T, u, vox):
    """Warped template values at ``vox`` and at its clamped neighbours, plus
    the template gradient at every such voxel.  Returns (lookup(ids) -> T_w,
    lookup_g(ids) -> g)."""
    nb = grid.voxel_neighbours(vox)
    need = np.unique(np.concatenate([np.asarray(vox, dtype=np.int64)] + [nb[d] for d in _DIRS]))
    tw, g = warped_template(grid, T, u, need)

    def at(ids):
        return tw[np.searchsorted(need, ids)]

    def g_at(ids):
        return g[np.searchsorted(need, ids)]

    return at, g_at


def residual_parts(grid, R, T, u, vox):
    """Numerator r1, norms ||grad T||_tau, ||grad R||_rho, the 6-vectors of
    short differences of T(P y) and R, and r = r1 / (nT nR) at ``vox``
    (eq. residual)."""
    vox = np.asarray(vox, dtype=np.int64)
    Rf = _flat(R)
    tw_at, _ = _warped_lookup(grid, T, u, vox)
    dTw = short_differences(grid, tw_at, vox)
    dR = short_differences(grid, lambda ids: Rf[ids], vox)
    r1 = 0.5 * np.sum(dTw * dR, axis=1) + grid.tau * grid.rho
    nT = np.sqrt(0.5 * np.sum(dTw * dTw, axis=1) + grid.tau ** 2)
    nR = np.sqrt(0.5 * np.sum(dR * dR, axis=1) + grid.rho ** 2)
    return dict(r=r1 / (nT * nR), r1=r1, nT=nT, nR=nR, dT=dTw, dR=dR)


def residual(grid, R, T, u):
    """r(T(P y)) over all voxels, shaped (mz, my, mx)."""
    parts = residual_parts(grid, R, T, u, np.arange(grid.mbar))
    return parts["r"].reshape(grid.m[2], grid.m[1], grid.m[0])


def distance(grid, R, T, u):
    """D(y) = hbar sum_i (1 - r_i^2)  (eq. NGF_discretized_ri)."""
    r = residual(grid, R, T, u).ravel()
    return grid.hbar * float(np.sum(1.0 - r * r))


def dr_rows(grid, R, T, u, rows):
    """Rows ``rows`` of dr/dT (len(rows) x mbar) from eq. ritcomp:
    dr_i/dT = 1/2 [grad R_i / (nT nR) - r1 grad T_i / (nT^3 nR)]^T d(grad_i)/dT,
    where d(grad_i)/dT is the 6 x mbar Jacobian of the short differences with
    clamped columns (entries of coinciding columns are summed).
    Also returns the residual values at ``rows``."""
    rows = np.asarray(rows, dtype=np.int64)
    p = residual_parts(grid, R, T, u, rows)
    coef = 0.5 * (p["dR"] / (p["nT"] * p["nR"])[:, None]
                  - (p["r1"] / (p["nT"] ** 3 * p["nR"]))[:, None] * p["dT"])
    nb = grid.voxel_neighbours(rows)
    ri, ci, vi = [], [], []
    loc = np.arange(len(rows))
    for j, d in enumerate(_DIRS):
        hk = grid.h[_AXIS[d]]
        cj = coef[:, j] / hk
        if d[0] == "-":      # (T_i - T_{i-k})/h_k
            ri += [loc, loc]
            ci += [rows, nb[d]]
            vi += [cj, -cj]
        else:                # (T_{i+k} - T_i)/h_k
            ri += [loc, loc]
            ci += [nb[d], rows]
            vi += [cj, -cj]
    M = sp.coo_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci))),
                      shape=(len(rows), grid.mbar)).tocsr()
    M.sum_duplicates()
    return M, p["r"]


def dTP_rows(grid, T, u, cols):
    """Rows ``cols`` of (dT/dP)(dP/dy): a len(cols) x 3 nbar matrix whose row j
    holds g_{j,d} P_{j,n} in column d*nbar + n (eq. dT and the block-diagonal P)."""
    cols = np.asarray(cols, dtype=np.int64)
    _, g = warped_template(grid, T, u, cols)
    Pr = grid.P_rows(cols)
    blocks = [sp.diags(g[:, d]) @ Pr for d in range(3)]
    return sp.hstack(blocks).tocsr()


def jacobian_rows(grid, R, T, u, rows):
    """Rows of J = dr/dT dT/dP dP/dy = dr/dy (len(rows) x 3 nbar) and r at
    those rows.  The product is taken over the distinct columns of dr only."""
    dr, r = dr_rows(grid, R, T, u, rows)
    used = np.unique(dr.indices)
    dtp = dTP_rows(grid, T, u, used)
    J = dr[:, used] @ dtp
    return J.tocsr(), r


def jacobian(grid, R, T, u):
    return jacobian_rows(grid, R, T, u, np.arange(grid.mbar))


def gradient_D(grid, R, T, u):
    """grad D = -2 hbar J^T r  (eq. dPsi with eq. NGF_discretized_gradient).
    Returns (3, nz, ny, nx)."""
    J, r = jacobian(grid, R, T, u)
    g = -2.0 * grid.hbar * (J.T @ r)
    return g.reshape(3, grid.my[2], grid.my[1], grid.my[0])


def hess_vec_D(grid, R, T, u, p, J=None):
    """H p = 2 hbar J^T (J p)  (eq. NGF_discretized_hessian, Gauss-Newton,
    sign flipped to the positive semi-definite form)."""
    if J is None:
        J, _ = jacobian(grid, R, T, u)
    pv = np.asarray(p, dtype=np.float64).ravel()
    q = 2.0 * grid.hbar * (J.T @ (J @ pv))
    return q.reshape(3, grid.my[2], grid.my[1], grid.my[0])


def hessian_diag_D(grid, R, T, u, J=None):
    """diag(H) = 2 hbar (column sums of J o J)."""
    if J is None:
        J, _ = jacobian(grid, R, T, u)
    d = 2.0 * grid.hbar * np.asarray(J.multiply(J).sum(axis=0)).ravel()
    return d.reshape(3, grid.my[2], grid.my[1], grid.my[0])


# --- exact evaluation of single outputs of very large problems ---------------

def rows_touching_node(grid, node):
    """Residual rows l whose Jacobian row has a non-zero in node ``node``:
    voxels whose 8-node conversion stencil contains the node, dilated by the
    7-point stencil of dr (columns of row l are l and its 6 neighbours)."""
    na, nb_, nc = grid.node_abc(node)
    ranges = []
    for k, n in enumerate((int(na), int(nb_), int(nc))):
        a = np.arange(grid.m[k])
        n0, _ = grid.conversion_1d(k, a)
        sup = a[(n0 == n) | (n0 + 1 == n)]
        lo = max(0, int(sup.min()) - 1)
        hi = min(grid.m[k] - 1, int(sup.max()) + 1)
        ranges.append(np.arange(lo, hi + 1))
    C, B, A = np.meshgrid(ranges[2], ranges[1], ranges[0], indexing="ij")
    return grid.voxel_id(A.ravel(), B.ravel(), C.ravel())


def node_outputs(grid, R, T, u, p, node):
    """Exact (grad D, H p, diag H) at one node (all 3 components) of a problem
    of any size, from the rows of J that touch the node."""
    rows = rows_touching_node(grid, node)
    J, r = jacobian_rows(grid, R, T, u, rows)
    cols = np.array([d * grid.nbar + node for d in range(3)])
    Jn = J[:, cols].toarray()                                   # (rows, 3)
    grad = -2.0 * grid.hbar * (Jn.T @ r)
    hv = 2.0 * grid.hbar * (Jn.T @ (J @ np.asarray(p, dtype=np.float64).ravel())) if p is not None else None
    diag = 2.0 * grid.hbar * np.sum(Jn * Jn, axis=0)
    return grad, hv, diag
