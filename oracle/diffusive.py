"""Diffusive regulariser on the nodal grid (Sec. 4.4 names it, with the
linear-elastic one, as a regulariser built from finite differences of the
deformation, like curvature).

The paper gives no formula; the oracle takes the usual discretisation of
S(y) = 1/2 int sum_d |grad (y_d - x_d)|^2 with forward differences between
neighbouring nodes (no difference across the grid border, the Neumann form):

    S(u) = hbar^y / 2 sum_d sum_k sum_{edges along k} ((u_{n+e_k} - u_n) / hy_k)^2
         = hbar^y / 2 sum_d sum_k ||D_k u_d||^2 / hy_k^2,

so grad S = hbar^y sum_k D_k^T D_k u / hy_k^2 and the (constant) Hessian is the
same operator on each component.  D_k is assembled entry by entry (one row per
edge, -1 and +1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def difference(grid, k):
    """Forward differences along axis k: one row per edge (n, n + e_k)."""
    n = np.arange(grid.nbar)
    abc = list(grid.node_abc(n))
    keep = abc[k] < grid.my[k] - 1
    src = n[keep]
    nb = list(a[keep] for a in abc)
    nb[k] = nb[k] + 1
    dst = grid.node_id(*nb)
    r = np.arange(len(src))
    return sp.coo_matrix((np.concatenate([-np.ones(len(src)), np.ones(len(src))]),
                          (np.concatenate([r, r]), np.concatenate([src, dst]))),
                         shape=(len(src), grid.nbar)).tocsr()


def operator(grid):
    """A = sum_k D_k^T D_k / hy_k^2 (nbar x nbar), so that grad S = hbar^y A u."""
    A = None
    for k in range(3):
        D = difference(grid, k)
        term = (D.T @ D) / grid.hy[k] ** 2
        A = term if A is None else A + term
    return A.tocsr()


def _comps(grid, u):
    return np.asarray(u, dtype=np.float64).reshape(3, grid.nbar)


def energy(grid, u, A=None):
    uc = _comps(grid, u)
    tot = 0.0
    for k in range(3):
        D = difference(grid, k)
        tot += sum(float(np.sum((D @ uc[d]) ** 2)) for d in range(3)) / grid.hy[k] ** 2
    return 0.5 * grid.hybar * tot


def gradient(grid, u, A=None):
    A = operator(grid) if A is None else A
    uc = _comps(grid, u)
    return np.stack([grid.hybar * (A @ uc[d]) for d in range(3)]).reshape(3, grid.my[2], grid.my[1], grid.my[0])


def hess_vec(grid, p, A=None):
    return gradient(grid, p, A)


def hessian_diag(grid, A=None):
    A = operator(grid) if A is None else A
    d = grid.hybar * A.diagonal()
    return np.stack([d, d, d]).reshape(3, grid.my[2], grid.my[1], grid.my[0])


def hessian_matrix(grid, A=None):
    """The per-component Hessian hbar^y A."""
    A = operator(grid) if A is None else A
    return grid.hybar * A


def node_outputs(grid, u, p, node):
    """Exact (grad S, (nabla^2 S) p, diag nabla^2 S) at one node: the edges at
    the node, each contributing (u_n - u_m) / hy_k^2."""
    abc = [int(x) for x in grid.node_abc(node)]
    uc = _comps(grid, u)
    pc = _comps(grid, p) if p is not None else None
    grad, hv, dg = np.zeros(3), np.zeros(3), 0.0
    for k in range(3):
        for s in (-1, 1):
            q = list(abc)
            q[k] += s
            if 0 <= q[k] < grid.my[k]:
                m = int(grid.node_id(*q))
                w = 1.0 / grid.hy[k] ** 2
                dg += w
                grad += w * (uc[:, node] - uc[:, m])
                if pc is not None:
                    hv += w * (pc[:, node] - pc[:, m])
    s = grid.hybar
    return s * grad, (s * hv if pc is not None else None), np.full(3, s * dg)
