"""Limited-memory BFGS on J = D + alpha S with the regulariser's Hessian as the
initial matrix (Sec. 2.3.2).

The paper builds L-BFGS from the objective and gradient alone and takes the
initial Hessian approximation H_0 = nabla^2 S + gamma I with gamma > 0 so
that H_0 is positive definite; it leaves the rest to the textbook method.
Readings taken here (listed in the design notes):

* nabla^2 S is the Hessian of the regulariser term of J, i.e.
  alpha 2 hbar^y L^T L (eq. curv_hessMult), so H_0 = 2 alpha hbar^y L^T L +
  gamma I, the same matrix for each displacement component.
* Search direction d = -H_k grad J by the two-loop recursion over the last
  ``mem`` pairs (s_i, y_i) with H_0^{-1} applied exactly (here: a sparse
  direct solve).
* A pair is stored only if s^T y > 1e-12 ||s|| ||y|| (curvature condition);
  otherwise it is skipped.  If d is not a descent direction the memory is
  cleared and d = -H_0^{-1} grad J.
* Step length: Armijo backtracking from eta = 1 as in the Gauss-Newton loop
  (c1 = 1e-4, halving at most ``max_ls`` times); a failed search ends the
  iteration.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import curvature, diffusive


class H0Solver:
    """x = H_0^{-1} v for H_0 = alpha nabla^2 S + gamma I (per component):
    2 alpha hbar^y L^T L + gamma I for curvature, alpha hbar^y sum_k D_k^T D_k / hy_k^2
    + gamma I for the diffusive regulariser."""

    def __init__(self, grid, gamma, L=None):
        if not gamma > 0:
            raise ValueError("gamma must be > 0")
        self.grid = grid
        if getattr(grid, "regulariser", "curvature") == "elastic":
            raise ValueError("the elastic regulariser's Hessian couples the components; no H_0 solve here")
        if getattr(grid, "regulariser", "curvature") == "diffusive":
            H = diffusive.hessian_matrix(grid)
        else:
            H = curvature.hessian_matrix(grid, curvature.laplacian(grid) if L is None else L)
        self.A = (grid.alpha * H + gamma * sp.identity(grid.nbar)).tocsc()
        self._solve = spla.factorized(self.A)

    def apply(self, v):
        """Per component (as many as v holds: three, or two on a two-dimensional grid)."""
        vc = np.asarray(v, dtype=np.float64).reshape(-1, self.grid.nbar)
        x = np.stack([self._solve(vc[d]) for d in range(len(vc))])
        return x.reshape(np.shape(v))

    def matvec(self, x):
        xc = np.asarray(x, dtype=np.float64).reshape(-1, self.grid.nbar)
        return np.stack([self.A @ xc[d] for d in range(len(xc))]).reshape(np.shape(x))


def two_loop(g, pairs, h0_inv):
    """-H g for the L-BFGS matrix H defined by H_0^{-1} = h0_inv and the pairs
    (s_i, y_i), oldest first (Nocedal & Wright, Algorithm 7.4)."""
    q = -np.asarray(g, dtype=np.float64).ravel()
    a = []
    for s, y in reversed(pairs):
        rho = 1.0 / float(s @ y)
        ai = rho * float(s @ q)
        q = q - ai * y
        a.append(ai)
    r = np.asarray(h0_inv(q.reshape(np.shape(g))), dtype=np.float64).ravel()
    for (s, y), ai in zip(pairs, reversed(a)):
        rho = 1.0 / float(s @ y)
        b = rho * float(y @ r)
        r = r + (ai - b) * s
    return r.reshape(np.shape(g))


def lbfgs(problem, u0, iters=10, mem=5, gamma=1.0, c1=1e-4, max_ls=10, callback=None):
    """L-BFGS iterations from u0.  Returns (u, history) with one dict per
    iteration (J before, gradient norm, step length, whether the pair was kept)."""
    # (a two-dimensional problem carries its 5-point Laplacian and no regulariser choice)
    h0 = H0Solver(problem.grid, gamma, problem.L if getattr(problem, "reg", curvature) is curvature else None)
    u = np.array(u0, dtype=np.float64, copy=True)
    Jv, g = problem.gradient(u)
    pairs = []
    hist = []
    for k in range(iters):
        d = two_loop(g, pairs, h0.apply)
        slope = float(np.sum(g * d))
        restarted = False
        if not slope < 0.0:
            pairs = []
            d = -h0.apply(g)
            slope = float(np.sum(g * d))
            restarted = True
        eta, accepted = 1.0, False
        for _ in range(max_ls):
            Jn = problem.objective(u + eta * d)[0]
            if Jn <= Jv + c1 * eta * slope:
                accepted = True
                break
            eta *= 0.5
        rec = dict(it=k, J=Jv, gnorm=float(np.linalg.norm(g)), eta=eta if accepted else 0.0, restarted=restarted)
        if callback is not None:
            callback(rec, u, d)
        if not accepted:
            rec["status"] = "line_search_failed"
            hist.append(rec)
            break
        s = eta * d
        u = u + s
        Jn2, gn = problem.gradient(u)
        y = gn - g
        sv, yv = s.ravel(), y.ravel()
        kept = float(sv @ yv) > 1e-12 * np.linalg.norm(sv) * np.linalg.norm(yv)
        if kept:
            pairs.append((sv.copy(), yv.copy()))
            if len(pairs) > mem:
                pairs.pop(0)
        rec.update(J_new=Jn2, kept=kept)
        hist.append(rec)
        Jv, g = Jn2, gn
    return u, hist
