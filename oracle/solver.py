"""Objective J = D + alpha S, its gradient, the Gauss-Newton system and the
solvers that drive it (Sec. 2.3).

* J(y) = D(y) + alpha S(y)  (eq. discreteenergy).
* Gauss-Newton (Sec. 2.3.1): the Hessian of D is replaced by its Gauss-Newton
  approximation H, the Hessian of S is exact; each step solves
  (H + alpha nabla^2 S) s = -(grad D + alpha grad S) (the Newton equation)
  with conjugate gradients, then y <- y + eta s with eta from an Armijo
  line search.
* Readings where the paper is silent: CG starts at s = 0 and stops on the
  relative residual ||b - A s_k|| / ||b|| of the recursively updated residual
  or after ``max_iter`` steps; it is preconditioned with the exact diagonal of
  the system matrix (Jacobi).  Armijo: eta_0 = 1, sufficient decrease
  J(y + eta s) <= J(y) + c1 eta grad J^T s with c1 = 1e-4, halving eta at most
  ``max_ls`` times; a failed search ends the Gauss-Newton loop.
"""
from __future__ import annotations

import numpy as np

from . import curvature, diffusive, elastic, ngf, ssd


class Problem:
    """One registration level: grid, reference R, template T (float64 copies).
    The distance term (NGF or SSD) and the regulariser (curvature or
    diffusive) are the grid's."""

    def __init__(self, grid, R, T):
        self.grid = grid
        self.R = np.asarray(R, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.float64)
        self.reg = {"diffusive": diffusive, "elastic": elastic}.get(grid.regulariser, curvature)
        if self.reg is curvature:
            self.L = curvature.laplacian(grid)
        elif self.reg is diffusive:
            self.L = diffusive.operator(grid)
        else:
            self.L = elastic.hessian_matrix(grid)
        self.dist = ssd if grid.distance == "ssd" else ngf

    def objective(self, u):
        """(J, D, S)."""
        D = self.dist.distance(self.grid, self.R, self.T, u)
        S = self.reg.energy(self.grid, u, self.L)
        return D + self.grid.alpha * S, D, S

    def gradient(self, u):
        """(J, grad J)."""
        Jv, _, _ = self.objective(u)
        g = self.dist.gradient_D(self.grid, self.R, self.T, u) + self.grid.alpha * self.reg.gradient(self.grid, u, self.L)
        return Jv, g

    def jacobian(self, u):
        return self.dist.jacobian(self.grid, self.R, self.T, u)[0]

    def hess_vec(self, u, p, Jac=None):
        """(H + alpha nabla^2 S) p."""
        return (self.dist.hess_vec_D(self.grid, self.R, self.T, u, p, Jac)
                + self.grid.alpha * self.reg.hess_vec(self.grid, p, self.L))

    def jacobi_diag(self, u, Jac=None):
        """diag(H + alpha nabla^2 S)."""
        return (self.dist.hessian_diag_D(self.grid, self.R, self.T, u, Jac)
                + self.grid.alpha * self.reg.hessian_diag(self.grid, self.L))


def pcg(apply_A, b, diag=None, max_iter=50, rtol=1e-3):
    """Preconditioned conjugate gradients for A s = b from s = 0.

    ``diag``: Jacobi preconditioner (None = plain CG; zero entries act as 1).  Returns
    (s, info) with info = dict(iters, relres, flag): flag 0 converged,
    1 reached max_iter, 2 breakdown (p^T A p <= 0 or not finite)."""
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    b = b.ravel()
    s = np.zeros_like(b)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return s.reshape(shape), dict(iters=0, relres=0.0, flag=0)
    if diag is not None:
        # a zero diagonal entry (no regulariser, no template derivative reaching the
        # node) is left unscaled
        diag = np.asarray(diag, dtype=np.float64).ravel()
        diag = np.where(diag == 0.0, 1.0, diag)
    Minv = (lambda r: r) if diag is None else (lambda r, d=diag: r / d)
    r = b.copy()
    z = Minv(r)
    p = z.copy()
    rz = float(r @ z)
    relres, flag, it = 1.0, 1, 0
    for it in range(1, max_iter + 1):
        q = np.asarray(apply_A(p.reshape(shape)), dtype=np.float64).ravel()
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            flag = 2
            it -= 1
            break
        alpha = rz / pq
        s += alpha * p
        r -= alpha * q
        relres = float(np.linalg.norm(r)) / bn
        if relres <= rtol:
            flag = 0
            break
        z = Minv(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return s.reshape(shape), dict(iters=it, relres=relres, flag=flag)


def fpcg(apply_A, b, precond, max_iter=50, rtol=1e-3, fallback=None, fallback_iters=0):
    """Flexible preconditioned CG for A s = b from s = 0, for a preconditioner
    z = precond(r) that may change from step to step or be nonlinear.

    The direction update uses the Polak-Ribiere form
    beta_k = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k), which equals the standard
    PCG beta when precond is linear, symmetric and fixed (then z_{k+1}^T r_k = 0).
    If ``fallback`` (a second preconditioner) is given and ``fallback_iters``
    > 0, the solve switches to it after that many steps without convergence,
    restarting the directions from the current iterate.  Stopping rule and
    info as in pcg, plus used_fallback."""
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    b = b.ravel()
    s = np.zeros_like(b)
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return s.reshape(shape), dict(iters=0, relres=0.0, flag=0, used_fallback=0)
    M = lambda r: np.asarray(precond(r.reshape(shape)), dtype=np.float64).ravel()
    r = b.copy()
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    relres, flag, it, used = 1.0, 1, 0, 0
    for it in range(1, max_iter + 1):
        q = np.asarray(apply_A(p.reshape(shape)), dtype=np.float64).ravel()
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            flag = 2
            it -= 1
            break
        alpha = rz / pq
        s += alpha * p
        r_old = r
        r = r - alpha * q
        relres = float(np.linalg.norm(r)) / bn
        if relres <= rtol:
            flag = 0
            break
        if fallback is not None and fallback_iters > 0 and it == fallback_iters and not used:
            used = 1
            M = lambda r: np.asarray(fallback(r.reshape(shape)), dtype=np.float64).ravel()
            z = M(r)
            p = z.copy()
            rz = float(r @ z)
            continue
        z = M(r)
        rz_new = float(r @ z)
        beta = (rz_new - float(r_old @ z)) / rz
        p = z + beta * p
        rz = rz_new
    return s.reshape(shape), dict(iters=it, relres=relres, flag=flag, used_fallback=used)


def gauss_newton(problem, u0, iters=10, pcg_max=50, pcg_rtol=1e-3, c1=1e-4, max_ls=10,
                 precond=True, callback=None):
    """Gauss-Newton with CG inner solves and Armijo line search.
    Returns (u, history) with one dict per accepted iteration."""
    u = np.array(u0, dtype=np.float64, copy=True)
    hist = []
    for k in range(iters):
        Jv, g = problem.gradient(u)
        Jac = problem.jacobian(u)
        diag = problem.jacobi_diag(u, Jac) if precond else None
        s, info = pcg(lambda p: problem.hess_vec(u, p, Jac), -g, diag, pcg_max, pcg_rtol)
        slope = float(np.sum(g * s))
        eta, accepted = 1.0, False
        for _ in range(max_ls):
            Jn = problem.objective(u + eta * s)[0]
            if Jn <= Jv + c1 * eta * slope:
                accepted = True
                break
            eta *= 0.5
        rec = dict(it=k, J=Jv, gnorm=float(np.linalg.norm(g)), pcg=info, eta=eta if accepted else 0.0)
        if callback is not None:
            callback(rec, u, s)
        if not accepted:
            rec["status"] = "line_search_failed"
            hist.append(rec)
            break
        u = u + eta * s
        rec["J_new"] = Jn
        hist.append(rec)
    return u, hist
