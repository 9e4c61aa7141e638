"""Float64 CPU oracle for the matrix-free NGF + curvature registration method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library, its
Python binding) may import, call or link anything in this package; only the
tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
use it.

The oracle computes the *definitions* the matrix-free scheme must reproduce:
the discretised NGF distance (Sec. 2.2, eq. NGF_discretized) and curvature
regulariser (eq. CURV_discretized), and their derivatives as products of
assembled sparse Jacobians (Sec. 3, eq. NGF_discretized_gradient and
eq. NGF_discretized_hessian): the grid conversion P, the template derivative
dT, the residual Jacobian dr and the Laplacian L are built entry by entry from
their definitions and multiplied with scipy.sparse.  It shares no code with
the HIP path: no kernels, no tables, no per-voxel recipe (the rho-hat
formulation of Sec. 4 is what the GPU computes; the oracle never uses it).
``ssd`` holds the same derivatives for the sum-of-squared-differences
distance (Sec. 4.4: the residual Jacobian becomes the identity).
``diffusive`` and ``elastic`` are the diffusive and linear-elastic regularisers (Sec. 4.4),
alternatives to curvature.
``lbfgs`` is the limited-memory BFGS alternative of Sec. 2.3.2 with the
regulariser's Hessian in the initial matrix.
``plane`` is the two-dimensional case (d = 2) of the whole path, written
separately (the paper's GPU experiments are 2D).
``cnn`` defines the learned preconditioner, an extension of the method
(convolutions, network, features, loss), and ``solver.fpcg`` the flexible CG
that uses it.
"""
from .grid import Grid  # noqa: F401
from . import interp, ngf, ssd, curvature, diffusive, elastic, solver, multilevel, lbfgs, cnn, plane  # noqa: F401
