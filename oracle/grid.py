"""Grids, lexicographic indexing, clamped neighbours and the grid conversion P.

Follows Sec. 2.2 (cell-centred image grid, nodal deformation grid,
lexicographic ordering with x fastest, component-major vectors) and
Sec. 4.3, eq. grid_conversion / eq. xi (trilinear conversion from nodes to
cell centres).  Indices are 0-based as in Algorithms 1 and 2.

Readings of the paper taken here (each listed in the design notes):
* ``my`` counts deformation grid NODES; the nodal grid spans the image domain,
  so the node spacing is ``hy_k = m_k h_k / (my_k - 1)``.
* The coordinate conversion of eq. grid_conversion is read as
  ``c_k(a) = (a + 1/2)(my_k - 1)/m_k`` (the node-space position of the voxel
  centre), and eq. xi's strides as the deformation grid's own strides.
* Neighbours follow eq. boundary_conditions with 0-based clamping to [0, m-1].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class Grid:
    """Image grid (``m`` cells, spacing ``h``), deformation grid (``my`` nodes),
    template grid (``mT`` cells, spacing ``hT``; default = image grid), the
    model parameters tau, rho (NGF) and alpha (curvature weight), and the
    distance measure: "ngf" (the paper's) or "ssd" (Sec. 4.4), and the
    regulariser: "curvature" (the paper's), "diffusive" or "elastic" (Sec. 4.4;
    elastic with the Lame parameters lame_mu, lame_lambda)."""

    def __init__(self, m, h, my, tau, rho, alpha, mT=None, hT=None, distance="ngf", regulariser="curvature",
                 lame_mu=1.0, lame_lambda=0.0):
        self.m = tuple(int(k) for k in m)
        self.h = tuple(float(k) for k in h)
        self.my = tuple(int(k) for k in my)
        self.mT = tuple(int(k) for k in (mT if mT is not None else m))
        self.hT = tuple(float(k) for k in (hT if hT is not None else h))
        self.tau, self.rho, self.alpha = float(tau), float(rho), float(alpha)
        if distance not in ("ngf", "ssd"):
            raise ValueError("distance must be 'ngf' or 'ssd'")
        self.distance = distance
        if regulariser not in ("curvature", "diffusive", "elastic"):
            raise ValueError("regulariser must be 'curvature', 'diffusive' or 'elastic'")
        self.regulariser = regulariser
        self.lame_mu, self.lame_lambda = float(lame_mu), float(lame_lambda)
        for k in range(3):
            if not (2 <= self.my[k] and self.my[k] - 1 <= self.m[k]):
                raise ValueError("need 2 <= my <= m + 1 in every dimension")

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.m, spec.h, spec.my, spec.tau, spec.rho, spec.alpha,
                   getattr(spec, "mT", None), getattr(spec, "hT", None),
                   getattr(spec, "distance", "ngf"), getattr(spec, "regulariser", "curvature"),
                   getattr(spec, "lame_mu", 1.0), getattr(spec, "lame_lambda", 0.0))

    # sizes -----------------------------------------------------------------
    @property
    def mbar(self):
        return self.m[0] * self.m[1] * self.m[2]

    @property
    def nbar(self):
        return self.my[0] * self.my[1] * self.my[2]

    @property
    def hbar(self):
        return self.h[0] * self.h[1] * self.h[2]

    @property
    def hy(self):
        """Node spacing: the nodal grid spans [0, m_k h_k] with my_k nodes."""
        return tuple(self.m[k] * self.h[k] / (self.my[k] - 1) for k in range(3))

    @property
    def hybar(self):
        hy = self.hy
        return hy[0] * hy[1] * hy[2]

    # voxel indexing ----------------------------------------------------------
    def voxel_abc(self, vox):
        vox = np.asarray(vox, dtype=np.int64)
        a = vox % self.m[0]
        b = (vox // self.m[0]) % self.m[1]
        c = vox // (self.m[0] * self.m[1])
        return a, b, c

    def voxel_id(self, a, b, c):
        return a + self.m[0] * (b + self.m[1] * c)

    def voxel_centres(self, vox):
        a, b, c = self.voxel_abc(vox)
        return np.stack([(a + 0.5) * self.h[0], (b + 0.5) * self.h[1], (c + 0.5) * self.h[2]], axis=-1)

    def voxel_neighbours(self, vox):
        """Clamped neighbours (eq. boundary_conditions), returned as a dict
        keyed by '-x', '+x', '-y', '+y', '-z', '+z'."""
        a, b, c = self.voxel_abc(vox)
        mx, my_, mz = self.m
        return {
            "-x": self.voxel_id(np.maximum(a - 1, 0), b, c),
            "+x": self.voxel_id(np.minimum(a + 1, mx - 1), b, c),
            "-y": self.voxel_id(a, np.maximum(b - 1, 0), c),
            "+y": self.voxel_id(a, np.minimum(b + 1, my_ - 1), c),
            "-z": self.voxel_id(a, b, np.maximum(c - 1, 0)),
            "+z": self.voxel_id(a, b, np.minimum(c + 1, mz - 1)),
        }

    # node indexing -----------------------------------------------------------
    def node_abc(self, node):
        node = np.asarray(node, dtype=np.int64)
        a = node % self.my[0]
        b = (node // self.my[0]) % self.my[1]
        c = node // (self.my[0] * self.my[1])
        return a, b, c

    def node_id(self, a, b, c):
        return a + self.my[0] * (b + self.my[1] * c)

    def node_positions(self):
        """x^y: (3, nz, ny, nx) physical node coordinates."""
        hy = self.hy
        zs = np.arange(self.my[2]) * hy[2]
        ys = np.arange(self.my[1]) * hy[1]
        xs = np.arange(self.my[0]) * hy[0]
        Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
        return np.stack([X, Y, Z])

    # grid conversion P (eq. grid_conversion, eq. xi) -------------------------
    def conversion_1d(self, k, a):
        """Lower node index and fraction along dimension k for voxel index a:
        c = (a + 1/2)(my_k - 1)/m_k, lower node min(floor(c), my_k - 2)."""
        a = np.asarray(a, dtype=np.float64)
        cpos = (a + 0.5) * (self.my[k] - 1) / self.m[k]
        n0 = np.minimum(np.floor(cpos), self.my[k] - 2).astype(np.int64)
        return n0, cpos - n0

    def conversion_rows(self, vox):
        """For each voxel: the 8 neighbouring node ids and trilinear weights
        w = w_x w_y w_z (weights (1 - f, f) per dimension)."""
        a, b, c = self.voxel_abc(vox)
        nx0, fx = self.conversion_1d(0, a)
        ny0, fy = self.conversion_1d(1, b)
        nz0, fz = self.conversion_1d(2, c)
        cols, wts = [], []
        for oz in (0, 1):
            wz = fz if oz else 1.0 - fz
            for oy in (0, 1):
                wy = fy if oy else 1.0 - fy
                for ox in (0, 1):
                    wx = fx if ox else 1.0 - fx
                    cols.append(self.node_id(nx0 + ox, ny0 + oy, nz0 + oz))
                    wts.append(wx * wy * wz)
        return np.stack(cols, axis=-1), np.stack(wts, axis=-1)

    def P_rows(self, vox):
        """Rows ``vox`` of one diagonal block of P (len(vox) x nbar, CSR)."""
        vox = np.asarray(vox, dtype=np.int64)
        cols, wts = self.conversion_rows(vox)
        rows = np.repeat(np.arange(len(vox)), 8)
        return sp.csr_matrix((wts.ravel(), (rows, cols.ravel())), shape=(len(vox), self.nbar))

    def P_matrix(self):
        """One diagonal block of P over all voxels (mbar x nbar)."""
        return self.P_rows(np.arange(self.mbar))

    def apply_P(self, y):
        """P y for a node field y (3, nz, ny, nx) -> (3, mz, my, mx)."""
        P = self.P_matrix()
        y = np.asarray(y, dtype=np.float64).reshape(3, self.nbar)
        return np.stack([P @ y[d] for d in range(3)]).reshape(3, self.m[2], self.m[1], self.m[0])

    def apply_PT(self, v):
        """P^T v for a voxel field v (3, mz, my, mx) -> (3, nz, ny, nx)."""
        P = self.P_matrix()
        v = np.asarray(v, dtype=np.float64).reshape(3, self.mbar)
        return np.stack([P.T @ v[d] for d in range(3)]).reshape(3, self.my[2], self.my[1], self.my[0])
