"""Synthetic volumes standing in for the paper's CT / histology data.

The paper evaluates on clinical thorax-abdomen CT crops, DIR-Lab 4DCT lungs and
histology sections (Sec. 6); none of these are available, so every workload
here is drawn from a seeded generator with the same shapes and value ranges.

Conventions
-----------
* Images are arrays shaped ``(m_z, m_y, m_x)`` (x fastest); voxel ``(a, b, c)``
  has centre ``((a+1/2) h_x, (b+1/2) h_y, (c+1/2) h_z)`` (Sec. 2.2).
* Node fields are arrays shaped ``(3, n_z, n_y, n_x)`` -- component-major, the
  paper's ordering of the deformation vector (Sec. 2.2).
* All random draws come from ``numpy.random.default_rng(seed)`` in the order
  documented in each function, so a seed gives the same inputs on any machine.
  Deterministic field evaluation runs in torch (on CPU or GPU); the values it
  returns are then handed unchanged to both the oracle and the GPU path.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


@dataclass(frozen=True)
class GridSpec:
    """Problem description: image cells, spacing, deformation nodes, parameters."""

    m: tuple            # image cells (m_x, m_y, m_z)
    h: tuple            # image spacing (h_x, h_y, h_z)
    my: tuple           # deformation grid NODES (n_x, n_y, n_z)
    tau: float          # NGF edge parameter of the template
    rho: float          # NGF edge parameter of the reference
    alpha: float        # curvature weight
    mT: tuple = None    # template cells (default: m)
    hT: tuple = None    # template spacing (default: h)
    distance: str = "ngf"   # distance measure: "ngf" or "ssd"
    regulariser: str = "curvature"   # "curvature", "diffusive" or "elastic"
    lame_mu: float = 1.0            # elastic regulariser: Lame parameters
    lame_lambda: float = 0.0

    def template_cells(self):
        return tuple(self.mT) if self.mT is not None else tuple(self.m)

    def template_spacing(self):
        return tuple(self.hT) if self.hT is not None else tuple(self.h)

    @property
    def voxels(self):
        return int(self.m[0]) * int(self.m[1]) * int(self.m[2])

    @property
    def nodes(self):
        return int(self.my[0]) * int(self.my[1]) * int(self.my[2])


def quarter_nodes(m):
    """Quarter-resolution deformation grid: ceil(m/4) cells, i.e. ceil(m/4)+1 nodes."""
    return tuple(int(math.ceil(k / 4)) + 1 for k in m)


def _centres(m, h, device, dtype):
    xs = (torch.arange(m[0], device=device, dtype=dtype) + 0.5) * h[0]
    ys = (torch.arange(m[1], device=device, dtype=dtype) + 0.5) * h[1]
    zs = (torch.arange(m[2], device=device, dtype=dtype) + 0.5) * h[2]
    return xs, ys, zs


def smooth_field(rng, nodes, amp, sigma=2.0):
    """Random smooth node field (3, n_z, n_y, n_x): N(0,1) per component,
    Gaussian-smoothed (sigma in nodes, reflecting boundary), scaled so that the
    largest per-node Euclidean norm equals ``amp``.  One draw of 3*prod(nodes)
    standard normals from ``rng``."""
    from scipy.ndimage import gaussian_filter

    nx, ny, nz = nodes
    raw = rng.standard_normal((3, nz, ny, nx))
    sm = np.stack([gaussian_filter(raw[d], sigma=sigma, mode="reflect") for d in range(3)])
    norm = np.sqrt((sm ** 2).sum(axis=0)).max()
    return sm * (amp / norm)


# ---------------------------------------------------------------------------
# Configuration 1: sum of Gaussians, sinusoidal warp (float64)
# ---------------------------------------------------------------------------

def blob_pair(seed, m=(32, 32, 32), n_blobs=20, noise=0.01, warp_amp=2.0,
              device="cpu", dtype=torch.float64):
    """Reference = sum of ``n_blobs`` isotropic Gaussians + N(0, noise) noise;
    template = the same sum evaluated at x - u*(x) (analytic, no resampling)
    + independent noise, with u*_d(x) = warp_amp * sin(2 pi x_{(d+1) mod 3}/L + phi_d).

    Draw order from default_rng(seed): centres (n_blobs, 3) ~ U[0, m]; sigmas
    (n_blobs) ~ U(2, 6); amplitudes (n_blobs) ~ U(0.2, 1); phases (3) ~ U[0, 2pi);
    reference noise (m_z, m_y, m_x); template noise (m_z, m_y, m_x).
    Returns (R, T, rng) with the rng positioned after these draws."""
    rng = np.random.default_rng(seed)
    mx, my_, mz = m
    cen = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * np.array([mx, my_, mz], dtype=np.float64)
    sig = rng.uniform(2.0, 6.0, size=n_blobs)
    amp = rng.uniform(0.2, 1.0, size=n_blobs)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=3)
    nR = rng.standard_normal((mz, my_, mx)) * noise
    nT = rng.standard_normal((mz, my_, mx)) * noise

    xs, ys, zs = _centres(m, (1.0, 1.0, 1.0), device, torch.float64)
    Z, Y, X = torch.meshgrid(zs, ys, xs, indexing="ij")
    L = (float(mx), float(my_), float(mz))

    def blobs(X, Y, Z):
        g = torch.zeros_like(X)
        for j in range(n_blobs):
            d2 = (X - cen[j, 0]) ** 2 + (Y - cen[j, 1]) ** 2 + (Z - cen[j, 2]) ** 2
            g = g + amp[j] * torch.exp(-d2 / (2.0 * sig[j] ** 2))
        return g

    comps = (X, Y, Z)
    ustar = [warp_amp * torch.sin(2 * math.pi * comps[(d + 1) % 3] / L[(d + 1) % 3] + phi[d])
             for d in range(3)]
    R = blobs(X, Y, Z) + torch.from_numpy(nR).to(device)
    T = blobs(X - ustar[0], Y - ustar[1], Z - ustar[2]) + torch.from_numpy(nT).to(device)
    return R.to(dtype), T.to(dtype), rng


def config_c1(seed=0, n_probes=10):
    """32^3 voxels (h = 1), 17^3 nodes, eps = 0.1, alpha = 1.  After the image
    draws: initial displacement (smooth, max norm 0.5 voxel), then ``n_probes``
    N(0,1) node vectors.  Everything float64 numpy."""
    spec = GridSpec(m=(32, 32, 32), h=(1.0, 1.0, 1.0), my=(17, 17, 17),
                    tau=0.1, rho=0.1, alpha=1.0)
    R, T, rng = blob_pair(seed, spec.m)
    u0 = smooth_field(rng, spec.my, 0.5)
    probes = rng.standard_normal((n_probes, 3, spec.my[2], spec.my[1], spec.my[0]))
    return dict(spec=spec, R=R.numpy(), T=T.numpy(), u0=u0, probes=probes)


# ---------------------------------------------------------------------------
# Configurations 2-4: CT-like phantom, cubic B-spline warp (float32)
# ---------------------------------------------------------------------------

_HU_AIR, _HU_LUNG, _HU_FAT, _HU_SOFT, _HU_BONE = -1000.0, -800.0, -100.0, 40.0, 400.0


def _bspline3(t):
    t = np.abs(t)
    out = np.zeros_like(t)
    a = t < 1
    b = (t >= 1) & (t < 2)
    out[a] = 2.0 / 3.0 - t[a] ** 2 + 0.5 * t[a] ** 3
    out[b] = (2.0 - t[b]) ** 3 / 6.0
    return out


def _bspline_basis(m, spacing):
    """(m, n_ctrl) matrix of cubic B-spline weights at voxel centres a + 1/2
    for control points at (j - 1) * spacing, j = 0 .. n_ctrl - 1."""
    n_ctrl = int(math.ceil(m / spacing)) + 3
    x = np.arange(m) + 0.5
    ctrl = (np.arange(n_ctrl) - 1) * spacing
    return _bspline3((x[:, None] - ctrl[None, :]) / spacing)


def _phantom_params(rng, m):
    """Draws 20 jitter factors U(0.9, 1.1) from ``rng`` (the only draws here)."""
    j = rng.uniform(0.9, 1.1, size=20)
    mx, my_, mz = (float(k) for k in m)
    c = np.array([mx / 2, my_ / 2, mz / 2])
    p = dict(
        body_c=c * np.array([j[0], j[1], 1.0]) * np.array([1.0, 1.0, 1.0]),
        body_a=np.array([0.44 * mx * j[2], 0.34 * my_ * j[3], 0.47 * mz * j[4]]),
        lung_dx=0.19 * mx * j[5],
        lung_a=np.array([0.13 * mx * j[6], 0.18 * my_ * j[7], 0.34 * mz * j[8]]),
        lung_dy=-0.04 * my_ * j[9],
        spine_r=0.055 * min(mx, my_) * j[10],
        spine_dy=0.21 * my_ * j[11],
        bones=[  # rib-like ellipsoids: (centre offset, semi-axes)
            (np.array([-0.33 * mx * j[12], -0.05 * my_, 0.10 * mz]), np.array([0.03 * mx, 0.10 * my_, 0.03 * mz]) * j[13]),
            (np.array([0.33 * mx * j[14], -0.05 * my_, 0.10 * mz]), np.array([0.03 * mx, 0.10 * my_, 0.03 * mz]) * j[15]),
            (np.array([-0.30 * mx * j[16], 0.05 * my_, -0.15 * mz]), np.array([0.03 * mx, 0.09 * my_, 0.03 * mz]) * j[17]),
            (np.array([0.30 * mx * j[18], 0.05 * my_, -0.15 * mz]), np.array([0.03 * mx, 0.09 * my_, 0.03 * mz]) * j[19]),
        ],
    )
    return p


def _phantom(X, Y, Z, p, width=1.0):
    """Piecewise-constant HU phantom with tanh edges of ``width`` voxels."""

    def step(sd):
        return 0.5 * (1.0 - torch.tanh(sd / width))

    def ell(c, a):
        q = torch.sqrt(((X - c[0]) / a[0]) ** 2 + ((Y - c[1]) / a[1]) ** 2 + ((Z - c[2]) / a[2]) ** 2)
        return (q - 1.0) * float(min(a))

    v = torch.full_like(X, _HU_AIR)
    bc, ba = p["body_c"], p["body_a"]
    s = step(ell(bc, ba))
    v = v + s * (_HU_FAT - v)
    s = step(ell(bc, ba - 4.0))
    v = v + s * (_HU_SOFT - v)
    for sgn in (-1.0, 1.0):
        lc = bc + np.array([sgn * p["lung_dx"], p["lung_dy"], 0.0])
        s = step(ell(lc, p["lung_a"]))
        v = v + s * (_HU_LUNG - v)
    rr = torch.sqrt((X - bc[0]) ** 2 + (Y - (bc[1] + p["spine_dy"])) ** 2)
    s = step(rr - p["spine_r"]) * step(ell(bc, ba))
    v = v + s * (_HU_BONE - v)
    for off, a in p["bones"]:
        s = step(ell(bc + off, a))
        v = v + s * (_HU_BONE - v)
    return v


def ct_pair(seed, m, max_disp=6.0, ctrl_spacing=16.0, noise=20.0, offset=1000.0,
            device="cpu", dtype=torch.float32, chunk=32):
    """CT-like reference/template pair on an h = 1 grid of ``m`` cells.

    Reference: nested HU regions (air, fat shell, soft tissue, lungs, spine,
    ribs) with tanh edges + N(0, noise).  Template: the phantom at x - u*(x)
    where u* is a cubic B-spline displacement (control spacing ``ctrl_spacing``
    voxels, N(0,1) coefficients scaled to max Euclidean norm ``max_disp``),
    + independent noise.  Both images get ``+offset`` so that air is 0 at the
    template's zero (Dirichlet) extension.

    Draw order from default_rng(seed): 20 phantom jitters; B-spline
    coefficients (3, ncz, ncy, ncx); reference noise; template noise (each
    (m_z, m_y, m_x), float32).  Returns (R, T, u_star, rng): images as torch
    tensors on ``device``; u_star (3, m_z, m_y, m_x) float32 on ``device``.
    """
    rng = np.random.default_rng(seed)
    mx, my_, mz = m
    p = _phantom_params(rng, m)
    Bx, By, Bz = (_bspline_basis(k, ctrl_spacing) for k in (mx, my_, mz))
    coef = rng.standard_normal((3, Bz.shape[1], By.shape[1], Bx.shape[1]))
    nR = rng.standard_normal((mz, my_, mx), dtype=np.float32)
    nT = rng.standard_normal((mz, my_, mx), dtype=np.float32)

    f64 = torch.float64
    tBx, tBy, tBz = (torch.from_numpy(B).to(device=device, dtype=f64) for B in (Bx, By, Bz))
    tc = torch.from_numpy(coef).to(device=device, dtype=f64)
    # u*(z,y,x) = sum_{k,j,i} c[k,j,i] Bz[z,k] By[y,j] Bx[x,i]
    ux = torch.einsum("dkji,xi->dkjx", tc, tBx)
    uxy = torch.einsum("dkjx,yj->dkyx", ux, tBy)
    ustar = torch.empty((3, mz, my_, mx), device=device, dtype=torch.float32)
    nmax = 0.0
    for z0 in range(0, mz, chunk):
        z1 = min(mz, z0 + chunk)
        blk = torch.einsum("dkyx,zk->dzyx", uxy, tBz[z0:z1])
        nmax = max(nmax, float(torch.sqrt((blk ** 2).sum(0)).max()))
        ustar[:, z0:z1] = blk.to(torch.float32)
    scale = max_disp / nmax
    ustar *= scale

    R = torch.empty((mz, my_, mx), device=device, dtype=dtype)
    T = torch.empty((mz, my_, mx), device=device, dtype=dtype)
    xs, ys, zs = _centres(m, (1.0, 1.0, 1.0), device, f64)
    for z0 in range(0, mz, chunk):
        z1 = min(mz, z0 + chunk)
        Z, Y, X = torch.meshgrid(zs[z0:z1], ys, xs, indexing="ij")
        u = ustar[:, z0:z1].to(f64)
        r = _phantom(X, Y, Z, p)
        t = _phantom(X - u[0], Y - u[1], Z - u[2], p)
        R[z0:z1] = (r + torch.from_numpy(nR[z0:z1]).to(device, f64) * noise + offset).to(dtype)
        T[z0:z1] = (t + torch.from_numpy(nT[z0:z1]).to(device, f64) * noise + offset).to(dtype)
    return R, T, ustar, rng


def ct_warp(seed, m, pts, max_disp=6.0, ctrl_spacing=16.0):
    """The generating displacement u* of ``ct_pair(seed, m)`` evaluated at
    arbitrary points ``pts`` (..., 3) in voxel units (x, y, z order): the same
    B-spline coefficients and scale, so at voxel centres it reproduces the
    u_star that ct_pair returns (up to its float32 rounding).  Returns
    (..., 3) float64.  Generator arithmetic only."""
    rng = np.random.default_rng(seed)
    mx, my_, mz = m
    _phantom_params(rng, m)
    Bx, By, Bz = (_bspline_basis(k, ctrl_spacing) for k in (mx, my_, mz))
    coef = rng.standard_normal((3, Bz.shape[1], By.shape[1], Bx.shape[1]))
    # the scale ct_pair applies: max Euclidean norm over voxel centres
    ux = np.einsum("dkji,xi->dkjx", coef, Bx)
    uxy = np.einsum("dkjx,yj->dkyx", ux, By)
    nmax = 0.0
    for z0 in range(0, mz, 32):
        blk = np.einsum("dkyx,zk->dzyx", uxy, Bz[z0:z0 + 32])
        nmax = max(nmax, float(np.sqrt((blk ** 2).sum(0)).max()))
    coef = coef * (max_disp / nmax)
    pts = np.asarray(pts, dtype=np.float64)
    flat = pts.reshape(-1, 3)

    def basis(x, n_ctrl):
        ctrl = (np.arange(n_ctrl) - 1) * ctrl_spacing
        return _bspline3((x[:, None] - ctrl[None, :]) / ctrl_spacing)

    wx = basis(flat[:, 0], Bx.shape[1])
    wy = basis(flat[:, 1], By.shape[1])
    wz = basis(flat[:, 2], Bz.shape[1])
    out = np.einsum("dkji,pi,pj,pk->pd", coef, wx, wy, wz, optimize=True)
    return out.reshape(pts.shape)


def ct_inverse_target(seed, m, pts, iters=60, **kw):
    """Displacement u at points x that aligns the pair of ``ct_pair(seed, m)``:
    the template is the phantom at x - u*(x), so T(x + u(x)) equals the
    reference phantom at x when u(x) = u*(x + u(x)).  Solved by the fixed-point
    iteration u <- u*(x + u) (a contraction while |grad u*| < 1).  Returns
    (..., 3) float64 in x, y, z order."""
    pts = np.asarray(pts, dtype=np.float64)
    u = ct_warp(seed, m, pts, **kw)
    for _ in range(iters):
        u = ct_warp(seed, m, pts + u, **kw)
    return u


def alignment_errors(seed, m, R, u_vox, n_sample=20000, edge_grad=100.0, body_level=500.0, sample_seed=0):
    """Registration error of a displacement against the one that aligns the pair
    of ``ct_pair(seed, m)`` (ct_inverse_target), where the images carry
    information: at a sample of edge voxels (central-difference |grad R| above
    ``edge_grad``) the RMS of the component along the edge normal grad R/|grad R|
    (the only component an edge determines), and at a sample of body voxels
    (R above ``body_level``) the RMS Euclidean error; each also for u = 0.
    R: (m_z, m_y, m_x) array; u_vox: callable mapping flat voxel indices to the
    displacement (n, 3) at those voxel centres (x, y, z order).  Generator-side
    evaluation only: R's differences and the warp, nothing of the method."""
    R = np.asarray(R, dtype=np.float64)
    gz, gy, gx = np.gradient(R)
    gm = np.sqrt(gx ** 2 + gy ** 2 + gz ** 2).ravel()
    rng = np.random.default_rng(sample_seed)
    mx, my_, mz = m
    out = {}
    for name, mask in (("edges", gm > edge_grad), ("body", R.ravel() > body_level)):
        idx = np.flatnonzero(mask)
        if len(idx) > n_sample:
            idx = np.sort(rng.choice(idx, n_sample, replace=False))
        a, b, c = idx % mx, (idx // mx) % my_, idx // (mx * my_)
        cen = np.stack([a + 0.5, b + 0.5, c + 0.5], axis=1)
        vstar = ct_inverse_target(seed, m, cen)
        e = np.asarray(u_vox(idx), dtype=np.float64) - vstar
        if name == "edges":
            n = np.stack([gx.ravel()[idx], gy.ravel()[idx], gz.ravel()[idx]], axis=1) / gm[idx][:, None]
            out[name] = (float(np.sqrt(np.mean(np.sum(vstar * n, 1) ** 2))),
                         float(np.sqrt(np.mean(np.sum(e * n, 1) ** 2))), len(idx))
        else:
            out[name] = (float(np.sqrt(np.mean(np.sum(vstar ** 2, 1)))), float(np.sqrt(np.mean(np.sum(e ** 2, 1)))),
                         len(idx))
    return out


def config_c2(seed=0, device="cpu"):
    """128 x 128 x 96 CT-like pair, finest grid 65 x 65 x 49 nodes, alpha 0.1,
    eps 50 HU; multilevel (3 levels) Gauss-Newton / Jacobi-PCG."""
    m = (128, 128, 96)
    spec = GridSpec(m=m, h=(1.0, 1.0, 1.0), my=(65, 65, 49), tau=50.0, rho=50.0, alpha=0.1)
    R, T, ustar, rng = ct_pair(seed, m, device=device)
    return dict(spec=spec, R=R, T=T, ustar=ustar, rng=rng, levels=3, gn_iters=10, pcg_max=50,
                pcg_rtol=1e-3)


def config_c3(seed=0, device="cpu", m=(512, 512, 900), my=(129, 129, 225), n_probes=20):
    """Large single-level GN step: 512 x 512 x 900 CT-like pair, 129 x 129 x 225
    nodes, smooth initial displacement of max norm 0.5 voxel, ``n_probes``
    N(0,1) probe vectors (float32).  ``m``/``my`` may be reduced for tests."""
    spec = GridSpec(m=tuple(m), h=(1.0, 1.0, 1.0), my=tuple(my), tau=50.0, rho=50.0, alpha=0.1)
    R, T, _, rng = ct_pair(seed, spec.m, device=device)
    u0 = smooth_field(rng, spec.my, 0.5).astype(np.float32)
    probes = rng.standard_normal((n_probes, 3, my[2], my[1], my[0]), dtype=np.float32)
    return dict(spec=spec, R=R, T=T, u0=u0, probes=probes)


def config_c4_sizes():
    """Image sizes of the ten-pair batched workload (deformation grids at quarter resolution)."""
    sizes = []
    for xy in (256, 512):
        for z in (94, 112, 120, 128, 136):
            sizes.append((xy, xy, z))
    return sizes


# ---------------------------------------------------------------------------
# Two-dimensional pairs: histology-section stand-in (Sec. 6.3 registers
# serial histology sections on the GPU in 2D)
# ---------------------------------------------------------------------------

def _section_shapes(rng, m):
    """Draws the shapes of a synthetic tissue section of m = (m_x, m_y) pixels:
    one tissue outline, glands and nuclei (ellipses: centre, semi-axes, angle,
    intensity change).  Draw order: outline (centre jitter 2, semi-axis
    factors 2, angle 1); glands (count from the area; centres, semi-axes,
    angles); nuclei (centres, radii)."""
    mx, my_ = (float(k) for k in m)
    shapes = []
    j = rng.uniform(-0.04, 0.04, size=2)
    a = rng.uniform(0.38, 0.46, size=2)
    ang = rng.uniform(0.0, math.pi)
    shapes.append((np.array([mx * (0.5 + j[0]), my_ * (0.5 + j[1])]), np.array([a[0] * mx, a[1] * my_]), ang, 0.55))
    n_gl = max(2, int(mx * my_) // 200000)
    cg = rng.uniform(0.2, 0.8, size=(n_gl, 2)) * np.array([mx, my_])
    ag = rng.uniform(0.01, 0.04, size=(n_gl, 2)) * min(mx, my_) + 2.0
    angg = rng.uniform(0.0, math.pi, size=n_gl)
    for k in range(n_gl):
        shapes.append((cg[k], ag[k], angg[k], -0.30))
    n_nu = max(8, int(mx * my_) // 10000)
    cn = rng.uniform(0.12, 0.88, size=(n_nu, 2)) * np.array([mx, my_])
    rn = rng.uniform(2.0, 5.0, size=n_nu)
    for k in range(n_nu):
        shapes.append((cn[k], np.array([rn[k], rn[k]]), 0.0, 0.40))
    return shapes


def _section_image(X, Y, shapes, width=1.0):
    """Sum of tanh-edged ellipses (value change per shape) at points (X, Y)."""
    v = np.zeros_like(X)
    for c, a, ang, dv in shapes:
        ca, sa = math.cos(ang), math.sin(ang)
        dx, dy = X - c[0], Y - c[1]
        q = np.sqrt(((ca * dx + sa * dy) / a[0]) ** 2 + ((-sa * dx + ca * dy) / a[1]) ** 2)
        v += dv * 0.5 * (1.0 - np.tanh((q - 1.0) * float(min(a)) / width))
    return v


def section_pair(seed, m, max_disp=6.0, ctrl_spacing=32.0, noise=0.02):
    """Two-dimensional reference/template pair of m = (m_x, m_y) pixels, h = 1
    (a stand-in for the paper's histology sections).

    Reference: a tissue outline (value 0.55 on a background of 0, so the
    template's zero extension is the background), darker glands (-0.30) and
    bright nuclei (+0.40), all with tanh edges of one pixel, + N(0, noise).
    Template: the same section at x - u*(x), u* a cubic B-spline displacement
    (control spacing ``ctrl_spacing`` pixels, N(0,1) coefficients scaled to max
    Euclidean norm ``max_disp``), + independent noise.  Shapes are evaluated
    only on pixels within reach of them (beyond 20 pixel widths the tanh step
    is 0 or 1 to within 1e-17).

    Draw order from default_rng(seed): the shapes (_section_shapes); B-spline
    coefficients (2, ncy, ncx); reference noise, template noise (each
    (m_y, m_x), float32).  Returns (R, T, u_star, rng) as float32 numpy arrays
    (images (m_y, m_x), u_star (2, m_y, m_x)), rng positioned after the draws."""
    rng = np.random.default_rng(seed)
    mx, my_ = int(m[0]), int(m[1])
    shapes = _section_shapes(rng, (mx, my_))
    Bx, By = _bspline_basis(mx, ctrl_spacing), _bspline_basis(my_, ctrl_spacing)
    coef = rng.standard_normal((2, By.shape[1], Bx.shape[1]))
    nR = rng.standard_normal((my_, mx), dtype=np.float32)
    nT = rng.standard_normal((my_, mx), dtype=np.float32)
    ustar = np.stack([By @ (coef[d] @ Bx.T) for d in range(2)])
    ustar *= max_disp / np.sqrt((ustar ** 2).sum(0)).max()
    xs, ys = np.arange(mx) + 0.5, np.arange(my_) + 0.5
    R = np.zeros((my_, mx))
    T = np.zeros((my_, mx))
    reach = 20.0
    for k, sh in enumerate(shapes):
        c, a = sh[0], sh[1]
        big = k == 0
        r = float(max(a)) + reach
        y0 = 0 if big else max(0, int(c[1] - r - max_disp - 1))
        y1 = my_ if big else min(my_, int(c[1] + r + max_disp + 2))
        x0 = 0 if big else max(0, int(c[0] - r - max_disp - 1))
        x1 = mx if big else min(mx, int(c[0] + r + max_disp + 2))
        if y0 >= y1 or x0 >= x1:
            continue
        Y, X = np.meshgrid(ys[y0:y1], xs[x0:x1], indexing="ij")
        R[y0:y1, x0:x1] += _section_image(X, Y, [sh])
        T[y0:y1, x0:x1] += _section_image(X - ustar[0, y0:y1, x0:x1], Y - ustar[1, y0:y1, x0:x1], [sh])
    R = (R + noise * nR).astype(np.float32)
    T = (T + noise * nT).astype(np.float32)
    return R, T, ustar.astype(np.float32), rng


def smooth_field_2d(rng, nodes, amp, sigma=2.0):
    """Random smooth two-component node field (2, n_y, n_x), as smooth_field:
    one draw of 2*n_x*n_y standard normals."""
    from scipy.ndimage import gaussian_filter

    nx, ny = int(nodes[0]), int(nodes[1])
    raw = rng.standard_normal((2, ny, nx))
    sm = np.stack([gaussian_filter(raw[d], sigma=sigma, mode="reflect") for d in range(2)])
    return sm * (amp / np.sqrt((sm ** 2).sum(axis=0)).max())


def config_section(seed=0, m=(4096, 4096), my=(2049, 2049), n_probes=3):
    """Two-dimensional workload: a section pair of m pixels (h = 1), a nodal
    grid of my nodes, eps = 0.05, alpha = 1, a smooth initial displacement of
    max norm 0.5 pixel and ``n_probes`` N(0,1) probe vectors (float32).  The
    problem is encoded with a trailing 1 (one cell and one node along z)."""
    spec = GridSpec(m=(int(m[0]), int(m[1]), 1), h=(1.0, 1.0, 1.0), my=(int(my[0]), int(my[1]), 1),
                    tau=0.05, rho=0.05, alpha=1.0)
    R, T, ustar, rng = section_pair(seed, m)
    u0 = smooth_field_2d(rng, my, 0.5).astype(np.float32)
    probes = rng.standard_normal((n_probes, 2, int(my[1]), int(my[0])), dtype=np.float32)
    return dict(spec=spec, R=R, T=T, ustar=ustar, u0=u0, probes=probes)
