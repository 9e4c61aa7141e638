"""Pure-Python loop evaluation of the discretised objective on tiny grids.

Written directly from eq. NGF_discretized (and the sum-of-squared-differences
distance hbar/2 sum (T(P y) - R)^2 for the SSD variant), eq. gradient_discretized,
eq. boundary_conditions (0-based clamping), eq. grid_conversion and the
trilinear template with zero extension (Sec. 2.2), scalar by scalar, with no
numpy vectorisation and no code shared with ``oracle/``.  Used to pin the
vectorised oracle on grids of a few dozen voxels.
"""
import math


def _node_weights_1d(a, m, n):
    c = (a + 0.5) * (n - 1) / m
    lo = min(int(math.floor(c)), n - 2)
    f = c - lo
    return [(lo, 1.0 - f), (lo + 1, f)]


def _tri(T, mT, hT, p):
    # continuous index and the 8 corners; samples outside are zero
    s = [p[d] / hT[d] - 0.5 for d in range(3)]
    k = [int(math.floor(s[d])) for d in range(3)]
    f = [s[d] - k[d] for d in range(3)]
    tot = 0.0
    for oz in (0, 1):
        for oy in (0, 1):
            for ox in (0, 1):
                ix, iy, iz = k[0] + ox, k[1] + oy, k[2] + oz
                if 0 <= ix < mT[0] and 0 <= iy < mT[1] and 0 <= iz < mT[2]:
                    w = (f[0] if ox else 1 - f[0]) * (f[1] if oy else 1 - f[1]) * (f[2] if oz else 1 - f[2])
                    tot += w * T[iz][iy][ix]
    return tot


def warped_template(m, h, my, T, u, mT=None, hT=None):
    """T(P y) on the image grid [z][y][x] for y = x^y + u, u: [3][nz][ny][nx]."""
    mT = mT or m
    hT = hT or h
    mx, my_, mz = m
    nx, ny, nz = my
    hy = [m[d] * h[d] / (my[d] - 1) for d in range(3)]
    Tw = [[[0.0] * mx for _ in range(my_)] for _ in range(mz)]
    for c in range(mz):
        for b in range(my_):
            for a in range(mx):
                yhat = [0.0, 0.0, 0.0]
                for (i, wi) in _node_weights_1d(a, mx, nx):
                    for (j, wj) in _node_weights_1d(b, my_, ny):
                        for (k, wk) in _node_weights_1d(c, mz, nz):
                            w = wi * wj * wk
                            node = (i * hy[0], j * hy[1], k * hy[2])
                            for d in range(3):
                                yhat[d] += w * (node[d] + u[d][k][j][i])
                Tw[c][b][a] = _tri(T, mT, hT, yhat)
    return Tw


def objective_ssd(m, h, my, R, T, u, mT=None, hT=None):
    """Sum-of-squared-differences distance hbar/2 sum_i (T(P y)_i - R_i)^2."""
    Tw = warped_template(m, h, my, T, u, mT, hT)
    hbar = h[0] * h[1] * h[2]
    D = 0.0
    for c in range(m[2]):
        for b in range(m[1]):
            for a in range(m[0]):
                r = Tw[c][b][a] - R[c][b][a]
                D += 0.5 * hbar * r * r
    return D


def objective_D(m, h, my, tau, rho, R, T, u, mT=None, hT=None):
    """D(y) for y = x^y + u.  R, T nested lists/arrays [z][y][x];
    u: [3][nz][ny][nx] displacement."""
    mx, my_, mz = m
    Tw = warped_template(m, h, my, T, u, mT, hT)

    def grad6(I, a, b, c):
        out = []
        for (da, db, dc, hh) in ((1, 0, 0, h[0]), (0, 1, 0, h[1]), (0, 0, 1, h[2])):
            am, bm, cm = max(a - da, 0), max(b - db, 0), max(c - dc, 0)
            out.append((I[c][b][a] - I[cm][bm][am]) / hh)
        for (da, db, dc, hh) in ((1, 0, 0, h[0]), (0, 1, 0, h[1]), (0, 0, 1, h[2])):
            ap, bp, cp = min(a + da, mx - 1), min(b + db, my_ - 1), min(c + dc, mz - 1)
            out.append((I[cp][bp][ap] - I[c][b][a]) / hh)
        return out

    hbar = h[0] * h[1] * h[2]
    D = 0.0
    for c in range(mz):
        for b in range(my_):
            for a in range(mx):
                gT = grad6(Tw, a, b, c)
                gR = grad6(R, a, b, c)
                num = 0.5 * sum(x * y for x, y in zip(gT, gR)) + tau * rho
                nT = math.sqrt(0.5 * sum(x * x for x in gT) + tau * tau)
                nR = math.sqrt(0.5 * sum(x * x for x in gR) + rho * rho)
                r = num / (nT * nR)
                D += hbar * (1.0 - r * r)
    return D


def curvature_S(my, hy, u):
    """S = hbar^y sum_n sum_d (Lap u_d)_n^2 with clamped (Neumann) neighbours."""
    nx, ny, nz = my
    hyb = hy[0] * hy[1] * hy[2]
    S = 0.0
    for d in range(3):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    c0 = u[d][k][j][i]
                    lap = ((u[d][k][j][max(i - 1, 0)] - 2 * c0 + u[d][k][j][min(i + 1, nx - 1)]) / hy[0] ** 2
                           + (u[d][k][max(j - 1, 0)][i] - 2 * c0 + u[d][k][min(j + 1, ny - 1)][i]) / hy[1] ** 2
                           + (u[d][max(k - 1, 0)][j][i] - 2 * c0 + u[d][min(k + 1, nz - 1)][j][i]) / hy[2] ** 2)
                    S += hyb * lap * lap
    return S


def diffusive_S(my, hy, u):
    """hbar^y / 2 sum_d sum over node edges ((u_{n+e_k} - u_n) / hy_k)^2, loop by loop."""
    nx, ny, nz = my
    hyb = hy[0] * hy[1] * hy[2]
    S = 0.0
    for d in range(3):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    for (di, dj, dk, h) in ((1, 0, 0, hy[0]), (0, 1, 0, hy[1]), (0, 0, 1, hy[2])):
                        a, b, c = i + di, j + dj, k + dk
                        if a < nx and b < ny and c < nz:
                            diff = (u[d][c][b][a] - u[d][k][j][i]) / h
                            S += 0.5 * hyb * diff * diff
    return S


def elastic_S(my, hy, u, mu, lam):
    """mu * diffusive_S + hbar^y/2 (lam + mu) sum over cells of the divergence squared, the
    divergence per cell being sum_d (mean of its four edge differences along d) / hy_d."""
    nx, ny, nz = my
    hyb = hy[0] * hy[1] * hy[2]
    S = mu * diffusive_S(my, hy, u)
    for k in range(nz - 1):
        for j in range(ny - 1):
            for i in range(nx - 1):
                div = 0.0
                for d in range(3):
                    tot = 0.0
                    for oz in (0, 1):
                        for oy in (0, 1):
                            for ox in (0, 1):
                                off = (ox, oy, oz)
                                sgn = 1.0 if off[d] else -1.0
                                tot += sgn * u[d][k + oz][j + oy][i + ox]
                    div += tot / (4.0 * hy[d])
                S += 0.5 * hyb * (lam + mu) * div * div
    return S


# --- two dimensions (d = 2), loop by loop -------------------------------------

def _bil(T, mT, hT, p):
    s = [p[d] / hT[d] - 0.5 for d in range(2)]
    k = [int(math.floor(s[d])) for d in range(2)]
    f = [s[d] - k[d] for d in range(2)]
    tot = 0.0
    for oy in (0, 1):
        for ox in (0, 1):
            ix, iy = k[0] + ox, k[1] + oy
            if 0 <= ix < mT[0] and 0 <= iy < mT[1]:
                tot += (f[0] if ox else 1 - f[0]) * (f[1] if oy else 1 - f[1]) * T[iy][ix]
    return tot


def objective_D_2d(m, h, my, tau, rho, R, T, u, mT=None, hT=None):
    """D(y) of a 2D problem: R, T [y][x]; u [2][ny][nx]; bilinear conversion
    and template, four short differences per voxel, clamped neighbours."""
    mT = mT or m
    hT = hT or h
    mx, my_ = m
    hy = [m[d] * h[d] / (my[d] - 1) for d in range(2)]
    Tw = [[0.0] * mx for _ in range(my_)]
    for b in range(my_):
        for a in range(mx):
            yhat = [0.0, 0.0]
            for (i, wi) in _node_weights_1d(a, mx, my[0]):
                for (j, wj) in _node_weights_1d(b, my_, my[1]):
                    node = (i * hy[0], j * hy[1])
                    for d in range(2):
                        yhat[d] += wi * wj * (node[d] + u[d][j][i])
            Tw[b][a] = _bil(T, mT, hT, yhat)

    def grad4(I, a, b):
        return [(I[b][a] - I[b][max(a - 1, 0)]) / h[0], (I[b][a] - I[max(b - 1, 0)][a]) / h[1],
                (I[b][min(a + 1, mx - 1)] - I[b][a]) / h[0], (I[min(b + 1, my_ - 1)][a] - I[b][a]) / h[1]]

    D = 0.0
    for b in range(my_):
        for a in range(mx):
            gT, gR = grad4(Tw, a, b), grad4(R, a, b)
            num = 0.5 * sum(x * y for x, y in zip(gT, gR)) + tau * rho
            nT = math.sqrt(0.5 * sum(x * x for x in gT) + tau * tau)
            nR = math.sqrt(0.5 * sum(x * x for x in gR) + rho * rho)
            r = num / (nT * nR)
            D += h[0] * h[1] * (1.0 - r * r)
    return D


def curvature_S_2d(my, hy, u):
    nx, ny = my
    S = 0.0
    for d in range(2):
        for j in range(ny):
            for i in range(nx):
                c0 = u[d][j][i]
                lap = ((u[d][j][max(i - 1, 0)] - 2 * c0 + u[d][j][min(i + 1, nx - 1)]) / hy[0] ** 2
                       + (u[d][max(j - 1, 0)][i] - 2 * c0 + u[d][min(j + 1, ny - 1)][i]) / hy[1] ** 2)
                S += hy[0] * hy[1] * lap * lap
    return S
