// Exact diagonal of the Gauss-Newton system, diag(H + alpha nabla^2 S), on
// node blocks (the Jacobi preconditioner of the conjugate-gradient solve).
//
// With J = dr dT P (eq. NGF_discretized_hessian), the NGF part is
//   diag_{(d,n)} = 2 hbar sum_l ( sum_{k in K} rho-hat_l(k) g_{l+k,d} W_n(l+k) )^2,
// a sum over the rows l of dr (eq. dr, eq. hatRho) whose 7-point stencil
// meets the support of node n; W_n is the trilinear conversion weight of the
// node (eq. grid_conversion) and g the template derivative (eq. dT).
//
// Each work-group owns a block of node columns (nodes in x and y) and a range
// of node planes, so every diagonal entry is written by exactly one group.  It
// covers the voxel rows of that block plus a one-voxel halo with one thread
// per voxel column, and marches through the voxel planes: per plane it
// samples the template (T(P y) and g) and computes the rho-hat rows of its
// voxels into LDS; then the threads assigned to each node column gather their
// rows' squared stencil sums from LDS into per-node-plane accumulators, and a
// node plane is reduced (fixed order) and written once no later voxel plane
// can touch it.
//
// For the sum-of-squared-differences distance (Sec. 4.4) dr is the identity:
// each row has the single coefficient 1 at its own voxel, so
//   diag_{(d,n)} = hbar sum_l (g_{l,d} W_n(l))^2.
#include "tile_common.h"

namespace mfr {

template <int AX, int AY, bool SSD>
__global__ __launch_bounds__(AX* AY) void jacobi_tile_kernel(const JacParams J, const float* __restrict__ u,
                                                             float* __restrict__ diag) {
  constexpr int NT = AX * AY;
  // Voxel-column arrays use a padded row stride SP: the gather's lanes read rows
  // of one node column (ten or so x-positions on consecutive y-rows), which an
  // unpadded stride of 32 floats maps onto the same LDS banks.
  constexpr int SP = AX + 10, NP = AY * SP;
  const TileParams& P = J.t;
  __shared__ float sTw[2][NP];
  __shared__ float sR[2][NP];
  __shared__ float sG[3][3][NP];   // template derivative, 3 plane slots
  __shared__ float sRho[7][NP];    // rho-hat rows: k = 0, -x, +x, -y, +y, -z, +z
  __shared__ float sPart[3][NT];
  __shared__ Conv1 sCx[AX], sCy[AY];
  // conversion weight of local voxel column la (row lb) for the block's node
  // column jc (row jr); 0 for columns outside the image (no stencil term there)
  __shared__ float sWx[AX][AX], sWy[AY][AY];

  const int tid = threadIdx.x;
  const int tx = tid % AX, ty = tid / AX;
  const int lid = ty * SP + tx;   // this thread's voxel column in the padded arrays
  const int bid = xcd_block_id();
  const int ib = bid % J.nbx;
  const int rest = bid / J.nbx;
  const int jb = rest % J.nby, kb = rest / J.nby;
  const NodeBlock BX = J.bx[ib], BY = J.by[jb], BZ = J.bz[kb];
  const int gx = BX.a0 + tx, gy = BY.a0 + ty;
  const bool in_img = (gx >= 0) && (gx < P.mx) && (gy >= 0) && (gy < P.my);
  const bool inB = (tx >= 1) && (tx < AX - 1) && (ty >= 1) && (ty < AY - 1);
  if (tid < AX) sCx[tid] = P.cx[min(max(BX.a0 + tid, 0), P.mx - 1)];
  if (tid < AY) sCy[tid] = P.cy[min(max(BY.a0 + tid, 0), P.my - 1)];

  // own column for the template samples
  const int cxi = min(max(gx, 0), P.mx - 1), cyi = min(max(gy, 0), P.my - 1);
  const Conv1 cvx = P.cx[cxi], cvy = P.cy[cyi];
  const Samp1 spx = P.sx[cxi], spy = P.sy[cyi];
  const float wx0 = 1.0f - cvx.f, wx1 = cvx.f, wy0 = 1.0f - cvy.f, wy1 = cvy.f;
  const int nodexy = cvy.n0 * P.nx + cvx.n0;
  const int nxy = P.nx * P.ny;
  const size_t plane = (size_t)P.mx * (size_t)P.my;
  const int colxy = gy * P.mx + gx;

  // node column of this thread for the gather
  const int ncx = BX.hi - BX.lo + 1, ncy = BY.hi - BY.lo + 1, NC = ncx * ncy;
  const int G = NT / NC;
  // consecutive threads take consecutive rows of one node column
  const int jcol = min(tid / G, NC - 1), kgrp = tid % G;
  const bool gathers = tid < NC * G;
  const int pslot = kgrp * NC + jcol;   // partial-sum slot (flush reads node column jc at jc + k NC)
  const int nxn = BX.lo + jcol % ncx, nyn = BY.lo + jcol / ncx;
  const Range1 rxr = J.rx[nxn], ryr = J.ry[nyn];
  const int rw = rxr.hi - rxr.lo + 1, rh = ryr.hi - ryr.lo + 1;
  // this thread's first row of the window (x fastest) and its stride G as (x, y) steps
  const int ra0 = kgrp % rw, rb0 = kgrp / rw, dra = G % rw, drb = G / rw;
  __syncthreads();   // sCx, sCy
  for (int q = tid; q < ncx * AX; q += NT) {
    const int jc = q / AX, la = q % AX, a = BX.a0 + la;
    sWx[jc][la] = (a >= 0 && a < P.mx) ? conv_weight(sCx[la], BX.lo + jc) : 0.0f;
  }
  for (int q = tid; q < ncy * AY; q += NT) {
    const int jr = q / AY, lb = q % AY, b = BY.a0 + lb;
    sWy[jr][lb] = (b >= 0 && b < P.my) ? conv_weight(sCy[lb], BY.lo + jr) : 0.0f;
  }
  const float* wxr = sWx[jcol % ncx];
  const float* wyr = sWy[jcol / ncx];

  // acc[q] accumulates node plane kflush + q (kflush: lowest plane not yet written)
  float acc[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0f;
  int kflush = BZ.lo;

  auto flush = [&](int K) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (gathers) sPart[d][pslot] = acc[0][d];
      acc[0][d] = acc[1][d];
      acc[1][d] = acc[2][d];
      acc[2][d] = acc[3][d];
      acc[3][d] = 0.0f;
    }
    __syncthreads();
    if (tid < NC) {
      const int i = BX.lo + tid % ncx, j = BY.lo + tid / ncx;
      const int cxn = (i > 0) + (i < P.nx - 1), cyn = (j > 0) + (j < P.ny - 1), czn = (K > 0) + (K < P.nz - 1);
      const float Lnn = -(cxn * J.ihy2x + cyn * J.ihy2y + czn * J.ihy2z);
      // curvature: (L^T L)_nn; diffusive: -L_nn; elastic: -L_nn + kappa (adjacent cells) / (16 hy_d^2)
      const float LL =
          P.reg ? -Lnn : Lnn * Lnn + cxn * J.ihy2x * J.ihy2x + cyn * J.ihy2y * J.ihy2y + czn * J.ihy2z * J.ihy2z;
      const float ncell = P.reg == 2 ? P.kappa * (float)(cxn * cyn * czn) * 0.0625f : 0.0f;
      const float ih2[3] = {J.ihy2x, J.ihy2y, J.ihy2z};
      const size_t n = (size_t)K * nxy + (size_t)j * P.nx + i;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float s = 0.0f;
        for (int k = 0; k < G; ++k) s += sPart[d][tid + k * NC];
        diag[(size_t)d * P.nbar + n] = fmaf(J.s_ngf, s, J.s_curv * fmaf(ncell, ih2[d], LL));
      }
    }
    __syncthreads();
  };

  float Tw_p = 0.f, Tw_c = 0.f, Tw_n = 0.f, R_p = 0.f, R_c = 0.f, R_n = 0.f;
  int Kp = -0x7fffffff;
  float ulo[3] = {0.f, 0.f, 0.f}, uhi[3] = {0.f, 0.f, 0.f};
  auto xy_interp = [&](int k, float (&o)[3]) {
    const int i00 = k * nxy + nodexy;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float* b = u + (size_t)d * P.nbar + i00;
      const float lo = fmaf(wx1, b[1], wx0 * b[0]);
      const float hi = fmaf(wx1, b[P.nx + 1], wx0 * b[P.nx]);
      o[d] = fmaf(wy1, hi, wy0 * lo);
    }
  };

  // stage-A inputs of the next plane, loaded one step ahead
  bool nx_ok = false;
  float nx_t[8];
  float nx_fx = 0.f, nx_fy = 0.f, nx_fz = 0.f, nx_R = 0.f;
  auto issue = [&](int tt) {
    nx_ok = tt >= 0 && tt < P.mz && in_img;
    if (!nx_ok) return;
    const Conv1 cvz = P.cz[tt];
    if (cvz.n0 != Kp) {
      if (cvz.n0 == Kp + 1) {
#pragma unroll
        for (int d = 0; d < 3; ++d) ulo[d] = uhi[d];
      } else {
        xy_interp(cvz.n0, ulo);
      }
      xy_interp(cvz.n0 + 1, uhi);
      Kp = cvz.n0;
    }
    const float fz = cvz.f;
    const int kx = template_cell(spx, fmaf(fz, uhi[0] - ulo[0], ulo[0]), P.ihTx, nx_fx);
    const int ky = template_cell(spy, fmaf(fz, uhi[1] - ulo[1], ulo[1]), P.ihTy, nx_fy);
    const int kz = template_cell(P.sz[tt], fmaf(fz, uhi[2] - ulo[2], ulo[2]), P.ihTz, nx_fz);
    template_corners(P, kx, ky, kz, nx_t);
    nx_R = P.R[(size_t)tt * plane + colxy];
  };

  const int zr0 = BZ.a0 + 1, zr1 = BZ.pad;   // voxel planes of the rows
  issue(zr0 - 1);
  for (int t = zr0 - 1; t <= zr1 + 1; ++t) {
    // ---- A: template value and derivative at plane t (inputs prefetched) ----
    {
      float Tv = 0.f, Rv = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
      if (nx_ok) {
        const Tri s = trilinear(P, nx_t, nx_fx, nx_fy, nx_fz);
        Tv = s.v;
        g0 = s.gx;
        g1 = s.gy;
        g2 = s.gz;
        Rv = nx_R;
      }
      const int sl = t & 1, s3 = (t + 3) % 3;
      sTw[sl][lid] = Tv;
      sR[sl][lid] = Rv;
      sG[s3][0][lid] = g0;
      sG[s3][1][lid] = g1;
      sG[s3][2][lid] = g2;
      Tw_n = Tv;
      R_n = Rv;
    }
    if (t < zr1 + 1) issue(t + 1);
    // No barrier here: stage B reads the plane t-1 slots written in the
    // previous step; the gather below waits (barrier after B) for this step's writes.

    const int c = t - 1;
    const bool row_plane = c >= zr0 && c <= zr1;
    // ---- B: rho-hat rows at plane c ----
    if (row_plane) {
      float rh[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (SSD) {
        rh[0] = (inB && in_img) ? 1.0f : 0.0f;
      } else if (inB && in_img) {
        const int s1 = c & 1;
        const float Tc = Tw_c, Rc = R_c;
        const bool hxm = gx > 0, hxp = gx < P.mx - 1, hym = gy > 0, hyp = gy < P.my - 1;
        const bool hzm = c > 0, hzp = c < P.mz - 1;
        const float dT[6] = {(hxm ? sTw[s1][lid - 1] : Tc) - Tc, (hxp ? sTw[s1][lid + 1] : Tc) - Tc,
                             (hym ? sTw[s1][lid - SP] : Tc) - Tc, (hyp ? sTw[s1][lid + SP] : Tc) - Tc,
                             (hzm ? Tw_p : Tc) - Tc, (hzp ? Tw_n : Tc) - Tc};
        const float dR[6] = {(hxm ? sR[s1][lid - 1] : Rc) - Rc, (hxp ? sR[s1][lid + 1] : Rc) - Rc,
                             (hym ? sR[s1][lid - SP] : Rc) - Rc, (hyp ? sR[s1][lid + SP] : Rc) - Rc,
                             (hzm ? R_p : Rc) - Rc, (hzp ? R_n : Rc) - Rc};
        const float ih2[3] = {P.ih2x, P.ih2y, P.ih2z};
        float sTT = 0.f, sRR = 0.f, sTR = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          sTT = fmaf(fmaf(dT[2 * a], dT[2 * a], dT[2 * a + 1] * dT[2 * a + 1]), ih2[a], sTT);
          sRR = fmaf(fmaf(dR[2 * a], dR[2 * a], dR[2 * a + 1] * dR[2 * a + 1]), ih2[a], sRR);
          sTR = fmaf(fmaf(dT[2 * a], dR[2 * a], dT[2 * a + 1] * dR[2 * a + 1]), ih2[a], sTR);
        }
        const float rnT = rsq_norm(fmaf(0.5f, sTT, P.tau2)), rnR = rsq_norm(fmaf(0.5f, sRR, P.rho2));
        const float r1 = fmaf(0.5f, sTR, P.taurho);
        const float c1 = rnT * rnR, c2 = r1 * rnT * rnT;
        const float hh[3] = {P.hhx, P.hhy, P.hhz};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          rh[1 + k] = hh[k / 2] * c1 * fmaf(-c2, dT[k], dR[k]);
          rh[0] -= rh[1 + k];
        }
      }
#pragma unroll
      for (int k = 0; k < 7; ++k) sRho[k][lid] = rh[k];
    }
    __syncthreads();

    // ---- gather of the rows at plane c into the node planes they touch ----
    if (row_plane) {
      const bool hzm = c > 0, hzp = c < P.mz - 1;
      const Conv1 czm = P.cz[max(c - 1, 0)], cz0 = P.cz[c], czp = P.cz[min(c + 1, P.mz - 1)];
      float wz0[4], wzp[4], wzm[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int nz = kflush + q;
        const bool ok = nz <= BZ.hi;
        wz0[q] = ok ? conv_weight(cz0, nz) : 0.0f;
        wzp[q] = (ok && hzp && !SSD) ? conv_weight(czp, nz) : 0.0f;
        wzm[q] = (ok && hzm && !SSD) ? conv_weight(czm, nz) : 0.0f;
      }
      // Node planes this row plane reaches: kflush (the lower node plane of row
      // plane c-1, the lowest any of its three planes touches) up to the upper
      // node plane of row plane c+1; the accumulators of planes beyond that
      // would only add exact zeros, so the row loop is instantiated per count.
      const int top = SSD ? cz0.n0 + 1 : max(cz0.n0, hzp ? czp.n0 : 0) + 1;
      const int nq = __builtin_amdgcn_readfirstlane(min(max(top - kflush + 1, 1), 4));
      const int sc = (c + 3) % 3, sp = (c + 4) % 3, sm = (c + 2) % 3;
      auto rows = [&](auto NQc) {
        constexpr int NQ = decltype(NQc)::value;
        if (!gathers) return;
        // row r = kgrp + i G of the node column's rw x (rows in y) window, as
        // (ra, rb) advanced by (G mod rw, G div rw) with a carry
        int ra = ra0, rb = rb0;
        while (rb < rh) {
          const int la = rxr.lo + ra - BX.a0, lb = ryr.lo + rb - BY.a0;
          ra += dra;
          rb += drb;
          if (ra >= rw) {
            ra -= rw;
            rb += 1;
          }
          const int li = lb * SP + la;
          const float vx0 = wxr[la], vxm = wxr[la - 1], vxp = wxr[la + 1];
          const float vy0 = wyr[lb], vym = wyr[lb - 1], vyp = wyr[lb + 1];
          const float w00 = vx0 * vy0;
          const float al0 = sRho[0][li] * w00;
          if constexpr (SSD) {   // the row's only coefficient sits at its own voxel
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float pxy = al0 * sG[sc][d][li];
#pragma unroll
              for (int q = 0; q < NQ; ++q) {
                const float zz = wz0[q] * pxy;
                acc[q][d] = fmaf(zz, zz, acc[q][d]);
              }
            }
            continue;
          }
          const float alxm = sRho[1][li] * vxm * vy0, alxp = sRho[2][li] * vxp * vy0;
          const float alym = sRho[3][li] * vx0 * vym, alyp = sRho[4][li] * vx0 * vyp;
          const float alzm = sRho[5][li] * w00, alzp = sRho[6][li] * w00;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const float* gc = sG[sc][d];
            float pxy = al0 * gc[li];
            pxy = fmaf(alxm, gc[li - 1], pxy);
            pxy = fmaf(alxp, gc[li + 1], pxy);
            pxy = fmaf(alym, gc[li - SP], pxy);
            pxy = fmaf(alyp, gc[li + SP], pxy);
            const float zp = alzp * sG[sp][d][li];
            const float zm = alzm * sG[sm][d][li];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              const float zz = fmaf(wz0[q], pxy, fmaf(wzp[q], zp, wzm[q] * zm));
              acc[q][d] = fmaf(zz, zz, acc[q][d]);
            }
          }
        }
      };
      switch (nq) {
        case 1: rows(std::integral_constant<int, 1>{}); break;
        case 2: rows(std::integral_constant<int, 2>{}); break;
        case 3: rows(std::integral_constant<int, 3>{}); break;
        default: rows(std::integral_constant<int, 4>{}); break;
      }
      // node planes below the window of the next row plane are complete
      while (kflush <= BZ.hi && kflush < cz0.n0) flush(kflush++);
    }

    Tw_p = Tw_c;
    Tw_c = Tw_n;
    R_p = R_c;
    R_c = R_n;
    __syncthreads();
  }
  while (kflush <= BZ.hi) flush(kflush++);
}

hipError_t launch_jacobi_tile(const JacParams& j, const float* u, float* diag, hipStream_t st) {
  const int blocks = j.nbx * j.nby * j.nbz;
  if (j.t.ssd)
    hipLaunchKernelGGL((jacobi_tile_kernel<32, 32, true>), dim3(blocks), dim3(1024), 0, st, j, u, diag);
  else
    hipLaunchKernelGGL((jacobi_tile_kernel<32, 32, false>), dim3(blocks), dim3(1024), 0, st, j, u, diag);
  return hipGetLastError();
}

}  // namespace mfr
