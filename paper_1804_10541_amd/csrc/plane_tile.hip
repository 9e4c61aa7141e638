// Fused matrix-free NGF kernel and exact Jacobi diagonal for two-dimensional
// problems (d = 2; the paper's GPU experiments of Sec. 6.3 are 2D).
//
// The discretisation of Sec. 2.2 with d = 2: bilinear grid conversion P of
// the two-component displacement (eq. grid_conversion), bilinear template with
// zero extension and its exact derivative (eq. dT), four short differences per
// pixel (eq. gradient_discretized, clamped neighbours of
// eq. boundary_conditions), so a row of dr has five entries (the d = 2 case of
// eq. hatRho) and dr^T dr thirteen (the d = 2 case of Table hessian_indices).
//
// A work-group of kPlaneNT threads covers kPlaneNT pixel columns: it owns the
// rows of dr at the inner kPlaneNT - 2 columns and samples the template on a
// one-column ring as well.  The group marches through a chunk of pixel rows;
// each thread keeps its column's values of the last three rows in registers,
// and the x neighbours of the current row go through LDS.  Per step t:
//
//  A(t)   P u (and P p) at row t, the template sample T(hat-y), its derivative
//         g = dT/dP and, for the Hessian product, a = g . (P p);
//  B(t-1) the four differences of T(P y) and R, the residual r (eq. residual)
//         and the row rho-hat of dr (eq. rho, eq. hatRho), z_l = (dr a)_l
//         (Hessian) or r_l (gradient), and the products rho-hat_l(k) z_l;
//  C(t-2) w_i = sum over the group's own rows l of dr_{l,i} z_l (eq. gradNGF,
//         eq. drTdr / eq. hessMult as a gather over the rows of dr), v = g w,
//         accumulated into the two node rows of the transposed conversion.
//
// A ring column is an own column of the neighbouring group, which adds the
// contributions of its rows there; the transposed conversion is linear, so the
// partial node blocks of the groups sum to the whole.  A complete node row is
// reduced over x in LDS and written to the group's slot of the partial buffer,
// in the layout the node pass of node_kernels.hip gathers (x tiles, one tile
// row, row chunks in place of z chunks), so the node pass, which also adds the
// curvature term, serves both dimensions.  Nothing per pixel reaches HBM.
#include <type_traits>

#include "tile_common.h"

namespace mfr {

namespace {

template <int MODE>
__global__ __launch_bounds__(kPlaneNT) void plane_tile_kernel(const TileParams P, const float* __restrict__ u,
                                                              const float* __restrict__ pv) {
  if (P.live && !ld_coherent(P.live)) return;   // a device-steered solve has stopped
  constexpr int NT = kPlaneNT, TX = NT - 2, MAXNX = NT + 1;
  constexpr bool HV = (MODE == MODE_HV), NEED_C = (MODE != MODE_OBJ);
  // row exchange with one zero pad at both ends, so every lane's neighbour reads
  // stay inside the arrays and read finite values
  __shared__ float sTw[2][NT + 2], sR[2][NT + 2];
  __shared__ float sA[HV ? 2 : 1][HV ? NT + 2 : 1];
  // x products of a row (+x, -x) with a zero pad at both ends: the reads of the
  // edge columns' missing neighbours then add exactly 0
  __shared__ float sE[NEED_C ? 2 : 1][2][NEED_C ? NT + 2 : 1];
  __shared__ float sV[NEED_C ? 2 : 1][NEED_C ? NT : 1];
  __shared__ int sColLo[NEED_C ? MAXNX : 1], sColHi[NEED_C ? MAXNX : 1];
  __shared__ Conv1 sCx[NEED_C ? NT : 1];
  __shared__ Conv1 sCy[kMaxChunk + 4];
  __shared__ Samp1 sSy[kMaxChunk + 4];
  __shared__ double sRed[NT / 64];

  const int tid = threadIdx.x;
  const int bid = xcd_block_id();
  const int tile_x = bid % P.tiles_x, chunk = bid / P.tiles_x;
  const int x0 = tile_x * TX;
  const int yb = chunk * P.chunk_len, ye = min(P.my, yb + P.chunk_len);

  const int gx = x0 - 1 + tid;
  const bool in_img = gx >= 0 && gx < P.mx;
  const bool inB = in_img && tid >= 1 && tid < NT - 1;
  const float own_row = inB ? 1.0f : 0.0f;   // scales z_l: 0 for rows this group does not own
  const int cxi = min(max(gx, 0), P.mx - 1);
  const Conv1 cvx = P.cx[cxi];
  const Samp1 spx = P.sx[cxi];
  const float wx0 = 1.0f - cvx.f, wx1 = cvx.f;
  const unsigned nb = (unsigned)P.nbar, nxu = (unsigned)P.nx;

  // local columns [lxa, lxb] of the group inside the image, first node column
  const int lxa = x0 == 0 ? 1 : 0;
  const int lxb = min(NT - 1, P.mx - x0);
  const int nox = P.cx[x0 - 1 + lxa].n0, noy = P.cy[yb].n0;
  for (int j = tid; j < ye - yb + 4; j += NT) {
    const int q = min(max(yb - 2 + j, 0), P.my - 1);
    sCy[j] = P.cy[q];
    sSy[j] = P.sy[q];
  }
  const int nxl = P.cx[x0 - 1 + lxb].n0 + 2 - nox;
  if (tid < 4) {   // pads of the row exchange
    const int sl = tid >> 1, q = (tid & 1) ? NT + 1 : 0;
    sTw[sl][q] = 0.f;
    sR[sl][q] = 0.f;
    if constexpr (HV) sA[sl][q] = 0.f;
  }
  if constexpr (NEED_C) {
    sCx[tid] = cvx;
    if (tid < 8) sE[tid >> 2][(tid >> 1) & 1][(tid & 1) ? NT + 1 : 0] = 0.f;   // the pads
    // Columns [lo, hi] touching node column nox + i (lower node ng - 1 or ng):
    // the lower node index grows by at most one per column, so the first column
    // of each lower node starts the range of the next node and the last column
    // of each lower node ends its range.
    if (tid >= lxa && tid <= lxb) {
      const int a = cvx.n0 - nox;
      const bool first = tid == lxa || P.cx[cxi - 1].n0 != cvx.n0;
      const bool last = tid == lxb || P.cx[cxi + 1].n0 != cvx.n0;
      if (tid == lxa) sColLo[0] = lxa;
      if (first) sColLo[a + 1] = tid;
      if (last) sColHi[a] = tid;
      if (tid == lxb) sColHi[a + 1] = lxb;
    }
  }
  __syncthreads();

  // the group's partial slot, one float per node and component (node index of
  // the grid: row-major), read coalesced by the node pass
  const int pslot = (chunk % P.smz) * P.smx + tile_x % P.smx;
  float* const part = P.part + (size_t)pslot * 3 * (size_t)P.nbar;
  const size_t dstride = (size_t)P.nbar;

  // Writes node row kloc of the transposed conversion: reduce the per-column
  // sums over x into the slot's node block.
  auto flush = [&](const float (&acc)[2], int kloc) {
    if constexpr (NEED_C) {   // (only the derivative modes gather)
      if (in_img) {
        sV[0][tid] = acc[0];
        sV[1][tid] = acc[1];
      }
      __syncthreads();
      for (int fj = tid; fj < nxl; fj += NT) {
        const int jg = nox + fj;
        float s0 = 0.f, s1 = 0.f;
        for (int l = sColLo[fj]; l <= sColHi[fj]; ++l) {
          const Conv1 c = sCx[l];
          const float wt = (c.n0 == jg) ? 1.0f - c.f : c.f;
          s0 = fmaf(wt, sV[0][l], s0);
          s1 = fmaf(wt, sV[1][l], s1);
        }
        const size_t o = (size_t)(noy + kloc) * P.nx + (nox + fj);
        part[o] = s0;
        part[o + dstride] = s1;
      }
      __syncthreads();
    }
  };

  // register windows of the column, slot (t - tfirst) mod 3
  float Tw[3] = {0.f, 0.f, 0.f}, Rv[3] = {0.f, 0.f, 0.f}, av[3] = {0.f, 0.f, 0.f};
  float g[3][2] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
  float e0[3] = {0.f, 0.f, 0.f}, eyp[3] = {0.f, 0.f, 0.f};
  float acc_lo[2] = {0.f, 0.f}, acc_hi[2] = {0.f, 0.f};
  int KL = noy;
  double obj = 0.0;

  // x-interpolated u and p at the two node rows bracketing the current row, and
  // their differences (the y interpolation of every row in between is one FMA)
  int Kp = -0x7fffffff;
  float ulo[2] = {0.f, 0.f}, uhi[2] = {0.f, 0.f}, udy[2] = {0.f, 0.f};
  float plo[2] = {0.f, 0.f}, phi[2] = {0.f, 0.f}, pdy[2] = {0.f, 0.f};
  // template and reference through buffer descriptors: the two corner loads share
  // one vector offset, the reference load needs only the row's scalar offset
  const __amdgpu_buffer_rsrc_t rsT = raw_buffer(P.Tp, P.Tbytes), rsR = raw_buffer(P.R, P.Rbytes);
  const unsigned rcol = (unsigned)cxi << 2;
  auto x_interp = [&](const float* __restrict__ f, int k, float (&o)[2]) {
    const unsigned i0 = (unsigned)k * nxu + (unsigned)cvx.n0;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const unsigned b = (unsigned)d * nb + i0;
      o[d] = fmaf(wx1, ld32(f, b + 1), wx0 * ld32(f, b));
    }
  };

  // stage A inputs of the next row, loaded one step ahead
  float nt00 = 0.f, nt10 = 0.f, nt01 = 0.f, nt11 = 0.f, nfx = 0.f, nfy = 0.f, nR = 0.f;
  float npp[2] = {0.f, 0.f};
  const unsigned PX = (unsigned)P.PX;
  auto issue = [&](int tt) {
    const int tc = min(max(tt, 0), P.my - 1);
    const int jy = tt - yb + 2;   // LDS slot of row tt (entries clamped into the image)
    Conv1 cvy = sCy[jy];
    cvy.n0 = __builtin_amdgcn_readfirstlane(cvy.n0);   // uniform: the row logic stays scalar
    cvy.f = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, cvy.f)));
    if (cvy.n0 != Kp) {
      if (cvy.n0 == Kp + 1) {
#pragma unroll
        for (int d = 0; d < 2; ++d) {
          ulo[d] = uhi[d];
          if (HV) plo[d] = phi[d];
        }
      } else {
        x_interp(u, cvy.n0, ulo);
        if (HV) x_interp(pv, cvy.n0, plo);
      }
      x_interp(u, cvy.n0 + 1, uhi);
      if (HV) x_interp(pv, cvy.n0 + 1, phi);
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        udy[d] = uhi[d] - ulo[d];
        if (HV) pdy[d] = phi[d] - plo[d];
      }
      Kp = cvy.n0;
    }
    const float fy = cvy.f;
    int kx = template_cell(spx, fmaf(fy, udy[0], ulo[0]), P.ihTx, nfx);
    int ky = template_cell(sSy[jy], fmaf(fy, udy[1], ulo[1]), P.ihTy, nfy);
    // clamping to [-2, mT] maps only samples entirely outside onto the zero border
    kx = clamp_m2(kx, P.mTx);
    ky = clamp_m2(ky, P.mTy);
    const unsigned v = (__umul24((unsigned)(ky + 2), PX) + (unsigned)(kx + 2)) << 2;
    const FPair a = buf_ld2(rsT, v, 0), b = buf_ld2(rsT, v, 4u * PX);
    nt00 = a.a;
    nt10 = a.b;
    nt01 = b.a;
    nt11 = b.b;
    nR = buf_ld(rsR, rcol, (unsigned)tc * (unsigned)P.mx * 4u);
    if (HV) {
#pragma unroll
      for (int d = 0; d < 2; ++d) npp[d] = fmaf(fy, pdy[d], plo[d]);
    }
  };

  const int tfirst = yb - 2, tlast = ye + 1;

  auto step = [&](auto Kc, int t) {
    constexpr int K = decltype(Kc)::value;   // slot of row t
    constexpr int K1 = (K + 2) % 3;          // slot of row t-1
    constexpr int K2 = (K + 1) % 3;          // slot of row t-2

    // ---------------- stage A: row t ----------------
    {
      const float d0 = nt10 - nt00, d1 = nt11 - nt01;
      const float f0 = fmaf(nfx, d0, nt00), f1 = fmaf(nfx, d1, nt01);
      Tw[K] = fmaf(nfy, f1 - f0, f0);
      g[K][0] = fmaf(nfy, d1 - d0, d0) * P.ihTx;
      g[K][1] = (f1 - f0) * P.ihTy;
      Rv[K] = nR;
      if (HV) av[K] = fmaf(g[K][0], npp[0], g[K][1] * npp[1]);
      const int sl = t & 1;
      sTw[sl][1 + tid] = Tw[K];
      sR[sl][1 + tid] = Rv[K];
      if (HV) sA[sl][1 + tid] = av[K];
    }
    if (t < tlast) issue(t + 1);
    // No barrier here: stage B reads only LDS slots of row t-1 (written in the
    // previous step); the slots written above were last read before the
    // barrier that ended the previous step.

    // ---------------- stage B: row yc = t-1 ----------------
    // Every lane evaluates its row (ring columns and columns outside the image read
    // finite neighbours: clamped samples or the zero pads); a lane that does not own
    // its row scales z by 0, which zeroes all its products.
    const int yc = t - 1;
    float eym = 0.f;
    e0[K1] = 0.f;
    eyp[K1] = 0.f;
    if (yc >= yb - 1 && yc <= ye && yc >= 0 && yc < P.my) {
      const int s1 = yc & 1;
      const int q = 1 + tid;
      const float Tc = Tw[K1], Rc = Rv[K1];
      const float dTxm = sTw[s1][q - 1] - Tc, dTxp = sTw[s1][q + 1] - Tc;
      const float dTym = Tw[K2] - Tc, dTyp = Tw[K] - Tc;
      const float dRxm = sR[s1][q - 1] - Rc, dRxp = sR[s1][q + 1] - Rc;
      const float dRym = Rv[K2] - Rc, dRyp = Rv[K] - Rc;
      const float sTT = fmaf(fmaf(dTxm, dTxm, dTxp * dTxp), P.ih2x, fmaf(dTym, dTym, dTyp * dTyp) * P.ih2y);
      const float sRR = fmaf(fmaf(dRxm, dRxm, dRxp * dRxp), P.ih2x, fmaf(dRym, dRym, dRyp * dRyp) * P.ih2y);
      const float sTR = fmaf(fmaf(dTxm, dRxm, dTxp * dRxp), P.ih2x, fmaf(dTym, dRym, dTyp * dRyp) * P.ih2y);
      const float nT2 = fmaf(0.5f, sTT, P.tau2);
      const float nR2 = fmaf(0.5f, sRR, P.rho2);
      const float r1 = fmaf(0.5f, sTR, P.taurho);
      const float rnT = rsq_norm(nT2), rnR = rsq_norm(nR2);
      const float c1 = rnT * rnR;
      const float r = r1 * c1;
      // 1 - r^2 from the float32 sums in float64: in float32 it cancels where r is
      // close to 1 (aligned images), and the bias of the hardware reciprocal
      // square root would add up over the voxels of the objective sum
      if (MODE != MODE_HV && inB && yc >= yb && yc < ye)
        obj += 1.0 - ((double)r1 * (double)r1) / ((double)nT2 * (double)nR2);
      if constexpr (NEED_C) {
        const float c2 = r1 * rnT * rnT;
        const float kx = P.hhx * c1, ky = P.hhy * c1;
        const float rxm = kx * fmaf(-c2, dTxm, dRxm), rxp = kx * fmaf(-c2, dTxp, dRxp);
        const float rym = ky * fmaf(-c2, dTym, dRym), ryp = ky * fmaf(-c2, dTyp, dRyp);
        const float r0 = -((rxm + rxp) + (rym + ryp));
        float zl;
        if constexpr (HV) {
          zl = r0 * av[K1];
          zl = fmaf(rxm, sA[s1][q - 1], zl);
          zl = fmaf(rxp, sA[s1][q + 1], zl);
          zl = fmaf(rym, av[K2], zl);
          zl = fmaf(ryp, av[K], zl);
        } else {
          zl = r;
        }
        zl *= own_row;
        sE[s1][0][1 + tid] = rxp * zl;
        sE[s1][1][1 + tid] = rxm * zl;
        eyp[K1] = ryp * zl;
        eym = rym * zl;
        e0[K1] = r0 * zl;
      }
    }

    // ---------------- stage C: row c = t-2 ----------------
    if constexpr (NEED_C) {
      const int c = t - 2;
      if (c >= yb && c < ye) {
        Conv1 cvy = sCy[c - yb + 2];
        cvy.n0 = __builtin_amdgcn_readfirstlane(cvy.n0);
        cvy.f = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, cvy.f)));
        if (cvy.n0 != KL) {   // node row KL is complete
          flush(acc_lo, KL - noy);
          acc_lo[0] = acc_hi[0];
          acc_lo[1] = acc_hi[1];
          acc_hi[0] = 0.f;
          acc_hi[1] = 0.f;
          KL = cvy.n0;
        }
        if (in_img) {
          // rows of the x neighbours (beyond the group's edge: the zero pad), then
          // the rows below (c+1, computed in this step) and above (c-1)
          const int s2 = c & 1;
          float w = e0[K2];
          w += sE[s2][1][1 + tid + 1];
          w += sE[s2][0][1 + tid - 1];
          w += eym;
          w += eyp[K];
          const float wy1 = cvy.f, wy0 = 1.0f - cvy.f;
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            const float v = g[K2][d] * w;
            acc_lo[d] = fmaf(wy0, v, acc_lo[d]);
            acc_hi[d] = fmaf(wy1, v, acc_hi[d]);
          }
        }
      }
    }
    __syncthreads();
  };

  issue(tfirst);
  for (int t = tfirst; t <= tlast; t += 3) {
    step(std::integral_constant<int, 0>{}, t);
    if (t + 1 <= tlast) step(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 <= tlast) step(std::integral_constant<int, 2>{}, t + 2);
  }

  if constexpr (NEED_C) {
    flush(acc_lo, KL - noy);
    flush(acc_hi, KL + 1 - noy);
  }
  if constexpr (MODE != MODE_HV) block_sum_store<NT>(obj, P.red + bid, sRed);
}

// Bilinear template value and derivative at pixel (x, y) for displacement u
// (the same conversion and sampling as stage A of the tile kernel).
struct PixelEval {
  float T, g[2];
};

__device__ __forceinline__ PixelEval eval_pixel(const TileParams& P, const float* __restrict__ u, int x, int y) {
  const Conv1 cx = P.cx[x], cy = P.cy[y];
  float dsp[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const float* b = u + (size_t)d * P.nbar + (size_t)cy.n0 * P.nx + cx.n0;
    const float lo = fmaf(cx.f, b[1], (1.0f - cx.f) * b[0]);
    const float hi = fmaf(cx.f, b[P.nx + 1], (1.0f - cx.f) * b[P.nx]);
    dsp[d] = fmaf(cy.f, hi - lo, lo);
  }
  float fx, fy;
  int kx = template_cell(P.sx[x], dsp[0], P.ihTx, fx);
  int ky = template_cell(P.sy[y], dsp[1], P.ihTy, fy);
  kx = min(max(kx, -2), P.mTx);
  ky = min(max(ky, -2), P.mTy);
  const float* b0 = P.Tp + (size_t)(ky + 2) * P.PX + (kx + 2);
  const float t00 = b0[0], t10 = b0[1], t01 = b0[P.PX], t11 = b0[P.PX + 1];
  const float d0 = t10 - t00, d1 = t11 - t01;
  const float f0 = fmaf(fx, d0, t00), f1 = fmaf(fx, d1, t01);
  PixelEval o;
  o.T = fmaf(fy, f1 - f0, f0);
  o.g[0] = fmaf(fy, d1 - d0, d0) * P.ihTx;
  o.g[1] = (f1 - f0) * P.ihTy;
  return o;
}

// Exact Jacobi diagonal, one thread per node:
// diag_{(d,n)} = 2 hbar sum_l (sum_k rho-hat_l(k) g_{l+k,d} W_n(l+k))^2 + 2 alpha hbar^y (L^T L)_{nn}
// over the rows l of dr whose five-point stencil meets the node's support.
__global__ __launch_bounds__(kNodeBlock) void plane_jacobi_kernel(const DiagParams D, const float* __restrict__ u,
                                                                  float* __restrict__ diag) {
  const TileParams& P = D.t;
  const int n = blockIdx.x * kNodeBlock + threadIdx.x;
  if (n >= P.nbar) return;
  const int ni = n % P.nx, nj = n / P.nx;
  const Range1 rx = D.rx[ni], ry = D.ry[nj];
  float acc[2] = {0.f, 0.f};
  for (int y = ry.lo; y <= ry.hi; ++y) {
    for (int x = rx.lo; x <= rx.hi; ++x) {
      // the five stencil points of row l = (x, y); clamped ones carry no weight
      const int px[5] = {x, x - 1, x + 1, x, x};
      const int py[5] = {y, y, y, y - 1, y + 1};
      bool ok[5];
      PixelEval ev[5];
      float Rv[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        ok[k] = px[k] >= 0 && px[k] < P.mx && py[k] >= 0 && py[k] < P.my;
        const int qx = ok[k] ? px[k] : x, qy = ok[k] ? py[k] : y;
        ev[k] = eval_pixel(P, u, qx, qy);
        Rv[k] = P.R[(size_t)qy * P.mx + qx];
      }
      float dT[5], dR[5];
#pragma unroll
      for (int k = 1; k < 5; ++k) {
        dT[k] = ev[k].T - ev[0].T;
        dR[k] = Rv[k] - Rv[0];
      }
      const float sTT = fmaf(fmaf(dT[1], dT[1], dT[2] * dT[2]), P.ih2x, fmaf(dT[3], dT[3], dT[4] * dT[4]) * P.ih2y);
      const float sRR = fmaf(fmaf(dR[1], dR[1], dR[2] * dR[2]), P.ih2x, fmaf(dR[3], dR[3], dR[4] * dR[4]) * P.ih2y);
      const float sTR = fmaf(fmaf(dT[1], dR[1], dT[2] * dR[2]), P.ih2x, fmaf(dT[3], dR[3], dT[4] * dR[4]) * P.ih2y);
      const float rnT = rsq_norm(fmaf(0.5f, sTT, P.tau2)), rnR = rsq_norm(fmaf(0.5f, sRR, P.rho2));
      const float r1 = fmaf(0.5f, sTR, P.taurho);
      const float c1 = rnT * rnR, c2 = r1 * rnT * rnT;
      const float hh[5] = {0.f, P.hhx, P.hhx, P.hhy, P.hhy};
      float rh[5];
      rh[0] = 0.f;
#pragma unroll
      for (int k = 1; k < 5; ++k) {
        rh[k] = hh[k] * c1 * fmaf(-c2, dT[k], dR[k]);
        rh[0] -= rh[k];
      }
      float zd[2] = {0.f, 0.f};
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        if (!ok[k]) continue;
        const float W = conv_weight(P.cx[px[k]], ni) * conv_weight(P.cy[py[k]], nj);
        const float c = rh[k] * W;
        zd[0] = fmaf(c, ev[k].g[0], zd[0]);
        zd[1] = fmaf(c, ev[k].g[1], zd[1]);
      }
      acc[0] = fmaf(zd[0], zd[0], acc[0]);
      acc[1] = fmaf(zd[1], zd[1], acc[1]);
    }
  }
  // curvature: (L^T L)_nn = (L_nn)^2 + sum over in-range neighbours 1/hy_k^4
  const int cxn = (ni > 0) + (ni < P.nx - 1), cyn = (nj > 0) + (nj < P.ny - 1);
  const float Lnn = -(cxn * D.ihy2x + cyn * D.ihy2y);
  const float LL = Lnn * Lnn + cxn * D.ihy2x * D.ihy2x + cyn * D.ihy2y * D.ihy2y;
  diag[n] = fmaf(D.s_ngf, acc[0], D.s_curv * LL);
  diag[(size_t)P.nbar + n] = fmaf(D.s_ngf, acc[1], D.s_curv * LL);
}

}  // namespace

hipError_t launch_plane_tile(int mode, const TileParams& p, const float* u, const float* pv, int grid,
                             hipStream_t st) {
  dim3 blk(kPlaneNT), grd(grid);
  switch (mode) {
    case MODE_OBJ:
      hipLaunchKernelGGL(plane_tile_kernel<MODE_OBJ>, grd, blk, 0, st, p, u, pv);
      break;
    case MODE_GRAD:
      hipLaunchKernelGGL(plane_tile_kernel<MODE_GRAD>, grd, blk, 0, st, p, u, pv);
      break;
    default:
      hipLaunchKernelGGL(plane_tile_kernel<MODE_HV>, grd, blk, 0, st, p, u, pv);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_plane_jacobi(const DiagParams& d, const float* u, float* diag, hipStream_t st) {
  const int blocks = (d.t.nbar + kNodeBlock - 1) / kNodeBlock;
  hipLaunchKernelGGL(plane_jacobi_kernel, dim3(blocks), dim3(kNodeBlock), 0, st, d, u, diag);
  return hipGetLastError();
}

}  // namespace mfr
