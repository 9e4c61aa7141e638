// Fused matrix-free NGF kernel on voxel tiles (CDNA4 / gfx950).
//
// One work-group owns a column block of BX x BY voxel columns: the inner
// (BX-4) x (BY-4) columns are its output voxels, the outer ring a two-voxel
// halo that is recomputed rather than exchanged.  The group marches through a
// chunk of z planes; each thread owns one column and keeps the values of its
// own column in registers across planes, while the x/y neighbours of the
// current plane are exchanged through LDS.  Per step t three stages run:
//
//  A(t)   conversion P of u (and of p) at plane t (Sec. 4.3,
//         eq. grid_conversion), trilinear template sample T(hat-y) and its
//         derivative g = dT/dP (eq. dT), and, for the Hessian product,
//         a = g . (P p);
//  B(t-1) the six short differences of T(P y) and R (eq. gradient_discretized
//         with clamped neighbours, eq. boundary_conditions), the residual r
//         (eq. residual) and the row rho-hat of dr (eq. rho, eq. hatRho);
//         then z_l = (dr a)_l (Hessian) or z_l = r_l (gradient) and the
//         products e_l(k) = rho-hat_l(k) z_l;
//  C(t-2) the column sum w_i = sum_{rows l} dr_{l,i} z_l = e_i(0) +
//         sum_k e_{i+k}(-k) over neighbours inside the image (eq. gradNGF and
//         eq. drTdr / eq. hessMult as a gather over the rows of dr), v = g w,
//         accumulated into the node planes of the transposed conversion P^T.
//
// P^T is a gather: each column accumulates its z contributions in registers;
// when a node plane is complete the group reduces it over x and y in LDS and
// writes the node block to its own slot of a partial buffer.  A node pass sums
// the slots that overlap each node in a fixed order, so results are
// deterministic and no atomics are used.  Nothing per voxel reaches HBM.
#include "tile_common.h"

namespace mfr {

template <int BX, int BY, int MODE>
__global__ __launch_bounds__(BX* BY) void ngf_tile_kernel(const TileParams P,
                                                          const float* __restrict__ u,
                                                          const float* __restrict__ pv) {
  constexpr int NT = BX * BY;
  constexpr int TX = BX - 4, TY = BY - 4;
  constexpr int MAXNX = TX + 1, MAXNY = TY + 1;
  constexpr bool HV = (MODE == MODE_HV);
  constexpr bool NEED_C = (MODE != MODE_OBJ);

  __shared__ float sTw[2][NT];
  __shared__ float sR[2][NT];
  __shared__ float sA[HV ? 2 : 1][HV ? NT : 1];
  __shared__ float sE[NEED_C ? 2 : 1][4][NEED_C ? NT : 1];
  __shared__ float sV[3][TX * TY];
  __shared__ float sW[3][TY * MAXNX];
  __shared__ int sColLo[MAXNX], sColHi[MAXNX], sRowLo[MAXNY], sRowHi[MAXNY];
  __shared__ Conv1 sCx[TX], sCy[TY];
  __shared__ double sRed[NT / 64];

  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;

  const int bid = xcd_block_id();
  const int tile_x = bid % P.tiles_x;
  const int rest = bid / P.tiles_x;
  const int tile_y = rest % P.tiles_y;
  const int chunk = rest / P.tiles_y;
  const int x0 = tile_x * TX, y0 = tile_y * TY;
  const int zb = chunk * P.chunk_len;
  const int ze = min(P.mz, zb + P.chunk_len);

  const int gx = x0 - 2 + tx, gy = y0 - 2 + ty;
  const bool in_img = (gx >= 0) && (gx < P.mx) && (gy >= 0) && (gy < P.my);
  const bool inB = (tx >= 1) && (tx < BX - 1) && (ty >= 1) && (ty < BY - 1);
  const bool inner = (tx >= 2) && (tx < BX - 2) && (ty >= 2) && (ty < BY - 2);
  const bool inC = inner && in_img;

  const int cxi = min(max(gx, 0), P.mx - 1), cyi = min(max(gy, 0), P.my - 1);
  const Conv1 cvx = P.cx[cxi], cvy = P.cy[cyi];
  const Samp1 spx = P.sx[cxi], spy = P.sy[cyi];
  const float wx0 = 1.0f - cvx.f, wx1 = cvx.f, wy0 = 1.0f - cvy.f, wy1 = cvy.f;
  const int nodexy = cvy.n0 * P.nx + cvx.n0;
  const int nxy = P.nx * P.ny;
  const size_t plane = (size_t)P.mx * (size_t)P.my;
  const int colxy = gy * P.mx + gx;

  // Tile node origins and the column / row ranges of each local node.
  const int TXv = min(TX, P.mx - x0), TYv = min(TY, P.my - y0);
  const int nox = P.cx[x0].n0, noy = P.cy[y0].n0, noz = P.cz[zb].n0;
  const int nxl = P.cx[x0 + TXv - 1].n0 + 2 - nox;
  const int nyl = P.cy[y0 + TYv - 1].n0 + 2 - noy;
  if constexpr (NEED_C) {
    if (tid < TX) sCx[tid] = P.cx[min(x0 + tid, P.mx - 1)];
    if (tid < TY) sCy[tid] = P.cy[min(y0 + tid, P.my - 1)];
    __syncthreads();
    if (tid < nxl) {
      const int jg = nox + tid;
      int lo = TXv, hi = -1;
      for (int l = 0; l < TXv; ++l) {
        const int n0 = sCx[l].n0;
        if (n0 == jg || n0 + 1 == jg) {
          lo = min(lo, l);
          hi = max(hi, l);
        }
      }
      sColLo[tid] = lo;
      sColHi[tid] = hi;
    }
    if (tid >= 64 && tid - 64 < nyl) {
      const int i = tid - 64, ig = noy + i;
      int lo = TYv, hi = -1;
      for (int l = 0; l < TYv; ++l) {
        const int n0 = sCy[l].n0;
        if (n0 == ig || n0 + 1 == ig) {
          lo = min(lo, l);
          hi = max(hi, l);
        }
      }
      sRowLo[i] = lo;
      sRowHi[i] = hi;
    }
  }

  const int slot = tile_x + P.tiles_x * (tile_y + P.tiles_y * chunk);
  float* const part = P.part + (size_t)slot * 3 * P.nzt * P.nyt * P.nxt;

  // Writes one node plane (local index kloc) of the transposed conversion:
  // reduce the per-column sums acc over x, then y, into the slot's node block.
  auto flush = [&](const float (&acc)[3], int kloc) {
    if (inner) {
      const int l = (ty - 2) * TX + (tx - 2);
      sV[0][l] = acc[0];
      sV[1][l] = acc[1];
      sV[2][l] = acc[2];
    }
    __syncthreads();
    for (int it = tid; it < nxl * TYv * 3; it += NT) {
      const int j = it % nxl;
      const int r = it / nxl;
      const int ly = r % TYv, d = r / TYv;
      const int jg = nox + j;
      float s = 0.0f;
      for (int l = sColLo[j]; l <= sColHi[j]; ++l) {
        const Conv1 c = sCx[l];
        const float w = (c.n0 == jg) ? 1.0f - c.f : c.f;
        s = fmaf(w, sV[d][ly * TX + l], s);
      }
      sW[d][ly * MAXNX + j] = s;
    }
    __syncthreads();
    for (int it = tid; it < nxl * nyl * 3; it += NT) {
      const int j = it % nxl;
      const int r = it / nxl;
      const int i = r % nyl, d = r / nyl;
      const int ig = noy + i;
      float s = 0.0f;
      for (int l = sRowLo[i]; l <= sRowHi[i]; ++l) {
        const Conv1 c = sCy[l];
        const float w = (c.n0 == ig) ? 1.0f - c.f : c.f;
        s = fmaf(w, sW[d][l * MAXNX + j], s);
      }
      part[(((size_t)d * P.nzt + kloc) * P.nyt + i) * P.nxt + j] = s;
    }
    __syncthreads();
  };

  // Register state of the own column.
  float Tw_p = 0.f, Tw_c = 0.f, Tw_n = 0.f;   // T(P y) at planes t-2, t-1, t
  float R_p = 0.f, R_c = 0.f, R_n = 0.f;
  float a_p = 0.f, a_c = 0.f, a_n = 0.f;      // g . P p (Hessian only)
  float g_p[3] = {0.f, 0.f, 0.f}, g_c[3] = {0.f, 0.f, 0.f}, g_n[3] = {0.f, 0.f, 0.f};
  float e0_prev = 0.f, ezp_p = 0.f, ezp_pp = 0.f;
  float acc_lo[3] = {0.f, 0.f, 0.f}, acc_hi[3] = {0.f, 0.f, 0.f};
  int KL = noz;
  double obj = 0.0;

  // xy-interpolated u and p at the two node planes bracketing the current plane.
  int Kp = -0x7fffffff;
  float ulo[3] = {0.f, 0.f, 0.f}, uhi[3] = {0.f, 0.f, 0.f};
  float plo[3] = {0.f, 0.f, 0.f}, phi[3] = {0.f, 0.f, 0.f};
  auto xy_interp = [&](const float* __restrict__ f, int k, float (&o)[3]) {
    const int i00 = k * nxy + nodexy;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float* b = f + (size_t)d * P.nbar + i00;
      const float lo = fmaf(wx1, b[1], wx0 * b[0]);
      const float hi = fmaf(wx1, b[P.nx + 1], wx0 * b[P.nx]);
      o[d] = fmaf(wy1, hi, wy0 * lo);
    }
  };

  const int tfirst = zb - 2, tlast = ze + 1;
  for (int t = tfirst; t <= tlast; ++t) {
    // ---------------- stage A: plane t ----------------
    {
      float Tv = 0.f, Rv = 0.f, av = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
      if (t >= 0 && t < P.mz && in_img) {
        const Conv1 cvz = P.cz[t];
        if (cvz.n0 != Kp) {
          if (cvz.n0 == Kp + 1) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              ulo[d] = uhi[d];
              if (HV) plo[d] = phi[d];
            }
          } else {
            xy_interp(u, cvz.n0, ulo);
            if (HV) xy_interp(pv, cvz.n0, plo);
          }
          xy_interp(u, cvz.n0 + 1, uhi);
          if (HV) xy_interp(pv, cvz.n0 + 1, phi);
          Kp = cvz.n0;
        }
        const float fz = cvz.f;
        const float dux = fmaf(fz, uhi[0] - ulo[0], ulo[0]);
        const float duy = fmaf(fz, uhi[1] - ulo[1], ulo[1]);
        const float duz = fmaf(fz, uhi[2] - ulo[2], ulo[2]);
        const Samp1 spz = P.sz[t];
        float fx, fy, fz2;
        const int kx = template_cell(spx, dux, P.ihTx, fx);
        const int ky = template_cell(spy, duy, P.ihTy, fy);
        const int kz = template_cell(spz, duz, P.ihTz, fz2);
        const Tri s = sample_template(P, kx, ky, kz, fx, fy, fz2);
        Tv = s.v;
        g0 = s.gx;
        g1 = s.gy;
        g2 = s.gz;
        Rv = P.R[(size_t)t * plane + colxy];
        if (HV) {
          const float ppx = fmaf(fz, phi[0] - plo[0], plo[0]);
          const float ppy = fmaf(fz, phi[1] - plo[1], plo[1]);
          const float ppz = fmaf(fz, phi[2] - plo[2], plo[2]);
          av = fmaf(g0, ppx, fmaf(g1, ppy, g2 * ppz));
        }
      }
      const int sl = t & 1;
      sTw[sl][tid] = Tv;
      sR[sl][tid] = Rv;
      if (HV) sA[sl][tid] = av;
      Tw_n = Tv;
      R_n = Rv;
      a_n = av;
      g_n[0] = g0;
      g_n[1] = g1;
      g_n[2] = g2;
    }
    __syncthreads();

    // ---------------- stage B: plane zc = t-1 ----------------
    const int zc = t - 1;
    float e0_new = 0.f, ezp_new = 0.f, ezm_new = 0.f;
    if (zc >= zb - 1 && zc <= ze && zc >= 0 && zc < P.mz) {
      const int s1 = zc & 1;
      float ex_p = 0.f, ex_m = 0.f, ey_p = 0.f, ey_m = 0.f;
      if (inB && in_img) {
        const float Tc = Tw_c, Rc = R_c;
        const bool hxm = gx > 0, hxp = gx < P.mx - 1, hym = gy > 0, hyp = gy < P.my - 1;
        const bool hzm = zc > 0, hzp = zc < P.mz - 1;
        const float dTxm = (hxm ? sTw[s1][tid - 1] : Tc) - Tc;
        const float dTxp = (hxp ? sTw[s1][tid + 1] : Tc) - Tc;
        const float dTym = (hym ? sTw[s1][tid - BX] : Tc) - Tc;
        const float dTyp = (hyp ? sTw[s1][tid + BX] : Tc) - Tc;
        const float dTzm = (hzm ? Tw_p : Tc) - Tc;
        const float dTzp = (hzp ? Tw_n : Tc) - Tc;
        const float dRxm = (hxm ? sR[s1][tid - 1] : Rc) - Rc;
        const float dRxp = (hxp ? sR[s1][tid + 1] : Rc) - Rc;
        const float dRym = (hym ? sR[s1][tid - BX] : Rc) - Rc;
        const float dRyp = (hyp ? sR[s1][tid + BX] : Rc) - Rc;
        const float dRzm = (hzm ? R_p : Rc) - Rc;
        const float dRzp = (hzp ? R_n : Rc) - Rc;
        const float sTT = fmaf(fmaf(dTxm, dTxm, dTxp * dTxp), P.ih2x,
                               fmaf(fmaf(dTym, dTym, dTyp * dTyp), P.ih2y,
                                    fmaf(dTzm, dTzm, dTzp * dTzp) * P.ih2z));
        const float sRR = fmaf(fmaf(dRxm, dRxm, dRxp * dRxp), P.ih2x,
                               fmaf(fmaf(dRym, dRym, dRyp * dRyp), P.ih2y,
                                    fmaf(dRzm, dRzm, dRzp * dRzp) * P.ih2z));
        const float sTR = fmaf(fmaf(dTxm, dRxm, dTxp * dRxp), P.ih2x,
                               fmaf(fmaf(dTym, dRym, dTyp * dRyp), P.ih2y,
                                    fmaf(dTzm, dRzm, dTzp * dRzp) * P.ih2z));
        const float nT2 = fmaf(0.5f, sTT, P.tau2);
        const float nR2 = fmaf(0.5f, sRR, P.rho2);
        const float r1 = fmaf(0.5f, sTR, P.taurho);
        const float rnT = rsqrtf(nT2), rnR = rsqrtf(nR2);
        const float c1 = rnT * rnR;
        const float r = r1 * c1;
        if (MODE != MODE_HV && inner && zc >= zb && zc < ze) obj += (double)fmaf(-r, r, 1.0f);
        if (NEED_C) {
          const float c2 = r1 * rnT * rnT;
          const float kx = P.hhx * c1, ky = P.hhy * c1, kz = P.hhz * c1;
          const float rxm = kx * fmaf(-c2, dTxm, dRxm), rxp = kx * fmaf(-c2, dTxp, dRxp);
          const float rym = ky * fmaf(-c2, dTym, dRym), ryp = ky * fmaf(-c2, dTyp, dRyp);
          const float rzm = kz * fmaf(-c2, dTzm, dRzm), rzp = kz * fmaf(-c2, dTzp, dRzp);
          const float r0 = -(((rxm + rxp) + (rym + ryp)) + (rzm + rzp));
          float zl;
          if (HV) {
            zl = r0 * a_c;
            zl = fmaf(rxm, sA[s1][tid - 1], zl);
            zl = fmaf(rxp, sA[s1][tid + 1], zl);
            zl = fmaf(rym, sA[s1][tid - BX], zl);
            zl = fmaf(ryp, sA[s1][tid + BX], zl);
            zl = fmaf(rzm, a_p, zl);
            zl = fmaf(rzp, a_n, zl);
          } else {
            zl = r;
          }
          ex_p = rxp * zl;
          ex_m = rxm * zl;
          ey_p = ryp * zl;
          ey_m = rym * zl;
          ezp_new = rzp * zl;
          ezm_new = rzm * zl;
          e0_new = r0 * zl;
        }
      }
      if (NEED_C) {
        sE[s1][0][tid] = ex_p;
        sE[s1][1][tid] = ex_m;
        sE[s1][2][tid] = ey_p;
        sE[s1][3][tid] = ey_m;
      }
    }

    // ---------------- stage C: plane c = t-2 ----------------
    if constexpr (NEED_C) {
      const int c = t - 2;
      if (c >= zb && c < ze) {
        const Conv1 cvz = P.cz[c];
        if (cvz.n0 != KL) {  // node plane KL is complete
          flush(acc_lo, KL - noz);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            acc_lo[d] = acc_hi[d];
            acc_hi[d] = 0.f;
          }
          KL = cvz.n0;
        }
        if (inC) {
          const int s2 = c & 1;
          float w = e0_prev;
          w += sE[s2][1][tid + 1];
          w += sE[s2][0][tid - 1];
          w += sE[s2][3][tid + BX];
          w += sE[s2][2][tid - BX];
          w += ezm_new;
          w += ezp_pp;
          const float wz1 = cvz.f, wz0 = 1.0f - cvz.f;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const float v = g_p[d] * w;
            acc_lo[d] = fmaf(wz0, v, acc_lo[d]);
            acc_hi[d] = fmaf(wz1, v, acc_hi[d]);
          }
        }
      }
    }

    // rotate the register windows
    Tw_p = Tw_c;
    Tw_c = Tw_n;
    R_p = R_c;
    R_c = R_n;
    a_p = a_c;
    a_c = a_n;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      g_p[d] = g_c[d];
      g_c[d] = g_n[d];
    }
    e0_prev = e0_new;
    ezp_pp = ezp_p;
    ezp_p = ezp_new;
    __syncthreads();
  }

  if constexpr (NEED_C) {
    flush(acc_lo, KL - noz);
    flush(acc_hi, KL + 1 - noz);
  }
  if constexpr (MODE != MODE_HV) block_sum_store<NT>(obj, P.red + bid, sRed);
}

template <int BX, int BY>
static hipError_t launch_tile_shape(int mode, const TileParams& p, const float* u, const float* pv,
                                    int grid, hipStream_t st) {
  dim3 blk(BX * BY), grd(grid);
  switch (mode) {
    case MODE_OBJ:
      hipLaunchKernelGGL((ngf_tile_kernel<BX, BY, MODE_OBJ>), grd, blk, 0, st, p, u, pv);
      break;
    case MODE_GRAD:
      hipLaunchKernelGGL((ngf_tile_kernel<BX, BY, MODE_GRAD>), grd, blk, 0, st, p, u, pv);
      break;
    default:
      hipLaunchKernelGGL((ngf_tile_kernel<BX, BY, MODE_HV>), grd, blk, 0, st, p, u, pv);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_tile(const TileShape& s, int mode, const TileParams& p, const float* u,
                       const float* pv, int grid, hipStream_t st) {
  if (s.bx == 32 && s.by == 16) return launch_tile_shape<32, 16>(mode, p, u, pv, grid, st);
  if (s.bx == 64 && s.by == 8) return launch_tile_shape<64, 8>(mode, p, u, pv, grid, st);
  if (s.bx == 32 && s.by == 32) return launch_tile_shape<32, 32>(mode, p, u, pv, grid, st);
  if (s.bx == 64 && s.by == 16) return launch_tile_shape<64, 16>(mode, p, u, pv, grid, st);
  return hipErrorInvalidValue;
}

}  // namespace mfr
