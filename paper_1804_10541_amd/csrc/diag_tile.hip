// Exact diagonal of the Gauss-Newton system, diag(H + alpha nabla^2 S), on
// voxel tiles (the Jacobi preconditioner of the conjugate-gradient solve).
//
// With J = dr dT P (eq. NGF_discretized_hessian) the NGF part of entry (d, n) is
//   2 hbar sum_l ( sum_{k in K} rho-hat_l(k) g_{l+k,d} W_n(l+k) )^2,
// a sum over the rows l of dr (eq. dr, eq. hatRho) whose 7-point stencil meets
// the support of node n; W_n is the trilinear conversion weight of the node
// (eq. grid_conversion) and g the template derivative (eq. dT).
//
// A work-group covers BX x BY voxel columns like the fused tile kernel: it
// owns the rows of dr at the inner (BX-2) x (BY-2) columns, samples the
// template on a one-column ring around them as well, and marches through a
// chunk of z planes.  Per plane t it samples T, g and R (stage A), and at the
// row plane t-1 each own column forms its row of dr and the 21 products
// rho-hat_l(k) g_{l+k,d} (k in K, d = x, y, z), which go to LDS.  Then the
// group's threads, split over the node columns its rows reach in proportion
// to the rows each one has, add (sum_k P_l(k, d) W_n(l+k))^2 over their rows
// for the (up to four) node planes the row plane reaches, in registers.  When
// no later row plane can reach a node plane, the threads of each node column
// are summed in a fixed order and the group writes its partial node block.  A
// node pass sums the blocks of the groups overlapping each node (fixed order)
// and adds the regulariser's diagonal: deterministic, no atomics, nothing per
// voxel in HBM.  Each row's products are formed once; a ring column's rows
// are the neighbouring group's.
//
// For the sum-of-squared-differences distance (Sec. 4.4) dr is the identity:
// each row has the single coefficient 1 at its own voxel, so the products are
// g_{l,d} and the entry is hbar sum_l (g_{l,d} W_n(l))^2.
#include <type_traits>

#include "tile_common.h"

#ifndef DIAG_WP
#define DIAG_WP 1
#endif

namespace mfr {

namespace {

template <bool SSD>
struct DiagSmem {
  static constexpr int BX = kDiagBX, BY = kDiagBY, NT = BX * BY;
  static constexpr int MAXNX = BX + 1, MAXNY = BY + 1, MAXNC = NT / 2;
  // plane exchange with a zero pad of one block row at both ends (NGF only)
  static constexpr int XP = SSD ? 0 : BX, NX = SSD ? 1 : NT + 2 * BX;
  // products of a row, index 7 d + k: the first NV in float4 groups per column
  // (a pitch of 20 floats keeps eight lanes' 16-byte reads on distinct banks),
  // the 21st apart; SSD: the three g_d and a pad
  static constexpr int NV = SSD ? 4 : 20;
  static constexpr int WX = BX + DIAG_WP, WY = BY + DIAG_WP;
  float sTw[2][NX];
  float sR[2][NX];
  float sG[2][3][NX];
  float4 sPv[NT][NV / 4];   // the flush reuses it as a flat float array
  float sPs[SSD ? 1 : NT];
  // conversion weight of local column la (row lb) for node column jx (row jy);
  // 0 for columns outside the image
  float sWx[MAXNX][WX];
  float sWy[MAXNY][WY];
  int sPre[MAXNC + 1];   // first gather thread of each node column (prefix of the thread counts)
  Conv1 sCx[BX], sCy[BY];
  Conv1 sCz[kMaxChunk + 4];
  Samp1 sSz[kMaxChunk + 4];
  int sTotal;
};

__device__ __forceinline__ float uniform_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ __forceinline__ Conv1 uniform_conv(Conv1 c) {
  c.n0 = __builtin_amdgcn_readfirstlane(c.n0);
  c.f = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, c.f)));
  return c;
}

}  // namespace

template <bool SSD>
__global__ __launch_bounds__(kDiagBX* kDiagBY) __attribute__((amdgpu_waves_per_eu(4))) void diag_tile_kernel(
    const DiagTileParams D,
                                                                     const float* __restrict__ u) {
  using Sm = DiagSmem<SSD>;
  constexpr int BX = Sm::BX, BY = Sm::BY, NT = Sm::NT, XP = Sm::XP;
  constexpr int TX = BX - 2, TY = BY - 2;
  __shared__ Sm S;
  const TileParams& P = D.t;

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

  const int gx = x0 - 1 + tx, gy = y0 - 1 + ty;
  const int cxi = min(max(gx, 0), P.mx - 1), cyi = min(max(gy, 0), P.my - 1);
  const Conv1 cvx = P.cx[cxi], cvy = P.cy[cyi];
  const Samp1 spx = P.sx[cxi], spy = P.sy[cyi];
  const float wx0 = 1.0f - cvx.f, wx1 = cvx.f, wy0 = 1.0f - cvy.f, wy1 = cvy.f;
  const unsigned nxy = (unsigned)(P.nx * P.ny);
  const unsigned nodexy = (unsigned)(cvy.n0 * P.nx + cvx.n0);
  const unsigned plane = (unsigned)(P.mx * P.my);
  const unsigned colxy = (unsigned)(cyi * P.mx + cxi);
  const unsigned nb = (unsigned)P.nbar, nxu = (unsigned)P.nx;

  // The group's node block: nodes of its columns inside the image (own and
  // ring) in x and y, and in z the node planes of the planes its rows' z
  // stencils reach.
  const int lxa = x0 == 0 ? 1 : 0, lya = y0 == 0 ? 1 : 0;
  const int lxb = min(BX - 1, P.mx - x0), lyb = min(BY - 1, P.my - y0);
  const int nox = P.cx[x0 - 1 + lxa].n0, noy = P.cy[y0 - 1 + lya].n0;
  const int nxl = P.cx[x0 - 1 + lxb].n0 + 2 - nox, nyl = P.cy[y0 - 1 + lyb].n0 + 2 - noy;
  const int NC = nxl * nyl;
  const int noz = P.cz[max(zb - 1, 0)].n0;
  const int nzend = P.cz[min(ze, P.mz - 1)].n0 + 2;   // one past the block's last node plane

  for (int j = tid; j < ze - zb + 4; j += NT) {
    const int q = min(max(zb - 2 + j, 0), P.mz - 1);
    S.sCz[j] = P.cz[q];
    S.sSz[j] = P.sz[q];
  }
  if (tid < BX) S.sCx[tid] = P.cx[min(max(x0 - 1 + tid, 0), P.mx - 1)];
  if (tid < BY) S.sCy[tid] = P.cy[min(max(y0 - 1 + tid, 0), P.my - 1)];
  if constexpr (XP > 0) {   // the pads of the plane exchange are never written by the march
    for (int w = tid; w < 2 * 2 * XP; w += NT) {
      const int r = w % (2 * XP), sl = w / (2 * XP);
      const int q = r < XP ? r : NT + r;
      S.sTw[sl][q] = 0.f;
      S.sR[sl][q] = 0.f;
      S.sG[sl][0][q] = S.sG[sl][1][q] = S.sG[sl][2][q] = 0.f;
    }
  }
  if (tid == 0) S.sTotal = 0;

  // Row window of node column j (local x node jx, y node jy): the own columns
  // inside the image whose dr rows touch the node's support.
  auto window = [&](int j, int& ax0, int& cw, int& ay0, int& ch) {
    const Range1 rx = D.rx[nox + j % nxl], ry = D.ry[noy + j / nxl];
    ax0 = max(rx.lo, x0);
    cw = max(0, min(rx.hi, min(x0 + TX - 1, P.mx - 1)) - ax0 + 1);
    ay0 = max(ry.lo, y0);
    ch = max(0, min(ry.hi, min(y0 + TY - 1, P.my - 1)) - ay0 + 1);
  };
  __syncthreads();   // tables, sTotal
  for (int q = tid; q < nxl * BX; q += NT) {
    const int jx = q / BX, la = q % BX, a = x0 - 1 + la;
    S.sWx[jx][la] = (a >= 0 && a < P.mx) ? conv_weight(S.sCx[la], nox + jx) : 0.0f;
  }
  for (int q = tid; q < nyl * BY; q += NT) {
    const int jy = q / BY, lb = q % BY, b = y0 - 1 + lb;
    S.sWy[jy][lb] = (b >= 0 && b < P.my) ? conv_weight(S.sCy[lb], noy + jy) : 0.0f;
  }
  // threads per node column: one each, the remaining NT - NC in proportion to the rows
  int rows_j = 0;
  if (tid < NC) {
    int ax0, cw, ay0, ch;
    window(tid, ax0, cw, ay0, ch);
    rows_j = cw * ch;
    atomicAdd(&S.sTotal, rows_j);   // an integer sum: order-free
  }
  __syncthreads();
  if (tid < NC) S.sPre[tid + 1] = 1 + (int)(((long long)rows_j * (NT - NC)) / max(S.sTotal, 1));
  __syncthreads();
  if (tid == 0) {
    S.sPre[0] = 0;
    for (int j = 0; j < NC; ++j) S.sPre[j + 1] += S.sPre[j];
  }
  __syncthreads();

  // This thread's node column (binary search in the prefix) and its rows:
  // r = s, s + G, ... of the column's cw x ch window (x fastest), stepped as
  // (x, y) increments with a carry.
  const bool gathers = tid < S.sPre[NC];
  int jc = 0;
  {
    int lo = 0, hi = NC - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (S.sPre[mid] <= tid) lo = mid; else hi = mid - 1;
    }
    jc = lo;
  }
  const int G = S.sPre[jc + 1] - S.sPre[jc], sidx = tid - S.sPre[jc];
  // the row walk, packed into two registers (every field < 256: windows are at
  // most BX columns, at most NT rows per thread); it is the same every plane
  unsigned walk0 = 0, walk1 = 1u << 16;   // (ra0, rb0, dra, drb), (la0, lb0, cw, trips)
  if (gathers) {
    int ax0, cw, ay0, ch;
    window(jc, ax0, cw, ay0, ch);
    const int rows = cw * ch;
    int trips = 0, ra0 = 0, rb0 = 0, dra = 0, drb = 0;
    if (rows > sidx) {
      trips = (rows - sidx + G - 1) / G;
      ra0 = sidx % cw;
      rb0 = sidx / cw;
      dra = G % cw;
      drb = G / cw;
    }
    walk0 = (unsigned)ra0 | ((unsigned)rb0 << 8) | ((unsigned)dra << 16) | ((unsigned)drb << 24);
    walk1 = (unsigned)(ax0 - (x0 - 1)) | ((unsigned)(ay0 - (y0 - 1)) << 8) | ((unsigned)max(cw, 1) << 16) |
            ((unsigned)trips << 24);
  }
  const float* const wxr = S.sWx[jc % nxl];
  const float* const wyr = S.sWy[jc / nxl];

  const int slot = tile_x + P.tiles_x * (tile_y + P.tiles_y * chunk);
  float* const part = P.part + (size_t)slot * 3 * P.nzt * P.nyt * P.nxt;
  const size_t dstride = (size_t)P.nzt * P.nyt * P.nxt;

  // acc[q][d]: node plane kflush + q (kflush: lowest node plane not yet written)
  float acc[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0f;
  int kflush = noz;
  auto flush = [&]() {
    __syncthreads();   // every gather of the plane is done with sP
    float* const buf = reinterpret_cast<float*>(S.sPv);   // 3 NT floats
    if (gathers) {
#pragma unroll
      for (int d = 0; d < 3; ++d) buf[d * NT + tid] = acc[0][d];
    }
    __syncthreads();
    for (int w = tid; w < 3 * NC; w += NT) {
      const int d = w / NC, j = w % NC;
      float s = 0.0f;
      for (int i = S.sPre[j]; i < S.sPre[j + 1]; ++i) s += buf[d * NT + i];
      part[(size_t)d * dstride + ((size_t)(kflush - noz) * P.nyt + j / nxl) * P.nxt + j % nxl] = s;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      acc[0][d] = acc[1][d];
      acc[1][d] = acc[2][d];
      acc[2][d] = acc[3][d];
      acc[3][d] = 0.0f;
    }
    ++kflush;
  };

  // Register windows of the own column; slot (t - tfirst) mod 3.
  float Tw[3] = {0.f, 0.f, 0.f}, Rv[3] = {0.f, 0.f, 0.f};
  float g[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};

  int Kp = -0x7fffffff;
  float ulo[3] = {0.f, 0.f, 0.f}, udz[3] = {0.f, 0.f, 0.f};
  const __amdgpu_buffer_rsrc_t rsT = raw_buffer(P.Tp, P.Tbytes), rsR = raw_buffer(P.R, P.Rbytes);
  const CornerOffsets co{4u * (unsigned)P.PX, 4u * (unsigned)P.PXY, 4u * (unsigned)(P.PX + P.PXY)};
  const unsigned rcol = colxy << 2;
  auto xy_interp = [&](int k, float (&o)[3]) {
    const unsigned i00 = (unsigned)k * nxy + nodexy;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const unsigned b = (unsigned)d * nb + i00;
      const float lo = fmaf(wx1, ld32(u, b + 1), wx0 * ld32(u, b));
      const float hi = fmaf(wx1, ld32(u, b + nxu + 1), wx0 * ld32(u, b + nxu));
      o[d] = fmaf(wy1, hi, wy0 * lo);
    }
  };

  // stage-A inputs of the next plane, loaded one step ahead
  float nx_t[8];
  float nx_fx = 0.f, nx_fy = 0.f, nx_fz = 0.f, nx_R = 0.f;
  auto issue = [&](int tt) {
    const int tc = min(max(tt, 0), P.mz - 1);
    const int jz = tt - zb + 2;
    const Conv1 cvz = uniform_conv(S.sCz[jz]);
    if (cvz.n0 != Kp) {   // both node planes are interpolated again (cached reads; fewer live registers)
      float uhi[3];
      xy_interp(cvz.n0, ulo);
      xy_interp(cvz.n0 + 1, uhi);
#pragma unroll
      for (int d = 0; d < 3; ++d) udz[d] = uhi[d] - ulo[d];
      Kp = cvz.n0;
    }
    const float fz = cvz.f;
    const int kx = template_cell(spx, fmaf(fz, udz[0], ulo[0]), P.ihTx, nx_fx);
    const int ky = template_cell(spy, fmaf(fz, udz[1], ulo[1]), P.ihTy, nx_fy);
    const int kz = template_cell(S.sSz[jz], fmaf(fz, udz[2], ulo[2]), P.ihTz, nx_fz);
    template_corners_buf(P, rsT, co, kx, ky, kz, nx_t);
    nx_R = buf_ld(rsR, rcol, (unsigned)tc * plane * 4u);
  };

  // The rows of row plane c, for NQ reached node planes from kflush.
  auto gather = [&](auto NQc, int c) {
    constexpr int NQ = decltype(NQc)::value;
    const bool hzm = c > 0, hzp = c < P.mz - 1;
    const Conv1 cz0 = uniform_conv(S.sCz[c - zb + 2]);
    const Conv1 czm = uniform_conv(S.sCz[c - zb + 1]), czp = uniform_conv(S.sCz[c - zb + 3]);
    float wz0[NQ], wzp[NQ], wzm[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      // uniform: scalar registers
      wz0[q] = uniform_f(conv_weight(cz0, kflush + q));
      wzp[q] = uniform_f((hzp && !SSD) ? conv_weight(czp, kflush + q) : 0.0f);
      wzm[q] = uniform_f((hzm && !SSD) ? conv_weight(czm, kflush + q) : 0.0f);
    }
    int ra = walk0 & 255, rb = (walk0 >> 8) & 255;
    const int dra = (walk0 >> 16) & 255, drb = walk0 >> 24;
    const int la0 = walk1 & 255, lb0 = (walk1 >> 8) & 255, cw = (walk1 >> 16) & 255, trips = walk1 >> 24;
    for (int it = 0; it < trips; ++it) {
      const int la = la0 + ra, lb = lb0 + rb;
      ra += dra;
      rb += drb;
      if (ra >= cw) {
        ra -= cw;
        rb += 1;
      }
      const int li = lb * BX + la;
      const float vx0 = wxr[la], vy0 = wyr[lb];
      const float w00 = vx0 * vy0;
      if constexpr (SSD) {
        const float4 gv = S.sPv[li][0];
        const float pv[3] = {gv.x, gv.y, gv.z};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float pxy = w00 * pv[d];
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const float zz = wz0[q] * pxy;
            acc[q][d] = fmaf(zz, zz, acc[q][d]);
          }
        }
      } else {
        float pv[21];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const float4 a = S.sPv[li][v];
          pv[4 * v] = a.x;
          pv[4 * v + 1] = a.y;
          pv[4 * v + 2] = a.z;
          pv[4 * v + 3] = a.w;
        }
        pv[20] = S.sPs[li];
        const float wxm = wxr[la - 1] * vy0, wxp = wxr[la + 1] * vy0;
        const float wym = vx0 * wyr[lb - 1], wyp = vx0 * wyr[lb + 1];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float* pd = pv + 7 * d;
          float pxy = w00 * pd[0];
          pxy = fmaf(wxm, pd[1], pxy);
          pxy = fmaf(wxp, pd[2], pxy);
          pxy = fmaf(wym, pd[3], pxy);
          pxy = fmaf(wyp, pd[4], pxy);
          const float zm = w00 * pd[5], zp = w00 * pd[6];
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const float zz = fmaf(wz0[q], pxy, fmaf(wzp[q], zp, wzm[q] * zm));
            acc[q][d] = fmaf(zz, zz, acc[q][d]);
          }
        }
      }
    }
  };

  const int tfirst = zb - 1, tlast = ze;

  auto step = [&](auto Kc, int t) {
    constexpr int K = decltype(Kc)::value;   // slot of plane t
    constexpr int K1 = (K + 2) % 3;          // slot of plane t-1
    constexpr int K2 = (K + 1) % 3;          // slot of plane t-2

    // ---------------- stage A: plane t ----------------
    {
      const Tri s = trilinear(P, nx_t, nx_fx, nx_fy, nx_fz);
      Tw[K] = s.v;
      g[K][0] = s.gx;
      g[K][1] = s.gy;
      g[K][2] = s.gz;
      Rv[K] = nx_R;
      if constexpr (!SSD) {
        const int sl = t & 1;
        S.sTw[sl][XP + tid] = Tw[K];
        S.sR[sl][XP + tid] = Rv[K];
        S.sG[sl][0][XP + tid] = s.gx;
        S.sG[sl][1][XP + tid] = s.gy;
        S.sG[sl][2][XP + tid] = s.gz;
      }
    }
    if (t < tlast) issue(t + 1);

    // ---------------- row plane c = t-1: products, then the gather ----------------
    const int c = t - 1;
    if (c < zb) {   // uniform: the first two steps sample planes zb-1 and zb only
      __syncthreads();
      return;
    }
    if constexpr (SSD) {
      S.sPv[tid][0] = make_float4(g[K1][0], g[K1][1], g[K1][2], 0.0f);
    } else {
      // the row of dr at this column (every lane evaluates it; the gather reads
      // own rows inside the image only)
      const int s1 = c & 1;
      const int q = XP + tid;
      const float Tc = Tw[K1], Rc = Rv[K1];
      const float dTxm = S.sTw[s1][q - 1] - Tc, dTxp = S.sTw[s1][q + 1] - Tc;
      const float dTym = S.sTw[s1][q - BX] - Tc, dTyp = S.sTw[s1][q + BX] - Tc;
      const float dTzm = Tw[K2] - Tc, dTzp = Tw[K] - Tc;
      const float dRxm = S.sR[s1][q - 1] - Rc, dRxp = S.sR[s1][q + 1] - Rc;
      const float dRym = S.sR[s1][q - BX] - Rc, dRyp = S.sR[s1][q + BX] - Rc;
      const float dRzm = Rv[K2] - Rc, dRzp = Rv[K] - Rc;
      const float sTT = fmaf(fmaf(dTxm, dTxm, dTxp * dTxp), P.ih2x,
                             fmaf(fmaf(dTym, dTym, dTyp * dTyp), P.ih2y, fmaf(dTzm, dTzm, dTzp * dTzp) * P.ih2z));
      const float sRR = fmaf(fmaf(dRxm, dRxm, dRxp * dRxp), P.ih2x,
                             fmaf(fmaf(dRym, dRym, dRyp * dRyp), P.ih2y, fmaf(dRzm, dRzm, dRzp * dRzp) * P.ih2z));
      const float sTR = fmaf(fmaf(dTxm, dRxm, dTxp * dRxp), P.ih2x,
                             fmaf(fmaf(dTym, dRym, dTyp * dRyp), P.ih2y, fmaf(dTzm, dRzm, dTzp * dRzp) * P.ih2z));
      const float nT2 = fmaf(0.5f, sTT, P.tau2);
      const float nR2 = fmaf(0.5f, sRR, P.rho2);
      const float r1 = fmaf(0.5f, sTR, P.taurho);
      const float rnT = rsq_norm(nT2), rnR = rsq_norm(nR2);
      const float c1 = rnT * rnR;
      const float c2 = r1 * rnT * rnT;
      const float kx = P.hhx * c1, ky = P.hhy * c1, kz = P.hhz * c1;
      const float rxm = kx * fmaf(-c2, dTxm, dRxm), rxp = kx * fmaf(-c2, dTxp, dRxp);
      const float rym = ky * fmaf(-c2, dTym, dRym), ryp = ky * fmaf(-c2, dTyp, dRyp);
      const float rzm = kz * fmaf(-c2, dTzm, dRzm), rzp = kz * fmaf(-c2, dTzp, dRzp);
      const float r0 = -(((rxm + rxp) + (rym + ryp)) + (rzm + rzp));
      float pv[21];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float* pd = pv + 7 * d;
        pd[0] = r0 * g[K1][d];
        pd[1] = rxm * S.sG[s1][d][q - 1];
        pd[2] = rxp * S.sG[s1][d][q + 1];
        pd[3] = rym * S.sG[s1][d][q - BX];
        pd[4] = ryp * S.sG[s1][d][q + BX];
        pd[5] = rzm * g[K2][d];
        pd[6] = rzp * g[K][d];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) S.sPv[tid][v] = make_float4(pv[4 * v], pv[4 * v + 1], pv[4 * v + 2], pv[4 * v + 3]);
      S.sPs[tid] = pv[20];
    }
    __syncthreads();   // the products of the row plane

    // node planes the row plane reaches: kflush (the lower node plane of plane
    // c-1, the lowest any of its three planes touches) up to the upper node
    // plane of plane c+1; the accumulators of further planes would add exact zeros
    const int n0c = __builtin_amdgcn_readfirstlane(S.sCz[c - zb + 2].n0);
    const int n0p = __builtin_amdgcn_readfirstlane(S.sCz[c - zb + 3].n0);
    const int top = (SSD ? n0c : max(n0c, n0p)) + 1;
    const int nq = min(max(top - kflush + 1, 1), 4);
    switch (nq) {
      case 1: gather(std::integral_constant<int, 1>{}, c); break;
      case 2: gather(std::integral_constant<int, 2>{}, c); break;
      case 3: gather(std::integral_constant<int, 3>{}, c); break;
      default: gather(std::integral_constant<int, 4>{}, c); break;
    }
    // node planes below those of the next row plane are complete
    while (kflush < n0c) flush();
    __syncthreads();   // sP and the plane-exchange slots are free for the next step
  };

  issue(tfirst);
  for (int t = tfirst; t <= tlast; t += 3) {
    step(std::integral_constant<int, 0>{}, t);
    if (t + 1 <= tlast) step(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 <= tlast) step(std::integral_constant<int, 2>{}, t + 2);
  }
  while (kflush < nzend) flush();
}

// The same for a two-dimensional problem (d = 2): a group of kPlaneNT threads
// covers kPlaneNT pixel columns (own inner columns and a one-column ring) and
// marches through a chunk of pixel rows; a row of dr has five entries (0, -x,
// +x, -y, +y), so ten products per pixel; the node columns are the x nodes the
// group's rows reach, and the up to four node rows a pixel row reaches take
// the place of the node planes.  Its partial blocks use the node pass's view
// of the node grid as n_x x n_y x 1 (x tiles, row chunks as y tiles).
__global__ __launch_bounds__(kPlaneNT) void plane_diag_kernel(const DiagTileParams D, const float* __restrict__ u) {
  constexpr int NT = kPlaneNT, TX = NT - 2;
  // row exchange with one zero pad at both ends
  __shared__ float sTw[2][NT + 2], sR[2][NT + 2], sG[2][2][NT + 2];
  // products of a row, index 5 d + k (k: 0, -x, +x, -y, +y); a pitch of ten
  // floats puts sixteen lanes' 8-byte reads on distinct banks
  __shared__ float2 sPv[NT][5];
  __shared__ Conv1 sCx[NT];
  __shared__ Conv1 sCy[kMaxChunk + 4];
  __shared__ Samp1 sSy[kMaxChunk + 4];
  __shared__ int sPre[NT + 1];
  __shared__ int sTotal;
  const TileParams& P = D.t;

  const int tid = threadIdx.x;
  const int bid = xcd_block_id();
  const int tile_x = bid % P.tiles_x, chunk = bid / P.tiles_x;
  const int x0 = tile_x * TX;
  const int yb = chunk * P.chunk_len, ye = min(P.my, yb + P.chunk_len);

  const int gx = x0 - 1 + tid;
  const int cxi = min(max(gx, 0), P.mx - 1);
  const Conv1 cvx = P.cx[cxi];
  const Samp1 spx = P.sx[cxi];
  const float wx0 = 1.0f - cvx.f, wx1 = cvx.f;
  const unsigned nb = (unsigned)P.nbar, nxu = (unsigned)P.nx;

  const int lxa = x0 == 0 ? 1 : 0;
  const int lxb = min(NT - 1, P.mx - x0);
  const int nox = P.cx[x0 - 1 + lxa].n0;
  const int NC = P.cx[x0 - 1 + lxb].n0 + 2 - nox;   // node columns of the block
  const int noy = P.cy[max(yb - 1, 0)].n0;
  const int nyend = P.cy[min(ye, P.my - 1)].n0 + 2;
  for (int j = tid; j < ye - yb + 4; j += NT) {
    const int q = min(max(yb - 2 + j, 0), P.my - 1);
    sCy[j] = P.cy[q];
    sSy[j] = P.sy[q];
  }
  // columns outside the image carry no conversion weight
  sCx[tid] = (gx >= 0 && gx < P.mx) ? cvx : Conv1{-8, 0.0f};
  if (tid < 4) {
    const int sl = tid >> 1, q = (tid & 1) ? NT + 1 : 0;
    sTw[sl][q] = sR[sl][q] = sG[sl][0][q] = sG[sl][1][q] = 0.f;
  }
  if (tid == 0) sTotal = 0;
  // the own columns inside the image whose dr rows touch node column j's support
  auto window = [&](int j, int& ax0, int& cw) {
    const Range1 rx = D.rx[nox + j];
    ax0 = max(rx.lo, x0);
    cw = max(0, min(rx.hi, min(x0 + TX - 1, P.mx - 1)) - ax0 + 1);
  };
  __syncthreads();
  int rows_j = 0;
  if (tid < NC) {
    int ax0;
    window(tid, ax0, rows_j);
    atomicAdd(&sTotal, rows_j);   // an integer sum: order-free
  }
  __syncthreads();
  if (tid < NC) sPre[tid + 1] = 1 + (int)(((long long)rows_j * (NT - NC)) / max(sTotal, 1));
  __syncthreads();
  if (tid == 0) {
    sPre[0] = 0;
    for (int j = 0; j < NC; ++j) sPre[j + 1] += sPre[j];
  }
  __syncthreads();
  const bool gathers = tid < sPre[NC];
  int jc = 0;
  {
    int lo = 0, hi = NC - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sPre[mid] <= tid) lo = mid; else hi = mid - 1;
    }
    jc = lo;
  }
  const int G = sPre[jc + 1] - sPre[jc], sidx = tid - sPre[jc];
  const int nodec = nox + jc;
  int la0 = 1, trips = 0;
  if (gathers) {
    int ax0, cw;
    window(jc, ax0, cw);
    la0 = ax0 - (x0 - 1) + sidx;   // this thread's columns: la0, la0 + G, ...
    trips = cw > sidx ? (cw - sidx + G - 1) / G : 0;
  }

  const int slot = tile_x + P.tiles_x * chunk;
  float* const part = P.part + (size_t)slot * 3 * P.nzt * P.nyt * P.nxt;
  const size_t dstride = (size_t)P.nzt * P.nyt * P.nxt;
  float acc[4][2];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q][0] = acc[q][1] = 0.0f;
  int kflush = noy;
  auto flush = [&]() {
    __syncthreads();
    float* const buf = reinterpret_cast<float*>(sPv);   // 2 NT floats
    if (gathers) {
      buf[tid] = acc[0][0];
      buf[NT + tid] = acc[0][1];
    }
    __syncthreads();
    for (int w = tid; w < 2 * NC; w += NT) {
      const int d = w / NC, j = w % NC;
      float s = 0.0f;
      for (int i = sPre[j]; i < sPre[j + 1]; ++i) s += buf[d * NT + i];
      part[(size_t)d * dstride + (size_t)(kflush - noy) * P.nxt + j] = s;
    }
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      acc[0][d] = acc[1][d];
      acc[1][d] = acc[2][d];
      acc[2][d] = acc[3][d];
      acc[3][d] = 0.0f;
    }
    ++kflush;
  };

  float Tw[3] = {0.f, 0.f, 0.f}, Rv[3] = {0.f, 0.f, 0.f};
  float g[3][2] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
  int Kp = -0x7fffffff;
  float ulo[2] = {0.f, 0.f}, udy[2] = {0.f, 0.f};
  const __amdgpu_buffer_rsrc_t rsT = raw_buffer(P.Tp, P.Tbytes), rsR = raw_buffer(P.R, P.Rbytes);
  const unsigned rcol = (unsigned)cxi << 2;
  const unsigned PX = (unsigned)P.PX;
  auto x_interp = [&](int k, float (&o)[2]) {
    const unsigned i0 = (unsigned)k * nxu + (unsigned)cvx.n0;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const unsigned b = (unsigned)d * nb + i0;
      o[d] = fmaf(wx1, ld32(u, b + 1), wx0 * ld32(u, b));
    }
  };
  float nt00 = 0.f, nt10 = 0.f, nt01 = 0.f, nt11 = 0.f, nfx = 0.f, nfy = 0.f, nR = 0.f;
  auto issue = [&](int tt) {
    const int tc = min(max(tt, 0), P.my - 1);
    const int jy = tt - yb + 2;
    const Conv1 cvy = uniform_conv(sCy[jy]);
    if (cvy.n0 != Kp) {
      float uhi[2];
      x_interp(cvy.n0, ulo);
      x_interp(cvy.n0 + 1, uhi);
      udy[0] = uhi[0] - ulo[0];
      udy[1] = uhi[1] - ulo[1];
      Kp = cvy.n0;
    }
    const float fy = cvy.f;
    int kx = template_cell(spx, fmaf(fy, udy[0], ulo[0]), P.ihTx, nfx);
    int ky = template_cell(sSy[jy], fmaf(fy, udy[1], ulo[1]), P.ihTy, nfy);
    kx = clamp_m2(kx, P.mTx);
    ky = clamp_m2(ky, P.mTy);
    const unsigned v = (__umul24((unsigned)(ky + 2), PX) + (unsigned)(kx + 2)) << 2;
    const FPair a = buf_ld2(rsT, v, 0), b = buf_ld2(rsT, v, 4u * PX);
    nt00 = a.a;
    nt10 = a.b;
    nt01 = b.a;
    nt11 = b.b;
    nR = buf_ld(rsR, rcol, (unsigned)tc * (unsigned)P.mx * 4u);
  };

  auto gather = [&](auto NQc, int c) {
    constexpr int NQ = decltype(NQc)::value;
    const bool hym = c > 0, hyp = c < P.my - 1;
    const Conv1 cy0 = uniform_conv(sCy[c - yb + 2]);
    const Conv1 cym = uniform_conv(sCy[c - yb + 1]), cyp = uniform_conv(sCy[c - yb + 3]);
    float wy0[NQ], wyp[NQ], wym[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      wy0[q] = uniform_f(conv_weight(cy0, kflush + q));
      wyp[q] = uniform_f(hyp ? conv_weight(cyp, kflush + q) : 0.0f);
      wym[q] = uniform_f(hym ? conv_weight(cym, kflush + q) : 0.0f);
    }
    int la = la0;
    for (int it = 0; it < trips; ++it, la += G) {
      const float vx0 = conv_weight(sCx[la], nodec);
      const float vxm = conv_weight(sCx[la - 1], nodec), vxp = conv_weight(sCx[la + 1], nodec);
      float pv[10];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const float2 a = sPv[la][v];
        pv[2 * v] = a.x;
        pv[2 * v + 1] = a.y;
      }
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const float* pd = pv + 5 * d;
        float px = vx0 * pd[0];
        px = fmaf(vxm, pd[1], px);
        px = fmaf(vxp, pd[2], px);
        const float ym = vx0 * pd[3], yp = vx0 * pd[4];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const float zz = fmaf(wy0[q], px, fmaf(wyp[q], yp, wym[q] * ym));
          acc[q][d] = fmaf(zz, zz, acc[q][d]);
        }
      }
    }
  };

  const int tfirst = yb - 1, tlast = ye;
  auto step = [&](auto Kc, int t) {
    constexpr int K = decltype(Kc)::value;   // slot of row t
    constexpr int K1 = (K + 2) % 3;          // slot of row t-1
    constexpr int K2 = (K + 1) % 3;          // slot of row t-2
    {
      const float d0 = nt10 - nt00, d1 = nt11 - nt01;
      const float f0 = fmaf(nfx, d0, nt00), f1 = fmaf(nfx, d1, nt01);
      Tw[K] = fmaf(nfy, f1 - f0, f0);
      g[K][0] = fmaf(nfy, d1 - d0, d0) * P.ihTx;
      g[K][1] = (f1 - f0) * P.ihTy;
      Rv[K] = nR;
      const int sl = t & 1;
      sTw[sl][1 + tid] = Tw[K];
      sR[sl][1 + tid] = Rv[K];
      sG[sl][0][1 + tid] = g[K][0];
      sG[sl][1][1 + tid] = g[K][1];
    }
    if (t < tlast) issue(t + 1);
    const int c = t - 1;
    if (c < yb) {   // uniform: the first two steps sample rows yb-1 and yb only
      __syncthreads();
      return;
    }
    {
      const int s1 = c & 1;
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
      const float c2 = r1 * rnT * rnT;
      const float kx = P.hhx * c1, ky = P.hhy * c1;
      const float rxm = kx * fmaf(-c2, dTxm, dRxm), rxp = kx * fmaf(-c2, dTxp, dRxp);
      const float rym = ky * fmaf(-c2, dTym, dRym), ryp = ky * fmaf(-c2, dTyp, dRyp);
      const float r0 = -((rxm + rxp) + (rym + ryp));
      float pv[10];
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        float* pd = pv + 5 * d;
        pd[0] = r0 * g[K1][d];
        pd[1] = rxm * sG[s1][d][q - 1];
        pd[2] = rxp * sG[s1][d][q + 1];
        pd[3] = rym * g[K2][d];
        pd[4] = ryp * g[K][d];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) sPv[tid][v] = make_float2(pv[2 * v], pv[2 * v + 1]);
    }
    __syncthreads();
    const int n0c = __builtin_amdgcn_readfirstlane(sCy[c - yb + 2].n0);
    const int n0p = __builtin_amdgcn_readfirstlane(sCy[c - yb + 3].n0);
    const int nq = min(max(max(n0c, n0p) + 1 - kflush + 1, 1), 4);
    switch (nq) {
      case 1: gather(std::integral_constant<int, 1>{}, c); break;
      case 2: gather(std::integral_constant<int, 2>{}, c); break;
      case 3: gather(std::integral_constant<int, 3>{}, c); break;
      default: gather(std::integral_constant<int, 4>{}, c); break;
    }
    while (kflush < n0c) flush();
    __syncthreads();
  };

  issue(tfirst);
  for (int t = tfirst; t <= tlast; t += 3) {
    step(std::integral_constant<int, 0>{}, t);
    if (t + 1 <= tlast) step(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 <= tlast) step(std::integral_constant<int, 2>{}, t + 2);
  }
  while (kflush < nyend) flush();
}

// Node pass of the diagonal: the partial blocks of every group overlapping
// node n (fixed order), scaled, plus the regulariser's diagonal:
// curvature (L^T L)_nn = L_nn^2 + sum over present neighbours of 1/hy^4,
// diffusive -L_nn, elastic -L_nn + kappa (adjacent cells) / (16 hy_d^2).
__global__ __launch_bounds__(256) void diag_node_kernel(const DiagTileParams D, float* __restrict__ diag) {
  const TileParams& P = D.t;
  const int n = blockIdx.x * 256 + threadIdx.x, d = blockIdx.y;
  if (n >= P.nbar) return;
  const int i = n % P.nx, j = (n / P.nx) % P.ny, k = n / (P.nx * P.ny);
  const Range1 rx = D.ntx[i], ry = D.nty[j], rz = D.ntz[k];
  float s = 0.0f;
  for (int cz = rz.lo; cz <= rz.hi; ++cz) {
    const int kz = k - D.orgz[cz];
    for (int cy = ry.lo; cy <= ry.hi; ++cy) {
      const int iy = j - D.orgy[cy];
      for (int cx = rx.lo; cx <= rx.hi; ++cx) {
        const int jx = i - D.orgx[cx];
        const size_t slot = (size_t)cx + (size_t)P.tiles_x * ((size_t)cy + (size_t)P.tiles_y * cz);
        s += P.part[(((slot * 3 + d) * P.nzt + kz) * P.nyt + iy) * P.nxt + jx];
      }
    }
  }
  const int cxn = (i > 0) + (i < P.nx - 1), cyn = (j > 0) + (j < P.ny - 1), czn = (k > 0) + (k < P.nz - 1);
  const float Lnn = -(cxn * D.ihy2x + cyn * D.ihy2y + czn * D.ihy2z);
  const float LL =
      P.reg ? -Lnn : Lnn * Lnn + cxn * D.ihy2x * D.ihy2x + cyn * D.ihy2y * D.ihy2y + czn * D.ihy2z * D.ihy2z;
  const float ncell = P.reg == 2 ? P.kappa * (float)(cxn * cyn * czn) * 0.0625f : 0.0f;
  const float ih2 = d == 0 ? D.ihy2x : d == 1 ? D.ihy2y : D.ihy2z;
  diag[(size_t)d * P.nbar + n] = fmaf(D.s_ngf, s, D.s_curv * fmaf(ncell, ih2, LL));
}

hipError_t launch_diag_tile(const DiagTileParams& d, const float* u, float* diag, hipStream_t st) {
  const int grid = d.t.tiles_x * d.t.tiles_y * d.t.chunks;
  if (d.plane) {   // two-dimensional: row chunks in place of y tiles
    hipLaunchKernelGGL(plane_diag_kernel, dim3(grid), dim3(kPlaneNT), 0, st, d, u);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_node_kernel, dim3((d.t.nbar + 255) / 256, 2), dim3(256), 0, st, d, diag);
    return hipGetLastError();
  }
  if (d.t.ssd)
    hipLaunchKernelGGL((diag_tile_kernel<true>), dim3(grid), dim3(kDiagBX * kDiagBY), 0, st, d, u);
  else
    hipLaunchKernelGGL((diag_tile_kernel<false>), dim3(grid), dim3(kDiagBX * kDiagBY), 0, st, d, u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_node_kernel, dim3((d.t.nbar + 255) / 256, 3), dim3(256), 0, st, d, diag);
  return hipGetLastError();
}

}  // namespace mfr
