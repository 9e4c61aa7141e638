// Fused matrix-free NGF kernel on voxel tiles (CDNA4 / gfx950).
//
// One work-group covers a column block of BX x BY voxel columns: it owns the
// rows of dr at the inner (BX-2) x (BY-2) columns and samples the template on
// a one-column ring around them as well, which the differences of its rows
// need.  The group marches through a chunk of z planes; each thread owns one
// column and keeps the values of its own column in registers across planes,
// while the x/y neighbours of the current plane are exchanged through LDS.
// Per step t three stages run:
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
//         A group gathers only its own rows, at every column it covers (own
//         columns and ring): a ring column is an own column of the
//         neighbouring group, which adds the contributions of its rows there,
//         and P^T is linear, so the two partial node blocks sum to the whole.
//         Each row's contributions are formed exactly once.
//
// Columns and planes outside the image sample the template at the clamped
// position, so every neighbour read in stage B already holds the clamped
// value of eq. boundary_conditions (differences across the border are 0).
// The stage-A inputs of plane t+1 (template corners, reference value) are
// loaded during step t.  The march is unrolled by three so the per-column
// register windows (planes t, t-1, t-2) sit in fixed registers.
//
// P^T is a gather: each column accumulates its z contributions in registers;
// when a node plane is complete the group reduces it over x and y in LDS and
// writes the node block to its own slot of a partial buffer.  A node pass sums
// the slots that overlap each node in a fixed order, so results are
// deterministic and no atomics are used.  Nothing per voxel reaches HBM.
//
// The same march evaluates the sum-of-squared-differences distance (SSD,
// Sec. 4.4), whose residual Jacobian dr/dT is the identity: stage B forms
// r = T(P y) - R and z_l = a_l (Hessian) or r_l (gradient) at the own columns,
// stage C takes w_i = z_i, and no plane data is exchanged through LDS.
#include <type_traits>

#include "tile_common.h"

namespace mfr {

// LDS of one work-group of the voxel-tile kernel.
template <int BX, int BY, int MODE, bool SSD>
struct TileSmem {
  static constexpr int NT = BX * BY, MAXNX = BX + 1, MAXNY = BY + 1;
  static constexpr bool HV = (MODE == MODE_HV), NEED_C = (MODE != MODE_OBJ);
  static constexpr int NX = SSD ? 1 : NT;   // plane exchange (NGF differences only)
  // with a zero pad of one block row at both ends, so that every lane's four
  // neighbour reads stay inside the arrays and read finite values
  static constexpr int XP = SSD ? 0 : BX;
  float sTw[2][NX + 2 * XP];
  float sR[2][NX + 2 * XP];
  float sA[HV ? 2 : 1][HV ? NX + 2 * XP : 1];
  // row products of the plane exchange, with a zero pad of one block row at both
  // ends: a neighbour read past the block's edge (or wrapping to the next row,
  // whose edge column is a ring column that writes 0) then adds exactly 0
  static constexpr int EP = (NEED_C && !SSD) ? BX : 0;
  float sE[NEED_C ? 2 : 1][4][NEED_C ? NX + 2 * EP : 1];
  float sV[NEED_C ? 3 : 1][NEED_C ? NT : 1];
  float sW[NEED_C ? 3 : 1][NEED_C ? BY * MAXNX : 1];
  int sColLo[MAXNX], sColHi[MAXNX], sRowLo[MAXNY], sRowHi[MAXNY];
  Conv1 sCx[BX], sCy[BY];
  // z conversion and template-coordinate entries of planes zb-2 .. ze+1 (clamped
  // into the image): read at a uniform index every plane, from LDS rather than
  // through a vector load whose latency would sit on every step's address path
  Conv1 sCz[kMaxChunk + 4];
  Samp1 sSz[kMaxChunk + 4];
  double sRed[NT / 64];
};

// One tile (work-group id `bid` of the problem P) of the fused kernel.
template <int BX, int BY, int MODE, bool SSD>
__device__ __forceinline__ void tile_body(const TileParams& P, const int bid, const float* __restrict__ u,
                                          const float* __restrict__ pv, TileSmem<BX, BY, MODE, SSD>& S) {
  constexpr int NT = BX * BY;
  constexpr int TX = BX - 2, TY = BY - 2;   // own columns per tile
  constexpr int MAXNX = BX + 1;
  constexpr bool HV = (MODE == MODE_HV);
  constexpr bool NEED_C = (MODE != MODE_OBJ);
  auto& sTw = S.sTw;
  auto& sR = S.sR;
  auto& sA = S.sA;
  auto& sE = S.sE;
  constexpr int EP = TileSmem<BX, BY, MODE, SSD>::EP;
  auto& sV = S.sV;
  auto& sW = S.sW;
  auto& sColLo = S.sColLo;
  auto& sColHi = S.sColHi;
  auto& sRowLo = S.sRowLo;
  auto& sRowHi = S.sRowHi;
  auto& sCx = S.sCx;
  auto& sCy = S.sCy;
  auto& sCz = S.sCz;
  auto& sSz = S.sSz;
  auto& sRed = S.sRed;

  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;

  const int tile_x = bid % P.tiles_x;
  const int rest = bid / P.tiles_x;
  const int tile_y = rest % P.tiles_y;
  const int chunk = rest / P.tiles_y;
  const int x0 = tile_x * TX, y0 = tile_y * TY;
  const int zb = chunk * P.chunk_len;
  const int ze = min(P.mz, zb + P.chunk_len);

  // Columns: the own columns tx in [1, BX-2] plus a one-column ring.  Stage B
  // forms the rows of dr at own columns only; stage C gathers, at every column
  // of the group inside the image, the contributions of the group's own rows
  // (the ring's other contributions come from the neighbouring group, whose
  // own columns they are) and the transposed conversion sums both groups'
  // partial node blocks.
  const int gx = x0 - 1 + tx, gy = y0 - 1 + ty;
  const bool in_img = (gx >= 0) && (gx < P.mx) && (gy >= 0) && (gy < P.my);
  const bool own = (tx >= 1) && (tx < BX - 1) && (ty >= 1) && (ty < BY - 1);
  const bool inB = own && in_img;
  const bool inC = in_img;
  const float own_row = inB ? 1.0f : 0.0f;   // scales z_l: 0 for rows this group does not own

  // own column, clamped into the image
  const int cxi = min(max(gx, 0), P.mx - 1), cyi = min(max(gy, 0), P.my - 1);
  const Conv1 cvx = P.cx[cxi], cvy = P.cy[cyi];
  const Samp1 spx = P.sx[cxi], spy = P.sy[cyi];
  const float wx0 = 1.0f - cvx.f, wx1 = cvx.f, wy0 = 1.0f - cvy.f, wy1 = cvy.f;
  const unsigned nxy = (unsigned)(P.nx * P.ny);
  const unsigned nodexy = (unsigned)(cvy.n0 * P.nx + cvx.n0);
  const unsigned plane = (unsigned)(P.mx * P.my);
  const unsigned colxy = (unsigned)(cyi * P.mx + cxi);
  const unsigned nb = (unsigned)P.nbar, nxu = (unsigned)P.nx;

  // Local columns [lxa, lxb] and rows [lya, lyb] of the group inside the image,
  // the first node they touch and the number of node columns / rows touched.
  const int lxa = x0 == 0 ? 1 : 0, lya = y0 == 0 ? 1 : 0;
  const int lxb = min(BX - 1, P.mx - x0), lyb = min(BY - 1, P.my - y0);
  const int nox = P.cx[x0 - 1 + lxa].n0, noy = P.cy[y0 - 1 + lya].n0, noz = P.cz[zb].n0;
  for (int j = tid; j < ze - zb + 4; j += NT) {
    const int q = min(max(zb - 2 + j, 0), P.mz - 1);
    sCz[j] = P.cz[q];
    sSz[j] = P.sz[q];
  }
  if constexpr (!NEED_C) __syncthreads();   // (with NEED_C the barrier after sCx / sCy covers it)
  constexpr int XP = TileSmem<BX, BY, MODE, SSD>::XP;
  if constexpr (XP > 0) {   // nor are the pads of the plane exchange
    for (int w = tid; w < 2 * 2 * XP; w += NT) {
      const int r = w % (2 * XP), sl = w / (2 * XP);
      const int q = r < XP ? r : NT + r;
      sTw[sl][q] = 0.f;
      sR[sl][q] = 0.f;
      if constexpr (HV) sA[sl][q] = 0.f;
    }
  }
  if constexpr (EP > 0) {   // the pads of sE are never written by the march
    for (int w = tid; w < 2 * 4 * 2 * EP; w += NT) {
      const int r = w % (2 * EP), k = (w / (2 * EP)) % 4, sl = w / (8 * EP);
      sE[sl][k][r < EP ? r : NT + r] = 0.f;
    }
  }
  const int nxl = P.cx[x0 - 1 + lxb].n0 + 2 - nox;
  const int nyl = P.cy[y0 - 1 + lyb].n0 + 2 - noy;
  if constexpr (NEED_C) {
    if (tid < BX) sCx[tid] = P.cx[min(max(x0 - 1 + tid, 0), P.mx - 1)];
    if (tid < BY) sCy[tid] = P.cy[min(max(y0 - 1 + tid, 0), P.my - 1)];
    __syncthreads();
    for (int w = tid; w < nxl + nyl; w += NT) {
      const bool isx = w < nxl;
      const int i = isx ? w : w - nxl;
      const int ng = (isx ? nox : noy) + i;
      const int la = isx ? lxa : lya, lb = isx ? lxb : lyb;
      int lo = lb + 1, hi = -1;
      for (int l = la; l <= lb; ++l) {
        const int n0 = isx ? sCx[l].n0 : sCy[l].n0;
        if (n0 == ng || n0 + 1 == ng) {
          lo = min(lo, l);
          hi = max(hi, l);
        }
      }
      if (isx) {
        sColLo[i] = lo;
        sColHi[i] = hi;
      } else {
        sRowLo[i] = lo;
        sRowHi[i] = hi;
      }
    }
  }

  // the group's partial slot: node n of component d at part[d nbar + n], n the
  // node's index in the grid, so the node pass reads its slots coalesced
  const int pslot = ((chunk % P.smz) * P.smy + tile_y % P.smy) * P.smx + tile_x % P.smx;
  float* const part = P.part + (size_t)pslot * 3 * (size_t)P.nbar;

  // Writes one node plane (local index kloc) of the transposed conversion:
  // reduce the per-column sums acc over x, then y, into the slot's node block.
  const int nrow = lyb - lya + 1;
  auto flush = [&](const float (&acc)[3], int kloc) {
    if constexpr (NEED_C) {   // (only the derivative modes gather)
      if (inC) {
        sV[0][tid] = acc[0];
        sV[1][tid] = acc[1];
        sV[2][tid] = acc[2];
      }
      __syncthreads();
      for (int w = tid; w < nxl * nrow; w += NT) {   // x reduction: node column fj, local row ly
        const int fj = w % nxl, ly = lya + w / nxl;
        const int jg = nox + fj;
        float s0 = 0.f, s1 = 0.f, s2 = 0.f;
        for (int l = sColLo[fj]; l <= sColHi[fj]; ++l) {
          const Conv1 c = sCx[l];
          const float wt = (c.n0 == jg) ? 1.0f - c.f : c.f;
          const int q = ly * BX + l;
          s0 = fmaf(wt, sV[0][q], s0);
          s1 = fmaf(wt, sV[1][q], s1);
          s2 = fmaf(wt, sV[2][q], s2);
        }
        sW[0][ly * MAXNX + fj] = s0;
        sW[1][ly * MAXNX + fj] = s1;
        sW[2][ly * MAXNX + fj] = s2;
      }
      __syncthreads();
      for (int w = tid; w < nxl * nyl; w += NT) {   // y reduction: node (fj, fr)
        const int fj = w % nxl, fr = w / nxl;
        const int ig = noy + fr;
        float s0 = 0.f, s1 = 0.f, s2 = 0.f;
        for (int l = sRowLo[fr]; l <= sRowHi[fr]; ++l) {
          const Conv1 c = sCy[l];
          const float wt = (c.n0 == ig) ? 1.0f - c.f : c.f;
          const int q = l * MAXNX + fj;
          s0 = fmaf(wt, sW[0][q], s0);
          s1 = fmaf(wt, sW[1][q], s1);
          s2 = fmaf(wt, sW[2][q], s2);
        }
        const size_t o = ((size_t)(noz + kloc) * P.ny + (noy + fr)) * P.nx + (nox + fj);
        part[o] = s0;
        part[o + (size_t)P.nbar] = s1;
        part[o + 2 * (size_t)P.nbar] = s2;
      }
      __syncthreads();
    }
  };

  // Register windows of the own column; slot (t - tfirst) mod 3.
  float Tw[3] = {0.f, 0.f, 0.f}, Rv[3] = {0.f, 0.f, 0.f}, av[3] = {0.f, 0.f, 0.f};
  float g[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  float e0[3] = {0.f, 0.f, 0.f}, ezp[3] = {0.f, 0.f, 0.f};
  float acc_lo[3] = {0.f, 0.f, 0.f}, acc_hi[3] = {0.f, 0.f, 0.f};
  int KL = noz;
  double obj = 0.0;

  // xy-interpolated u and p at the two node planes bracketing the current plane,
  // and their differences (the z interpolation of every plane in between is one FMA)
  int Kp = -0x7fffffff;
  float ulo[3] = {0.f, 0.f, 0.f}, uhi[3] = {0.f, 0.f, 0.f}, udz[3] = {0.f, 0.f, 0.f};
  float plo[3] = {0.f, 0.f, 0.f}, phi[3] = {0.f, 0.f, 0.f}, pdz[3] = {0.f, 0.f, 0.f};
  // template and reference through buffer descriptors: the corner loads share one
  // vector offset, the reference load needs only the plane's scalar offset
  const __amdgpu_buffer_rsrc_t rsT = raw_buffer(P.Tp, P.Tbytes), rsR = raw_buffer(P.R, P.Rbytes);
  const CornerOffsets co{4u * (unsigned)P.PX, 4u * (unsigned)P.PXY, 4u * (unsigned)(P.PX + P.PXY)};
  const unsigned rcol = colxy << 2;
  auto xy_interp = [&](const float* __restrict__ f, int k, float (&o)[3]) {
    const unsigned i00 = (unsigned)k * nxy + nodexy;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const unsigned b = (unsigned)d * nb + i00;
      const float lo = fmaf(wx1, ld32(f, b + 1), wx0 * ld32(f, b));
      const float hi = fmaf(wx1, ld32(f, b + nxu + 1), wx0 * ld32(f, b + nxu));
      o[d] = fmaf(wy1, hi, wy0 * lo);
    }
  };

  // Stage A inputs of the next plane, loaded one step ahead.
  float nx_t[8];
  float nx_fx = 0.f, nx_fy = 0.f, nx_fz = 0.f, nx_R = 0.f;
  float nx_pp[3] = {0.f, 0.f, 0.f};
  auto issue = [&](int tt) {
    const int tc = min(max(tt, 0), P.mz - 1);
    const int jz = tt - zb + 2;   // LDS slot of plane tt (entries are clamped into the image)
    Conv1 cvz = sCz[jz];
    cvz.n0 = __builtin_amdgcn_readfirstlane(cvz.n0);   // uniform: keeps the plane logic scalar
    cvz.f = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, cvz.f)));
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
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        udz[d] = uhi[d] - ulo[d];
        if (HV) pdz[d] = phi[d] - plo[d];
      }
      Kp = cvz.n0;
    }
    const float fz = cvz.f;
    const int kx = template_cell(spx, fmaf(fz, udz[0], ulo[0]), P.ihTx, nx_fx);
    const int ky = template_cell(spy, fmaf(fz, udz[1], ulo[1]), P.ihTy, nx_fy);
    const int kz = template_cell(sSz[jz], fmaf(fz, udz[2], ulo[2]), P.ihTz, nx_fz);
    template_corners_buf(P, rsT, co, kx, ky, kz, nx_t);
    nx_R = buf_ld(rsR, rcol, (unsigned)tc * plane * 4u);
    if (HV) {
#pragma unroll
      for (int d = 0; d < 3; ++d) nx_pp[d] = fmaf(fz, pdz[d], plo[d]);
    }
  };

  const int tfirst = zb - 2, tlast = ze + 1;

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
      if (HV) av[K] = fmaf(s.gx, nx_pp[0], fmaf(s.gy, nx_pp[1], s.gz * nx_pp[2]));
      if constexpr (!SSD) {
        const int sl = t & 1;
        sTw[sl][XP + tid] = Tw[K];
        sR[sl][XP + tid] = Rv[K];
        if (HV) sA[sl][XP + tid] = av[K];
      }
    }
    if (t < tlast) issue(t + 1);
    // No barrier here: stage B reads only LDS slots of plane t-1 (written in the
    // previous step) and the slots written above were last read before the
    // barrier that ends the previous step.

    // ---------------- stage B: plane zc = t-1 ----------------
    const int zc = t - 1;
    float ezm = 0.f;
    e0[K1] = 0.f;
    ezp[K1] = 0.f;
    const bool zin = zc >= zb - 1 && zc <= ze && zc >= 0 && zc < P.mz;   // uniform
    if (SSD && zin) {
      if (inB) {
        const float r = Tw[K1] - Rv[K1];
        if (MODE != MODE_HV && zc >= zb && zc < ze) {
          const double rd = r;
          obj += 0.5 * rd * rd;
        }
        if constexpr (NEED_C) e0[K1] = HV ? av[K1] : r;
      }
    } else if (!SSD && zin) {
      // Every lane evaluates the row (ring columns and columns outside the image
      // read finite neighbours: clamped samples or the zero pads), and a lane
      // that does not own its row scales z by 0, which zeroes all its products:
      // no divergent branch and no per-step clearing of the products.
      const int s1 = zc & 1;
      const int q = XP + tid;
      const float Tc = Tw[K1], Rc = Rv[K1];
      const float dTxm = sTw[s1][q - 1] - Tc, dTxp = sTw[s1][q + 1] - Tc;
      const float dTym = sTw[s1][q - BX] - Tc, dTyp = sTw[s1][q + BX] - Tc;
      const float dTzm = Tw[K2] - Tc, dTzp = Tw[K] - Tc;
      const float dRxm = sR[s1][q - 1] - Rc, dRxp = sR[s1][q + 1] - Rc;
      const float dRym = sR[s1][q - BX] - Rc, dRyp = sR[s1][q + BX] - Rc;
      const float dRzm = Rv[K2] - Rc, dRzp = Rv[K] - Rc;
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
      const float rnT = rsq_norm(nT2), rnR = rsq_norm(nR2);
      const float c1 = rnT * rnR;
      const float r = r1 * c1;
      // 1 - r^2 from the float32 sums in float64: in float32 it cancels where r is
      // close to 1 (aligned images), and the bias of the hardware reciprocal
      // square root would add up over the voxels of the objective sum
      if (MODE != MODE_HV && inB && zc >= zb && zc < ze)
        obj += 1.0 - ((double)r1 * (double)r1) / ((double)nT2 * (double)nR2);
      if constexpr (NEED_C) {
        const float c2 = r1 * rnT * rnT;
        const float kx = P.hhx * c1, ky = P.hhy * c1, kz = P.hhz * c1;
        const float rxm = kx * fmaf(-c2, dTxm, dRxm), rxp = kx * fmaf(-c2, dTxp, dRxp);
        const float rym = ky * fmaf(-c2, dTym, dRym), ryp = ky * fmaf(-c2, dTyp, dRyp);
        const float rzm = kz * fmaf(-c2, dTzm, dRzm), rzp = kz * fmaf(-c2, dTzp, dRzp);
        const float r0 = -(((rxm + rxp) + (rym + ryp)) + (rzm + rzp));
        float zl;
        if constexpr (HV) {
          zl = r0 * av[K1];
          zl = fmaf(rxm, sA[s1][q - 1], zl);
          zl = fmaf(rxp, sA[s1][q + 1], zl);
          zl = fmaf(rym, sA[s1][q - BX], zl);
          zl = fmaf(ryp, sA[s1][q + BX], zl);
          zl = fmaf(rzm, av[K2], zl);
          zl = fmaf(rzp, av[K], zl);
        } else {
          zl = r;
        }
        zl *= own_row;
        sE[s1][0][EP + tid] = rxp * zl;
        sE[s1][1][EP + tid] = rxm * zl;
        sE[s1][2][EP + tid] = ryp * zl;
        sE[s1][3][EP + tid] = rym * zl;
        ezp[K1] = rzp * zl;
        ezm = rzm * zl;
        e0[K1] = r0 * zl;
      }
    }

    // ---------------- stage C: plane c = t-2 ----------------
    if constexpr (NEED_C) {
      const int c = t - 2;
      if (c >= zb && c < ze) {
        Conv1 cvz = sCz[c - zb + 2];
        cvz.n0 = __builtin_amdgcn_readfirstlane(cvz.n0);
        cvz.f = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, cvz.f)));
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
          float w = e0[K2];
          if constexpr (!SSD) {
            // rows of the neighbours within the group (beyond its edge: the zero pad,
            // or a ring column of the next row, which holds 0)
            const int s2 = c & 1;
            w += sE[s2][1][EP + tid + 1];
            w += sE[s2][0][EP + tid - 1];
            w += sE[s2][3][EP + tid + BX];
            w += sE[s2][2][EP + tid - BX];
            w += ezm;
            w += ezp[K];
          }
          const float wz1 = cvz.f, wz0 = 1.0f - cvz.f;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const float v = g[K2][d] * w;
            acc_lo[d] = fmaf(wz0, v, acc_lo[d]);
            acc_hi[d] = fmaf(wz1, v, acc_hi[d]);
          }
        }
      }
    }
    // SSD exchanges nothing between columns within a step (flush has its own barriers)
    if constexpr (!SSD) __syncthreads();
  };

  issue(tfirst);
  for (int t = tfirst; t <= tlast; t += 3) {
    step(std::integral_constant<int, 0>{}, t);
    if (t + 1 <= tlast) step(std::integral_constant<int, 1>{}, t + 1);
    if (t + 2 <= tlast) step(std::integral_constant<int, 2>{}, t + 2);
  }

  if constexpr (NEED_C) {
    flush(acc_lo, KL - noz);
    flush(acc_hi, KL + 1 - noz);
  }
  if constexpr (MODE != MODE_HV) block_sum_store<NT>(obj, P.red + bid, sRed);
  __syncthreads();   // LDS may be reused by the next tile of a persistent group
}

template <int BX, int BY, int MODE, bool SSD>
__global__ __launch_bounds__(BX* BY) void ngf_tile_kernel(const TileParams P, const float* __restrict__ u,
                                                          const float* __restrict__ pv) {
  if (P.live && !ld_coherent(P.live)) return;   // a device-steered solve has stopped
  __shared__ TileSmem<BX, BY, MODE, SSD> S;
  tile_body<BX, BY, MODE, SSD>(P, xcd_block_id(), u, pv, S);
}

// Persistent form over a batch of problems: every group takes tiles from a
// shared work counter until all tiles of all active problems are done.  A
// tile's results depend only on its problem and tile id, so the output equals
// one launch per problem bit for bit.  At most 128 VGPRs (four waves per SIMD):
// two groups of 512 threads per CU, as for the single-problem kernel.
template <int BX, int BY, int MODE>
__global__ __launch_bounds__(BX* BY) __attribute__((amdgpu_waves_per_eu(4))) void ngf_tile_batch_kernel(const BatchJobs J) {
  __shared__ TileSmem<BX, BY, MODE, false> S;
  __shared__ int sItem;
  for (;;) {
    if (threadIdx.x == 0) sItem = atomicAdd(J.counter, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(sItem);   // uniform across the group
    __syncthreads();
    if (item >= J.total) break;
    int pr = 0;
    while (pr + 1 < J.n && J.prefix[pr + 1] <= item) ++pr;
    if (J.active && !ld_coherent(J.active + pr)) continue;
    const BatchJob& jb = J.jobs[pr];
    tile_body<BX, BY, MODE, false>(jb.t, item - J.prefix[pr], jb.u, jb.p, S);
  }
}

template <int BX, int BY, bool SSD>
static void launch_tile_dist(int mode, const TileParams& p, const float* u, const float* pv, int grid,
                             hipStream_t st) {
  dim3 blk(BX * BY), grd(grid);
  switch (mode) {
    case MODE_OBJ:
      hipLaunchKernelGGL((ngf_tile_kernel<BX, BY, MODE_OBJ, SSD>), grd, blk, 0, st, p, u, pv);
      break;
    case MODE_GRAD:
      hipLaunchKernelGGL((ngf_tile_kernel<BX, BY, MODE_GRAD, SSD>), grd, blk, 0, st, p, u, pv);
      break;
    default:
      hipLaunchKernelGGL((ngf_tile_kernel<BX, BY, MODE_HV, SSD>), grd, blk, 0, st, p, u, pv);
      break;
  }
}

template <int BX, int BY>
static hipError_t launch_tile_shape(int mode, const TileParams& p, const float* u, const float* pv,
                                    int grid, hipStream_t st) {
  if (p.ssd)
    launch_tile_dist<BX, BY, true>(mode, p, u, pv, grid, st);
  else
    launch_tile_dist<BX, BY, false>(mode, p, u, pv, grid, st);
  return hipGetLastError();
}

static int resident_groups(const void* kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
    return 0;
  return cus * per_cu;
}

template <int BX, int BY>
static hipError_t launch_tile_batch_shape(int mode, const BatchJobs& j, int groups, hipStream_t st) {
  if (groups <= 0) {
    // resident capacity of each mode, queried once per process (one device)
    static int cap[3] = {-1, -1, -1};
    const int mi = mode == MODE_OBJ ? 0 : mode == MODE_GRAD ? 1 : 2;
    if (cap[mi] < 0) {
      const void* k = mi == 0   ? reinterpret_cast<const void*>(ngf_tile_batch_kernel<BX, BY, MODE_OBJ>)
                      : mi == 1 ? reinterpret_cast<const void*>(ngf_tile_batch_kernel<BX, BY, MODE_GRAD>)
                                : reinterpret_cast<const void*>(ngf_tile_batch_kernel<BX, BY, MODE_HV>);
      cap[mi] = resident_groups(k, BX * BY);
    }
    groups = cap[mi] > 0 ? cap[mi] : 512;
  }
  groups = groups < j.total ? groups : j.total;
  if (groups <= 0) return hipSuccess;
  dim3 blk(BX * BY), grd(groups);
  switch (mode) {
    case MODE_OBJ:
      hipLaunchKernelGGL((ngf_tile_batch_kernel<BX, BY, MODE_OBJ>), grd, blk, 0, st, j);
      break;
    case MODE_GRAD:
      hipLaunchKernelGGL((ngf_tile_batch_kernel<BX, BY, MODE_GRAD>), grd, blk, 0, st, j);
      break;
    default:
      hipLaunchKernelGGL((ngf_tile_batch_kernel<BX, BY, MODE_HV>), grd, blk, 0, st, j);
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

hipError_t launch_tile_batch(const TileShape& s, int mode, const BatchJobs& j, int groups, hipStream_t st) {
  if (s.bx == 32 && s.by == 16) return launch_tile_batch_shape<32, 16>(mode, j, groups, st);
  if (s.bx == 64 && s.by == 8) return launch_tile_batch_shape<64, 8>(mode, j, groups, st);
  if (s.bx == 32 && s.by == 32) return launch_tile_batch_shape<32, 32>(mode, j, groups, st);
  if (s.bx == 64 && s.by == 16) return launch_tile_batch_shape<64, 16>(mode, j, groups, st);
  return hipErrorInvalidValue;
}

}  // namespace mfr
