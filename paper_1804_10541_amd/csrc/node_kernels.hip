// Node-grid kernels: the gather that completes the transposed grid conversion
// (Sec. 4.3), the curvature stencils (Sec. 3.1 eq. curvatureMF, Sec. 4.2
// eq. curv_hessMult), fixed-order float64 reductions, the zero-bordered
// template copy, the exact Jacobi diagonal, and image / displacement
// pyramid transfers.
#include <algorithm>

#include "mfr_internal.h"

namespace mfr {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum in a fixed order (lane tree, then waves in index order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sred) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sred[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += sred[w];
  }
  return s;
}

// 7-point Laplacian with clamped (Neumann) neighbours at node (i, j, k)
// (eq. laplace_discretized).
__device__ __forceinline__ float lap7(const float* __restrict__ f, int i, int j, int k, int nx, int ny,
                                      int nz, float ix2, float iy2, float iz2) {
  const int nxy = nx * ny;
  const int c = i + nx * j + nxy * k;
  const float f0 = f[c];
  const float fxm = f[c - (i > 0)], fxp = f[c + (i < nx - 1)];
  const float fym = f[c - nx * (j > 0)], fyp = f[c + nx * (j < ny - 1)];
  const float fzm = f[c - nxy * (k > 0)], fzp = f[c + nxy * (k < nz - 1)];
  const float m2 = -2.0f * f0;
  return fmaf(fxm + fxp + m2, ix2, fmaf(fym + fyp + m2, iy2, (fzm + fzp + m2) * iz2));
}

// Squared forward differences at node (i, j, k), sum_k ((f_{n+e_k} - f_n)/hy_k)^2
// (none past the last node: the clamped neighbour gives 0).  The diffusive
// regulariser's value is the sum of these over the nodes; summing f . (-L f)
// instead would cancel large terms whenever f has a large mean.
__device__ __forceinline__ float fwd_sq(const float* __restrict__ f, int i, int j, int k, int nx, int ny, int nz,
                                        float ix2, float iy2, float iz2) {
  const int nxy = nx * ny;
  const int c = i + nx * j + nxy * k;
  const float f0 = f[c];
  const float dx = f[c + (i < nx - 1)] - f0, dy = f[c + nx * (j < ny - 1)] - f0, dz = f[c + nxy * (k < nz - 1)] - f0;
  return fmaf(dx * dx, ix2, fmaf(dy * dy, iy2, dz * dz * iz2));
}

// Divergence of f at cell (a, b, c) of the nodal grid (cells: one fewer per
// axis than nodes): sum over d of the mean of the cell's four edge differences
// of f_d along d, divided by hy_d (ih4 = 1 / (4 hy)).
__device__ __forceinline__ float cell_div(const float* __restrict__ f, int nbar, int a, int b, int c, int nx, int ny,
                                          float ih4x, float ih4y, float ih4z) {
  const int nxy = nx * ny;
  const int n0 = a + nx * b + nxy * c;
  const float* fx = f;
  const float* fy = f + nbar;
  const float* fz = f + 2 * (size_t)nbar;
  float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    const int p = o & 1, q = o >> 1;
    const int ex = n0 + nx * p + nxy * q;   // edge along x at (y + p, z + q)
    const int ey = n0 + p + nxy * q;        // edge along y at (x + p, z + q)
    const int ez = n0 + p + nx * q;         // edge along z at (x + p, y + q)
    sx += fx[ex + 1] - fx[ex];
    sy += fy[ey + nx] - fy[ey];
    sz += fz[ez + nxy] - fz[ez];
  }
  return fmaf(sx, ih4x, fmaf(sy, ih4y, sz * ih4z));
}

}  // namespace

// The curvature part runs in two passes over the nodes: the first stores the
// 7-point Laplacian L f_d of every node (eq. laplace_discretized) in Q.lap and,
// for the regulariser value, sums (L f_d)^2; the second reads the Laplacians of
// the node and its six neighbours (clamped, so a missing neighbour contributes
// its own value) for L L f_d and adds the gathered tile partials.  Each
// Laplacian is evaluated once instead of seven times; the floats are the same
// as evaluating them in place.
template <int MODE>
__device__ __forceinline__ void lap_body(const NodeParams& Q, const float* __restrict__ f, const int blk,
                                         double* sred) {
  const int n = blk * kNodeBlock + threadIdx.x;
  double local = 0.0;
  if (n < Q.nbar) {
    const int i = n % Q.nx;
    const int j = (n / Q.nx) % Q.ny;
    const int k = n / (Q.nx * Q.ny);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d >= Q.nc) break;
      const float L0 = lap7(f + (size_t)d * Q.nbar, i, j, k, Q.nx, Q.ny, Q.nz, Q.ihy2x, Q.ihy2y, Q.ihy2z);
      Q.lap[(size_t)d * Q.nbar + n] = L0;
      // curvature: sum (L f)^2; diffusive and elastic: the squared edge differences
      if (MODE == NP_S)
        local += Q.reg ? (double)fwd_sq(f + (size_t)d * Q.nbar, i, j, k, Q.nx, Q.ny, Q.nz, Q.ihy2x, Q.ihy2y, Q.ihy2z)
                       : (double)L0 * (double)L0;
    }
  }
  if (Q.reg == 2) {   // elastic: divergence of the cell with linear index n, kept for the second pass
    const int cx = Q.nx - 1, cy = Q.ny - 1, cz = Q.nz - 1;
    if (n < cx * cy * cz) {
      const int a = n % cx, b = (n / cx) % cy, c = n / (cx * cy);
      const float dv = cell_div(f, Q.nbar, a, b, c, Q.nx, Q.ny, 0.25f * sqrtf(Q.ihy2x), 0.25f * sqrtf(Q.ihy2y),
                                0.25f * sqrtf(Q.ihy2z));
      Q.div[n] = dv;
      if (MODE == NP_S) local += (double)Q.kappa * (double)dv * (double)dv;
    }
  }
  if (MODE == NP_S) {
    const double s = block_sum<kNodeBlock>(local, sred);
    if (threadIdx.x == 0) Q.red[blk] = s;
  }
}

// One thread per node, all its components d: q_d = s_ngf * (sum of the tile
// partials of component d) + s_curv * (L L f_d).  The node's indices and the
// walk over the tile slots that overlap it are formed once for all components.
// Partials: red[blk] (the components summed in order within the thread).
template <int MODE>
__device__ __forceinline__ void node_pass_body(const NodeParams& Q, const float* __restrict__ f,
                                               float* __restrict__ out, const int blk, double* sred) {
  const int n = blk * kNodeBlock + threadIdx.x;
  double local = 0.0;
  if (n < Q.nbar) {
    const int i = n % Q.nx;
    const int j = (n / Q.nx) % Q.ny;
    const int k = n / (Q.nx * Q.ny);
    const int nxy = Q.nx * Q.ny;
    const size_t nb3 = (size_t)Q.nbar;
    // gather of the transposed conversion: every tile slot overlapping node n
    // (the groups overlapping a node have distinct slots: at most smx of them
    // along x, and so on)
    const Range1 rx = Q.ntx[i], ry = Q.nty[j], rz = Q.ntz[k];
    // slot indices c % sm advance with c (one remainder per axis)
    float sg[3] = {0.0f, 0.0f, 0.0f};
    const int sx0 = rx.lo % Q.smx, sy0 = ry.lo % Q.smy;
    for (int cz = rz.lo, sz = rz.lo % Q.smz; cz <= rz.hi; ++cz, sz = sz + 1 == Q.smz ? 0 : sz + 1) {
      for (int cy = ry.lo, sy = sy0; cy <= ry.hi; ++cy, sy = sy + 1 == Q.smy ? 0 : sy + 1) {
        const size_t pzy = (size_t)sz * Q.smy + sy;
        for (int cx = rx.lo, sx = sx0; cx <= rx.hi; ++cx, sx = sx + 1 == Q.smx ? 0 : sx + 1) {
          const float* pp = Q.part + (pzy * Q.smx + sx) * 3 * nb3 + n;
#pragma unroll
          for (int d = 0; d < 3; ++d)
            if (d < Q.nc) sg[d] += pp[d * nb3];
        }
      }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d >= Q.nc) break;
      const float* fd = f + (size_t)d * nb3;
      const float* Ld = Q.lap + (size_t)d * nb3;
      const float L0 = Ld[n];
      const float Lxm = i > 0 ? Ld[n - 1] : L0;
      const float Lxp = i < Q.nx - 1 ? Ld[n + 1] : L0;
      const float Lym = j > 0 ? Ld[n - Q.nx] : L0;
      const float Lyp = j < Q.ny - 1 ? Ld[n + Q.nx] : L0;
      const float Lzm = k > 0 ? Ld[n - nxy] : L0;
      const float Lzp = k < Q.nz - 1 ? Ld[n + nxy] : L0;
      const float m2 = -2.0f * L0;
      // curvature: L L f; diffusive: -L f (its Hessian is -hbar^y L); elastic: -L f + kappa (B^T B f)_d
      float LL = Q.reg ? -L0 : fmaf(Lxm + Lxp + m2, Q.ihy2x, fmaf(Lym + Lyp + m2, Q.ihy2y, (Lzm + Lzp + m2) * Q.ihy2z));
      if (Q.reg == 2) {
        const int cx = Q.nx - 1, cy = Q.ny - 1;
        const int nd = d == 0 ? i : d == 1 ? j : k;
        const float ih4 = 0.25f * sqrtf(d == 0 ? Q.ihy2x : d == 1 ? Q.ihy2y : Q.ihy2z);
        float bt = 0.f;
        for (int c = max(k - 1, 0); c <= min(k, Q.nz - 2); ++c)
          for (int b = max(j - 1, 0); b <= min(j, Q.ny - 2); ++b)
            for (int a = max(i - 1, 0); a <= min(i, Q.nx - 2); ++a) {
              const int cd = d == 0 ? a : d == 1 ? b : c;
              const float dv = Q.div[a + cx * (b + cy * c)];
              bt += cd == nd - 1 ? dv : -dv;   // the node is the upper (+) or lower (-) corner along d
            }
        LL = fmaf(Q.kappa * ih4, bt, LL);
      }
      const float q = fmaf(Q.s_ngf, sg[d], Q.s_curv * LL);
      out[(size_t)d * nb3 + n] = q;
      if (MODE == NP_GRAD) {
        local += Q.reg ? (double)fwd_sq(fd, i, j, k, Q.nx, Q.ny, Q.nz, Q.ihy2x, Q.ihy2y, Q.ihy2z)
                       : (double)L0 * (double)L0;
        if (Q.reg == 2 && d == 0 && n < (Q.nx - 1) * (Q.ny - 1) * (Q.nz - 1))
          local += (double)Q.kappa * (double)Q.div[n] * (double)Q.div[n];   // once per cell (component row 0)
      }
      if (MODE == NP_HV) local += (double)fd[n] * (double)q;
    }
  }
  const double s = block_sum<kNodeBlock>(local, sred);
  if (threadIdx.x == 0) Q.red[blk] = s;
}

template <int MODE>
__global__ __launch_bounds__(kNodeBlock) void lap_kernel(const NodeParams Q, const float* __restrict__ f) {
  if (Q.live && !ld_coherent(Q.live)) return;   // a device-steered solve has stopped
  __shared__ double sred[kNodeBlock / 64];
  lap_body<MODE>(Q, f, blockIdx.x, sred);
}

template <int MODE>
__global__ __launch_bounds__(kNodeBlock) void lap_batch_kernel(const NodeJobs J) {
  __shared__ double sred[kNodeBlock / 64];
  int pr = 0;
  while (pr + 1 < J.n && J.prefix[pr + 1] <= (int)blockIdx.x) ++pr;
  if (J.active && !ld_coherent(J.active + pr)) return;
  const NodeJob& jb = J.jobs[pr];
  lap_body<MODE>(jb.q, jb.f, blockIdx.x - J.prefix[pr], sred);
}

template <int MODE>
__global__ __launch_bounds__(kNodeBlock) void node_pass_kernel(const NodeParams Q,
                                                               const float* __restrict__ f,
                                                               float* __restrict__ out) {
  if (Q.live && !ld_coherent(Q.live)) return;   // a device-steered solve has stopped
  __shared__ double sred[kNodeBlock / 64];
  node_pass_body<MODE>(Q, f, out, blockIdx.x, sred);
}

// The same per-node arithmetic for a table of problems (batched path).
template <int MODE>
__global__ __launch_bounds__(kNodeBlock) void node_pass_batch_kernel(const NodeJobs J) {
  __shared__ double sred[kNodeBlock / 64];
  int pr = 0;
  while (pr + 1 < J.n && J.prefix[pr + 1] <= (int)blockIdx.x) ++pr;
  if (J.active && !ld_coherent(J.active + pr)) return;
  const NodeJob& jb = J.jobs[pr];
  node_pass_body<MODE>(jb.q, jb.f, jb.out, blockIdx.x - J.prefix[pr], sred);
}

hipError_t launch_node_pass_batch(int mode, const NodeJobs& j, hipStream_t st) {
  const int blocks = j.prefix[j.n];
  if (mode == NP_S) {
    hipLaunchKernelGGL(lap_batch_kernel<NP_S>, dim3(blocks), dim3(kNodeBlock), 0, st, j);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(lap_batch_kernel<NP_HV>, dim3(blocks), dim3(kNodeBlock), 0, st, j);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == NP_GRAD)
    hipLaunchKernelGGL(node_pass_batch_kernel<NP_GRAD>, dim3(blocks), dim3(kNodeBlock), 0, st, j);
  else
    hipLaunchKernelGGL(node_pass_batch_kernel<NP_HV>, dim3(blocks), dim3(kNodeBlock), 0, st, j);
  return hipGetLastError();
}


hipError_t launch_node_pass(int mode, const NodeParams& q, const float* f, float* out, int blocks,
                            hipStream_t st) {
  if (mode == NP_S) {
    hipLaunchKernelGGL(lap_kernel<NP_S>, dim3(blocks), dim3(kNodeBlock), 0, st, q, f);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(lap_kernel<NP_HV>, dim3(blocks), dim3(kNodeBlock), 0, st, q, f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (mode == NP_GRAD)
    hipLaunchKernelGGL(node_pass_kernel<NP_GRAD>, dim3(blocks), dim3(kNodeBlock), 0, st, q, f, out);
  else
    hipLaunchKernelGGL(node_pass_kernel<NP_HV>, dim3(blocks), dim3(kNodeBlock), 0, st, q, f, out);
  return hipGetLastError();
}

// Fixed-order sum of n float64 partials by one work-group.
__global__ __launch_bounds__(256) void sum_kernel(const double* __restrict__ parts, int n,
                                                  double* __restrict__ out) {
  __shared__ double sred[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += parts[i];
  s = block_sum<256>(s, sred);
  if (threadIdx.x == 0) *out = s;
}

hipError_t launch_sum(const double* parts, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, parts, n, out);
  return hipGetLastError();
}

// Objective scalars into caller memory (the graph-capturable entry points):
// D = dmul sums[0], S = (smul sums[1]) sk, J = D + alpha S; out = {J, D, S} (count
// 3) or {J} (count 1).  Separate roundings, as the host evaluates them.
__global__ void objective_out_kernel(const double* __restrict__ sums, double dmul, double smul, double sk,
                                     double alpha, double* __restrict__ out, int count) {
  if (threadIdx.x != 0) return;
  const double D = __dmul_rn(dmul, sums[0]), S = __dmul_rn(__dmul_rn(smul, sums[1]), sk);
  out[0] = __dadd_rn(D, __dmul_rn(alpha, S));
  if (count == 3) {
    out[1] = D;
    out[2] = S;
  }
}

hipError_t launch_objective_out(const double* sums, double dmul, double smul, double sk, double alpha, double* out,
                                int count, hipStream_t st) {
  hipLaunchKernelGGL(objective_out_kernel, dim3(1), dim3(64), 0, st, sums, dmul, smul, sk, alpha, out, count);
  return hipGetLastError();
}

// Copy T into an (mx + 4) x (my + 4) x (mz + 2 bz) array with a two-cell zero
// border in x and y and bz cells in z.
__global__ void pad_template_kernel(const float* __restrict__ T, float* __restrict__ Tp, int mx, int my,
                                    int mz, int bz) {
  const int PX = mx + 4, PY = my + 4, PZ = mz + 2 * bz;
  const size_t total = (size_t)PX * PY * PZ;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(idx % PX) - 2;
    const int y = (int)((idx / PX) % PY) - 2;
    const int z = (int)(idx / ((size_t)PX * PY)) - bz;
    float v = 0.0f;
    if (x >= 0 && x < mx && y >= 0 && y < my && z >= 0 && z < mz) v = T[((size_t)z * my + y) * mx + x];
    Tp[idx] = v;
  }
}

hipError_t launch_pad_template(const float* T, float* Tp, int mx, int my, int mz, int bz, hipStream_t st) {
  const size_t total = (size_t)(mx + 4) * (my + 4) * (mz + 2 * bz);
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(pad_template_kernel, dim3(blocks), dim3(256), 0, st, T, Tp, mx, my, mz, bz);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact Jacobi diagonal: diag_{(d,n)} = 2 hbar sum_l (sum_k drow_l(k) g_{l+k,d}
// W_n(l+k))^2 + 2 alpha hbar^y (L^T L)_{nn}; one thread per node, rows l of
// dr whose 7-point stencil meets the node's support, everything recomputed.
// SSD: drow_l is the unit row at l and the scale is hbar.
// ---------------------------------------------------------------------------
namespace {

struct VoxelEval {
  float T, g[3];
};

__device__ __forceinline__ VoxelEval eval_voxel(const TileParams& P, const float* __restrict__ u, int x,
                                                int y, int z) {
  const Conv1 cx = P.cx[x], cy = P.cy[y], cz = P.cz[z];
  const int nxy = P.nx * P.ny;
  float dsp[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float* b = u + (size_t)d * P.nbar + cz.n0 * nxy + cy.n0 * P.nx + cx.n0;
    const float l00 = fmaf(cx.f, b[1] - b[0], b[0]);
    const float l10 = fmaf(cx.f, b[P.nx + 1] - b[P.nx], b[P.nx]);
    const float l01 = fmaf(cx.f, b[nxy + 1] - b[nxy], b[nxy]);
    const float l11 = fmaf(cx.f, b[nxy + P.nx + 1] - b[nxy + P.nx], b[nxy + P.nx]);
    const float m0 = fmaf(cy.f, l10 - l00, l00), m1 = fmaf(cy.f, l11 - l01, l01);
    dsp[d] = fmaf(cz.f, m1 - m0, m0);
  }
  const Samp1 sx = P.sx[x], sy = P.sy[y], sz = P.sz[z];
  const float qx = fminf(fmaxf(fmaf(dsp[0], P.ihTx, sx.frac), -1.0e7f), 1.0e7f);
  const float qy = fminf(fmaxf(fmaf(dsp[1], P.ihTy, sy.frac), -1.0e7f), 1.0e7f);
  const float qz = fminf(fmaxf(fmaf(dsp[2], P.ihTz, sz.frac), -1.0e7f), 1.0e7f);
  const float flx = floorf(qx), fly = floorf(qy), flz = floorf(qz);
  int kx = min(max(sx.base + (int)flx, -2), P.mTx);
  int ky = min(max(sy.base + (int)fly, -2), P.mTy);
  int kz = min(max(sz.base + (int)flz, -2), P.mTz);
  const float fx = qx - flx, fy = qy - fly, fz = qz - flz;
  const float* b0 = P.Tp + (size_t)(kz + 2) * (size_t)P.PXY + (size_t)((ky + 2) * P.PX + (kx + 2));
  const float* b1 = b0 + P.PXY;
  const float t000 = b0[0], t100 = b0[1], t010 = b0[P.PX], t110 = b0[P.PX + 1];
  const float t001 = b1[0], t101 = b1[1], t011 = b1[P.PX], t111 = b1[P.PX + 1];
  const float d00 = t100 - t000, d10 = t110 - t010, d01 = t101 - t001, d11 = t111 - t011;
  const float e00 = fmaf(fx, d00, t000), e10 = fmaf(fx, d10, t010);
  const float e01 = fmaf(fx, d01, t001), e11 = fmaf(fx, d11, t011);
  const float dy0 = e10 - e00, dy1 = e11 - e01;
  const float f0 = fmaf(fy, dy0, e00), f1 = fmaf(fy, dy1, e01);
  const float dxa = fmaf(fy, d10 - d00, d00), dxb = fmaf(fy, d11 - d01, d01);
  VoxelEval o;
  o.T = fmaf(fz, f1 - f0, f0);
  o.g[2] = (f1 - f0) * P.ihTz;
  o.g[1] = fmaf(fz, dy1 - dy0, dy0) * P.ihTy;
  o.g[0] = fmaf(fz, dxb - dxa, dxa) * P.ihTx;
  return o;
}

// weight of node index n for voxel index a along one axis
__device__ __forceinline__ float w1(const Conv1 c, int n) {
  return (c.n0 == n) ? 1.0f - c.f : ((c.n0 + 1 == n) ? c.f : 0.0f);
}

}  // namespace

__global__ __launch_bounds__(kNodeBlock) void jacobi_diag_kernel(const DiagParams D,
                                                                 const float* __restrict__ u,
                                                                 float* __restrict__ diag) {
  const TileParams& P = D.t;
  const int n = blockIdx.x * kNodeBlock + threadIdx.x;
  if (n >= P.nbar) return;
  const int ni = n % P.nx, nj = (n / P.nx) % P.ny, nk = n / (P.nx * P.ny);
  const Range1 rx = D.rx[ni], ry = D.ry[nj], rz = D.rz[nk];
  const size_t plane = (size_t)P.mx * P.my;
  float acc[3] = {0.f, 0.f, 0.f};
  for (int z = rz.lo; z <= rz.hi; ++z) {
    for (int y = ry.lo; y <= ry.hi; ++y) {
      for (int x = rx.lo; x <= rx.hi; ++x) {
        // the seven stencil points of row l = (x, y, z); clamped ones carry no weight
        const int px[7] = {x, x - 1, x + 1, x, x, x, x};
        const int py[7] = {y, y, y, y - 1, y + 1, y, y};
        const int pz[7] = {z, z, z, z, z, z - 1, z + 1};
        bool ok[7];
        VoxelEval ev[7];
        float Rv[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) {
          ok[k] = px[k] >= 0 && px[k] < P.mx && py[k] >= 0 && py[k] < P.my && pz[k] >= 0 && pz[k] < P.mz;
          const int qx = ok[k] ? px[k] : x, qy = ok[k] ? py[k] : y, qz = ok[k] ? pz[k] : z;
          ev[k] = eval_voxel(P, u, qx, qy, qz);
          Rv[k] = P.R[(size_t)qz * plane + (size_t)qy * P.mx + qx];
        }
        float dT[7], dR[7];
#pragma unroll
        for (int k = 1; k < 7; ++k) {
          dT[k] = ev[k].T - ev[0].T;
          dR[k] = Rv[k] - Rv[0];
        }
        const float sTT = fmaf(fmaf(dT[1], dT[1], dT[2] * dT[2]), P.ih2x,
                               fmaf(fmaf(dT[3], dT[3], dT[4] * dT[4]), P.ih2y, fmaf(dT[5], dT[5], dT[6] * dT[6]) * P.ih2z));
        const float sRR = fmaf(fmaf(dR[1], dR[1], dR[2] * dR[2]), P.ih2x,
                               fmaf(fmaf(dR[3], dR[3], dR[4] * dR[4]), P.ih2y, fmaf(dR[5], dR[5], dR[6] * dR[6]) * P.ih2z));
        const float sTR = fmaf(fmaf(dT[1], dR[1], dT[2] * dR[2]), P.ih2x,
                               fmaf(fmaf(dT[3], dR[3], dT[4] * dR[4]), P.ih2y, fmaf(dT[5], dR[5], dT[6] * dR[6]) * P.ih2z));
        const float rnT = rsqrtf(fmaf(0.5f, sTT, P.tau2)), rnR = rsqrtf(fmaf(0.5f, sRR, P.rho2));
        const float r1 = fmaf(0.5f, sTR, P.taurho);
        const float c1 = rnT * rnR, c2 = r1 * rnT * rnT;
        const float hh[7] = {0.f, P.hhx, P.hhx, P.hhy, P.hhy, P.hhz, P.hhz};
        float rh[7];
        rh[0] = 0.f;
#pragma unroll
        for (int k = 1; k < 7; ++k) {
          rh[k] = hh[k] * c1 * fmaf(-c2, dT[k], dR[k]);
          rh[0] -= rh[k];
        }
        if (P.ssd) {   // sum of squared differences: dr/dT is the identity
          rh[0] = 1.0f;
#pragma unroll
          for (int k = 1; k < 7; ++k) rh[k] = 0.0f;
        }
        float zd[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < 7; ++k) {
          if (!ok[k]) continue;
          const float W = w1(P.cx[px[k]], ni) * w1(P.cy[py[k]], nj) * w1(P.cz[pz[k]], nk);
          const float c = rh[k] * W;
#pragma unroll
          for (int d = 0; d < 3; ++d) zd[d] = fmaf(c, ev[k].g[d], zd[d]);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[d] = fmaf(zd[d], zd[d], acc[d]);
      }
    }
  }
  // curvature part: (L^T L)_{nn} = (L_nn)^2 + sum over in-range neighbours 1/hy_k^4
  const int cxn = (ni > 0) + (ni < P.nx - 1), cyn = (nj > 0) + (nj < P.ny - 1), czn = (nk > 0) + (nk < P.nz - 1);
  const float Lnn = -(cxn * D.ihy2x + cyn * D.ihy2y + czn * D.ihy2z);
  // curvature: (L^T L)_nn; diffusive: -L_nn; elastic: -L_nn + kappa (B^T B)_nn, the latter
  // (adjacent cells) / (16 hy_d^2)
  const float LL = P.reg ? -Lnn : Lnn * Lnn + cxn * D.ihy2x * D.ihy2x + cyn * D.ihy2y * D.ihy2y + czn * D.ihy2z * D.ihy2z;
  const float ncell = P.reg == 2 ? P.kappa * (float)(cxn * cyn * czn) * 0.0625f : 0.0f;
  const float ih2[3] = {D.ihy2x, D.ihy2y, D.ihy2z};
#pragma unroll
  for (int d = 0; d < 3; ++d) diag[(size_t)d * P.nbar + n] = fmaf(D.s_ngf, acc[d], D.s_curv * fmaf(ncell, ih2[d], LL));
}

hipError_t launch_jacobi_diag(const DiagParams& d, const float* u, float* diag, hipStream_t st) {
  const int blocks = (d.t.nbar + kNodeBlock - 1) / kNodeBlock;
  hipLaunchKernelGGL(jacobi_diag_kernel, dim3(blocks), dim3(kNodeBlock), 0, st, d, u, diag);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// PCG vector kernels (float32 vectors, float64 dots and step lengths)
// ---------------------------------------------------------------------------
// Jacobi preconditioner of the CG solves: a zero diagonal entry (possible only
// without the regulariser, at a node that no row of dr reaches with a non-zero
// template derivative) is replaced by 1, i.e. that entry is left unscaled.
__global__ __launch_bounds__(kVecBlock) void safe_diag_kernel(int n3, float* __restrict__ d) {
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock)
    if (d[i] == 0.0f) d[i] = 1.0f;
}

hipError_t launch_safe_diag(int n3, float* d, hipStream_t st) {
  const int blocks = std::min((n3 + kVecBlock - 1) / kVecBlock, 4096);
  hipLaunchKernelGGL(safe_diag_kernel, dim3(blocks), dim3(kVecBlock), 0, st, n3, d);
  return hipGetLastError();
}

__global__ __launch_bounds__(kVecBlock) void pcg_init_kernel(int n3, const float* __restrict__ b,
                                                             const float* __restrict__ diag,
                                                             float* __restrict__ s, float* __restrict__ r,
                                                             float* __restrict__ z, float* __restrict__ p,
                                                             double* __restrict__ red) {
  __shared__ double sred[kVecBlock / 64];
  double bb = 0.0, rz = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock) {
    const float bi = b[i];
    const float zi = diag ? bi / diag[i] : bi;
    s[i] = 0.0f;
    r[i] = bi;
    z[i] = zi;
    p[i] = zi;
    bb += (double)bi * bi;
    rz += (double)bi * zi;
  }
  const double sb = block_sum<kVecBlock>(bb, sred);
  __syncthreads();
  const double sz = block_sum<kVecBlock>(rz, sred);
  if (threadIdx.x == 0) {
    red[2 * blockIdx.x] = sb;
    red[2 * blockIdx.x + 1] = sz;
  }
}

hipError_t launch_pcg_init(int n3, const float* b, const float* diag, float* s, float* r, float* z,
                           float* p, double* red, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(pcg_init_kernel, dim3(blocks), dim3(kVecBlock), 0, st, n3, b, diag, s, r, z, p, red);
  return hipGetLastError();
}

// sums pairs of partials (bb, rz) -> sc[SC_BB], sc[SC_RZ]
__global__ __launch_bounds__(256) void pcg_init_finish_kernel(const double* __restrict__ red, int nred,
                                                              double* __restrict__ sc) {
  __shared__ double sred[4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nred; i += 256) {
    a += red[2 * i];
    b += red[2 * i + 1];
  }
  const double sa = block_sum<256>(a, sred);
  __syncthreads();
  const double sb = block_sum<256>(b, sred);
  if (threadIdx.x == 0) {
    sc[SC_BB] = sa;
    sc[SC_RZ] = sb;
    sc[SC_RR] = sa;
  }
}

hipError_t launch_pcg_init_finish(const double* red, int nred, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(pcg_init_finish_kernel, dim3(1), dim3(256), 0, st, red, nred, sc);
  return hipGetLastError();
}

// pq = sum of node-pass partials; alpha = rz / pq (0 on breakdown)
__global__ __launch_bounds__(256) void pcg_alpha_kernel(const double* __restrict__ red, int nred,
                                                        double* __restrict__ sc) {
  __shared__ double sred[4];
  double a = 0.0;
  for (int i = threadIdx.x; i < nred; i += 256) a += red[i];
  const double pq = block_sum<256>(a, sred);
  if (threadIdx.x == 0) {
    sc[SC_PQ] = pq;
    sc[SC_ALPHA] = (pq > 0.0 && isfinite(pq)) ? ld_coherent(sc + SC_RZ) / pq : 0.0;
  }
}

hipError_t launch_pcg_alpha(const double* red_pq, int nred, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(pcg_alpha_kernel, dim3(1), dim3(256), 0, st, red_pq, nred, sc);
  return hipGetLastError();
}

__global__ __launch_bounds__(kVecBlock) void pcg_update_kernel(int n3, const float* __restrict__ diag,
                                                               const float* __restrict__ p,
                                                               const float* __restrict__ q,
                                                               float* __restrict__ s, float* __restrict__ r,
                                                               float* __restrict__ z,
                                                               const double* __restrict__ sc,
                                                               double* __restrict__ red) {
  __shared__ double sred[kVecBlock / 64];
  const float alpha = (float)ld_coherent(sc + SC_ALPHA);
  double rr = 0.0, rz = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock) {
    const float ri = fmaf(-alpha, q[i], r[i]);
    s[i] = fmaf(alpha, p[i], s[i]);
    r[i] = ri;
    const float zi = diag ? ri / diag[i] : ri;
    z[i] = zi;
    rr += (double)ri * ri;
    rz += (double)ri * zi;
  }
  const double a = block_sum<kVecBlock>(rr, sred);
  __syncthreads();
  const double b = block_sum<kVecBlock>(rz, sred);
  if (threadIdx.x == 0) {
    red[2 * blockIdx.x] = a;
    red[2 * blockIdx.x + 1] = b;
  }
}

hipError_t launch_pcg_update(int n3, const float* diag, const float* p, const float* q, float* s,
                             float* r, float* z, const double* sc, double* red, int blocks,
                             hipStream_t st) {
  hipLaunchKernelGGL(pcg_update_kernel, dim3(blocks), dim3(kVecBlock), 0, st, n3, diag, p, q, s, r, z, sc,
                     red);
  return hipGetLastError();
}

// rr, rz_new; beta = rz_new / rz; rz <- rz_new
__global__ __launch_bounds__(256) void pcg_beta_kernel(const double* __restrict__ red, int nred,
                                                       double* __restrict__ sc) {
  __shared__ double sred[4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nred; i += 256) {
    a += red[2 * i];
    b += red[2 * i + 1];
  }
  const double rr = block_sum<256>(a, sred);
  __syncthreads();
  const double rz = block_sum<256>(b, sred);
  if (threadIdx.x == 0) {
    sc[SC_RR] = rr;
    sc[SC_RZNEW] = rz;
    sc[SC_BETA] = rz / ld_coherent(sc + SC_RZ);
    sc[SC_RZ] = rz;
  }
}

hipError_t launch_pcg_beta(const double* red, int nred, double* sc, hipStream_t st) {
  hipLaunchKernelGGL(pcg_beta_kernel, dim3(1), dim3(256), 0, st, red, nred, sc);
  return hipGetLastError();
}

__global__ __launch_bounds__(kVecBlock) void pcg_direction_kernel(int n3, const float* __restrict__ z,
                                                                  float* __restrict__ p,
                                                                  const double* __restrict__ sc) {
  const float beta = (float)ld_coherent(sc + SC_BETA);
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n3; i += gridDim.x * kVecBlock)
    p[i] = fmaf(beta, p[i], z[i]);
}

hipError_t launch_pcg_direction(int n3, const float* z, float* p, const double* sc, int blocks,
                                hipStream_t st) {
  hipLaunchKernelGGL(pcg_direction_kernel, dim3(blocks), dim3(kVecBlock), 0, st, n3, z, p, sc);
  return hipGetLastError();
}

// partial sums of x . y per work-group
__global__ __launch_bounds__(kVecBlock) void dot_kernel(int n, const float* __restrict__ x,
                                                        const float* __restrict__ y, double* __restrict__ red) {
  __shared__ double sred[kVecBlock / 64];
  double a = 0.0;
  for (int i = blockIdx.x * kVecBlock + threadIdx.x; i < n; i += gridDim.x * kVecBlock) a += (double)x[i] * y[i];
  const double s = block_sum<kVecBlock>(a, sred);
  if (threadIdx.x == 0) red[blockIdx.x] = s;
}

hipError_t launch_dot(int n, const float* x, const float* y, double* red, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(dot_kernel, dim3(blocks), dim3(kVecBlock), 0, st, n, x, y, red);
  return hipGetLastError();
}

__global__ void axpy_kernel(int n, const float* __restrict__ x, float eta, const float* __restrict__ s,
                            float* __restrict__ y) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    y[i] = fmaf(eta, s[i], x[i]);
}

// ---- the line search of the capturable Gauss-Newton step ----------------------
// info (device double[9]) = {J_before, J_after, eta, slope, pcg iterations, pcg
// relative residual, pcg flag, accepted, line-search trials}; *search is 1 while
// no step length has been accepted.  J = D + alpha S from the sums at sums[0]
// (distance) and sums[1] (regulariser), rounded as the host evaluates it.
__device__ __forceinline__ double objective_of(const double* sums, double dmul, double smul, double sk,
                                               double alpha) {
  const double D = __dmul_rn(dmul, sums[0]), S = __dmul_rn(__dmul_rn(smul, sums[1]), sk);
  return __dadd_rn(D, __dmul_rn(alpha, S));
}

__global__ void ls_begin_kernel(const double* __restrict__ sums, double dmul, double smul, double sk, double alpha,
                                int* __restrict__ search, double* __restrict__ info) {
  if (threadIdx.x != 0) return;
  const double J = objective_of(sums, dmul, smul, sk, alpha);
  info[0] = J;
  info[1] = J;
  info[2] = 0.0;
  info[7] = 0.0;
  info[8] = 0.0;
  *search = 1;
}

// slope = grad J . s = -(b . s), from the sum of b . s
__global__ void ls_slope_kernel(const double* __restrict__ dot, double* __restrict__ info) {
  if (threadIdx.x == 0) info[3] = -dot[0];
}

__global__ void ls_trial_kernel(int n, const float* __restrict__ u, float eta, const float* __restrict__ s,
                                float* __restrict__ trial, const int* search) {
  if (!ld_coherent(search)) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    trial[i] = fmaf(eta, s[i], u[i]);   // the arithmetic of axpy_kernel
}

// Armijo test of trial k at step length eta (J(u + eta s) <= J + c1 eta slope,
// evaluated as the host does); a non-finite J is rejected
__global__ void ls_check_kernel(const double* __restrict__ sums, double dmul, double smul, double sk, double alpha,
                                double c1, double eta, int k, int* __restrict__ search, double* __restrict__ info) {
  if (threadIdx.x != 0 || !ld_coherent(search)) return;
  const double J = objective_of(sums, dmul, smul, sk, alpha);
  info[8] = (double)(k + 1);
  if (isfinite(J) && J <= __dadd_rn(info[0], __dmul_rn(__dmul_rn(c1, eta), info[3]))) {
    info[1] = J;
    info[2] = eta;
    info[7] = 1.0;
    *search = 0;
  }
}

__global__ void ls_commit_kernel(int n, const float* __restrict__ trial, float* __restrict__ u,
                                 const double* __restrict__ info) {
  if (info[7] != 1.0) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) u[i] = trial[i];
}

hipError_t launch_ls_begin(const double* sums, double dmul, double smul, double sk, double alpha, int* search,
                           double* info, hipStream_t st) {
  hipLaunchKernelGGL(ls_begin_kernel, dim3(1), dim3(64), 0, st, sums, dmul, smul, sk, alpha, search, info);
  return hipGetLastError();
}

hipError_t launch_ls_slope(const double* dot, double* info, hipStream_t st) {
  hipLaunchKernelGGL(ls_slope_kernel, dim3(1), dim3(64), 0, st, dot, info);
  return hipGetLastError();
}

hipError_t launch_ls_trial(int n, const float* u, float eta, const float* s, float* trial, const int* search,
                           hipStream_t st) {
  const int blocks = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(ls_trial_kernel, dim3(blocks), dim3(256), 0, st, n, u, eta, s, trial, search);
  return hipGetLastError();
}

hipError_t launch_ls_check(const double* sums, double dmul, double smul, double sk, double alpha, double c1, double eta,
                           int k, int* search, double* info, hipStream_t st) {
  hipLaunchKernelGGL(ls_check_kernel, dim3(1), dim3(64), 0, st, sums, dmul, smul, sk, alpha, c1, eta, k, search, info);
  return hipGetLastError();
}

hipError_t launch_ls_commit(int n, const float* trial, float* u, const double* info, hipStream_t st) {
  const int blocks = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(ls_commit_kernel, dim3(blocks), dim3(256), 0, st, n, trial, u, info);
  return hipGetLastError();
}

hipError_t launch_axpy(int n, const float* x, float eta, const float* s, float* y, hipStream_t st) {
  const int blocks = std::min((n + 255) / 256, 4096);
  hipLaunchKernelGGL(axpy_kernel, dim3(blocks), dim3(256), 0, st, n, x, eta, s, y);
  return hipGetLastError();
}

// y[i] = v for i < n (a kernel rather than a memset, so that a captured
// sequence holds no memset node)
__global__ void fill_kernel(size_t n, float v, float* __restrict__ y) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = v;
}

hipError_t launch_fill(size_t n, float v, float* y, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, st, n, v, y);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pyramid transfers
// ---------------------------------------------------------------------------
__global__ void restrict_kernel(const float* __restrict__ f, int mx, int my, int mz, float* __restrict__ c) {
  const int cx = (mx + 1) / 2, cy = (my + 1) / 2, cz = (mz + 1) / 2;
  const size_t total = (size_t)cx * cy * cz;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(idx % cx), b = (int)((idx / cx) % cy), k = (int)(idx / ((size_t)cx * cy));
    const int x0 = 2 * a, x1 = min(2 * a + 1, mx - 1);
    const int y0 = 2 * b, y1 = min(2 * b + 1, my - 1);
    const int z0 = 2 * k, z1 = min(2 * k + 1, mz - 1);
    auto at = [&](int x, int y, int z) { return f[((size_t)z * my + y) * mx + x]; };
    const float s = ((at(x0, y0, z0) + at(x1, y0, z0)) + (at(x0, y1, z0) + at(x1, y1, z0))) +
                    ((at(x0, y0, z1) + at(x1, y0, z1)) + (at(x0, y1, z1) + at(x1, y1, z1)));
    c[idx] = 0.125f * s;
  }
}

hipError_t launch_restrict(const float* fine, int mx, int my, int mz, float* coarse, hipStream_t st) {
  const size_t total = (size_t)((mx + 1) / 2) * ((my + 1) / 2) * ((mz + 1) / 2);
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(restrict_kernel, dim3(blocks), dim3(256), 0, st, fine, mx, my, mz, coarse);
  return hipGetLastError();
}

__global__ void prolong_kernel(const float* __restrict__ c, int cnx, int cny, int cnz, float* __restrict__ f,
                               int fnx, int fny, int fnz, const Conv1* __restrict__ tx,
                               const Conv1* __restrict__ ty, const Conv1* __restrict__ tz, int nc) {
  const size_t fb = (size_t)fnx * fny * fnz, cb = (size_t)cnx * cny * cnz;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < fb;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % fnx), j = (int)((idx / fnx) % fny), k = (int)(idx / ((size_t)fnx * fny));
    const Conv1 a = tx[i], b = ty[j];
    // a two-dimensional field (one node plane): no second plane to interpolate towards
    const Conv1 e = cnz > 1 ? tz[k] : Conv1{0, 0.0f};
    for (int d = 0; d < nc; ++d) {
      const float* s = c + d * cb + ((size_t)e.n0 * cny + b.n0) * cnx + a.n0;
      const size_t sy = cnx, sz = cnz > 1 ? (size_t)cnx * cny : 0;
      const float l00 = fmaf(a.f, s[1] - s[0], s[0]);
      const float l10 = fmaf(a.f, s[sy + 1] - s[sy], s[sy]);
      const float l01 = fmaf(a.f, s[sz + 1] - s[sz], s[sz]);
      const float l11 = fmaf(a.f, s[sz + sy + 1] - s[sz + sy], s[sz + sy]);
      const float m0 = fmaf(b.f, l10 - l00, l00), m1 = fmaf(b.f, l11 - l01, l01);
      f[d * fb + idx] = fmaf(e.f, m1 - m0, m0);
    }
  }
}

hipError_t launch_prolong(const float* coarse, int cnx, int cny, int cnz, float* fine, int fnx, int fny,
                          int fnz, const Conv1* tx, const Conv1* ty, const Conv1* tz, int nc, hipStream_t st) {
  const size_t total = (size_t)fnx * fny * fnz;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(prolong_kernel, dim3(blocks), dim3(256), 0, st, coarse, cnx, cny, cnz, fine, fnx, fny,
                     fnz, tx, ty, tz, nc);
  return hipGetLastError();
}

}  // namespace mfr
