// Kernels of the L-BFGS initial-matrix solve (Sec. 2.3.2):
// x = H_0^{-1} v with H_0 = 2 alpha hbar^y L^T L + gamma I (curvature) or
// -alpha hbar^y L + gamma I (diffusive regulariser).
//
// The 7-point Laplacian with clamped (Neumann) neighbours is the Kronecker sum
// of one-dimensional second-difference matrices whose eigenvectors are the
// DCT-II cosines, so H_0 is diagonal in the separable cosine basis: the solve
// is a forward transform along z, y and x, a division by the eigenvalues
// 2 alpha hbar^y (lx + ly + lz)^2 + gamma (curvature) or
// -alpha hbar^y (lx + ly + lz) + gamma (diffusive), and the inverse transform.  Each
// axis transform is a small dense product (the n x n cosine matrix against
// all lines of that axis), done here as an LDS-tiled float32 product.
#include "mfr_internal.h"

namespace mfr {

namespace {

constexpr int TK = 32;   // output rows (transformed index) per tile
constexpr int TC = 64;   // lines per tile
constexpr int TI = 32;   // summation chunk

// out[b][k][c] = sum_i M[k][i] in[b][i][c] with element offsets
// b * bs + i * is + c * cs (the same for in and out).  ISTRIDE1: the summed
// index is the contiguous one (the x axis), else the line index is.
template <bool ISTRIDE1>
__global__ __launch_bounds__(256) void axis_transform_kernel(const float* __restrict__ M, int n, const float* __restrict__ in,
                                                             float* __restrict__ out, long long bs, long long is,
                                                             long long cs, int C) {
  __shared__ float sM[TK][TI + 1];
  __shared__ float sIn[TI][TC + 4];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * TC, k0 = blockIdx.y * TK;
  const long long base = (long long)blockIdx.z * bs;
  const int tk = tid / 16, tc = tid % 16;   // rows 2 tk, 2 tk + 1; columns 4 tc .. 4 tc + 3
  float acc[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  for (int i0 = 0; i0 < n; i0 += TI) {
    for (int e = tid; e < TK * TI; e += 256) {
      const int kk = e / TI, ii = e % TI;
      const int k = k0 + kk, i = i0 + ii;
      sM[kk][ii] = (k < n && i < n) ? M[(size_t)k * n + i] : 0.0f;
    }
    for (int e = tid; e < TI * TC; e += 256) {
      int ii, cc;
      if (ISTRIDE1) {
        ii = e % TI;
        cc = e / TI;
      } else {
        ii = e / TC;
        cc = e % TC;
      }
      const int i = i0 + ii, c = c0 + cc;
      sIn[ii][cc] = (i < n && c < C) ? in[base + (long long)i * is + (long long)c * cs] : 0.0f;
    }
    __syncthreads();
#pragma unroll 8
    for (int ii = 0; ii < TI; ++ii) {
      const float m0 = sM[2 * tk][ii], m1 = sM[2 * tk + 1][ii];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float v = sIn[ii][4 * tc + j];
        acc[0][j] = fmaf(m0, v, acc[0][j]);
        acc[1][j] = fmaf(m1, v, acc[1][j]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int k = k0 + 2 * tk + r;
    if (k >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = c0 + 4 * tc + j;
      if (c < C) out[base + (long long)k * is + (long long)c * cs] = acc[r][j];
    }
  }
}

// x = v / (c2 l^2 + c1 l + gamma), l = lx[i] + ly[j] + lz[k], in the cosine basis.
__global__ __launch_bounds__(256) void h0_scale_kernel(float* __restrict__ x, const float* __restrict__ lam, int nx,
                                                       int ny, int nz, int nc, float c2, float c1, float gamma) {
  const size_t nb = (size_t)nx * ny * nz, total = (size_t)nc * nb;
  const float* lx = lam;
  const float* ly = lam + nx;
  const float* lz = lam + nx + ny;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
    const size_t n = idx % nb;
    const int i = (int)(n % nx), j = (int)((n / nx) % ny), k = (int)(n / ((size_t)nx * ny));
    const float l = lx[i] + ly[j] + lz[k];
    x[idx] = x[idx] / fmaf(fmaf(c2, l, c1), l, gamma);
  }
}

hipError_t transform(const float* M, int n, const float* in, float* out, long long bs, long long is, long long cs,
                     int C, int batches, bool istride1, hipStream_t st) {
  dim3 grid((C + TC - 1) / TC, (n + TK - 1) / TK, batches);
  if (istride1)
    hipLaunchKernelGGL(axis_transform_kernel<true>, grid, dim3(256), 0, st, M, n, in, out, bs, is, cs, C);
  else
    hipLaunchKernelGGL(axis_transform_kernel<false>, grid, dim3(256), 0, st, M, n, in, out, bs, is, cs, C);
  return hipGetLastError();
}

}  // namespace

// x = H_0^{-1} v.  tab: the cosine matrices and their transposes (x, y, z)
// followed by the per-axis Laplacian eigenvalues; ta, tb: scratch node vectors.
// x may alias v.
hipError_t launch_h0_solve(const H0Tables& t, const float* v, float* x, float* ta, float* tb, float c2, float c1,
                           float gamma, hipStream_t st) {
  const int nx = t.n[0], ny = t.n[1], nz = t.n[2], nc = t.nc;
  const long long nxy = (long long)nx * ny, nb = nxy * nz;
  hipError_t e;
  // forward: z (per component), y (per component and plane), x (all lines); a
  // two-dimensional field (nz = 1) has no z transform (its cosine matrix is 1)
  const float* in = v;
  if (nz > 1) {
    if ((e = transform(t.C[2], nz, v, tb, nb, nxy, 1, (int)nxy, nc, false, st)) != hipSuccess) return e;
    in = tb;
  }
  if ((e = transform(t.C[1], ny, in, ta, nxy, nx, 1, nx, nc * nz, false, st)) != hipSuccess) return e;
  if ((e = transform(t.C[0], nx, ta, tb, 0, 1, nx, (int)(nc * nz * ny), 1, true, st)) != hipSuccess) return e;
  const int blocks = (int)std::min<long long>((nc * nb + 255) / 256, 8192);
  hipLaunchKernelGGL(h0_scale_kernel, dim3(blocks), dim3(256), 0, st, tb, t.lam, nx, ny, nz, nc, c2, c1, gamma);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // inverse: the transposed matrices in reverse order
  if ((e = transform(t.Ct[0], nx, tb, ta, 0, 1, nx, (int)(nc * nz * ny), 1, true, st)) != hipSuccess) return e;
  if (nz == 1) return transform(t.Ct[1], ny, ta, x, nxy, nx, 1, nx, nc, false, st);
  if ((e = transform(t.Ct[1], ny, ta, tb, nxy, nx, 1, nx, nc * nz, false, st)) != hipSuccess) return e;
  return transform(t.Ct[2], nz, tb, x, nb, nxy, 1, (int)nxy, nc, false, st);
}

}  // namespace mfr
