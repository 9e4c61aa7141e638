// Node-grid kernels of the learned preconditioner around the convolutions:
// input features, RMS scales, the training loss and its gradient, the
// restriction of |grad R| to the nodes, and the flexible-CG coefficients.
// Reductions: float64 per-block partials in a fixed layout, summed in a fixed
// order by one group, so every result is run-to-run deterministic.
#include <algorithm>

#include "mfr_internal.h"

namespace mfr {

namespace {

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum over 256 threads; result valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* sred) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (sred[0] + sred[1]) + (sred[2] + sred[3]);
  __syncthreads();
  return s;
}

constexpr int kPB = 256;          // threads per block of the vector kernels
constexpr int kMaxPartials = 1024;

int vec_blocks_for(size_t n) { return (int)std::max<size_t>(1, std::min<size_t>((n + kPB - 1) / kPB, kMaxPartials)); }

}  // namespace

// ---- up to four float64 dot products per launch -------------------------------------
// red[k * blocks + b] = partial of sum_i a_k[i] * b_k[i]; b_k null means a_k . a_k;
// den_k (nullable) divides a_k elementwise first (Jacobi-scaled vectors).
__global__ __launch_bounds__(kPB) void pc_dots_kernel(const DotsArgs d, double* __restrict__ red) {
  if (d.live && !ld_coherent(d.live)) return;
  __shared__ double sred[4];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t i = (size_t)blockIdx.x * kPB + threadIdx.x; i < d.n; i += (size_t)gridDim.x * kPB) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k < d.count) {
        float a = d.a[k][i];
        if (d.den[k]) a = a / d.den[k][i];
        const float b = d.b[k] ? d.b[k][i] : a;
        acc[k] += (double)a * b;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (k < d.count) {
      const double s = block_sum256(acc[k], sred);
      if (threadIdx.x == 0) red[(size_t)k * gridDim.x + blockIdx.x] = s;
    }
  }
}

// out[k] = sum_b red[k * blocks + b] (fixed order); sqrt_scale[k] > 0 stores
// sqrt(sum * sqrt_scale[k]) instead (an RMS).
__global__ __launch_bounds__(256) void pc_dots_finish_kernel(const double* __restrict__ red, int blocks, int count,
                                                             DotsOut o, const int* live) {
  if (live && !ld_coherent(live)) return;
  __shared__ double sred[4];
  for (int k = 0; k < count; ++k) {
    double a = 0.0;
    for (int b = threadIdx.x; b < blocks; b += 256) a += red[(size_t)k * blocks + b];
    const double s = block_sum256(a, sred);
    if (threadIdx.x == 0 && o.out[k]) *o.out[k] = o.rms_scale[k] > 0.0 ? sqrt(s * o.rms_scale[k]) : s;
  }
}

int pc_dots_blocks(size_t n) { return vec_blocks_for(n); }

hipError_t launch_pc_dots(const DotsArgs& d, const DotsOut& o, double* red, hipStream_t st) {
  const int blocks = vec_blocks_for(d.n);
  hipLaunchKernelGGL(pc_dots_kernel, dim3(blocks), dim3(kPB), 0, st, d, red);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pc_dots_finish_kernel, dim3(1), dim3(256), 0, st, red, blocks, d.count, o, d.live);
  return hipGetLastError();
}

// ---- network input ---------------------------------------------------------------
// h0[n][0..2] = (r/diag)/rms_y, [3..5] = r/rms_r, [6..8] = diag/rms_d, [9] = gR/rms_g, rest 0.
__global__ __launch_bounds__(kPB) void pc_features_kernel(int n, const float* __restrict__ r,
                                                          const float* __restrict__ diag,
                                                          const float* __restrict__ gR,
                                                          const double* __restrict__ sc,
                                                          uint16_t* __restrict__ h0, const int* live) {
  if (live && !ld_coherent(live)) return;
  const int i = blockIdx.x * kPB + threadIdx.x;
  if (i >= n) return;
  const double sy = ld_coherent(sc + PC_RMS_Y), sr = ld_coherent(sc + PC_RMS_R);
  const double sd = ld_coherent(sc + PC_RMS_D), sg = ld_coherent(sc + PC_RMS_G);
  const float iy = sy > 0.0 ? (float)(1.0 / sy) : 0.f, ir = sr > 0.0 ? (float)(1.0 / sr) : 0.f;
  const float id = sd > 0.0 ? (float)(1.0 / sd) : 0.f, ig = sg > 0.0 ? (float)(1.0 / sg) : 0.f;
  float f[16];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float rv = r[(size_t)d * n + i], dv = diag[(size_t)d * n + i];
    f[d] = (rv / dv) * iy;
    f[3 + d] = rv * ir;
    f[6 + d] = dv * id;
  }
  f[9] = gR[i] * ig;
#pragma unroll
  for (int c = 10; c < 16; ++c) f[c] = 0.f;
  uint32_t w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = f2bf(f[2 * k]) | ((uint32_t)f2bf(f[2 * k + 1]) << 16);
  uint4* dst = reinterpret_cast<uint4*>(h0 + (size_t)i * 16);
  dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
  dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

hipError_t launch_pc_features(int n, const float* r, const float* diag, const float* gR, const double* sc,
                              uint16_t* h0, hipStream_t st, const int* live) {
  hipLaunchKernelGGL(pc_features_kernel, dim3((n + kPB - 1) / kPB), dim3(kPB), 0, st, n, r, diag, gR, sc, h0,
                     live);
  return hipGetLastError();
}

// y = r / diag (node vector, 3n)
__global__ __launch_bounds__(kPB) void pc_jacobi_kernel(int n3, const float* __restrict__ r,
                                                        const float* __restrict__ diag, float* __restrict__ y) {
  for (int i = blockIdx.x * kPB + threadIdx.x; i < n3; i += gridDim.x * kPB) y[i] = r[i] / diag[i];
}

hipError_t launch_pc_jacobi(int n3, const float* r, const float* diag, float* y, hipStream_t st) {
  const int blocks = std::min((n3 + kPB - 1) / kPB, 4096);
  hipLaunchKernelGGL(pc_jacobi_kernel, dim3(blocks), dim3(kPB), 0, st, n3, r, diag, y);
  return hipGetLastError();
}

__global__ __launch_bounds__(kPB) void pc_fallback_kernel(int n3, const float* __restrict__ r,
                                                          const float* __restrict__ diag, float* __restrict__ z,
                                                          float* __restrict__ p, const int* live, int* state) {
  if (!ld_coherent(live)) return;
  for (int i = blockIdx.x * kPB + threadIdx.x; i < n3; i += gridDim.x * kPB) {
    const float zi = r[i] / diag[i];
    z[i] = zi;
    p[i] = zi;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) state[ST_FALLBACK] = 1;
}

hipError_t launch_pc_fallback(int n3, const float* r, const float* diag, float* z, float* p, const int* live,
                              int* state, hipStream_t st) {
  const int blocks = std::min((n3 + kPB - 1) / kPB, 4096);
  hipLaunchKernelGGL(pc_fallback_kernel, dim3(blocks), dim3(kPB), 0, st, n3, r, diag, z, p, live, state);
  return hipGetLastError();
}

// ---- training loss --------------------------------------------------------------
// From sc[PC_ZR] = z.r, sc[PC_ZAZ] = z.Az, sc[PC_YR] = y.r, sc[PC_YAY] = y.Ay:
// L = -(z.r)^2 / z.Az / E_J with E_J = (y.r)^2 / y.Ay, and dL/dz = cA Az + cR r.
__global__ void pc_loss_kernel(double* sc) {
  if (threadIdx.x != 0) return;
  const double zr = ld_coherent(sc + PC_ZR), zAz = ld_coherent(sc + PC_ZAZ);
  const double yr = ld_coherent(sc + PC_YR), yAy = ld_coherent(sc + PC_YAY);
  const double EJ = yr * yr / yAy;
  const double s = zr / zAz;
  sc[PC_LOSS] = -(zr * s) / EJ;
  sc[PC_CA] = 2.0 * s * s / EJ;
  sc[PC_CR] = -2.0 * s / EJ;
}

hipError_t launch_pc_loss(double* sc, hipStream_t st) {
  hipLaunchKernelGGL(pc_loss_kernel, dim3(1), dim3(64), 0, st, sc);
  return hipGetLastError();
}

// Gradient at the network output: z = y + rms_y o, so dL/do[c] = rms_y (cA Az + cR r)[c], c < 3.
__global__ __launch_bounds__(kPB) void pc_grad_out_kernel(int n, const float* __restrict__ Az,
                                                          const float* __restrict__ r,
                                                          const double* __restrict__ sc,
                                                          uint16_t* __restrict__ g16) {
  const int i = blockIdx.x * kPB + threadIdx.x;
  if (i >= n) return;
  const double sy = ld_coherent(sc + PC_RMS_Y);
  const float cA = (float)(ld_coherent(sc + PC_CA) * sy), cR = (float)(ld_coherent(sc + PC_CR) * sy);
  float v[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) v[d] = fmaf(cA, Az[(size_t)d * n + i], cR * r[(size_t)d * n + i]);
  uint4* dst = reinterpret_cast<uint4*>(g16 + (size_t)i * 16);
  dst[0] = make_uint4(f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16), f2bf(v[2]), 0u, 0u);
  dst[1] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_pc_grad_out(int n, const float* Az, const float* r, const double* sc, uint16_t* g16,
                              hipStream_t st) {
  hipLaunchKernelGGL(pc_grad_out_kernel, dim3((n + kPB - 1) / kPB), dim3(kPB), 0, st, n, Az, r, sc, g16);
  return hipGetLastError();
}

// ---- |grad R| restricted to the nodes: (P^T g) / (P^T 1), separable ---------------
// |grad R| per voxel from the short differences (eq. NGF_discretized, no edge
// parameter), neighbours clamped; then three 1D gathers with the weights of the
// grid conversion (eq. grid_conversion), x first.
__global__ __launch_bounds__(kPB) void pc_gm_x_kernel(GmArgs g, float* __restrict__ out) {
  const size_t total = (size_t)g.mz * g.my * g.nx;
  for (size_t idx = (size_t)blockIdx.x * kPB + threadIdx.x; idx < total; idx += (size_t)gridDim.x * kPB) {
    const int j = (int)(idx % g.nx);
    const size_t row = idx / g.nx;          // z * my + y
    const int y = (int)(row % g.my), z = (int)(row / g.my);
    const Range1 rg = g.rx[j];
    float s = 0.f;
    for (int a = rg.lo; a <= rg.hi; ++a) {
      const Conv1 c = g.cx[a];
      const float w = (c.n0 == j) ? 1.0f - c.f : c.f;
      const size_t v = row * g.mx + a;
      const float R0 = g.R[v];
      const float xp = g.R[v - a + min(a + 1, g.mx - 1)] - R0, xm = g.R[v - a + max(a - 1, 0)] - R0;
      const size_t pl = (size_t)g.mx * g.my;
      const size_t yb = v - (size_t)y * g.mx, zb = v - (size_t)z * pl;
      const float yp = g.R[yb + (size_t)min(y + 1, g.my - 1) * g.mx] - R0;
      const float ym = g.R[yb + (size_t)max(y - 1, 0) * g.mx] - R0;
      const float zp = g.R[zb + (size_t)min(z + 1, g.mz - 1) * pl] - R0;
      const float zm = g.R[zb + (size_t)max(z - 1, 0) * pl] - R0;
      const float q = fmaf(fmaf(xp, xp, xm * xm), g.ih2x,
                           fmaf(fmaf(yp, yp, ym * ym), g.ih2y, fmaf(zp, zp, zm * zm) * g.ih2z));
      s = fmaf(w, sqrtf(0.5f * q), s);
    }
    out[idx] = s;
  }
}

// out[(z * ny + jy) * nx + x] = sum_b w_y(b, jy) in[(z * my + b) * nx + x]
__global__ __launch_bounds__(kPB) void pc_gm_y_kernel(GmArgs g, const float* __restrict__ in, float* __restrict__ out) {
  const size_t total = (size_t)g.mz * g.ny * g.nx;
  for (size_t idx = (size_t)blockIdx.x * kPB + threadIdx.x; idx < total; idx += (size_t)gridDim.x * kPB) {
    const int x = (int)(idx % g.nx);
    const int jy = (int)((idx / g.nx) % g.ny);
    const int z = (int)(idx / ((size_t)g.nx * g.ny));
    const Range1 rg = g.ry[jy];
    float s = 0.f;
    for (int b = rg.lo; b <= rg.hi; ++b) {
      const Conv1 c = g.cy[b];
      const float w = (c.n0 == jy) ? 1.0f - c.f : c.f;
      s = fmaf(w, in[((size_t)z * g.my + b) * g.nx + x], s);
    }
    out[idx] = s;
  }
}

// gR[(jz * ny + y) * nx + x] = sum_c w_z(c, jz) in[(c * ny + y) * nx + x] / (sx[x] sy[y] sz[jz])
__global__ __launch_bounds__(kPB) void pc_gm_z_kernel(GmArgs g, const float* __restrict__ in, float* __restrict__ gR) {
  const size_t total = (size_t)g.nz * g.ny * g.nx;
  for (size_t idx = (size_t)blockIdx.x * kPB + threadIdx.x; idx < total; idx += (size_t)gridDim.x * kPB) {
    const int x = (int)(idx % g.nx);
    const int y = (int)((idx / g.nx) % g.ny);
    const int jz = (int)(idx / ((size_t)g.nx * g.ny));
    const Range1 rg = g.rz[jz];
    float s = 0.f;
    for (int c = rg.lo; c <= rg.hi; ++c) {
      const Conv1 cv = g.cz[c];
      const float w = (cv.n0 == jz) ? 1.0f - cv.f : cv.f;
      s = fmaf(w, in[((size_t)c * g.ny + y) * g.nx + x], s);
    }
    gR[idx] = s / (g.wsx[x] * g.wsy[y] * g.wsz[jz]);
  }
}

hipError_t launch_pc_gradmag(const GmArgs& g, float* tmp1, float* tmp2, float* gR, hipStream_t st) {
  auto blocks = [](size_t n) { return (int)std::min<size_t>((n + kPB - 1) / kPB, 8192); };
  hipLaunchKernelGGL(pc_gm_x_kernel, dim3(blocks((size_t)g.mz * g.my * g.nx)), dim3(kPB), 0, st, g, tmp1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pc_gm_y_kernel, dim3(blocks((size_t)g.mz * g.ny * g.nx)), dim3(kPB), 0, st, g, tmp1, tmp2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pc_gm_z_kernel, dim3(blocks((size_t)g.nz * g.ny * g.nx)), dim3(kPB), 0, st, g, tmp2, gR);
  return hipGetLastError();
}

// ---- flexible CG (Polak-Ribiere) --------------------------------------------------
__global__ __launch_bounds__(kPB) void fpcg_update_kernel(int n3, const float* __restrict__ diag,
                                                          const float* __restrict__ p, const float* __restrict__ q,
                                                          float* __restrict__ s, float* __restrict__ r,
                                                          float* __restrict__ rprev, const double* __restrict__ sc,
                                                          double* __restrict__ red, const int* live) {
  if (live && !ld_coherent(live)) return;
  __shared__ double sred[4];
  const float alpha = (float)ld_coherent(sc + SC_ALPHA);
  double rr = 0.0, yy = 0.0;
  for (int i = blockIdx.x * kPB + threadIdx.x; i < n3; i += gridDim.x * kPB) {
    const float r0 = r[i];
    const float ri = fmaf(-alpha, q[i], r0);
    s[i] = fmaf(alpha, p[i], s[i]);
    rprev[i] = r0;
    r[i] = ri;
    const float yi = ri / diag[i];
    rr += (double)ri * ri;
    yy += (double)yi * yi;
  }
  const double a = block_sum256(rr, sred);
  const double b = block_sum256(yy, sred);
  if (threadIdx.x == 0) {
    red[2 * blockIdx.x] = a;
    red[2 * blockIdx.x + 1] = b;
  }
}

hipError_t launch_fpcg_update(int n3, const float* diag, const float* p, const float* q, float* s, float* r,
                              float* rprev, const double* sc, double* red, int blocks, hipStream_t st,
                              const int* live) {
  hipLaunchKernelGGL(fpcg_update_kernel, dim3(blocks), dim3(kPB), 0, st, n3, diag, p, q, s, r, rprev, sc, red, live);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fpcg_scales_kernel(const double* __restrict__ red, int blocks, int n3,
                                                          double* __restrict__ sc, double* __restrict__ pc_sc,
                                                          int* state, int* active) {
  if (active && !ld_coherent(active)) return;
  __shared__ double sred[4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < blocks; i += 256) {
    a += red[2 * i];
    b += red[2 * i + 1];
  }
  const double rr = block_sum256(a, sred);
  const double yy = block_sum256(b, sred);
  if (threadIdx.x == 0) {
    sc[SC_RR] = rr;
    pc_sc[PC_RMS_R] = sqrt(rr / n3);
    pc_sc[PC_RMS_Y] = sqrt(yy / n3);
    if (state) {   // the convergence test of a device-steered solve
      const int iters = ld_coherent(state + ST_ITERS) + 1;
      const double rel = sqrt(rr) / sqrt(ld_coherent(sc + SC_BB));
      state[ST_ITERS] = iters;
      sc[SC_RELRES] = rel;
      if (rel <= ld_coherent(sc + SC_RTOL)) {
        state[ST_FLAG] = 0;
        state[ST_ACTIVE] = 0;
        *active = 0;
      } else if (iters >= ld_coherent(state + ST_MAXIT)) {
        state[ST_FLAG] = 1;
        state[ST_ACTIVE] = 0;
        *active = 0;
      }
    }
  }
}

hipError_t launch_fpcg_scales(const double* red, int blocks, int n3, double* sc, double* pc_sc, hipStream_t st,
                              int* state, int* active) {
  hipLaunchKernelGGL(fpcg_scales_kernel, dim3(1), dim3(256), 0, st, red, blocks, n3, sc, pc_sc, state, active);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fpcg_beta_sum_kernel(const double* __restrict__ zred, int blocks,
                                                            double* __restrict__ sc, const int* live) {
  if (live && !ld_coherent(live)) return;
  __shared__ double sred[4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < blocks; i += 256) {
    a += zred[2 * i];
    b += zred[2 * i + 1];
  }
  const double zr = block_sum256(a, sred);
  const double zrp = block_sum256(b, sred);
  if (threadIdx.x == 0) {
    sc[SC_ZR] = zr;
    sc[SC_ZRP] = zrp;
    sc[SC_BETA] = (zr - zrp) / ld_coherent(sc + SC_RZ);
    sc[SC_RZ] = zr;
  }
}

hipError_t launch_fpcg_beta_sum(const double* zred, int blocks, double* sc, hipStream_t st, const int* live) {
  hipLaunchKernelGGL(fpcg_beta_sum_kernel, dim3(1), dim3(256), 0, st, zred, blocks, sc, live);
  return hipGetLastError();
}

}  // namespace mfr
