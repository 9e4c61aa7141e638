// Kernels of the batched path: several independent registration problems of
// different sizes advance together, one launch per phase.  Problem tables sit
// in kernel-argument memory (uniform, scalar loads); each problem keeps its
// own float64 partial sums in the same block layout as a single-problem
// launch, so sums (and results) equal the single-problem path bit for bit.
//
// The conjugate-gradient iteration (Sec. 2.3.1) is steered on the device:
// per problem an active flag, iteration count, status and relative residual
// live in device memory, so a fixed sequence of launches can be captured once
// into a HIP graph and replayed; finished problems turn into no-ops.
#include "mfr_internal.h"

namespace mfr {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

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
  __syncthreads();
  return s;
}

template <int N>
__device__ __forceinline__ int find_job(const int (&prefix)[N], int n, int item) {
  int j = 0;
  while (j + 1 < n && prefix[j + 1] <= item) ++j;
  return j;
}

}  // namespace

// ---- per-problem fixed-order sums: one group per problem -------------------------
__global__ __launch_bounds__(256) void sum_batch_kernel(const SumJobs J) {
  __shared__ double sred[4];
  const SumJob& s = J.jobs[blockIdx.x];
  if (J.active && !ld_coherent(J.active + blockIdx.x)) return;
  double a = 0.0;
  for (int i = threadIdx.x; i < s.n; i += 256) a += s.parts[i * s.stride];
  a = block_sum<256>(a, sred);
  if (threadIdx.x == 0) *s.out = a;
}

hipError_t launch_sum_batch(const SumJobs& j, hipStream_t st) {
  hipLaunchKernelGGL(sum_batch_kernel, dim3(j.n), dim3(256), 0, st, j);
  return hipGetLastError();
}

__global__ void zero_ints_kernel(int* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

// ---- batched vector kernels ------------------------------------------------------
// y_j = x_j + eta_j s_j for active problems
__global__ __launch_bounds__(kVecBlock) void axpy_batch_kernel(const AxpyJobs J) {
  const int pr = find_job(J.prefix, J.n, blockIdx.x);
  if (J.active && !ld_coherent(J.active + pr)) return;
  const AxpyJob& a = J.jobs[pr];
  const int nb = J.prefix[pr + 1] - J.prefix[pr];
  for (int i = (blockIdx.x - J.prefix[pr]) * kVecBlock + threadIdx.x; i < a.n; i += nb * kVecBlock)
    a.y[i] = fmaf(a.eta, a.s[i], a.x[i]);
}

hipError_t launch_axpy_batch(const AxpyJobs& j, hipStream_t st) {
  hipLaunchKernelGGL(axpy_batch_kernel, dim3(j.prefix[j.n]), dim3(kVecBlock), 0, st, j);
  return hipGetLastError();
}

// x_j . y_j partials (one per block of the problem, same layout as launch_dot)
__global__ __launch_bounds__(kVecBlock) void dot_batch_kernel(const VecJobs J) {
  __shared__ double sred[kVecBlock / 64];
  const int pr = find_job(J.prefix, J.n, blockIdx.x);
  const VecJob& v = J.jobs[pr];
  const int lb = blockIdx.x - J.prefix[pr], nb = J.prefix[pr + 1] - J.prefix[pr];
  double a = 0.0;
  for (int i = lb * kVecBlock + threadIdx.x; i < v.n3; i += nb * kVecBlock) a += (double)v.r[i] * v.z[i];
  const double s = block_sum<kVecBlock>(a, sred);
  if (threadIdx.x == 0) v.red[lb] = s;
}

hipError_t launch_dot_batch(const VecJobs& j, hipStream_t st) {
  hipLaunchKernelGGL(dot_batch_kernel, dim3(j.prefix[j.n]), dim3(kVecBlock), 0, st, j);
  return hipGetLastError();
}

// PCG start: s = 0, r = b, z = M^-1 r, p = z; partials (b.b, r.z); state reset.
__global__ __launch_bounds__(kVecBlock) void pcg_init_batch_kernel(const VecJobs J) {
  __shared__ double sred[kVecBlock / 64];
  const int pr = find_job(J.prefix, J.n, blockIdx.x);
  const VecJob& v = J.jobs[pr];
  const int lb = blockIdx.x - J.prefix[pr], nb = J.prefix[pr + 1] - J.prefix[pr];
  double bb = 0.0, rz = 0.0;
  for (int i = lb * kVecBlock + threadIdx.x; i < v.n3; i += nb * kVecBlock) {
    const float bi = v.b[i];
    const float zi = v.diag ? bi / v.diag[i] : bi;
    v.s[i] = 0.0f;
    v.r[i] = bi;
    v.z[i] = zi;
    v.p[i] = zi;
    bb += (double)bi * bi;
    rz += (double)bi * zi;
  }
  const double sb = block_sum<kVecBlock>(bb, sred);
  const double sz = block_sum<kVecBlock>(rz, sred);
  if (threadIdx.x == 0) {
    v.red[2 * lb] = sb;
    v.red[2 * lb + 1] = sz;
  }
}

// One group per problem: ||b||, r.z, and the per-problem control state.
__global__ __launch_bounds__(256) void pcg_init_finish_batch_kernel(const VecJobs J) {
  __shared__ double sred[4];
  const int pr = blockIdx.x;
  const VecJob& v = J.jobs[pr];
  const int nb = J.prefix[pr + 1] - J.prefix[pr];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += v.red[2 * i];
    b += v.red[2 * i + 1];
  }
  const double bb = block_sum<256>(a, sred);
  const double rz = block_sum<256>(b, sred);
  if (threadIdx.x == 0) {
    double* sc = v.sc;
    sc[SC_BB] = bb;
    sc[SC_RZ] = rz;
    sc[SC_RR] = bb;
    sc[SC_RELRES] = (bb > 0.0) ? 1.0 : 0.0;
    int* st = v.state;
    const bool live = bb > 0.0 && isfinite(bb) && v.max_iter > 0;
    st[ST_ITERS] = 0;
    st[ST_MAXIT] = v.max_iter;
    st[ST_FALLBACK] = 0;
    sc[SC_RTOL] = v.rtol;
    st[ST_FLAG] = (bb == 0.0) ? 0 : 1;
    st[ST_ACTIVE] = live ? 1 : 0;
    J.active_out[pr] = live ? 1 : 0;
  }
}

// The result of a device-steered solve into caller memory: {iterations,
// relative residual, flag} (the capturable solve).
__global__ void pcg_info_out_kernel(const int* __restrict__ state, const double* __restrict__ sc,
                                    double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  out[0] = (double)state[ST_ITERS];
  out[1] = sc[SC_RELRES];
  out[2] = (double)state[ST_FLAG];
}

hipError_t launch_pcg_info_out(const int* state, const double* sc, double* out, hipStream_t st) {
  hipLaunchKernelGGL(pcg_info_out_kernel, dim3(1), dim3(64), 0, st, state, sc, out);
  return hipGetLastError();
}

hipError_t launch_pcg_init_batch(const VecJobs& j, hipStream_t st) {
  hipLaunchKernelGGL(pcg_init_batch_kernel, dim3(j.prefix[j.n]), dim3(kVecBlock), 0, st, j);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pcg_init_finish_batch_kernel, dim3(j.n), dim3(256), 0, st, j);
  return hipGetLastError();
}

// alpha = r.z / p.q from the node-pass partials; breakdown ends the problem.
// One 1024-thread group per problem with two independent running sums per thread
// (a fixed order, so the result does not depend on timing).
__global__ __launch_bounds__(1024) void pcg_alpha_batch_kernel(const VecJobs J) {
  __shared__ double sred[16];
  const int pr = blockIdx.x;
  const VecJob& v = J.jobs[pr];
  if (!ld_coherent(v.state + ST_ACTIVE)) return;
  double a = 0.0, b = 0.0;
  int i = threadIdx.x;
  for (; i + 1024 < v.n_pq; i += 2048) {
    a += v.red_pq[i];
    b += v.red_pq[i + 1024];
  }
  if (i < v.n_pq) a += v.red_pq[i];
  const double pq = block_sum<1024>(a + b, sred);
  if (threadIdx.x == 0) {
    double* sc = v.sc;
    sc[SC_PQ] = pq;
    if (pq > 0.0 && isfinite(pq)) {
      sc[SC_ALPHA] = ld_coherent(sc + SC_RZ) / pq;
    } else {
      sc[SC_ALPHA] = 0.0;
      v.state[ST_FLAG] = 2;
      v.state[ST_ACTIVE] = 0;
      J.active_out[pr] = 0;
    }
  }
}

hipError_t launch_pcg_alpha_batch(const VecJobs& j, hipStream_t st) {
  hipLaunchKernelGGL(pcg_alpha_batch_kernel, dim3(j.n), dim3(1024), 0, st, j);
  return hipGetLastError();
}

__global__ __launch_bounds__(kVecBlock) void pcg_update_batch_kernel(const VecJobs J) {
  __shared__ double sred[kVecBlock / 64];
  const int pr = find_job(J.prefix, J.n, blockIdx.x);
  const VecJob& v = J.jobs[pr];
  if (!ld_coherent(v.state + ST_ACTIVE)) return;
  const int lb = blockIdx.x - J.prefix[pr], nb = J.prefix[pr + 1] - J.prefix[pr];
  const float alpha = (float)ld_coherent(v.sc + SC_ALPHA);
  double rr = 0.0, rz = 0.0;
  for (int i = lb * kVecBlock + threadIdx.x; i < v.n3; i += nb * kVecBlock) {
    const float ri = fmaf(-alpha, v.q[i], v.r[i]);
    v.s[i] = fmaf(alpha, v.p[i], v.s[i]);
    v.r[i] = ri;
    const float zi = v.diag ? ri / v.diag[i] : ri;
    v.z[i] = zi;
    rr += (double)ri * ri;
    rz += (double)ri * zi;
  }
  const double a = block_sum<kVecBlock>(rr, sred);
  const double b = block_sum<kVecBlock>(rz, sred);
  if (threadIdx.x == 0) {
    v.red[2 * lb] = a;
    v.red[2 * lb + 1] = b;
  }
}

hipError_t launch_pcg_update_batch(const VecJobs& j, hipStream_t st) {
  hipLaunchKernelGGL(pcg_update_batch_kernel, dim3(j.prefix[j.n]), dim3(kVecBlock), 0, st, j);
  return hipGetLastError();
}

// rr, rz_new, beta; convergence and iteration limit end the problem.
__global__ __launch_bounds__(256) void pcg_beta_batch_kernel(const VecJobs J) {
  __shared__ double sred[4];
  const int pr = blockIdx.x;
  const VecJob& v = J.jobs[pr];
  if (!ld_coherent(v.state + ST_ACTIVE)) return;
  const int nb = J.prefix[pr + 1] - J.prefix[pr];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += v.red[2 * i];
    b += v.red[2 * i + 1];
  }
  const double rr = block_sum<256>(a, sred);
  const double rz = block_sum<256>(b, sred);
  if (threadIdx.x == 0) {
    double* sc = v.sc;
    int* st = v.state;
    const double rz_old = ld_coherent(sc + SC_RZ), bb = ld_coherent(sc + SC_BB), rtol = ld_coherent(sc + SC_RTOL);
    const int iters = ld_coherent(st + ST_ITERS) + 1, maxit = ld_coherent(st + ST_MAXIT);
    sc[SC_RR] = rr;
    sc[SC_RZNEW] = rz;
    sc[SC_BETA] = rz / rz_old;
    sc[SC_RZ] = rz;
    st[ST_ITERS] = iters;
    const double rel = sqrt(rr) / sqrt(bb);
    sc[SC_RELRES] = rel;
    if (rel <= rtol) {
      st[ST_FLAG] = 0;
      st[ST_ACTIVE] = 0;
    } else if (iters >= maxit) {
      st[ST_FLAG] = 1;
      st[ST_ACTIVE] = 0;
    }
    J.active_out[pr] = (rel <= rtol || iters >= maxit) ? 0 : 1;
  }
}

hipError_t launch_pcg_beta_batch(const VecJobs& j, hipStream_t st) {
  hipLaunchKernelGGL(pcg_beta_batch_kernel, dim3(j.n), dim3(256), 0, st, j);
  return hipGetLastError();
}

__global__ __launch_bounds__(kVecBlock) void pcg_direction_batch_kernel(const VecJobs J) {
  const int pr = find_job(J.prefix, J.n, blockIdx.x);
  const VecJob& v = J.jobs[pr];
  if (!ld_coherent(v.state + ST_ACTIVE)) return;
  const int lb = blockIdx.x - J.prefix[pr], nb = J.prefix[pr + 1] - J.prefix[pr];
  const float beta = (float)ld_coherent(v.sc + SC_BETA);
  for (int i = lb * kVecBlock + threadIdx.x; i < v.n3; i += nb * kVecBlock) v.p[i] = fmaf(beta, v.p[i], v.z[i]);
}

hipError_t launch_pcg_direction_batch(const VecJobs& j, hipStream_t st) {
  hipLaunchKernelGGL(pcg_direction_batch_kernel, dim3(j.prefix[j.n]), dim3(kVecBlock), 0, st, j);
  return hipGetLastError();
}

}  // namespace mfr
