// 3x3x3 convolutions of the learned preconditioner on the deformation-node
// grid, as implicit GEMMs on the bf16 matrix cores of gfx950
// (v_mfma_f32_16x16x32_bf16, fp32 accumulation).
//
// Layouts: activations channels-last [z][y][x][16] bf16 (one node = 32 bytes);
// weights [27 taps][16 in][16 out] bf16 with tap t = 9 (dz+1) + 3 (dy+1) + (dx+1);
// zero padding outside the grid.  One wave computes a 16 x 16 output tile:
// 16 output channels x 16 consecutive nodes of one x-row, reducing over
// K = 27 taps x 16 input channels = 14 MFMA steps of 32 (two taps each, the
// last half zero).  Operands: A = weights (row = output channel), B = the
// shifted activations (column = node), so each lane loads 16 contiguous bytes
// of one node per step and stores 4 contiguous output channels of one node.
#include <algorithm>

#include "mfr_internal.h"

namespace mfr {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kTaps = 27;
constexpr int kCh = 16;
constexpr int kSteps = 14;   // ceil(27 / 2)

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to nearest, ties to even; NaN stays NaN.
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ void tap_offset(int t, int& dz, int& dy, int& dx) {
  dz = t / 9 - 1;
  dy = (t / 3) % 3 - 1;
  dx = t % 3 - 1;
}

__device__ __forceinline__ bf16x8 zero8() {
  uint4 z = make_uint4(0u, 0u, 0u, 0u);
  return __builtin_bit_cast(bf16x8, z);
}

}  // namespace

// ---- forward and backward-data convolution --------------------------------------
__global__ __launch_bounds__(256) void cnn_conv_kernel(const ConvArgs a) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, quad = lane >> 4;
  const int nwaves = gridDim.x * 4;
  const int gxn = (a.nx + 15) >> 4;
  const int groups = gxn * a.ny * a.nz;
  const size_t nn = (size_t)a.nx * a.ny * a.nz;

  // A operand (weights): row = output channel col, k = 8 quad + e within the step:
  // tap 2 j + (quad >> 1), input channel 8 (quad & 1) + e.
  bf16x8 wa[kSteps];
#pragma unroll
  for (int j = 0; j < kSteps; ++j) {
    const int t = 2 * j + (quad >> 1);
    const int c0 = 8 * (quad & 1);
    if (t >= kTaps) {
      wa[j] = zero8();
    } else if (a.transpose) {
      // W'[t][c][o] = W[26 - t][o][c]: contiguous in c
      const uint4 v = *reinterpret_cast<const uint4*>(a.w + ((size_t)(kTaps - 1 - t) * kCh + col) * kCh + c0);
      wa[j] = __builtin_bit_cast(bf16x8, v);
    } else {
      uint16_t e[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) e[i] = a.w[((size_t)t * kCh + c0 + i) * kCh + col];
      uint4 v;
      v.x = e[0] | ((uint32_t)e[1] << 16);
      v.y = e[2] | ((uint32_t)e[3] << 16);
      v.z = e[4] | ((uint32_t)e[5] << 16);
      v.w = e[6] | ((uint32_t)e[7] << 16);
      wa[j] = __builtin_bit_cast(bf16x8, v);
    }
  }
  float bias[4] = {0.f, 0.f, 0.f, 0.f};
  if (a.bias) {
#pragma unroll
    for (int i = 0; i < 4; ++i) bias[i] = a.bias[4 * quad + i];
  }
  const float scale = a.z ? (float)*a.scale : 0.f;

  for (int g = blockIdx.x * 4 + (threadIdx.x >> 6); g < groups; g += nwaves) {
    const int gx = g % gxn;
    const int rest = g / gxn;
    const int y = rest % a.ny, z = rest / a.ny;
    const int x = gx * 16 + col;   // node of this lane's B column
    bf16x8 xb[kSteps];
#pragma unroll
    for (int j = 0; j < kSteps; ++j) {
      const int t = 2 * j + (quad >> 1);
      xb[j] = zero8();
      if (t < kTaps) {
        int dz, dy, dx;
        tap_offset(t, dz, dy, dx);
        const int xx = x + dx, yy = y + dy, zz = z + dz;
        if (x < a.nx && xx >= 0 && xx < a.nx && yy >= 0 && yy < a.ny && zz >= 0 && zz < a.nz) {
          const size_t node = ((size_t)zz * a.ny + yy) * a.nx + xx;
          xb[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(a.x + node * kCh + 8 * (quad & 1)));
        }
      }
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < kSteps; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[j], xb[j], acc, 0, 0, 0);
    if (x >= a.nx) continue;
    // this lane holds output channels 4 quad + i of node x
    const size_t node = ((size_t)z * a.ny + y) * a.nx + x;
    float v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = acc[i] + bias[i];
      if (a.relu) v[i] = fmaxf(v[i], 0.f);
    }
    if (a.mask) {
      const uint2 m = *reinterpret_cast<const uint2*>(a.mask + node * kCh + 4 * quad);
      const uint16_t mh[4] = {(uint16_t)(m.x & 0xffff), (uint16_t)(m.x >> 16), (uint16_t)(m.y & 0xffff),
                              (uint16_t)(m.y >> 16)};
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (!(bf2f(mh[i]) > 0.f)) v[i] = 0.f;
    }
    if (a.y16) {
      uint2 o;
      o.x = f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
      o.y = f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
      *reinterpret_cast<uint2*>(a.y16 + node * kCh + 4 * quad) = o;
    }
    if (a.y32) *reinterpret_cast<float4*>(a.y32 + node * kCh + 4 * quad) = make_float4(v[0], v[1], v[2], v[3]);
    if (a.z && quad == 0) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const size_t i = (size_t)d * nn + node;
        a.z[i] = fmaf(scale, v[d], a.r[i] / a.diag[i]);
      }
    }
  }
}

hipError_t launch_cnn_conv(const ConvArgs& a, hipStream_t st) {
  const long groups = (long)((a.nx + 15) / 16) * a.ny * a.nz;
  const int blocks = (int)std::min<long>((groups + 3) / 4, 4096);
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(cnn_conv_kernel, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---- weight and bias gradients ---------------------------------------------------
// dW[t][c][o] = sum_n x[n + off_t][c] g[n][o], db[o] = sum_n g[n][o].  A work-group
// takes segments of 32 nodes of one x-row: it stages the 3 x 3 neighbouring rows
// of x (34 nodes each, zero outside) and the segment of g in LDS; wave w owns the
// taps t = w (mod 4) and accumulates D[c][o] over K = 32 nodes per MFMA.
// Per-group partials (fp32, fixed layout) are summed in a fixed order afterwards.
constexpr int kSeg = 32;
constexpr int kSegW = kSeg + 2;
constexpr int kTapsPerWave = 7;

__global__ __launch_bounds__(256) void cnn_wgrad_kernel(int nx, int ny, int nz, const uint16_t* __restrict__ x,
                                                        const uint16_t* __restrict__ g, float* __restrict__ part) {
  __shared__ __align__(16) uint16_t xs[9][kSegW][kCh];
  __shared__ __align__(16) uint16_t gs[kSeg][kCh];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, quad = lane >> 4;
  const int sxn = (nx + kSeg - 1) / kSeg;
  const int nseg = sxn * ny * nz;
  f32x4 acc[kTapsPerWave];
#pragma unroll
  for (int i = 0; i < kTapsPerWave; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  float db = 0.f;

  for (int s = blockIdx.x; s < nseg; s += gridDim.x) {
    const int sx = s % sxn, rest = s / sxn;
    const int y = rest % ny, z = rest / ny;
    const int x0 = sx * kSeg;
    // stage x: 9 rows x 34 nodes x 2 halves of 16 bytes
    for (int q = tid; q < 9 * kSegW * 2; q += 256) {
      const int row = q / (kSegW * 2), w = q % (kSegW * 2);
      const int ni = w >> 1, half = w & 1;
      const int xx = x0 - 1 + ni, yy = y + row % 3 - 1, zz = z + row / 3 - 1;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (xx >= 0 && xx < nx && yy >= 0 && yy < ny && zz >= 0 && zz < nz)
        v = *reinterpret_cast<const uint4*>(x + (((size_t)zz * ny + yy) * nx + xx) * kCh + 8 * half);
      *reinterpret_cast<uint4*>(&xs[row][ni][8 * half]) = v;
    }
    if (tid < kSeg * 2) {
      const int ni = tid >> 1, half = tid & 1;
      const int xx = x0 + ni;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (xx < nx) v = *reinterpret_cast<const uint4*>(g + (((size_t)z * ny + y) * nx + xx) * kCh + 8 * half);
      *reinterpret_cast<uint4*>(&gs[ni][8 * half]) = v;
    }
    __syncthreads();
    // B operand: g[n][o], column o = col, k = node 8 quad + e
    uint16_t be[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) be[e] = gs[8 * quad + e][col];
    uint4 bv;
    bv.x = be[0] | ((uint32_t)be[1] << 16);
    bv.y = be[2] | ((uint32_t)be[3] << 16);
    bv.z = be[4] | ((uint32_t)be[5] << 16);
    bv.w = be[6] | ((uint32_t)be[7] << 16);
    const bf16x8 B = __builtin_bit_cast(bf16x8, bv);
#pragma unroll
    for (int i = 0; i < kTapsPerWave; ++i) {
      const int t = wave + 4 * i;
      if (t < kTaps) {
        int dz, dy, dx;
        tap_offset(t, dz, dy, dx);
        const int row = (dz + 1) * 3 + (dy + 1);
        // A operand: x[n + off_t][c], row c = col, k = node 8 quad + e
        uint16_t ae[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) ae[e] = xs[row][8 * quad + e + dx + 1][col];
        uint4 av;
        av.x = ae[0] | ((uint32_t)ae[1] << 16);
        av.y = ae[2] | ((uint32_t)ae[3] << 16);
        av.z = ae[4] | ((uint32_t)ae[5] << 16);
        av.w = ae[6] | ((uint32_t)ae[7] << 16);
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), B, acc[i], 0, 0, 0);
      }
    }
    if (tid < kCh) {
      for (int n = 0; n < kSeg; ++n) db += bf2f(gs[n][tid]);
    }
    __syncthreads();
  }
  float* p = part + (size_t)blockIdx.x * kCnnLayerParams;
#pragma unroll
  for (int i = 0; i < kTapsPerWave; ++i) {
    const int t = wave + 4 * i;
    if (t < kTaps) {
#pragma unroll
      for (int r = 0; r < 4; ++r) p[(size_t)t * kCh * kCh + (4 * quad + r) * kCh + col] = acc[i][r];
    }
  }
  if (tid < kCh) p[kTaps * kCh * kCh + tid] = db;
}

// out[i] = sum over groups b (in order) of part[b][i]
__global__ __launch_bounds__(256) void cnn_wgrad_reduce_kernel(const float* __restrict__ part, int groups,
                                                               float* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kCnnLayerParams) return;
  float s = 0.f;
  for (int b = 0; b < groups; ++b) s += part[(size_t)b * kCnnLayerParams + i];
  out[i] = s;
}

int cnn_wgrad_groups(int nx, int ny, int nz) {
  const long nseg = (long)((nx + kSeg - 1) / kSeg) * ny * nz;
  return (int)std::max<long>(1, std::min<long>(nseg, 512));
}

hipError_t launch_cnn_wgrad(int nx, int ny, int nz, const uint16_t* x, const uint16_t* g, float* part,
                            float* out, hipStream_t st) {
  const int groups = cnn_wgrad_groups(nx, ny, nz);
  hipLaunchKernelGGL(cnn_wgrad_kernel, dim3(groups), dim3(256), 0, st, nx, ny, nz, x, g, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cnn_wgrad_reduce_kernel, dim3((kCnnLayerParams + 255) / 256), dim3(256), 0, st, part, groups,
                     out);
  return hipGetLastError();
}

// ---- parameters: bf16 copies and Adam --------------------------------------------
// Parameter vector: per layer [27][16][16] weights then [16] biases.  The output
// channels 3..15 of the last layer are unused and held at zero.
__device__ __forceinline__ bool frozen_param(int i) {
  const int layer = i / kCnnLayerParams, j = i % kCnnLayerParams;
  if (layer != kCnnLayers - 1) return false;
  const int o = j < kCnnWeights ? j % kCh : j - kCnnWeights;
  return o >= 3;
}

__global__ __launch_bounds__(256) void cnn_cast_kernel(float* __restrict__ p, uint16_t* __restrict__ w16) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kCnnParams) return;
  if (frozen_param(i)) p[i] = 0.f;
  const int layer = i / kCnnLayerParams, j = i % kCnnLayerParams;
  if (j < kCnnWeights) w16[(size_t)layer * kCnnWeights + j] = f2bf(p[i]);
}

hipError_t launch_cnn_cast(float* params, uint16_t* w16, hipStream_t st) {
  hipLaunchKernelGGL(cnn_cast_kernel, dim3((kCnnParams + 255) / 256), dim3(256), 0, st, params, w16);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void cnn_adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                       float* __restrict__ m, float* __restrict__ v,
                                                       uint16_t* __restrict__ w16, AdamArgs h) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kCnnParams) return;
  float pi = p[i];
  if (!frozen_param(i)) {
    const float gi = g[i];
    const float mi = fmaf(h.beta1, m[i], (1.0f - h.beta1) * gi);
    const float vi = fmaf(h.beta2, v[i], (1.0f - h.beta2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    pi -= h.lr * (mi / h.bc1) / (sqrtf(vi / h.bc2) + h.eps);
  } else {
    pi = 0.f;
  }
  p[i] = pi;
  const int layer = i / kCnnLayerParams, j = i % kCnnLayerParams;
  if (j < kCnnWeights) w16[(size_t)layer * kCnnWeights + j] = f2bf(pi);
}

hipError_t launch_cnn_adam(float* p, const float* g, float* m, float* v, uint16_t* w16, const AdamArgs& h,
                           hipStream_t st) {
  hipLaunchKernelGGL(cnn_adam_kernel, dim3((kCnnParams + 255) / 256), dim3(256), 0, st, p, g, m, v, w16, h);
  return hipGetLastError();
}

}  // namespace mfr
