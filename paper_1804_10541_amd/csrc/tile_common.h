// Device helpers shared by the voxel-tile kernels.
#pragma once

#include "mfr_internal.h"

namespace mfr {
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NT>
__device__ __forceinline__ void block_sum_store(double v, double* out, double* sred) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sred[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += sred[w];
    *out = s;
  }
}

// XCD-aware block order: hardware dispatches block b to XCD b % 8, so give each
// XCD a contiguous range of tile ids (neighbouring tiles share its L2).
__device__ __forceinline__ int xcd_block_id() {
  const int G = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, per = G >> 3, rem = G & 7;
  return xcd * per + min(xcd, rem) + (b >> 3);
}

struct Tri {
  float v, gx, gy, gz;
};

// Trilinear sample of the zero-bordered template and its exact derivative.
// (kx, ky, kz) is the lower corner in template cells, (fx, fy, fz) the
// fractions; indices are clamped to [-2, mT] which only ever maps fully
// outside samples onto the zero border (value and derivative stay 0).
__device__ __forceinline__ Tri sample_template(const TileParams& P, int kx, int ky, int kz, float fx,
                                               float fy, float fz) {
  kx = min(max(kx, -2), P.mTx);
  ky = min(max(ky, -2), P.mTy);
  kz = min(max(kz, -2), P.mTz);
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
  Tri o;
  o.v = fmaf(fz, f1 - f0, f0);
  o.gz = (f1 - f0) * P.ihTz;
  o.gy = fmaf(fz, dy1 - dy0, dy0) * P.ihTy;
  o.gx = fmaf(fz, dxb - dxa, dxa) * P.ihTx;
  return o;
}


// Template coordinate along one axis for voxel-table entry s and displacement d:
// returns the lower template cell and writes the fraction.
__device__ __forceinline__ int template_cell(const Samp1 s, float d, float ihT, float& frac) {
  const float q = fminf(fmaxf(fmaf(d, ihT, s.frac), -1.0e7f), 1.0e7f);
  const float fl = floorf(q);
  frac = q - fl;
  return s.base + (int)fl;
}

// Weight of node index n for a voxel with conversion entry c (0 outside its pair).
__device__ __forceinline__ float conv_weight(const Conv1 c, int n) {
  return (c.n0 == n) ? 1.0f - c.f : ((c.n0 + 1 == n) ? c.f : 0.0f);
}

}  // namespace mfr
