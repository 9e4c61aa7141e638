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

// Two consecutive floats loaded together (one 8-byte load; 4-byte alignment
// suffices on this GPU).
struct __attribute__((aligned(4))) FPair {
  float a, b;
};

// Loads the 8 corner samples of the zero-bordered template for the cell with
// lower corner (kx, ky, kz) (template cells).  Indices are clamped to [-2, mT],
// which only ever maps fully outside samples onto the zero border, so value
// and derivative stay exactly 0 there (the Dirichlet extension).
__device__ __forceinline__ void template_corners(const TileParams& P, int kx, int ky, int kz, float (&t)[8]) {
  kx = min(max(kx, -2), P.mTx);
  ky = min(max(ky, -2), P.mTy);
  kz = min(max(kz, -2), P.mTz);
  const float* b0 = P.Tp + (size_t)(kz + 2) * (size_t)P.PXY + (size_t)((ky + 2) * P.PX + (kx + 2));
  const float* b1 = b0 + P.PXY;
  // x-pairs of corners with one 8-byte load each (4-byte alignment suffices)
  const FPair a = *reinterpret_cast<const FPair*>(b0), b = *reinterpret_cast<const FPair*>(b0 + P.PX);
  const FPair c = *reinterpret_cast<const FPair*>(b1), d = *reinterpret_cast<const FPair*>(b1 + P.PX);
  t[0] = a.a;
  t[1] = a.b;
  t[2] = b.a;
  t[3] = b.b;
  t[4] = c.a;
  t[5] = c.b;
  t[6] = d.a;
  t[7] = d.b;
}

// Trilinear value and exact derivative from the 8 corners (x fastest) and
// the fractions (fx, fy, fz); the derivative is scaled by 1/hT.
__device__ __forceinline__ Tri trilinear(const TileParams& P, const float (&t)[8], float fx, float fy, float fz) {
  const float d00 = t[1] - t[0], d10 = t[3] - t[2], d01 = t[5] - t[4], d11 = t[7] - t[6];
  const float e00 = fmaf(fx, d00, t[0]), e10 = fmaf(fx, d10, t[2]);
  const float e01 = fmaf(fx, d01, t[4]), e11 = fmaf(fx, d11, t[6]);
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

// Loads of a float at a 32-bit byte offset from a uniform base pointer (the
// library limits images and node vectors to < 2^32 bytes, checked on the host).
__device__ __forceinline__ float ld32(const float* __restrict__ base, unsigned idx) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (idx << 2));
}

// Two consecutive floats at a 32-bit element offset: one 8-byte load (4-byte
// alignment suffices on this GPU), which halves the address work of a gather
// in the texture addresser (the voxel-tile kernel's vector-memory bottleneck).
__device__ __forceinline__ FPair ld32x2(const float* __restrict__ base, unsigned idx) {
  return *reinterpret_cast<const FPair*>(reinterpret_cast<const char*>(base) + (idx << 2));
}

// template_corners with 32-bit offsets; the x-pairs of corners are loaded together.
__device__ __forceinline__ void template_corners32(const TileParams& P, int kx, int ky, int kz, float (&t)[8]) {
  kx = min(max(kx, -2), P.mTx);
  ky = min(max(ky, -2), P.mTy);
  kz = min(max(kz, -2), P.mTz);
  const unsigned PX = (unsigned)P.PX, PXY = (unsigned)P.PXY;
  const unsigned i0 = (unsigned)(kz + 2) * PXY + (unsigned)__mul24(ky + 2, (int)PX) + (unsigned)(kx + 2);
  const unsigned i1 = i0 + PXY;
  const FPair a = ld32x2(P.Tp, i0), b = ld32x2(P.Tp, i0 + PX), c = ld32x2(P.Tp, i1), d = ld32x2(P.Tp, i1 + PX);
  t[0] = a.a;
  t[1] = a.b;
  t[2] = b.a;
  t[3] = b.b;
  t[4] = c.a;
  t[5] = c.b;
  t[6] = d.a;
  t[7] = d.b;
}

__device__ __forceinline__ Tri sample_template(const TileParams& P, int kx, int ky, int kz, float fx, float fy,
                                               float fz) {
  float t[8];
  template_corners(P, kx, ky, kz, t);
  return trilinear(P, t, fx, fy, fz);
}

// floor(q) as an integer in one instruction (convert with round-down).
__device__ __forceinline__ int floor_to_int(float q) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(q));
  return r;
}

// max(-2, min(k, hi)) for hi >= -2 in one instruction.
__device__ __forceinline__ int clamp_m2(int k, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, -2, %2" : "=v"(r) : "v"(k), "s"(hi));
  return r;
}

// Template coordinate along one axis for voxel-table entry s and displacement d:
// returns the lower template cell and writes the fraction (q - floor(q), at most
// the float below 1).
__device__ __forceinline__ int template_cell(const Samp1 s, float d, float ihT, float& frac) {
  const float q = __builtin_amdgcn_fmed3f(fmaf(d, ihT, s.frac), -1.0e7f, 1.0e7f);
  frac = __builtin_amdgcn_fractf(q);
  return s.base + floor_to_int(q);
}

// 1/sqrt(x) by the hardware reciprocal square root.  Its NGF arguments are
// sums of squares plus tau^2 or rho^2, which the host raises to at least the
// smallest normal float, so no denormal ever reaches it.
__device__ __forceinline__ float rsq_norm(float x) { return __builtin_amdgcn_rsqf(x); }

// Buffer descriptor of a raw float array of `bytes` bytes: loads at byte
// offsets voffset (vector) + soffset (scalar); loads past the end return 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const float* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float buf_ld(const __amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 0));
}

__device__ __forceinline__ FPair buf_ld2(const __amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(FPair, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}

// The eight corners of the template cell (kx, ky, kz) through the template's
// buffer descriptor: one vector byte offset for the lower x-pair of corners,
// the other three x-pairs at the scalar offsets of the next row, plane and both.
struct CornerOffsets {
  unsigned row, plane, both;   // bytes: 4 PX, 4 PXY, 4 (PX + PXY)
};
__device__ __forceinline__ void template_corners_buf(const TileParams& P, const __amdgpu_buffer_rsrc_t rs,
                                                     const CornerOffsets o, int kx, int ky, int kz, float (&t)[8]) {
  kx = clamp_m2(kx, P.mTx);
  ky = clamp_m2(ky, P.mTy);
  kz = clamp_m2(kz, P.mTz);
  // a 24-bit multiply (full rate) for planes below 2^24 elements, else a 32-bit one
  const unsigned zo = P.pxy24 ? __umul24((unsigned)(kz + 2), (unsigned)P.PXY) : (unsigned)(kz + 2) * (unsigned)P.PXY;
  const unsigned i0 = zo + __umul24((unsigned)(ky + 2), (unsigned)P.PX) + (unsigned)(kx + 2);
  const unsigned v = i0 << 2;
  const FPair a = buf_ld2(rs, v, 0), b = buf_ld2(rs, v, o.row), c = buf_ld2(rs, v, o.plane), d = buf_ld2(rs, v, o.both);
  t[0] = a.a;
  t[1] = a.b;
  t[2] = b.a;
  t[3] = b.b;
  t[4] = c.a;
  t[5] = c.b;
  t[6] = d.a;
  t[7] = d.b;
}

// Weight of node index n for a voxel with conversion entry c (0 outside its pair).
__device__ __forceinline__ float conv_weight(const Conv1 c, int n) {
  return (c.n0 == n) ? 1.0f - c.f : ((c.n0 + 1 == n) ? c.f : 0.0f);
}

}  // namespace mfr
