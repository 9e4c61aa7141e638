// 3x3x3 convolutions of the learned preconditioner on the deformation-node
// grid, as implicit GEMMs on the bf16 matrix cores of gfx950
// (v_mfma_f32_16x16x32_bf16, fp32 accumulation).
//
// Layouts: activations channels-last [z][y][x][16] bf16 (one node = 32 bytes);
// weights [27 taps][16 in][16 out] bf16 with tap t = 9 (dz+1) + 3 (dy+1) + (dx+1);
// zero padding outside the grid.  One MFMA computes 16 output channels x 16
// consecutive nodes of one x-row over K = 32: two taps x 16 input channels.
// Operands: A = weights (row = output channel), B = the shifted activations
// (column = node), so each lane loads 16 contiguous bytes of one node and
// stores 4 contiguous output channels of one node.
#include <algorithm>

#include "mfr_internal.h"
#include "tile_common.h"

namespace mfr {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2;
typedef short __attribute__((ext_vector_type(2))) s16x2;

constexpr int kTaps = 27;
constexpr int kCh = 16;
constexpr int kTx = 16, kTy = 8, kTz = 4;   // output tile of the convolution kernel
constexpr int kHx = kTx + 2, kHy = kTy + 2, kHz = kTz + 2;   // with its one-node halo
constexpr int kTile = kTx * kTy * kTz;
static_assert(kTz == 4 && kTile % 256 == 0, "one wave per z plane of the tile");
static_assert(3 * kTile * 4 <= kHz * kHy * kHx * 32, "the last layer stages z over the input tile");
// The nine (dz, dx) offsets m = 3 (dz+1) + (dx+1) go in pairs (2p, 2p+1) into
// the two K halves of an MFMA; m = 9 is a zero-weight half.  The three dy
// offsets of a pair share one activation load per x-row.
constexpr int kPairs = 5;

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

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

}  // namespace

// ---- forward and backward-data convolution --------------------------------------
// One kernel body, specialised per use so that each instance keeps only the
// registers and branches it needs: kGeneric takes every option at run time (the
// public convolution entry points); the others are the preconditioner's own
// layers with out-major weights: kHidden (bf16 input; ReLU; bf16 output), kLast
// (bf16 input; output z = r / diag + scale * y[0..2]) and kBwd (transposed
// weights, ReLU mask, bf16 output: backward-data of the training pass) and
// kFirst (kHidden whose input, the network features, is computed from r, the
// diagonal and |grad R| while the tile is staged: no separate feature pass).
//
// A work-group takes output tiles of 16 (x) x 8 (y) x 4 (z) nodes; wave w owns
// the plane z = w of the tile, eight x-rows with one accumulator each.  For each
// (dz, dx) pair the wave walks the ten staged rows y = -1 .. 8 of its shifted
// planes once: the activations of row s serve dy = -1, 0, +1 of output rows
// s, s - 1, s - 2 (three MFMAs per LDS load).
enum ConvMode : int { kGeneric = 0, kFirst = 1, kHidden = 2, kLast = 3, kBwd = 4 };

template <int kMode>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void cnn_conv_kernel(const ConvArgs a) {
  constexpr bool kRelu = kMode == kHidden || kMode == kFirst;
  constexpr bool kOutZ = kMode == kLast;
  constexpr bool kOut16 = kMode == kHidden || kMode == kFirst || kMode == kBwd;
  constexpr bool kFeat = kMode == kFirst;
  if (a.live && !ld_coherent(a.live)) return;   // a device-steered solve has stopped
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = lane & 15, quad = lane >> 4;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int nn = nx * ny * nz;   // < 2^26 nodes
  const bool transpose = kMode == kBwd || (kMode == kGeneric && a.transpose);
  const bool out_major = kMode == kHidden || kMode == kFirst || kMode == kLast || (kMode == kGeneric && a.w_out_major);

  // LDS: the A operands [pair][dy][quad][row][8 k] (a lane's 16 bytes of one
  // step are contiguous, a wave's 1 KB too), and the input tile with its halo
  // as [z][y][channel half][x][8], so that the 16 lanes of one half read 256
  // contiguous bytes.
  __shared__ __align__(16) uint16_t wl[kPairs][3][4][kCh][8];
  __shared__ __align__(16) uint16_t xs[kHz][kHy][2][kHx][8];
  constexpr int kWChunks = kPairs * 3 * 4 * kCh;   // 16-byte chunks of wl
  constexpr int kWPer = (kWChunks + 255) / 256;
  constexpr unsigned kNowhere = 0x80000000u;   // past every array here (< 2^26 nodes of 32 bytes)
  const __amdgpu_buffer_rsrc_t rx = raw_buffer(reinterpret_cast<const float*>(a.x), (unsigned)nn * 32u);
  // inputs of the first layer's features (r, diag: 3 x nn floats; |grad R|: nn)
  __amdgpu_buffer_rsrc_t rr = rx, rd = rx, rg = rx;
  if constexpr (kFeat) {
    rr = raw_buffer(a.fr, (unsigned)nn * 12u);
    rd = raw_buffer(a.fdiag, (unsigned)nn * 12u);
    rg = raw_buffer(a.fgR, (unsigned)nn * 4u);
  }
  // halo staging by rows: 36 chunks of 16 bytes per staged x-row, 7 rows per pass
  constexpr int kRowChunks = 2 * kHx, kRowStep = 256 / kRowChunks, kRows = kHz * kHy;
  constexpr int kRowPasses = (kRows + kRowStep - 1) / kRowStep;
  constexpr int kRowBytes = 2 * kHx * 16;
  static_assert(kRowStep < kHy, "one carry per pass at most");
  const int srow_r0 = tid / kRowChunks, srow_c = tid % kRowChunks;
  const bool srow_ok = srow_r0 < kRowStep;   // the last 256 - 7 * 36 threads stage nothing
  const int srow_x = srow_c >> 1;
  const unsigned srow_half16 = 16u * (srow_c & 1);
  unsigned char* const srow_lds = reinterpret_cast<unsigned char*>(&xs[0][0][0][0][0]) + srow_r0 * kRowBytes +
                                  ((srow_c & 1) * kHx + srow_x) * 16;

  // weight chunk q of this thread: its tap, or -1 for the zero half
  auto w_tap = [&](int q) {
    const int p = q / 192, dyi = (q / 64) % 3, qd = (q / 16) % 4;
    const int m = 2 * p + (qd >> 1);
    return m > 8 ? -1 : 9 * (m / 3) + 3 * dyi + m % 3;
  };
  if (!(transpose || out_major)) {
    // in-major forward weights [t][in][out] (public entry point): gather each
    // row's input channels; once per work-group
    for (int q = tid; q < kWChunks; q += 256) {
      const int t = w_tap(q), row = q % 16, c0 = 8 * ((q / 16) % 2);
      uint16_t* dst = &wl[0][0][0][0][0] + 8 * q;
#pragma unroll
      for (int e = 0; e < 8; ++e) dst[e] = t < 0 ? (uint16_t)0 : a.w[((size_t)t * kCh + c0 + e) * kCh + row];
    }
  }
  float bias[4] = {0.f, 0.f, 0.f, 0.f};
  if (a.bias) {
    const float4 b4 = *reinterpret_cast<const float4*>(a.bias + 4 * quad);
    bias[0] = b4.x;
    bias[1] = b4.y;
    bias[2] = b4.z;
    bias[3] = b4.w;
  }
  float scale = 0.f;
  if constexpr (kOutZ) scale = (float)ld_coherent(a.scale);
  // feature scales: 1 / RMS of r / diag, r, diag and |grad R| (0 for a zero RMS)
  float fs[4] = {0.f, 0.f, 0.f, 0.f};
  if constexpr (kFeat) {
    const int slot[4] = {PC_RMS_Y, PC_RMS_R, PC_RMS_D, PC_RMS_G};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double sv = ld_coherent(a.fsc + slot[i]);
      fs[i] = sv > 0.0 ? (float)(1.0 / sv) : 0.f;
    }
  }
  double zr = 0.0, zrp = 0.0;

  const int tnx = (nx + kTx - 1) / kTx, tny = (ny + kTy - 1) / kTy, tnz = (nz + kTz - 1) / kTz;
  const int tiles = tnx * tny * tnz;
  bool first = true;
#pragma clang loop unroll(disable)
  for (int tile = xcd_block_id(); tile < tiles; tile += gridDim.x) {
    const int x0 = (tile % tnx) * kTx, y0 = ((tile / tnx) % tny) * kTy, z0 = (tile / (tnx * tny)) * kTz;
    // all loads first (the weights with the first tile), then the LDS stores:
    // one memory latency per tile
    uint4 wv[kWPer];
    if (first && (transpose || out_major)) {
#pragma unroll
      for (int k = 0; k < kWPer; ++k) {
        const int q = tid + 256 * k;
        wv[k] = make_uint4(0u, 0u, 0u, 0u);
        if (q < kWChunks) {
          const int t = w_tap(q);
          if (t >= 0)
            wv[k] = *reinterpret_cast<const uint4*>(a.w + ((unsigned)(transpose ? kTaps - 1 - t : t) * kCh * kCh +
                                                            (q % 16) * kCh + 8 * ((q / 16) % 2)));
        }
      }
    }
    // network input of the halo nodes (kFirst): r, diag and |grad R| of node x
    // = tid % 18 of the staged rows tid / 18, + 14, ... (zero outside the grid,
    // where a node gets an offset past the arrays)
    constexpr int kFStep = 256 / kHx, kFPasses = (kRows + kFStep - 1) / kFStep;
    static_assert(kFStep < 2 * kHy, "at most two carries per pass");
    float fin[kFeat ? kFPasses : 1][7];
    bool fok[kFeat ? kFPasses : 1];
    if constexpr (kFeat) {
      const int fr0 = tid / kHx, fx = tid % kHx;
      const int fxx = x0 + fx - 1;
      const bool fxok = fr0 < kFStep && (unsigned)fxx < (unsigned)nx;
#pragma unroll
      for (int j = 0, ly = fr0 % kHy, lz = fr0 / kHy; j < kFPasses; ++j) {
        const int yy = y0 + ly - 1, zz = z0 + lz - 1;
        fok[j] = fxok && lz < kHz && (unsigned)yy < (unsigned)ny && (unsigned)zz < (unsigned)nz;
        const unsigned o = fok[j] ? 4u * (unsigned)((zz * ny + yy) * nx + fxx) : kNowhere;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          fin[j][d] = buf_ld(rr, o, 4u * d * nn);
          fin[j][3 + d] = buf_ld(rd, o, 4u * d * nn);
        }
        fin[j][6] = buf_ld(rg, o, 0u);
        ly += kFStep % kHy;   // the next row of this thread: row + 14
        lz += kFStep / kHy;
        if (ly >= kHy) {
          ly -= kHy;
          ++lz;
        }
      }
    }
    // halo chunks through a buffer descriptor: a chunk outside the grid gets an
    // offset past the array's end, for which the hardware returns zeros.  Thread
    // (r0, c) = (tid / 36, tid % 36) loads chunk c (x = c / 2, channel half c % 2)
    // of the staged rows r0, r0 + 7, ... (row = lz * kHy + ly)
    uint4 v[kRowPasses];
    const int xx = x0 + srow_x - 1;
    const bool xok = srow_ok && (unsigned)xx < (unsigned)nx;
#pragma unroll
    for (int j = 0, ly = srow_r0, lz = 0; j < (kFeat ? 0 : kRowPasses); ++j) {
      const int yy = y0 + ly - 1, zz = z0 + lz - 1;
      const bool ok = xok && lz < kHz && (unsigned)yy < (unsigned)ny && (unsigned)zz < (unsigned)nz;
      const unsigned off = ok ? (unsigned)((zz * ny + yy) * nx + xx) * 32u + srow_half16 : kNowhere;
      v[j] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rx, (int)off, 0, 0));
      ly += kRowStep;   // the next row of this thread: row + 7
      if (ly >= kHy) {
        ly -= kHy;
        ++lz;
      }
    }
    if (first && (transpose || out_major)) {
#pragma unroll
      for (int k = 0; k < kWPer; ++k) {
        const int q = tid + 256 * k;
        if (q < kWChunks) *reinterpret_cast<uint4*>(&wl[0][0][0][0][0] + 8 * q) = wv[k];
      }
    }
    first = false;
    if constexpr (kFeat) {
      // channels (r/diag)/rms_y [0..2], r/rms_r [3..5], diag/rms_d [6..8],
      // |grad R|/rms_g [9], zero [10..15], rounded to bf16 (to nearest even)
      const int fr0 = tid / kHx, fx = tid % kHx;
#pragma unroll
      for (int j = 0; j < kFPasses; ++j) {
        const int row = fr0 + kFStep * j;
        if (fr0 < kFStep && row < kRows) {
          uint4 lo = make_uint4(0u, 0u, 0u, 0u), hi = make_uint4(0u, 0u, 0u, 0u);
          if (fok[j]) {
            float f[10];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              f[d] = (fin[j][d] / fin[j][3 + d]) * fs[0];
              f[3 + d] = fin[j][d] * fs[1];
              f[6 + d] = fin[j][3 + d] * fs[2];
            }
            f[9] = fin[j][6] * fs[3];
            auto pk = [](float u, float w) {
              return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){u, w}, bf16x2));
            };
            lo = make_uint4(pk(f[0], f[1]), pk(f[2], f[3]), pk(f[4], f[5]), pk(f[6], f[7]));
            hi = make_uint4(pk(f[8], f[9]), 0u, 0u, 0u);
          }
          *reinterpret_cast<uint4*>(&xs[0][0][0][0][0] + 8 * (row * 2 * kHx + fx)) = lo;
          *reinterpret_cast<uint4*>(&xs[0][0][0][0][0] + 8 * ((row * 2 + 1) * kHx + fx)) = hi;
        }
      }
    }
    if (srow_ok) {
#pragma unroll
      for (int j = 0; j < (kFeat ? 0 : kRowPasses); ++j)
        if (srow_r0 + kRowStep * j < kRows) *reinterpret_cast<uint4*>(srow_lds + j * kRowStep * kRowBytes) = v[j];
    }
    __syncthreads();
    // row s first receives pair 0, dy = -1 at staged row s: that MFMA starts from 0
    f32x4 acc[kTy];
    const f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
      // this lane's (dz, dx): the first or second member of the pair; the zero
      // half reads any staged row (its weights are zero)
      const int m0 = 2 * p + (quad >> 1), m = m0 > 8 ? 4 : m0;
      const uint16_t* brow = &xs[wave + m / 3][0][quad & 1][col + m % 3][0];
      const uint4 a0 = *reinterpret_cast<const uint4*>(&wl[p][0][quad][col][0]);
      const uint4 a1 = *reinterpret_cast<const uint4*>(&wl[p][1][quad][col][0]);
      const uint4 a2 = *reinterpret_cast<const uint4*>(&wl[p][2][quad][col][0]);
#pragma unroll
      for (int s = 0; s < kHy; ++s) {
        const uint4 b = *reinterpret_cast<const uint4*>(brow + s * (2 * kHx * 8));
        if (s < kTy)
          acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a0), as_bf16x8(b), p == 0 ? zero4 : acc[s], 0, 0, 0);
        if (s >= 1 && s <= kTy)
          acc[s - 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a1), as_bf16x8(b), acc[s - 1], 0, 0, 0);
        if (s >= 2)
          acc[s - 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a2), as_bf16x8(b), acc[s - 2], 0, 0, 0);
      }
    }
    if constexpr (kOutZ) {
      // z = r / diag + scale * y[0..2] over the whole tile: the three channels go
      // through LDS (over the staged input) so that every lane takes one node
      __syncthreads();
      float* zs = reinterpret_cast<float*>(&xs[0][0][0][0][0]);   // [3][kTile]
      if (quad == 0) {
#pragma unroll
        for (int i = 0; i < kTy; ++i) {
          const int nl = (wave * kTy + i) * kTx + col;
#pragma unroll
          for (int r = 0; r < 3; ++r) zs[r * kTile + nl] = acc[i][r] + bias[r];
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kTile / 256; ++k) {
        const int nl = tid + 256 * k, row = nl / kTx;
        const int x = x0 + nl % kTx, y = y0 + row % kTy, z = z0 + row / kTy;
        if (x < nx && y < ny && z < nz) {
          const int node = (z * ny + y) * nx + x;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int id = d * nn + node;
            const float rv = a.r[id];
            const float zi = fmaf(scale, zs[d * kTile + nl], rv / a.diag[id]);
            a.z[id] = zi;
            if (a.zred) {
              zr += (double)zi * rv;
              zrp += (double)zi * a.rprev[id];
            }
          }
        }
      }
    } else {
      // this lane holds output channels 4 quad + r of node (x0 + col, y0 + i, z0 + w)
      const int x = x0 + col, z = z0 + wave;
      const int rows = min(kTy, ny - y0);   // wave-uniform
      if (x < nx && z < nz) {
        unsigned node = (unsigned)((z * ny + y0) * nx + x);
#pragma unroll
        for (int i = 0; i < kTy; ++i, node += nx) {
          if (i >= rows) break;
          float v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            v[r] = acc[i][r] + bias[r];
            if (kMode == kGeneric && a.relu) v[r] = fmaxf(v[r], 0.f);
          }
          if (kMode == kBwd || (kMode == kGeneric && a.mask)) {
            const uint2 mk = *reinterpret_cast<const uint2*>(a.mask + (node * kCh + 4 * quad));
            const uint16_t mh[4] = {(uint16_t)(mk.x & 0xffff), (uint16_t)(mk.x >> 16), (uint16_t)(mk.y & 0xffff),
                                    (uint16_t)(mk.y >> 16)};
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (!(bf2f(mh[r]) > 0.f)) v[r] = 0.f;
          }
          if (kOut16 || (kMode == kGeneric && a.y16)) {
            // round to nearest even in hardware (the same rounding as f2bf for non-NaN values)
            s16x2 lo = __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2){v[0], v[1]}, bf16x2));
            s16x2 hi = __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2){v[2], v[3]}, bf16x2));
            if constexpr (kRelu) {
              // ReLU on the rounded values, two per instruction: a bf16 pattern is
              // negative exactly when it is negative as a 16-bit integer (NaN
              // patterns with the sign clear pass through, as the reference's max)
              const s16x2 z2 = {0, 0};
              lo = __builtin_elementwise_max(lo, z2);
              hi = __builtin_elementwise_max(hi, z2);
            }
            *reinterpret_cast<uint2*>(a.y16 + (node * kCh + 4 * quad)) =
                make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
          }
          if (kMode == kGeneric && a.y32)
            *reinterpret_cast<float4*>(a.y32 + (node * kCh + 4 * quad)) = make_float4(v[0], v[1], v[2], v[3]);
        }
      }
    }
    __syncthreads();   // the next tile overwrites the staged input
  }
  if (kOutZ && a.zred) {   // per-group partials of z.r and z.r_prev (flexible CG)
    __shared__ double sred[2][4];
    zr = wave_sum(zr);
    zrp = wave_sum(zrp);
    if (lane == 0) {
      sred[0][wave] = zr;
      sred[1][wave] = zrp;
    }
    __syncthreads();
    if (tid == 0) {
      a.zred[2 * blockIdx.x] = (sred[0][0] + sred[0][1]) + (sred[0][2] + sred[0][3]);
      a.zred[2 * blockIdx.x + 1] = (sred[1][0] + sred[1][1]) + (sred[1][2] + sred[1][3]);
    }
  }
}

int cnn_conv_blocks(int nx, int ny, int nz) {
  const long tiles = (long)((nx + kTx - 1) / kTx) * ((ny + kTy - 1) / kTy) * ((nz + kTz - 1) / kTz);
  return (int)std::min<long>(tiles, kCnnMaxConvGroups);
}

hipError_t launch_cnn_conv(const ConvArgs& a, hipStream_t st) {
  const int blocks = cnn_conv_blocks(a.nx, a.ny, a.nz);
  if (blocks <= 0) return hipSuccess;
  int mode = kGeneric;
  if (!a.y32 && a.bias) {
    if (!a.transpose && a.w_out_major && !a.mask) {
      if (a.x && a.relu && a.y16 && !a.z) mode = kHidden;
      else if (a.x && !a.relu && !a.y16 && a.z) mode = kLast;
      else if (!a.x && a.fr && a.fdiag && a.fgR && a.fsc && a.relu && a.y16 && !a.z) mode = kFirst;
    }
  }
  // the computed input exists only in its specialisation, every other mode reads x
  if ((a.fr != nullptr) != (mode == kFirst) || (mode != kFirst && !a.x)) return hipErrorInvalidValue;
  if (a.transpose && a.mask && a.y16 && !a.y32 && !a.relu && !a.bias && !a.z) mode = kBwd;
  // the z output exists only in its specialisation
  if (a.z && mode != kLast) return hipErrorInvalidValue;
  switch (mode) {
    case kFirst: hipLaunchKernelGGL(cnn_conv_kernel<kFirst>, dim3(blocks), dim3(256), 0, st, a); break;
    case kHidden: hipLaunchKernelGGL(cnn_conv_kernel<kHidden>, dim3(blocks), dim3(256), 0, st, a); break;
    case kLast: hipLaunchKernelGGL(cnn_conv_kernel<kLast>, dim3(blocks), dim3(256), 0, st, a); break;
    case kBwd: hipLaunchKernelGGL(cnn_conv_kernel<kBwd>, dim3(blocks), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL(cnn_conv_kernel<kGeneric>, dim3(blocks), dim3(256), 0, st, a); break;
  }
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

// bf16 weights in both layouts: [layer][t][in][out] (backward-data operand), then
// [layer][t][out][in] (forward operand), so either product loads 16 contiguous bytes.
__device__ __forceinline__ void store_weight(uint16_t* w16, int layer, int j, uint16_t v) {
  const int t = j / (kCh * kCh), c = (j / kCh) % kCh, o = j % kCh;
  w16[(size_t)layer * kCnnWeights + j] = v;
  w16[(size_t)(kCnnLayers + layer) * kCnnWeights + (t * kCh + o) * kCh + c] = v;
}

__global__ __launch_bounds__(256) void cnn_cast_kernel(float* __restrict__ p, uint16_t* __restrict__ w16) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kCnnParams) return;
  if (frozen_param(i)) p[i] = 0.f;
  const int layer = i / kCnnLayerParams, j = i % kCnnLayerParams;
  if (j < kCnnWeights) store_weight(w16, layer, j, f2bf(p[i]));
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
  if (j < kCnnWeights) store_weight(w16, layer, j, f2bf(pi));
}

hipError_t launch_cnn_adam(float* p, const float* g, float* m, float* v, uint16_t* w16, const AdamArgs& h,
                           hipStream_t st) {
  hipLaunchKernelGGL(cnn_adam_kernel, dim3((kCnnParams + 255) / 256), dim3(256), 0, st, p, g, m, v, w16, h);
  return hipGetLastError();
}

}  // namespace mfr
