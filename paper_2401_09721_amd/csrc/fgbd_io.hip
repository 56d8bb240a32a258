// Steps on either side of the per-frame path.
//
// Quantisation (Sec. 2.2 takes integer voxel coordinates; a capture with float
// coordinates is first brought onto a 2^b grid): one isotropic scale for the
// three axes so the shape is not distorted,
//   lo_c = min_i x_ic,  ext = max_c (max_i x_ic - lo_c),  s = 2^b / ext,
//   g_ic = min(floor((x_ic - lo_c) s), 2^b - 1),
// in FP64 with IEEE division, so the result is fixed to the bit.  Points that
// fall on one voxel are all kept (the scan-line graph handles equal
// coordinates as neighbours at distance 0).  Bounds: per-block minima and
// maxima of order-preserving 32-bit keys, combined with integer atomics (exact
// and order-free); NaN coordinates take no part in the bounds and map to 0.
//
// Geometry as the signal: the integer coordinates as float32, which the
// filter then smooths like colours.
//
// Output rounding: colours to uint8 by round-half-to-even and clipping to
// 0..255 (NaN to 0).
#include "fgbd_internal.h"

namespace fgbd {

namespace {

// Monotone map of float onto uint32: a < b (as floats, not NaN) iff key(a) < key(b).
__device__ __forceinline__ uint32_t order_key(float x) {
  const uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__global__ void k_bounds_init(uint32_t *__restrict__ keys) {
  const int t = threadIdx.x;
  if (t < 6) keys[t] = t < 3 ? 0xffffffffu : 0u;  // minima start high, maxima low
}

__global__ __launch_bounds__(kBlock) void k_bounds(const float *__restrict__ xyz, int64_t n,
                                                   uint32_t *__restrict__ keys) {
  __shared__ uint32_t s_k[6][kBlock];
  uint32_t mn[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, mx[3] = {0u, 0u, 0u};
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float x = xyz[3 * i + c];
      if (x == x) {
        const uint32_t k = order_key(x);
        mn[c] = k < mn[c] ? k : mn[c];
        mx[c] = k > mx[c] ? k : mx[c];
      }
    }
  }
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s_k[c][t] = mn[c];
    s_k[3 + c][t] = mx[c];
  }
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if (t < h) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const uint32_t a = s_k[c][t + h], b = s_k[3 + c][t + h];
        s_k[c][t] = a < s_k[c][t] ? a : s_k[c][t];
        s_k[3 + c][t] = b > s_k[3 + c][t] ? b : s_k[3 + c][t];
      }
    }
    __syncthreads();
  }
  if (t < 3) atomicMin(&keys[t], s_k[t][0]);
  else if (t < 6) atomicMax(&keys[t], s_k[t][0]);
}

__global__ __launch_bounds__(kBlock) void k_quantize(const float *__restrict__ xyz, int64_t n, int bits,
                                                     const uint32_t *__restrict__ keys, int32_t *__restrict__ out,
                                                     double *__restrict__ frame) {
  double lo[3], ext = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lo[c] = (double)key_value(keys[c]);
    const double e = (double)key_value(keys[3 + c]) - lo[c];
    ext = e > ext ? e : ext;  // NaN (no finite value on an axis) never wins
  }
  const double cells = (double)(1 << bits);
  const double s = ext > 0.0 ? cells / ext : 0.0;
  const int32_t top = (1 << bits) - 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    frame[0] = lo[0];
    frame[1] = lo[1];
    frame[2] = lo[2];
    frame[3] = s;
  }
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = ((double)xyz[3 * i + c] - lo[c]) * s;
      int32_t g = 0;
      if (v >= 0.0) g = v < cells ? (int32_t)floor(v) : top;  // NaN fails the test: 0
      out[3 * i + c] = g < top ? g : top;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_round_u8(const float *__restrict__ x, int64_t m,
                                                     uint8_t *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m; e += stride) {
    const float v = rintf(x[e]);
    out[e] = v >= 0.0f ? (v < 255.0f ? (uint8_t)v : (uint8_t)255) : (uint8_t)0;
  }
}

__global__ __launch_bounds__(kBlock) void k_coords_f32(const int32_t *__restrict__ g, int64_t m,
                                                       float *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m; e += stride) out[e] = (float)g[e];
}

int grid_for(int64_t items) {
  const int64_t b = (items + kBlock - 1) / kBlock;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

hipError_t launch_quantize(const float *xyz, int64_t n, int32_t bits, int32_t *out, double *frame, uint32_t *keys,
                           hipStream_t st) {
  k_bounds_init<<<1, 64, 0, st>>>(keys);
  if (n > 0) {
    // few blocks: each adds six atomics on the same six words
    const int gb = grid_for(n) < 512 ? grid_for(n) : 512;
    k_bounds<<<gb, kBlock, 0, st>>>(xyz, n, keys);
  }
  k_quantize<<<grid_for(n), kBlock, 0, st>>>(xyz, n, bits, keys, out, frame);
  return hipGetLastError();
}

hipError_t launch_coords_f32(const int32_t *g, int64_t m, float *out, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  k_coords_f32<<<grid_for(m), kBlock, 0, st>>>(g, m, out);
  return hipGetLastError();
}

hipError_t launch_round_u8(const float *x, int64_t m, uint8_t *out, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  k_round_u8<<<grid_for(m), kBlock, 0, st>>>(x, m, out);
  return hipGetLastError();
}

}  // namespace fgbd
