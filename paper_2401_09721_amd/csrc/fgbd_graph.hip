// Neighbour selection and edge weights of the scan-line graph (Sec. 2.2).
//
// k_merge: one thread per point i.  For each direction it looks up i's sorted
// position r (rank array from the last radix pass), reads the items at
// r-w..r+w (their codes decode to coordinates, so no coordinate gather is
// needed), and keeps the K smallest distinct (squared distance, index) pairs
// in a register-resident sorted list (packed as d2 << 32 | j, so one 64-bit
// compare orders by distance then index).  It writes the fixed-K CSR row and
// accumulates the FP64 sum of edge lengths for sigma_g; the last block to
// finish reduces the per-block sums in a fixed order (eq. 4 bandwidth).
//
// k_weights: one thread per point, row-normalised Gaussian weights of eq. 4
// computed in FP64 with the row's smallest squared distance subtracted in the
// exponent (same ratio, no underflow of the whole row) and stored as float.
#include "fgbd_internal.h"

namespace fgbd {

namespace {

template <int KM>
__device__ __forceinline__ void topk_insert(uint64_t (&lst)[KM], int K, uint64_t c) {
  if (c >= lst[K - 1]) return;
#pragma unroll
  for (int k = 0; k < KM; ++k)
    if (k < K && lst[k] == c) return;
#pragma unroll
  for (int k = KM - 1; k > 0; --k) {
    if (k < K) {
      const uint64_t prev = lst[k - 1];
      if (prev > c)
        lst[k] = prev;
      else if (lst[k] > c)
        lst[k] = c;
    }
  }
  if (lst[0] > c) lst[0] = c;
}

template <int KM>
__global__ __launch_bounds__(kBlock) void k_merge(DirTable dt, int32_t n, int32_t window, int32_t K,
                                                  const int32_t *__restrict__ xyz, const uint64_t *__restrict__ sorted,
                                                  const uint32_t *__restrict__ rank, int32_t *__restrict__ col,
                                                  int32_t *__restrict__ dist2, double *__restrict__ part,
                                                  Counters *__restrict__ cnt, double sigma_g_fixed,
                                                  fgbd_result *__restrict__ res) {
  __shared__ double s_red[8];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double acc[2] = {0.0, 0.0};
  if (i < n) {
    uint64_t lst[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) lst[k] = ~0ull;
    const int gi0 = xyz[3 * i + 0], gi1 = xyz[3 * i + 1], gi2 = xyz[3 * i + 2];
    for (int d = 0; d < dt.num_dirs; ++d) {
      const DirInfo di = dt.d[d];
      const int r = (int)rank[(size_t)d * n + i];
      const uint64_t *srt = sorted + (size_t)d * n;
      const int lo = max(r - window, 0);
      const int hi = min(r + window, n - 1);
      for (int rr = lo; rr <= hi; ++rr) {
        if (rr == r) continue;
        const uint64_t it = srt[rr];
        int gj[3];
        scan_decode((uint32_t)(it >> 32), di, dt.bits, gj);
        const int dx = gj[0] - gi0, dy = gj[1] - gi1, dz = gj[2] - gi2;
        const uint32_t d2 = (uint32_t)(dx * dx + dy * dy + dz * dz);
        topk_insert<KM>(lst, K, ((uint64_t)d2 << 32) | (uint32_t)it);
      }
    }
    int32_t *crow = col + (size_t)i * K;
    int32_t *drow = dist2 + (size_t)i * K;
    for (int k = 0; k < KM; ++k) {
      if (k < K) {
        const bool ok = lst[k] != ~0ull;
        const uint32_t d2 = (uint32_t)(lst[k] >> 32);
        crow[k] = ok ? (int32_t)(uint32_t)lst[k] : -1;
        drow[k] = ok ? (int32_t)d2 : 0;
        if (ok) {
          acc[0] += sqrt((double)d2);
          acc[1] += 1.0;
        }
      }
    }
  }
  block_sum_f64<2>(acc, s_red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x + 0] = acc[0];
    part[2 * blockIdx.x + 1] = acc[1];
  }
  if (last_block_arrival(&cnt->merge, gridDim.x)) {
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) {
      v[0] += part[2 * b + 0];
      v[1] += part[2 * b + 1];
    }
    block_sum_f64<2>(v, s_red);
    if (threadIdx.x == 0) {
      double sg = sigma_g_fixed > 0.0 ? sigma_g_fixed : (v[1] > 0.0 ? v[0] / v[1] : 0.0);
      res->sigma_g = sg;
    }
  }
}

template <int KT>
__global__ __launch_bounds__(kBlock) void k_weights(int32_t n, int32_t k_rt, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ dist2,
                                                    const fgbd_result *__restrict__ res, float *__restrict__ p) {
  const int K = KT > 0 ? KT : k_rt;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double sg = res->sigma_g;
  const double inv = sg > 0.0 ? 1.0 / (sg * sg) : 0.0;
  const int32_t *crow = col + (size_t)i * K;
  const int32_t *drow = dist2 + (size_t)i * K;
  float *prow = p + (size_t)i * K;
  constexpr int KB = KT > 0 ? KT : kMaxK;
  double w[KB];
  double s = 0.0;
  const int d0 = drow[0];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    w[k] = 0.0;
    if (k < K && crow[k] >= 0) {
      const int delta = drow[k] - d0;
      w[k] = sg > 0.0 ? exp(-(double)delta * inv) : (delta == 0 ? 1.0 : 0.0);
      s += w[k];
    }
  }
  const double rs = s > 0.0 ? 1.0 / s : 0.0;
#pragma unroll
  for (int k = 0; k < KB; ++k)
    if (k < K) prow[k] = (float)(w[k] * rs);
}

}  // namespace

hipError_t launch_merge(const int32_t *xyz, int64_t n, const DirTable &dt, int window, int k, const uint64_t *sorted,
                        const uint32_t *rank, int32_t *col, int32_t *dist2, double *part, int nblocks,
                        Counters *cnt, double sigma_g_fixed, fgbd_result *res, hipStream_t stream) {
  if (k <= 8)
    k_merge<8><<<nblocks, kBlock, 0, stream>>>(dt, (int32_t)n, window, k, xyz, sorted, rank, col, dist2, part, cnt,
                                               sigma_g_fixed, res);
  else if (k <= 16)
    k_merge<16><<<nblocks, kBlock, 0, stream>>>(dt, (int32_t)n, window, k, xyz, sorted, rank, col, dist2, part, cnt,
                                                sigma_g_fixed, res);
  else
    k_merge<32><<<nblocks, kBlock, 0, stream>>>(dt, (int32_t)n, window, k, xyz, sorted, rank, col, dist2, part, cnt,
                                                sigma_g_fixed, res);
  return hipGetLastError();
}

hipError_t launch_weights(int64_t n, int k, const int32_t *col, const int32_t *dist2, const fgbd_result *res,
                          float *p, hipStream_t stream) {
  const int nb = (int)((n + kBlock - 1) / kBlock);
  if (nb == 0) return hipSuccess;
  if (k == 8)
    k_weights<8><<<nb, kBlock, 0, stream>>>((int32_t)n, k, col, dist2, res, p);
  else
    k_weights<0><<<nb, kBlock, 0, stream>>>((int32_t)n, k, col, dist2, res, p);
  return hipGetLastError();
}

}  // namespace fgbd
