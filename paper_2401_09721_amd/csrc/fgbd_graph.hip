// Neighbour selection and edge weights of the scan-line graph (Sec. 2.2).
//
// k_merge: one thread per point i.  For each direction it looks up i's sorted
// position r (rank array from the last radix pass), reads the items at
// r-w..r+w (their codes decode to coordinates, so no coordinate gather is
// needed), and keeps the K smallest distinct (squared distance, index) pairs
// in a register-resident sorted list (packed as d2 << 32 | j, so one 64-bit
// compare orders by distance then index).  It writes the fixed-K CSR row and
// writes per-block FP64 sums of edge lengths and edge counts for sigma_g.
//
// k_weights: every block first sums the merge partials in block order (all
// blocks get the same sigma_g, the mean edge length of eq. 4's bandwidth rule),
// then computes row-normalised Gaussian weights of eq. 4 in FP64 with the row's
// smallest squared distance subtracted in the exponent (same ratio, no
// underflow of the whole row), stored as float.  Squared-distance gaps are
// integers, so exp(-gap / sigma_g^2) comes from a per-block table for small
// gaps.  Both kernels are grid-stride over XCD-contiguous shares of points.
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
                                                  int32_t *__restrict__ dist2, double *__restrict__ part) {
  __shared__ double s_red[8];
  double acc[2] = {0.0, 0.0};
  const Share sh = xcd_share(n, kBlock);
  for (int64_t base = sh.first; base < sh.end; base += sh.step) {
    const int i = (int)(base + threadIdx.x);
    if (i >= sh.end) continue;
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
        const uint32_t dx = (uint32_t)(gj[0] - gi0), dy = (uint32_t)(gj[1] - gi1), dz = (uint32_t)(gj[2] - gi2);
        const uint32_t d2 = dx * dx + dy * dy + dz * dz;
        topk_insert<KM>(lst, K, ((uint64_t)d2 << 32) | (uint32_t)it);
      }
    }
    int cv[KM], dv[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const bool ok = lst[k] != ~0ull;
      const uint32_t d2 = (uint32_t)(lst[k] >> 32);
      cv[k] = ok ? (int32_t)(uint32_t)lst[k] : -1;
      dv[k] = ok ? (int32_t)d2 : 0;
      if (ok && k < K) {
        acc[0] += sqrt((double)d2);
        acc[1] += 1.0;
      }
    }
    if (KM == 8 && K == 8) {
      int4 *cr = reinterpret_cast<int4 *>(col + (size_t)i * 8);
      int4 *dr = reinterpret_cast<int4 *>(dist2 + (size_t)i * 8);
      cr[0] = make_int4(cv[0], cv[1], cv[2], cv[3]);
      cr[1] = make_int4(cv[4], cv[5], cv[6], cv[7]);
      dr[0] = make_int4(dv[0], dv[1], dv[2], dv[3]);
      dr[1] = make_int4(dv[4], dv[5], dv[6], dv[7]);
    } else {
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k < K) {
          col[(size_t)i * K + k] = cv[k];
          dist2[(size_t)i * K + k] = dv[k];
        }
      }
    }
  }
  block_sum_f64<2>(acc, s_red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x + 0] = acc[0];
    part[2 * blockIdx.x + 1] = acc[1];
  }
}

constexpr int kExpTable = 256;

template <int KT>
__global__ __launch_bounds__(kBlock) void k_weights(int32_t n, int32_t k_rt, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ dist2,
                                                    const double *__restrict__ merge_part, int merge_blocks,
                                                    double sigma_g_fixed, fgbd_result *__restrict__ res,
                                                    float *__restrict__ p) {
  __shared__ double s_red[8];
  __shared__ double s_exp[kExpTable];
  const int K = KT > 0 ? KT : k_rt;
  double sg = sigma_g_fixed;
  if (!(sg > 0.0)) {
    double t[2];
    reduce_partials<2>(merge_part, merge_blocks, 2, t, s_red);
    sg = t[1] > 0.0 ? t[0] / t[1] : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) res->sigma_g = sg;
  const double inv = sg > 0.0 ? 1.0 / (sg * sg) : 0.0;
  // squared-distance gaps are integers: tabulate exp(-gap / sigma_g^2) for small gaps
  for (int g = threadIdx.x; g < kExpTable; g += kBlock) s_exp[g] = sg > 0.0 ? exp(-(double)g * inv) : (g == 0 ? 1.0 : 0.0);
  __syncthreads();
  constexpr int KB = KT > 0 ? KT : kMaxK;
  const Share sh = xcd_share(n, kBlock);
  for (int64_t base = sh.first; base < sh.end; base += sh.step) {
    const int64_t i = base + threadIdx.x;
    if (i >= sh.end) continue;
    int cv[KB], dv[KB];
    if (KT == 8) {
      const int4 *cr = reinterpret_cast<const int4 *>(col + i * 8);
      const int4 *dr = reinterpret_cast<const int4 *>(dist2 + i * 8);
      const int4 c0 = cr[0], c1 = cr[1], e0 = dr[0], e1 = dr[1];
      cv[0] = c0.x; cv[1] = c0.y; cv[2] = c0.z; cv[3] = c0.w;
      cv[4] = c1.x; cv[5] = c1.y; cv[6] = c1.z; cv[7] = c1.w;
      dv[0] = e0.x; dv[1] = e0.y; dv[2] = e0.z; dv[3] = e0.w;
      dv[4] = e1.x; dv[5] = e1.y; dv[6] = e1.z; dv[7] = e1.w;
    } else {
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        cv[k] = k < K ? col[i * K + k] : -1;
        dv[k] = k < K ? dist2[i * K + k] : 0;
      }
    }
    double w[KB];
    double s = 0.0;
    const int d0 = dv[0];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      w[k] = 0.0;
      if (cv[k] >= 0) {
        const int gap = dv[k] - d0;
        w[k] = gap < kExpTable ? s_exp[gap] : (sg > 0.0 ? exp(-(double)gap * inv) : 0.0);
        s += w[k];
      }
    }
    const double rs = s > 0.0 ? 1.0 / s : 0.0;
    if (KT == 8) {
      float4 *pr = reinterpret_cast<float4 *>(p + i * 8);
      pr[0] = make_float4((float)(w[0] * rs), (float)(w[1] * rs), (float)(w[2] * rs), (float)(w[3] * rs));
      pr[1] = make_float4((float)(w[4] * rs), (float)(w[5] * rs), (float)(w[6] * rs), (float)(w[7] * rs));
    } else {
#pragma unroll
      for (int k = 0; k < KB; ++k)
        if (k < K) p[i * K + k] = (float)(w[k] * rs);
    }
  }
}

}  // namespace

hipError_t launch_merge(const int32_t *xyz, int64_t n, const DirTable &dt, int window, int k, const uint64_t *sorted,
                        const uint32_t *rank, int32_t *col, int32_t *dist2, double *part, int nblocks,
                        hipStream_t stream) {
  if (k <= 8)
    k_merge<8><<<nblocks, kBlock, 0, stream>>>(dt, (int32_t)n, window, k, xyz, sorted, rank, col, dist2, part);
  else if (k <= 16)
    k_merge<16><<<nblocks, kBlock, 0, stream>>>(dt, (int32_t)n, window, k, xyz, sorted, rank, col, dist2, part);
  else
    k_merge<32><<<nblocks, kBlock, 0, stream>>>(dt, (int32_t)n, window, k, xyz, sorted, rank, col, dist2, part);
  return hipGetLastError();
}

hipError_t launch_weights(int64_t n, int k, const int32_t *col, const int32_t *dist2, const double *merge_part,
                          int merge_blocks, double sigma_g_fixed, fgbd_result *res, float *p, int nblocks,
                          hipStream_t stream) {
  if (k == 8)
    k_weights<8><<<nblocks, kBlock, 0, stream>>>((int32_t)n, k, col, dist2, merge_part, merge_blocks, sigma_g_fixed,
                                                 res, p);
  else
    k_weights<0><<<nblocks, kBlock, 0, stream>>>((int32_t)n, k, col, dist2, merge_part, merge_blocks, sigma_g_fixed,
                                                 res, p);
  return hipGetLastError();
}

}  // namespace fgbd
