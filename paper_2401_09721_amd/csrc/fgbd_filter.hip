// Low-pass graph filter (eq. 5) with integer filter selection (eq. 6) and
// FSLR (Sec. 2.4).
//
// One launch = one sweep x_q = T x_{q-1}, (T x)_i = x_i/2 + sum_k p_ik x_{col_ik}/2,
// one thread per point, colours held as float4 (r, g, b, FSLR flag) so each
// neighbour gather is a single 16-byte load.  The sweep also accumulates the
// FP64 sums of |x_q|^2 over the FSLR subset and over all points; the last block
// to finish reduces the block sums in block order and updates the selection
// state in device memory:
//   E(q) = (sum_S |y|^2 - sum_S |x_q|^2) / (3 |S|),
//   best q so far = argmin |sigma_est^2 - E(q)| (ties keep the smaller q),
//   done when E(q) >= sigma_est^2, q reaches q_max, or the loss is 0.
// Later launches read `done` and return at once, so the host can enqueue up to
// q_max sweeps without reading anything back.  Three rotating float4 buffers
// hold x_q, the best iterate and the output, so the best iterate is never
// copied: the output buffer is always the one holding neither.
// The first sweep reads the caller's float32 [n][3] colours directly and marks
// FSLR membership (spread_i <= kappa * sigma_est) in the fourth lane.
#include "fgbd_internal.h"

namespace fgbd {

namespace {

struct SweepArgs {
  int32_t n, k;
  int32_t select, q_limit;
  double kappa;
  int64_t buf_stride;  // float4 elements per buffer
};

__device__ __forceinline__ int free_buffer(int in_buf, int best_buf) {
  for (int b = 0; b < 3; ++b)
    if (b != in_buf && b != best_buf) return b;
  return 0;
}

template <int KT, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs a, const int32_t *__restrict__ col,
                                                  const float *__restrict__ p, const float *__restrict__ rgb_in,
                                                  float4 *__restrict__ xbuf, const double *__restrict__ spread,
                                                  const fgbd_result *__restrict__ noise, double *__restrict__ part,
                                                  Counters *__restrict__ cnt, SweepCtrl *__restrict__ ctrl) {
  __shared__ double s_red[4 * kSweepParts];
  const int K = KT > 0 ? KT : a.k;
  int in_buf = 3, best_buf = 3;
  double thr = 0.0;
  bool fslr = false;
  if (FIRST) {
    if (a.select && a.kappa > 0.0) {
      fslr = true;
      thr = a.kappa * noise->sigma_est;
    }
  } else {
    if (ctrl->done) return;
    in_buf = ctrl->in_buf;
    best_buf = ctrl->best_buf;
  }
  const int out_buf = free_buffer(in_buf, best_buf);
  const float4 *xin = xbuf + (size_t)(in_buf < 3 ? in_buf : 0) * a.buf_stride;
  float4 *xout = xbuf + (size_t)out_buf * a.buf_stride;

  double v[kSweepParts] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < a.n) {
    float xr, xg, xb, member;
    if (FIRST) {
      xr = rgb_in[3 * (size_t)i + 0];
      xg = rgb_in[3 * (size_t)i + 1];
      xb = rgb_in[3 * (size_t)i + 2];
      member = fslr ? (spread[i] <= thr ? 1.0f : 0.0f) : 1.0f;
    } else {
      const float4 xi = xin[i];
      xr = xi.x;
      xg = xi.y;
      xb = xi.z;
      member = xi.w;
    }
    const int32_t *crow = col + (size_t)i * K;
    const float *prow = p + (size_t)i * K;
    float ar = 0.f, ag = 0.f, ab = 0.f;
    const int c0 = crow[0];
#pragma unroll
    for (int k = 0; k < (KT > 0 ? KT : kMaxK); ++k) {
      if (k < K) {
        const int c = crow[k];
        if (c >= 0) {
          const float w = prow[k];
          if (FIRST) {
            ar = fmaf(w, rgb_in[3 * (size_t)c + 0], ar);
            ag = fmaf(w, rgb_in[3 * (size_t)c + 1], ag);
            ab = fmaf(w, rgb_in[3 * (size_t)c + 2], ab);
          } else {
            const float4 xc = xin[c];
            ar = fmaf(w, xc.x, ar);
            ag = fmaf(w, xc.y, ag);
            ab = fmaf(w, xc.z, ab);
          }
        }
      }
    }
    float orr = xr, og = xg, ob = xb;
    if (c0 >= 0) {
      orr = 0.5f * xr + 0.5f * ar;
      og = 0.5f * xg + 0.5f * ag;
      ob = 0.5f * xb + 0.5f * ab;
    }
    xout[i] = make_float4(orr, og, ob, member);
    const double x2 = (double)orr * orr + (double)og * og + (double)ob * ob;
    v[0] = member != 0.0f ? x2 : 0.0;
    v[1] = x2;
    if (FIRST) {
      const double y2 = (double)xr * xr + (double)xg * xg + (double)xb * xb;
      v[2] = member != 0.0f ? y2 : 0.0;
      v[3] = y2;
      v[4] = member != 0.0f ? 1.0 : 0.0;
    }
  }
  block_sum_f64<kSweepParts>(v, s_red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < kSweepParts; ++j) part[(size_t)blockIdx.x * kSweepParts + j] = v[j];
  }
  if (!last_block_arrival(&cnt->sweep, gridDim.x)) return;

  double tsum[kSweepParts] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) {
#pragma unroll
    for (int j = 0; j < kSweepParts; ++j) tsum[j] += part[(size_t)b * kSweepParts + j];
  }
  block_sum_f64<kSweepParts>(tsum, s_red);
  if (threadIdx.x != 0) return;

  SweepCtrl c;
  if (FIRST) {
    c.sigma_est = a.select ? noise->sigma_est : 0.0;
    c.target = c.sigma_est * c.sigma_est;
    const int n_sel = (int)tsum[4];
    c.use_all = (!fslr || n_sel == 0) ? 1 : 0;
    c.n_sel = c.use_all ? a.n : n_sel;
    c.y2_sel = c.use_all ? tsum[3] : tsum[2];
    c.q = 0;
    c.best_q = 0;
    c.best_loss = c.target;
    c.best_buf = 3;
    c.select = a.select;
    c.q_limit = a.q_limit;
    c.pad = 0;
  } else {
    c = *ctrl;
  }
  const double x2 = c.use_all ? tsum[1] : tsum[0];
  c.q += 1;
  const double energy = c.n_sel > 0 ? (c.y2_sel - x2) / (3.0 * (double)c.n_sel) : 0.0;
  c.last_energy = energy;
  if (c.q > c.q_limit) {  // q_limit == 0: the sweep only counted the subset
    c.done = 1;
  } else if (c.select) {
    const double loss = fabs(c.target - energy);
    if (loss < c.best_loss) {
      c.best_loss = loss;
      c.best_q = c.q;
      c.best_buf = out_buf;
    }
    c.done = (energy >= c.target || c.q >= c.q_limit || c.best_loss == 0.0) ? 1 : 0;
  } else {
    c.best_q = c.q;
    c.best_buf = out_buf;
    c.best_loss = 0.0;
    c.done = c.q >= c.q_limit ? 1 : 0;
  }
  c.in_buf = out_buf;
  *ctrl = c;
}

__global__ __launch_bounds__(kBlock) void k_finalize(int32_t n, int64_t buf_stride, const float *__restrict__ rgb_in,
                                                     const float4 *__restrict__ xbuf,
                                                     const SweepCtrl *__restrict__ ctrl,
                                                     const fgbd_result *__restrict__ noise, float *__restrict__ rgb_out,
                                                     fgbd_result *__restrict__ res) {
  const int best = ctrl->best_buf;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    if (best == 3) {
      rgb_out[3 * (size_t)i + 0] = rgb_in[3 * (size_t)i + 0];
      rgb_out[3 * (size_t)i + 1] = rgb_in[3 * (size_t)i + 1];
      rgb_out[3 * (size_t)i + 2] = rgb_in[3 * (size_t)i + 2];
    } else {
      const float4 x = xbuf[(size_t)best * buf_stride + i];
      rgb_out[3 * (size_t)i + 0] = x.x;
      rgb_out[3 * (size_t)i + 1] = x.y;
      rgb_out[3 * (size_t)i + 2] = x.z;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    res->q = ctrl->best_q;
    res->loss = ctrl->best_loss;
    res->n_fslr = ctrl->n_sel;
    res->sweeps = ctrl->q;
    if (noise != nullptr && noise != res) res->sigma_est = noise->sigma_est;
  }
}

}  // namespace

hipError_t launch_sweep(int64_t n, int k, const int32_t *col, const float *p, const float *rgb_in, float4 *xbuf,
                        const double *spread, const fgbd_result *noise, double kappa, int select, int q_limit,
                        int first, double *part, int nblocks, Counters *cnt, SweepCtrl *ctrl, hipStream_t stream) {
  SweepArgs a;
  a.n = (int32_t)n;
  a.k = k;
  a.select = select;
  a.q_limit = q_limit;
  a.kappa = kappa;
  a.buf_stride = n;
  if (k == 8) {
    if (first)
      k_sweep<8, true><<<nblocks, kBlock, 0, stream>>>(a, col, p, rgb_in, xbuf, spread, noise, part, cnt, ctrl);
    else
      k_sweep<8, false><<<nblocks, kBlock, 0, stream>>>(a, col, p, rgb_in, xbuf, spread, noise, part, cnt, ctrl);
  } else {
    if (first)
      k_sweep<0, true><<<nblocks, kBlock, 0, stream>>>(a, col, p, rgb_in, xbuf, spread, noise, part, cnt, ctrl);
    else
      k_sweep<0, false><<<nblocks, kBlock, 0, stream>>>(a, col, p, rgb_in, xbuf, spread, noise, part, cnt, ctrl);
  }
  return hipGetLastError();
}

hipError_t launch_finalize(int64_t n, const float *rgb_in, const float4 *xbuf, const SweepCtrl *ctrl,
                           const fgbd_result *noise, int q_none, float *rgb_out, fgbd_result *res,
                           hipStream_t stream) {
  (void)q_none;
  const int nb = (int)((n + kBlock - 1) / kBlock);
  k_finalize<<<nb > 0 ? nb : 1, kBlock, 0, stream>>>((int32_t)n, n, rgb_in, xbuf, ctrl, noise, rgb_out, res);
  return hipGetLastError();
}

}  // namespace fgbd
