// Low-pass graph filter (eq. 5) with integer filter selection (eq. 6) and
// FSLR (Sec. 2.4).
//
// One launch = one sweep x_q = T x_{q-1}, (T x)_i = x_i/2 + sum_k p_ik x_{col_ik}/2,
// colours held as float4 (r, g, b, FSLR flag) so each neighbour gather is one
// 16-byte load.  Each sweep also sums |x_q|^2 over the FSLR subset and over
// all points.  Every point's term is rounded to a fixed-point integer (units of
// 2^-12) and blocks add their integer sums with 64-bit atomics into a few
// slots per cloud; integer addition is exact, so the totals do not depend on
// the order, the grid or the device schedule (deterministic, no floating-point
// atomics, no fences).  Three slot buffers rotate: launch q reads the sums of
// q-1, adds into q, and clears the buffer of q+1.  Every block works on one
// cloud, and every cloud has its own selection state.
//
// Selection without inter-block synchronisation: launch q starts by reading
// the sums of launch q-1 (every block reads the same integers) and advancing
// the selection state
//   E(q-1) = (sum_S |y|^2 - sum_S |x_{q-1}|^2) / (3 |S|),
//   best = argmin |sigma_est^2 - E| so far (ties keep the smaller q),
//   done when E >= sigma_est^2, q reaches q_max, or the loss is 0;
// the first block of each cloud stores the state for the next launch (ping-pong buffers, so no
// block reads a state another block of the same launch is writing).  A launch
// that finds the state done returns at once, so the host enqueues up to q_max
// launches without reading anything back.  Three rotating float4 buffers hold
// x_q, the best iterate and the output, so the best iterate is never copied.
// The first sweep reads the caller's float32 [n][3] colours directly and marks
// FSLR membership (spread_i <= kappa * sigma_est) in the fourth lane; its
// partials also carry sum |y|^2 and |S|.  The finalising launch applies the
// last sweep's partials the same way and writes the chosen iterate out.
// In the fused per-frame path x_1 comes from the noise launch, and when the
// selection has at least two separate sweeps one launch covers sweeps 1 and
// 2: it marks membership, adds x_1's and the input's sums into a fourth sums
// buffer outside the rotation (cleared by the call's setup) and computes x_2;
// its stored state is flagged so that the next state load applies x_1's sums
// before x_2's, exactly as two launches would have.
//
// Launch count: a launch that finds the selection done still costs about two
// microseconds, and q_max of them are enqueued.  So only the first few sweeps
// (the schedule's sweep_launches) are launches of their own; the rest, if the
// selection has not finished by then, run in one launch that loops over the
// remaining sweeps, its blocks waiting for each other between sweeps (a
// counter in device memory; the grid is sized to be resident at once).  That
// launch first reads the done flags the last separate launch stored and skips
// the loop when every cloud is done, which is the usual case; either way it
// then does the finalising work (so no separate launch follows it).  The
// wait between sweeps costs far more than a kernel boundary on this GPU (it
// writes back and invalidates the L2 of every XCD), so the loop is the
// fallback, not the main path.  A plain launch is used because a cooperative
// launch measured about 40 us of overhead even when it returned at once.
// With fixed q the host knows the sweep count and launches every sweep, then
// the finalising launch.
#include "fgbd_internal.h"

namespace fgbd {

namespace {

struct SweepArgs {
  SegArgs sa;
  int32_t k;
  int32_t select, q_limit;
  double kappa;
  int64_t buf_stride;  // float4 elements per buffer
  unsigned long long *sums3;  // [4][B][slots][parts]: 0-2 rotate by sweep, 3 holds x_1's sums
                              // when the fused first launch also computes x_2
  SweepCtrl *ctrl;            // [2][B], ping-pong by sweep
  // weights derived by the first sweep (the fused per-frame path): the
  // squared distances, the merge launch's edge-length sums, a fixed sigma_g
  // (<= 0: the mean edge length), the results that receive sigma_g, and
  // where to store the weights for the later sweeps
  const int32_t *dist2;
  const unsigned long long *edge_acc;
  double sigma_g_fixed;
  fgbd_result *res;
  float *p_out;
  // per cloud: set when the cloud was renumbered along scan order 0 (NULL:
  // never); its graph and input colours are then read from col_w, dist2_w
  // and rgb_w, and the output of point i is the iterate at rank0[i]
  const int32_t *relabel;
  const float *rgb_w;
  const int32_t *col_w, *dist2_w;
  const uint32_t *rank0;
};

constexpr int kSlotVals = kSweepSlots * kSweepParts;  // integers per cloud and sweep

// The rotating buffers of sweep q (1-based): it reads the sums and state of
// q-1, adds into the sums of q, clears the sums of q+1 and stores its state.
struct SweepIO {
  const unsigned long long *sums_prev;
  unsigned long long *sums_out, *sums_clear;
  unsigned long long *sums_first;  // x_1's sums of the fused first launch (never rotated)
  const SweepCtrl *ctrl_prev;
  SweepCtrl *ctrl_out;
};
__device__ __forceinline__ SweepIO sweep_io(const SweepArgs &a, int q) {
  const size_t S = (size_t)a.sa.B * kSlotVals;
  return {a.sums3 + ((q - 1) % 3) * S, a.sums3 + (q % 3) * S, a.sums3 + ((q + 1) % 3) * S, a.sums3 + 3 * S,
          a.ctrl + ((q - 1) & 1) * a.sa.B, a.ctrl + (q & 1) * a.sa.B};
}

constexpr double kFix = 4096.0;  // fixed-point scale of the energy sums (2^12)

__device__ __forceinline__ unsigned long long to_fix(double v) { return (unsigned long long)llrint(v * kFix); }

__device__ __forceinline__ int free_buffer(int in_buf, int best_buf) {
  for (int b = 0; b < 3; ++b)
    if (b != in_buf && b != best_buf) return b;
  return 0;
}

// Apply the sums of the sweep that produced x_{c.q+1} (written to out_buf).
__device__ __forceinline__ void advance(SweepCtrl &c, const double (&t)[kSweepParts], int n, int out_buf) {
  if (c.q == 0) {  // partials of the first sweep also carry |y|^2 and |S|
    const int n_sel = (int)t[4];
    c.use_all = (!c.fslr || n_sel == 0) ? 1 : 0;
    c.n_sel = c.use_all ? n : n_sel;
    c.y2_sel = c.use_all ? t[3] : t[2];
  }
  const double x2 = c.use_all ? t[1] : t[0];
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
}

// Selection state at the start of a launch: the stored state advanced by the
// previous sweep's integer sums (identical in every block).  A state stored
// by the fused first launch (first_pending) is first advanced by x_1's sums
// from sums_first, then, unless that ended the selection, by x_2's.  The
// state and both sets of slots are loaded at once (one round trip before the
// sweep); only the sets the state needs are then reduced, and a state that
// is already done returns before any reduction.  A wave reduces a set with
// every lane holding one slot, by shuffles, so every lane holds the totals.
__device__ __forceinline__ void load_slots(const unsigned long long *__restrict__ sums,
                                           unsigned long long (&u)[kSweepParts]) {
  const int sl = (int)lane_id();
#pragma unroll
  for (int j = 0; j < kSweepParts; ++j) u[j] = sl < kSweepSlots ? sums[sl * kSweepParts + j] : 0ull;
}
__device__ __forceinline__ void wave_sum(unsigned long long (&u)[kSweepParts]) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int j = 0; j < kSweepParts; ++j) u[j] += __shfl_xor(u[j], o, kWave);
  }
}
__device__ __forceinline__ void sums_to_double(const unsigned long long *u, double (&t)[kSweepParts]) {
#pragma unroll
  for (int j = 0; j < kSweepParts; ++j) t[j] = j < 4 ? (double)u[j] / kFix : (double)u[j];
}
// Advance a state that is not done by the reduced sums (see above).
__device__ __forceinline__ void advance_loaded(SweepCtrl &c, const unsigned long long *f,
                                               const unsigned long long *u, int n) {
  double t[kSweepParts];
  if (c.first_pending) {  // x_1 sits in buffer 0, where the noise launch wrote it
    sums_to_double(f, t);
    advance(c, t, n, 0);
    c.first_pending = 0;
    if (c.done) return;
  }
  sums_to_double(u, t);
  advance(c, t, n, free_buffer(c.in_buf, c.best_buf));
}
// Called by every thread of the block (the state, and so c.done, is the
// same for all of them); wave 0 loads and reduces the slots.
__device__ __forceinline__ void load_state(SweepCtrl &c, const SweepCtrl *__restrict__ prev,
                                           const unsigned long long *__restrict__ sums_prev,
                                           const unsigned long long *__restrict__ sums_first, int n) {
  __shared__ unsigned long long s_tot[2 * kSweepParts];
  c = *prev;
  if (threadIdx.x < kWave) {
    unsigned long long f[kSweepParts], u[kSweepParts];
    load_slots(sums_first, f);
    load_slots(sums_prev, u);
    if (!c.done) {
      if (c.first_pending) wave_sum(f);
      wave_sum(u);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < kSweepParts; ++j) {
          s_tot[j] = f[j];
          s_tot[kSweepParts + j] = u[j];
        }
      }
    }
  }
  if (c.done) return;
  __syncthreads();
  unsigned long long f[kSweepParts], u[kSweepParts];
#pragma unroll
  for (int j = 0; j < kSweepParts; ++j) {
    f[j] = s_tot[j];
    u[j] = s_tot[kSweepParts + j];
  }
  __syncthreads();  // s_tot is written again by the next call (the in-launch sweep loop)
  advance_loaded(c, f, u, n);
}
// The same advance by one wave alone (no block barrier).
__device__ __forceinline__ void wave_advance(SweepCtrl &c, const SweepCtrl *__restrict__ prev,
                                             const unsigned long long *__restrict__ sums_prev,
                                             const unsigned long long *__restrict__ sums_first, int n) {
  c = *prev;
  unsigned long long f[kSweepParts], u[kSweepParts];
  load_slots(sums_first, f);
  load_slots(sums_prev, u);
  if (c.done) return;
  if (c.first_pending) wave_sum(f);
  wave_sum(u);
  advance_loaded(c, f, u, n);
}

// Block-sum of per-thread integer sums, then one atomic per value per block
// into slot `slot` of the cloud's sums.
__device__ __forceinline__ void add_sums(unsigned long long (&v)[kSweepParts], unsigned long long *__restrict__ out,
                                         int slot, unsigned long long *s_buf) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int j = 0; j < kSweepParts; ++j) v[j] += __shfl_down(v[j], o, kWave);
  }
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
#pragma unroll
    for (int j = 0; j < kSweepParts; ++j) s_buf[w * kSweepParts + j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x < kSweepParts) {
    unsigned long long a = 0;
    for (int ww = 0; ww < (int)blockDim.x / kWave; ++ww) a += s_buf[ww * kSweepParts + threadIdx.x];
    if (a) atomicAdd(&out[slot * kSweepParts + threadIdx.x], a);
  }
}

template <bool D2>
struct SweepLds {
  unsigned long long red[4 * kSweepParts];
  double exp[D2 ? kExpTable : 1];
  unsigned long long eu[D2 ? kEdgeVals : 1];
};

// One sweep (number q, buffers io) by one block of cloud sb.s.  Every thread
// of the block calls it; it returns without touching the colours when the
// cloud's selection is already done (uniform over the block).
// D2 (first sweep only): sigma_g and the row weights come from the merge's
// edge-length sums and the squared distances (eq. 4, the graph builder's own
// arithmetic) instead of a stored p; sigma_g goes to the results and the
// weights into p_out for the later sweeps.
// MERGED (the fused path's first launch when it runs more than one sweep):
// x_1 is already in buffer 0 (the noise launch wrote it); the launch marks
// FSLR membership, adds x_1's and the input's sums into sums_first and
// computes x_2 (into buffer 1, its sums into the launch's own buffer), so the
// launch of x_1's flags and sums alone is saved; the next launch applies both
// sets of sums (load_state).
template <int KT, bool FIRST, bool D2, bool PRE = false, bool MERGED = false>
__device__ __forceinline__ void sweep_step(const SweepArgs &a, const SegBlock &sb, const SweepIO &io,
                                           const int32_t *__restrict__ col, const float *__restrict__ p,
                                           const float *__restrict__ rgb_in, float4 *__restrict__ xbuf,
                                           const double *__restrict__ spread, const fgbd_result *__restrict__ noise,
                                           SweepLds<D2> &lds) {
  const int K = KT > 0 ? KT : a.k;
  constexpr int KB = KT > 0 ? KT : kMaxK;  // slots per row held in registers
  const unsigned long long *sums_prev = io.sums_prev + (size_t)sb.s * kSlotVals;
  unsigned long long *sums_out = io.sums_out + (size_t)sb.s * kSlotVals;
  unsigned long long *sums_clear = io.sums_clear + (size_t)sb.s * kSlotVals;
  SweepCtrl *ctrl_out = io.ctrl_out;
  SweepCtrl c;
  static_assert(FIRST || !D2, "only the first sweep derives the weights");
  static_assert(!PRE || (FIRST && !D2), "precomputed colours: first sweep, weights already stored");
  static_assert(!MERGED || (FIRST && !D2 && !PRE), "the merged first launch reads x_1 and stored weights");
  constexpr bool FROM_X = !FIRST || MERGED;  // colours (own and gathered) from a float4 iterate
  if (FIRST) {
    c.sigma_g = 0.0;
    if (D2) {
      c.sigma_g = cloud_sigma_g(a.edge_acc + (size_t)kEdgeSlots * kEdgeVals * sb.s, a.sigma_g_fixed, lds.eu);
      if (sb.lb == 0 && threadIdx.x == 0) a.res[sb.s].sigma_g = c.sigma_g;
    }
    c.sigma_est = a.select ? noise[sb.s].sigma_est : 0.0;
    c.target = c.sigma_est * c.sigma_est;
    c.y2_sel = 0.0;
    c.best_loss = c.target;
    c.last_energy = 0.0;
    c.n_sel = 0;
    c.use_all = 1;
    c.q = 0;
    c.best_q = 0;
    c.in_buf = 3;
    c.best_buf = 3;
    c.done = 0;
    c.select = a.select;
    c.q_limit = a.q_limit;
    c.fslr = (a.select && a.kappa > 0.0) ? 1 : 0;
    c.first_pending = MERGED ? 1 : 0;
    c.pad_ = 0;
  } else {
    load_state(c, io.ctrl_prev + sb.s, sums_prev, io.sums_first + (size_t)sb.s * kSlotVals, (int)(sb.end - sb.begin));
  }
  if (sb.lb == 0) {
    if (threadIdx.x == 0) ctrl_out[sb.s] = c;
    for (int j = threadIdx.x; j < kSlotVals; j += blockDim.x) sums_clear[j] = 0ull;
  }
  if (c.done) return;
  if (D2) {
    fill_exp_table(c.sigma_g, lds.exp);
    __syncthreads();
  }

  const double thr = c.fslr ? a.kappa * c.sigma_est : 0.0;
  // MERGED: x_1 in buffer 0, x_2 to buffer 1 (the buffer the next launch's
  // second advance names: free_buffer(0, best) is 1 for best 0 or none)
  const int out_buf = MERGED ? 1 : free_buffer(c.in_buf, c.best_buf);
  const float4 *xin = xbuf + (size_t)(MERGED ? 0 : (c.in_buf < 3 ? c.in_buf : 0)) * a.buf_stride;
  float4 *xout = xbuf + (size_t)out_buf * a.buf_stride;

  unsigned long long v[kSweepParts] = {0, 0, 0, 0, 0};
  unsigned long long vf[kSweepParts] = {0, 0, 0, 0, 0};  // MERGED: x_1's sums
  const Share sh = seg_share(sb, kBlock);
  for (int64_t base = sh.first; base < sh.end; base += sh.step) {
    const int64_t i = base + threadIdx.x;
    if (i >= sh.end) continue;
    float xr, xg, xb, member;
    if (MERGED) {
      const float4 xi = xin[i];
      xr = xi.x;
      xg = xi.y;
      xb = xi.z;
      member = c.fslr ? (spread[i] <= thr ? 1.0f : 0.0f) : 1.0f;
      const float y0 = rgb_in[3 * i + 0], y1 = rgb_in[3 * i + 1], y2 = rgb_in[3 * i + 2];
      const unsigned long long x1s = to_fix((double)xr * xr + (double)xg * xg + (double)xb * xb);
      vf[0] += member != 0.0f ? x1s : 0ull;
      vf[1] += x1s;
      const unsigned long long ys = to_fix((double)y0 * y0 + (double)y1 * y1 + (double)y2 * y2);
      vf[2] += member != 0.0f ? ys : 0ull;
      vf[3] += ys;
      vf[4] += member != 0.0f ? 1ull : 0ull;
    } else if (FIRST) {
      xr = rgb_in[3 * i + 0];
      xg = rgb_in[3 * i + 1];
      xb = rgb_in[3 * i + 2];
      member = c.fslr ? (spread[i] <= thr ? 1.0f : 0.0f) : 1.0f;
    } else {
      const float4 xi = xin[i];
      xr = xi.x;
      xg = xi.y;
      xb = xi.z;
      member = xi.w;
    }
    if (PRE) {  // x1 from the noise launch; the flag and the sums only
      const float4 x1 = xout[i];
      xout[i] = make_float4(x1.x, x1.y, x1.z, member);
      const unsigned long long x2 = to_fix((double)x1.x * x1.x + (double)x1.y * x1.y + (double)x1.z * x1.z);
      v[0] += member != 0.0f ? x2 : 0ull;
      v[1] += x2;
      const unsigned long long y2 = to_fix((double)xr * xr + (double)xg * xg + (double)xb * xb);
      v[2] += member != 0.0f ? y2 : 0ull;
      v[3] += y2;
      v[4] += member != 0.0f ? 1ull : 0ull;
      continue;
    }
    int cc[KT > 0 ? KT : kMaxK];
    float ww[KT > 0 ? KT : kMaxK];
    if (D2) {
      int dv[KB];
      if (KT == 8) {
        const int4 *cr = reinterpret_cast<const int4 *>(col + i * 8);
        const int4 *dr = reinterpret_cast<const int4 *>(a.dist2 + i * 8);
        const int4 c0 = cr[0], c1 = cr[1], e0 = dr[0], e1 = dr[1];
        cc[0] = c0.x; cc[1] = c0.y; cc[2] = c0.z; cc[3] = c0.w;
        cc[4] = c1.x; cc[5] = c1.y; cc[6] = c1.z; cc[7] = c1.w;
        dv[0] = e0.x; dv[1] = e0.y; dv[2] = e0.z; dv[3] = e0.w;
        dv[4] = e1.x; dv[5] = e1.y; dv[6] = e1.z; dv[7] = e1.w;
      } else {
#pragma unroll
        for (int k = 0; k < (KT > 0 ? KT : kMaxK); ++k) {
          cc[k] = k < K ? col[i * K + k] : -1;
          dv[k] = k < K ? a.dist2[i * K + k] : 0;
        }
      }
      row_weights<KB>(cc, dv, c.sigma_g, lds.exp, ww);
      if (KT == 8) {
        float4 *pr = reinterpret_cast<float4 *>(a.p_out + i * 8);
        pr[0] = make_float4(ww[0], ww[1], ww[2], ww[3]);
        pr[1] = make_float4(ww[4], ww[5], ww[6], ww[7]);
      } else {
#pragma unroll
        for (int k = 0; k < KB; ++k)
          if (k < K) a.p_out[i * K + k] = ww[k];
      }
    } else if (KT == 8) {
      const int4 *cr = reinterpret_cast<const int4 *>(col + i * 8);
      const float4 *pr = reinterpret_cast<const float4 *>(p + i * 8);
      const int4 c0 = cr[0], c1 = cr[1];
      const float4 p0 = pr[0], p1 = pr[1];
      cc[0] = c0.x; cc[1] = c0.y; cc[2] = c0.z; cc[3] = c0.w;
      cc[4] = c1.x; cc[5] = c1.y; cc[6] = c1.z; cc[7] = c1.w;
      ww[0] = p0.x; ww[1] = p0.y; ww[2] = p0.z; ww[3] = p0.w;
      ww[4] = p1.x; ww[5] = p1.y; ww[6] = p1.z; ww[7] = p1.w;
    } else {
#pragma unroll
      for (int k = 0; k < (KT > 0 ? KT : kMaxK); ++k) {
        cc[k] = k < K ? col[i * K + k] : -1;
        ww[k] = k < K ? p[i * K + k] : 0.0f;
      }
    }
    // Branch-free gathers: an empty slot (col = -1, weight 0) reads the point
    // itself.  All neighbour loads are issued before any is consumed.
    float gx[KB], gy[KB], gz[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const int64_t cj = cc[k] >= 0 ? (int64_t)cc[k] : i;
      if (!FROM_X) {
        gx[k] = rgb_in[3 * cj + 0];
        gy[k] = rgb_in[3 * cj + 1];
        gz[k] = rgb_in[3 * cj + 2];
      } else {
        const float4 xc = xin[cj];
        gx[k] = xc.x;
        gy[k] = xc.y;
        gz[k] = xc.z;
      }
    }
    float ar = 0.f, ag = 0.f, ab = 0.f;
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const float w = cc[k] >= 0 ? ww[k] : 0.0f;
      ar = fmaf(w, gx[k], ar);
      ag = fmaf(w, gy[k], ag);
      ab = fmaf(w, gz[k], ab);
    }
    float orr = xr, og = xg, ob = xb;
    if (cc[0] >= 0) {
      orr = 0.5f * xr + 0.5f * ar;
      og = 0.5f * xg + 0.5f * ag;
      ob = 0.5f * xb + 0.5f * ab;
    }
    xout[i] = make_float4(orr, og, ob, member);
    const unsigned long long x2 = to_fix((double)orr * orr + (double)og * og + (double)ob * ob);
    v[0] += member != 0.0f ? x2 : 0ull;
    v[1] += x2;
    if (FIRST && !MERGED) {
      const unsigned long long y2 = to_fix((double)xr * xr + (double)xg * xg + (double)xb * xb);
      v[2] += member != 0.0f ? y2 : 0ull;
      v[3] += y2;
      v[4] += member != 0.0f ? 1ull : 0ull;
    }
  }
  add_sums(v, sums_out, sb.lb % kSweepSlots, lds.red);
  if (MERGED) {
    __syncthreads();  // lds.red is reused
    add_sums(vf, io.sums_first + (size_t)sb.s * kSlotVals, sb.lb % kSweepSlots, lds.red);
  }
}

template <int KT, bool FIRST, bool D2, bool PRE = false, bool MERGED = false>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs a, int q, const int32_t *__restrict__ col,
                                                  const float *__restrict__ p, const float *__restrict__ rgb_in,
                                                  float4 *__restrict__ xbuf, const double *__restrict__ spread,
                                                  const fgbd_result *__restrict__ noise) {
  __shared__ SweepLds<D2> lds;
  const SegBlock sb = seg_block(a.sa, kGridSweep);
  const float *y = rgb_in;
  if (a.relabel && a.relabel[sb.s]) {  // a renumbered cloud: its graph and colours in scan-order-0 numbering
    y = a.rgb_w;
    col = a.col_w;
    a.dist2 = a.dist2_w;
  }
  sweep_step<KT, FIRST, D2, PRE, MERGED>(a, sb, sweep_io(a, q), col, p, y, xbuf, spread, noise, lds);
}

// Waits until every block of the grid has arrived `epoch` times at this
// barrier (count starts at 0 for the launch), with this block's writes
// released before its arrival and the others' acquired after.  The wait is
// bounded by `limit` ticks of the constant-rate clock; false when it gave up.
__device__ bool grid_barrier(uint32_t *count, uint32_t epoch, long long limit, int *s_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t target = epoch * gridDim.x;
    const long long t0 = wall_clock64();
    int ok = 1;
    while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (wall_clock64() - t0 > limit) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

// True when the selection of every cloud is done in states[0..B).  Each wave
// reads the B flags (one per lane) and votes, so the answer is uniform.
__device__ __forceinline__ bool all_clouds_done(const SweepCtrl *states, int B) {
  const int l = (int)lane_id();
  const bool open = l < B && !states[l].done;
  return __builtin_amdgcn_ballot_w64(open) == 0;
}

// Sweeps q0..q_last in one launch (same grid and block-to-cloud map as the
// separate launches; all blocks resident), every block waiting for all
// others after each sweep.  States are left where the finalising launch looks
// for them: in the buffer of q_last.  If a wait gives up, every block's cloud
// is flagged FGBD_ST_SWEEP_STALL and the loop ends.
// The finalising work of one block, from the cloud's final state c: the
// chosen iterate (or the input for q = 0) out, and block 0 of the cloud
// writes its results (and its sweep count to hint when given).
__device__ __forceinline__ void finalize_block(const SegBlock &sb, const SweepCtrl &c, int64_t buf_stride,
                                               const float *__restrict__ rgb_in, const float4 *__restrict__ xbuf,
                                               const fgbd_result *__restrict__ noise, float *__restrict__ rgb_out,
                                               fgbd_result *__restrict__ res, int32_t *hint,
                                               const uint32_t *__restrict__ rank0) {
  const int best = c.best_buf;
  const Share sh = seg_share(sb, kBlock);
  if (best == 3) {
    for (int64_t base = sh.first; base < sh.end; base += sh.step) {
      const int64_t i = base + threadIdx.x;
      if (i >= sh.end) continue;
      rgb_out[3 * i + 0] = rgb_in[3 * i + 0];
      rgb_out[3 * i + 1] = rgb_in[3 * i + 1];
      rgb_out[3 * i + 2] = rgb_in[3 * i + 2];
    }
  } else {
    // four chunks per pass, all their loads in flight before any store
    constexpr int U = 4;
    const float4 *xs = xbuf + (size_t)best * buf_stride;
    for (int64_t base = sh.first; base < sh.end; base += U * sh.step) {
      float4 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = base + u * sh.step + threadIdx.x;
        if (i < sh.end) x[u] = xs[rank0 ? (int64_t)rank0[i] : i];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = base + u * sh.step + threadIdx.x;
        if (i >= sh.end) continue;
        rgb_out[3 * i + 0] = x[u].x;
        rgb_out[3 * i + 1] = x[u].y;
        rgb_out[3 * i + 2] = x[u].z;
      }
    }
  }
  if (sb.lb == 0 && threadIdx.x == 0) {
    fgbd_result *r = res + sb.s;
    r->q = c.best_q;
    r->loss = c.best_loss;
    r->n_fslr = c.n_sel;
    r->sweeps = c.q;
    if (rank0) r->status |= FGBD_ST_RELABELED;
    if (noise != nullptr && noise != res) r->sigma_est = noise[sb.s].sigma_est;
    if (hint != nullptr) hint[sb.s] = c.q;
  }
}

__global__ __launch_bounds__(kBlock) void k_finalize(SegArgs sa, int64_t buf_stride, const float *__restrict__ rgb_in,
                                                     const float4 *__restrict__ xbuf,
                                                     const unsigned long long *__restrict__ sums_prev,
                                                     const unsigned long long *__restrict__ sums_first,
                                                     const SweepCtrl *__restrict__ ctrl_prev,
                                                     const fgbd_result *__restrict__ noise,
                                                     float *__restrict__ rgb_out, fgbd_result *__restrict__ res,
                                                     int32_t *hint, const int32_t *__restrict__ relabel,
                                                     const uint32_t *__restrict__ rank0) {
  const SegBlock sb = seg_block(sa, kGridSweep);
  SweepCtrl c;
  load_state(c, ctrl_prev + sb.s, sums_prev + (size_t)sb.s * kSlotVals, sums_first + (size_t)sb.s * kSlotVals,
             (int)(sb.end - sb.begin));
  finalize_block(sb, c, buf_stride, rgb_in, xbuf, noise, rgb_out, res, hint,
                 relabel && relabel[sb.s] ? rank0 : nullptr);
}

template <int KT>
__global__ __launch_bounds__(kBlock) void k_sweep_tail(SweepArgs a, int q0, int q_last, uint32_t *barrier,
                                                       long long wait_limit, const int32_t *__restrict__ col,
                                                       const float *__restrict__ p, const float *__restrict__ rgb_in,
                                                       float4 *__restrict__ xbuf, const double *__restrict__ spread,
                                                       const fgbd_result *__restrict__ noise,
                                                       float *__restrict__ rgb_out, int32_t *hint) {
  __shared__ SweepLds<false> lds;
  __shared__ int s_flag;
  const SegBlock sb = seg_block(a.sa, kGridSweep);
  if (a.relabel && a.relabel[sb.s]) col = a.col_w;  // a renumbered cloud's graph
  const int B = a.sa.B;
  // state at the start of the last separate sweep, written by that launch
  const SweepCtrl *last = a.ctrl + ((q0 - 1) & 1) * B;
  {
    // Those states advanced by that sweep's sums, one wave per cloud: when
    // every cloud is then done (the usual case once the schedule launches as
    // many separate sweeps as the selection needs), finalise at once, with no
    // loop and no wait for the other blocks.
    __shared__ int s_open;
    __shared__ SweepCtrl s_mine;  // this block's cloud, as the wave that advanced it left it
    if (threadIdx.x == 0) s_open = 0;
    __syncthreads();
    const size_t S = (size_t)B * kSlotVals;
    const unsigned long long *sums_sep = a.sums3 + (size_t)((q0 - 1) % 3) * S;
    const unsigned long long *sums_first = a.sums3 + 3 * S;
    for (int s2 = (int)threadIdx.x / kWave; s2 < B; s2 += kBlock / kWave) {
      const int n2 = a.sa.n_fixed >= 0 ? a.sa.n_fixed : a.sa.segs->start[s2 + 1] - a.sa.segs->start[s2];
      SweepCtrl cs;
      wave_advance(cs, last + s2, sums_sep + (size_t)s2 * kSlotVals, sums_first + (size_t)s2 * kSlotVals, n2);
      if (!cs.done && lane_id() == 0) s_open = 1;
      if (s2 == sb.s && lane_id() == 0) s_mine = cs;
    }
    __syncthreads();
    if (s_open == 0) {  // uniform over the grid: every block read the same states and sums
      const SweepCtrl c = s_mine;
      finalize_block(sb, c, a.buf_stride, rgb_in, xbuf, noise, rgb_out, a.res, hint,
                     a.relabel && a.relabel[sb.s] ? a.rank0 : nullptr);
      return;
    }
  }
  int q = q0;
  bool done = all_clouds_done(last, B);
  uint32_t epoch = 0;
  while (!done && q <= q_last) {
    sweep_step<KT, false, false>(a, sb, sweep_io(a, q), col, p, rgb_in, xbuf, spread, noise, lds);
    if (!grid_barrier(barrier, ++epoch, wait_limit, &s_flag)) {
      // The selection cannot be completed: flag the cloud and leave every
      // point of this block's share defined (its input colour).
      if (threadIdx.x == 0) atomicOr(&a.res[sb.s].status, FGBD_ST_SWEEP_STALL);
      const Share sh = seg_share(sb, kBlock);
      for (int64_t base = sh.first; base < sh.end; base += sh.step) {
        const int64_t i = base + threadIdx.x;
        if (i >= sh.end) continue;
        rgb_out[3 * i + 0] = rgb_in[3 * i + 0];
        rgb_out[3 * i + 1] = rgb_in[3 * i + 1];
        rgb_out[3 * i + 2] = rgb_in[3 * i + 2];
      }
      return;
    }
    last = a.ctrl + (q & 1) * B;
    done = all_clouds_done(last, B);
    ++q;
  }
  // Finalise.  Every sweep this launch computed ended at a grid barrier, and
  // the earlier ones were launches of their own.  Stopped early: the last
  // states read are final; else the states of q_last with its sums applied.
  SweepCtrl c;
  if (done) {
    c = last[sb.s];
  } else {
    const unsigned long long *sums_last = a.sums3 + (size_t)(q_last % 3) * B * kSlotVals;
    load_state(c, a.ctrl + (q_last & 1) * B + sb.s, sums_last + (size_t)sb.s * kSlotVals,
               a.sums3 + (size_t)3 * B * kSlotVals + (size_t)sb.s * kSlotVals, (int)(sb.end - sb.begin));
  }
  finalize_block(sb, c, a.buf_stride, rgb_in, xbuf, noise, rgb_out, a.res, hint,
                 a.relabel && a.relabel[sb.s] ? a.rank0 : nullptr);
}

SweepArgs sweep_args(const Run &r, const int32_t *dist2, float *p_out, fgbd_result *res, int select, int q_limit) {
  SweepArgs a;
  a.sa = r.sa;
  a.k = r.prm.k;
  a.select = select;
  a.q_limit = q_limit;
  a.kappa = r.prm.fslr_kappa;
  a.buf_stride = r.pl.n_cap;
  a.sums3 = r.b.sums;
  a.ctrl = r.b.ctrl;
  a.dist2 = dist2;
  a.edge_acc = r.b.edge_acc;
  a.sigma_g_fixed = r.prm.sigma_g;
  a.res = res;
  a.p_out = p_out;
  a.relabel = r.relabel_ok ? r.b.segs->relabel : nullptr;
  a.rgb_w = r.b.rgb_w;
  a.col_w = r.b.col_w;
  a.dist2_w = r.b.dist2_w;
  a.rank0 = r.b.rank;
  return a;
}

template <int KT, bool FIRST, bool D2, bool PRE = false, bool MERGED = false>
void sweep_kernel(int nb, hipStream_t st, const SweepArgs &a, int q, const int32_t *col, const float *p,
                  const float *rgb_in, float4 *xbuf, const double *spread, const fgbd_result *noise) {
  k_sweep<KT, FIRST, D2, PRE, MERGED><<<nb, kBlock, 0, st>>>(a, q, col, p, rgb_in, xbuf, spread, noise);
}

// Per device: blocks of k_sweep_tail<KT> resident at once, and ticks of the
// constant-rate clock in `us` microseconds (negative: half a second).
constexpr int kMaxDevices = 64;
template <int KT>
int tail_capacity() {
  static int cap[kMaxDevices];  // 0: not yet queried
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
  if (cap[dev] == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_sweep_tail<KT>, kBlock, 0) !=
            hipSuccess)
      cap[dev] = -1;
    else
      cap[dev] = cus * per_cu > 0 ? cus * per_cu : -1;
  }
  return cap[dev];
}
long long wait_ticks(int64_t us) {
  static long long khz_of[kMaxDevices];  // 0: not yet queried
  if (us < 0) us = 500000;
  int dev = 0;
  long long khz = 100000;  // 100 MHz when the rate cannot be read
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices) {
    if (khz_of[dev] == 0) {
      int k = 0;
      khz_of[dev] = hipDeviceGetAttribute(&k, hipDeviceAttributeWallClockRate, dev) == hipSuccess && k > 0 ? k : khz;
    }
    khz = khz_of[dev];
  }
  return (long long)(us > 10000000 ? 10000000 : us) * khz / 1000;
}

template <int KT>
hipError_t tail_kernel(int nb, hipStream_t st, const SweepArgs &a, int q0, int q_last, uint32_t *barrier,
                       long long ticks, const int32_t *col, const float *p, const float *rgb_in, float4 *xbuf,
                       const double *spread, const fgbd_result *noise, float *rgb_out, int32_t *hint) {
  k_sweep_tail<KT><<<nb, kBlock, 0, st>>>(a, q0, q_last, barrier, ticks, col, p, rgb_in, xbuf, spread, noise, rgb_out,
                                          hint);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep(const Run &r, const int32_t *col, const float *p, const int32_t *dist2,
                        const float *rgb_in, const double *spread, const fgbd_result *noise, fgbd_result *res,
                        int select, int q_limit, int q, bool pre, bool merged) {
  const bool first = q == 1, d2 = dist2 != nullptr;
  if (d2 && !first) return hipErrorInvalidValue;  // only the first sweep derives the weights
  if (merged) {  // sweeps 1 and 2 of the fused path in one launch (buffers of sweep 2)
    if (q != 2 || d2 || pre || r.prm.k != 8) return hipErrorInvalidValue;
    const SweepArgs a = sweep_args(r, nullptr, nullptr, res, select, q_limit);
    sweep_kernel<8, true, false, false, true>(r.pl.grid[kGridSweep], r.stream, a, q, col, p, rgb_in, r.b.xbuf,
                                              spread, noise);
    return hipGetLastError();
  }
  if (pre && (!first || d2 || r.prm.k != 8)) return hipErrorInvalidValue;
  if (pre) {
    const SweepArgs a = sweep_args(r, nullptr, nullptr, res, select, q_limit);
    sweep_kernel<8, true, false, true>(r.pl.grid[kGridSweep], r.stream, a, q, col, p, rgb_in, r.b.xbuf, spread,
                                       noise);
    return hipGetLastError();
  }
  // the first sweep of the fused path stores the weights it derives into p
  const SweepArgs a = sweep_args(r, dist2, d2 ? const_cast<float *>(p) : nullptr, res, select, q_limit);
  const int nb = r.pl.grid[kGridSweep];
  using Fn = void (*)(int, hipStream_t, const SweepArgs &, int, const int32_t *, const float *, const float *,
                      float4 *, const double *, const fgbd_result *);
  // [k == 8][later sweep, first sweep, first sweep deriving the weights]
  static const Fn table[2][3] = {
      {sweep_kernel<0, false, false>, sweep_kernel<0, true, false>, sweep_kernel<0, true, true>},
      {sweep_kernel<8, false, false>, sweep_kernel<8, true, false>, sweep_kernel<8, true, true>}};
  table[a.k == 8][first ? (d2 ? 2 : 1) : 0](nb, r.stream, a, q, col, p, rgb_in, r.b.xbuf, spread, noise);
  return hipGetLastError();
}

bool sweep_tail_fits(const Run &r) {
  return (r.prm.k == 8 ? tail_capacity<8>() : tail_capacity<0>()) >= r.pl.grid[kGridSweep];
}

hipError_t launch_sweep_tail(const Run &r, const int32_t *col, const float *p, const float *rgb_in,
                             const double *spread, const fgbd_result *noise, fgbd_result *res, int select,
                             int q_limit, int q0, int q_last, float *rgb_out) {
  const SweepArgs a = sweep_args(r, nullptr, nullptr, res, select, q_limit);
  const int nb = r.pl.grid[kGridSweep];
  using Fn = hipError_t (*)(int, hipStream_t, const SweepArgs &, int, int, uint32_t *, long long,
                            const int32_t *, const float *, const float *, float4 *, const double *,
                            const fgbd_result *, float *, int32_t *);
  static const Fn table[2] = {tail_kernel<0>, tail_kernel<8>};
  return table[a.k == 8](nb, r.stream, a, q0, q_last, &r.b.segs->sweep_barrier, wait_ticks(r.wait_us), col, p,
                         rgb_in, r.b.xbuf, spread, noise, rgb_out, r.hint);
}

hipError_t launch_finalize(const Run &r, const float *rgb_in, int q_launches, const fgbd_result *noise,
                           float *rgb_out, fgbd_result *res) {
  const size_t S = (size_t)r.pl.B * kSlotVals;
  const unsigned long long *sp = r.b.sums + (q_launches % 3) * S;
  const SweepCtrl *cp = r.b.ctrl + (q_launches & 1) * r.pl.B;
  k_finalize<<<r.pl.grid[kGridSweep], kBlock, 0, r.stream>>>(r.sa, r.pl.n_cap, rgb_in, r.b.xbuf, sp, r.b.sums + 3 * S, cp,
                                                              noise,
                                                              rgb_out, res, r.hint,
                                                              r.relabel_ok ? r.b.segs->relabel : nullptr, r.b.rank);
  return hipGetLastError();
}

}  // namespace fgbd
