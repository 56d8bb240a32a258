// Polynomial graph filter and its adjoint.
//
// out = sum_{k=0}^{n-1} c_k T^k x with T = D_g^{-1} W_g of eq. 5 built from the
// graph's squared distances and a bandwidth sigma_g held in device memory
// (eq. 4), so sigma_g can be a trained parameter.  c = e_q gives eq. 5.
//
// Forward: x_0 = x, x_k = T x_{k-1}; all iterates x_0..x_{n-1} are saved, and
// the last sweep also forms out from them.  Each sweep also saves
// u_k = sum_k' dp_ik' x_{k-1}[col_ik'] (2 (dT/dsigma_g) x_{k-1}, the per-slot
// coefficients dp from the weights launch), from the neighbour values it
// gathers anyway, so the backward's sigma_g term needs no gather.
// Backward, for L = <g, out>:
//   dL/dc_k     = <g, x_k>
//   z_{n-1} = c_{n-1} g,  z_k = c_k g + T^T z_{k+1},  dL/dx = z_0
//   dL/dsigma_g = sum_{m=1}^{n-1} <z_m, (dT/dsigma_g) x_{m-1}> = sum_m <z_m, u_m> / 2, where
//     dT/dsigma_g = (1/2) dP/dsigma_g and dp_ik/dsigma_g = p_ik (a_ik - sum_k' p_ik' a_ik'),
//     a_ik = 2 (d2_ik - d2_i0) / sigma_g^3 (the row shift cancels).
// T^T pulls along an explicit transpose of the directed graph: for every point
// j the edge ids e = i * K + slot with col[e] = j, in increasing order (built
// once per graph by fgbd_graph_transpose, or per call); the backward call
// first lays the weights out in that order (p_T[u] = p[edge[u]] / 2), so a
// step reads them contiguously and gathers only the adjoint.  One launch per
// backward step computes z_{m-1}, the step's sigma_g term and the
// coefficient products <g, x_{m-1}> together.  Scalar gradients are FP64
// per-block partials summed in block order by a one-block kernel.  No
// floating-point atomics anywhere, so every result is deterministic.
#include "fgbd_internal.h"

namespace fgbd {

namespace {

// Row-normalised weights of eq. 4 from squared distances and a device
// bandwidth, with the graph builder's row_weights (the same bits as the
// weights fgbd_build_slg stores for that bandwidth).
// With dp given (the forward call), also the per-slot derivative coefficients
//   dp_ik = p_ik (a_ik - sum_k' p_ik' a_ik'),  a_ik = 2 (d2_ik - d2_i0) / sigma_g^3
// (FP64, rounded to float; 0 for an empty slot and for a row without edges),
// so that dT/dsigma_g x = (1/2) sum_k dp_ik x[col_ik].  With diag given, also
// T's diagonal per point (the forward call stores it with p in saved, so the
// backward steps read 4 bytes per point instead of the first slot of each
// neighbour row).
template <int KT>
__global__ __launch_bounds__(kBlock) void k_poly_weights(int32_t n, int32_t k_rt, const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ dist2,
                                                         const double *__restrict__ sigma_g,
                                                         float *__restrict__ p, float *__restrict__ dp,
                                                         float *__restrict__ diag) {
  __shared__ double s_exp[kExpTable];
  const int K = KT > 0 ? KT : k_rt;
  const double sg = *sigma_g;
  fill_exp_table(sg, s_exp);
  __syncthreads();
  constexpr int KB = KT > 0 ? KT : kMaxK;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
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
    float pw[KB];
    row_weights<KB>(cv, dv, sg, s_exp, pw);
    if (diag) diag[i] = cv[0] >= 0 ? 0.5f : 1.0f;  // T's diagonal: 1/2 with edges, 1 without
    if (KT == 8) {
      float4 *pr = reinterpret_cast<float4 *>(p + i * 8);
      pr[0] = make_float4(pw[0], pw[1], pw[2], pw[3]);
      pr[1] = make_float4(pw[4], pw[5], pw[6], pw[7]);
    } else {
#pragma unroll
      for (int k = 0; k < KB; ++k)
        if (k < K) p[i * K + k] = pw[k];
    }
    if (dp) {
      const double a_scale = sg > 0.0 ? 2.0 / (sg * sg * sg) : 0.0;
      float dw[KB];
      double pa = 0.0;
#pragma unroll
      for (int k = 0; k < KB; ++k)
        if (k < K && cv[0] >= 0 && cv[k] >= 0) pa += (double)pw[k] * a_scale * (double)(dv[k] - dv[0]);
#pragma unroll
      for (int k = 0; k < KB; ++k)
        dw[k] = (k < K && cv[0] >= 0 && cv[k] >= 0) ? (float)((double)pw[k] * (a_scale * (double)(dv[k] - dv[0]) - pa))
                                                    : 0.0f;
      if (KT == 8) {
        float4 *dr = reinterpret_cast<float4 *>(dp + i * 8);
        dr[0] = make_float4(dw[0], dw[1], dw[2], dw[3]);
        dr[1] = make_float4(dw[4], dw[5], dw[6], dw[7]);
      } else {
#pragma unroll
        for (int k = 0; k < KB; ++k)
          if (k < K) dp[i * K + k] = dw[k];
      }
    }
  }
}

// ---------------------------------------------------------------- transpose
__global__ __launch_bounds__(kBlock) void k_zero_i32(int32_t *__restrict__ a, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) a[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_indegree(int32_t n, int32_t K, const int32_t *__restrict__ col,
                                                     int32_t *__restrict__ indeg) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < (int64_t)n * K; e += (int64_t)gridDim.x * kBlock) {
    const int j = col[e];
    if (j >= 0) atomicAdd(&indeg[j], 1);
  }
}

// Exclusive scan of n counts into off[0..n] in three launches: each block
// sums one chunk of kScanChunk counts, one block scans the chunk sums, each
// block rescans its chunk from its chunk's offset.
constexpr int kScanPer = 8;
constexpr int kScanChunkLen = kBlock * kScanPer;
__global__ __launch_bounds__(kBlock) void k_chunk_sums(int32_t n, const int32_t *__restrict__ cnt,
                                                       int32_t *__restrict__ sums) {
  __shared__ uint32_t s_tmp[4];
  const int64_t i0 = (int64_t)blockIdx.x * kScanChunkLen + (int64_t)threadIdx.x * kScanPer;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) s += i0 + j < n ? (uint32_t)cnt[i0 + j] : 0u;
  uint32_t tot;
  (void)block_exclusive_scan_256(s, s_tmp, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = (int32_t)tot;
}

__global__ __launch_bounds__(1024) void k_scan_sums(int32_t m, int32_t *__restrict__ sums, int32_t *__restrict__ total) {
  __shared__ uint32_t s_tmp[16];
  uint32_t carry = 0;
  for (int64_t base = 0; base < m; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint32_t v = i < m ? (uint32_t)sums[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, s_tmp, &tot);
    if (i < m) sums[i] = (int32_t)(carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0) *total = (int32_t)carry;
}

__global__ __launch_bounds__(kBlock) void k_chunk_apply(int32_t n, const int32_t *__restrict__ cnt,
                                                        const int32_t *__restrict__ sums, int32_t *__restrict__ off) {
  __shared__ uint32_t s_tmp[4];
  const int64_t i0 = (int64_t)blockIdx.x * kScanChunkLen + (int64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer], s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    v[j] = i0 + j < n ? (uint32_t)cnt[i0 + j] : 0u;
    s += v[j];
  }
  uint32_t tot;
  uint32_t run = (uint32_t)sums[blockIdx.x] + block_exclusive_scan_256(s, s_tmp, &tot);
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    if (i0 + j < n) off[i0 + j] = (int32_t)run;
    run += v[j];
  }
}

__global__ __launch_bounds__(kBlock) void k_fill(int32_t n, int32_t K, const int32_t *__restrict__ col,
                                                 const int32_t *__restrict__ off, int32_t *__restrict__ fill,
                                                 int32_t *__restrict__ tsrc) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < (int64_t)n * K; e += (int64_t)gridDim.x * kBlock) {
    const int j = col[e];
    if (j >= 0) tsrc[off[j] + atomicAdd(&fill[j], 1)] = (int32_t)e;
  }
}

// Sort each transposed row by edge id (= source * K + slot), giving a fixed
// order independent of the atomics above.  Rows of up to 16 entries are
// sorted in registers; longer ones in place.
constexpr int kRowReg = 16;
__global__ __launch_bounds__(kBlock) void k_sort_rows(int32_t n, const int32_t *__restrict__ off,
                                                      int32_t *__restrict__ tsrc) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
    const int a = off[j], b = off[j + 1];
    const int len = b - a;
    if (len <= kRowReg) {
      int v[kRowReg];
#pragma unroll
      for (int u = 0; u < kRowReg; ++u) v[u] = u < len ? tsrc[a + u] : 0x7fffffff;
      // odd-even transposition: kRowReg rounds sort kRowReg entries
#pragma unroll
      for (int r = 0; r < kRowReg; ++r) {
#pragma unroll
        for (int u = r & 1; u + 1 < kRowReg; u += 2) {
          const int x = v[u], y = v[u + 1];
          v[u] = min(x, y);
          v[u + 1] = max(x, y);
        }
      }
#pragma unroll
      for (int u = 0; u < kRowReg; ++u)
        if (u < len) tsrc[a + u] = v[u];
    } else {
      for (int u = a + 1; u < b; ++u) {
        const int v = tsrc[u];
        int w = u - 1;
        while (w >= a && tsrc[w] > v) {
          tsrc[w + 1] = tsrc[w];
          --w;
        }
        tsrc[w + 1] = v;
      }
    }
  }
}

// ---------------------------------------------------------------- forward
__device__ __forceinline__ void ld3(const float *__restrict__ x, int64_t i, float &a, float &b, float &c) {
  a = x[3 * i + 0];
  b = x[3 * i + 1];
  c = x[3 * i + 2];
}
__device__ __forceinline__ void st3(float *__restrict__ x, int64_t i, float a, float b, float c) {
  x[3 * i + 0] = a;
  x[3 * i + 1] = b;
  x[3 * i + 2] = c;
}

// One sweep x_k = T x_{k-1} (k >= 1) into saved[k].  The last sweep
// (k == ncoef - 1) also forms out = sum_k c_k x_k from the saved iterates.
template <int KT>
__global__ __launch_bounds__(kBlock) void k_poly_step(int32_t n, int32_t k_rt, int k, int ncoef,
                                                      const int32_t *__restrict__ col, const float *__restrict__ p,
                                                      const float *__restrict__ dp, const float *__restrict__ coef,
                                                      float *__restrict__ saved, float *__restrict__ out) {
  const int K = KT > 0 ? KT : k_rt;
  const size_t S = (size_t)n * 3;
  const float *xp = saved + (size_t)(k - 1) * S;
  float *xs = saved + (size_t)k * S;
  float *us = saved + (size_t)(ncoef + k - 1) * S;  // u_k after the ncoef iterates
  const bool last = k == ncoef - 1;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    float u0 = 0.f, u1 = 0.f, u2 = 0.f;
    int c0;
    if (KT == 8) {
      const int4 *cr = reinterpret_cast<const int4 *>(col + i * 8);
      const float4 *pr = reinterpret_cast<const float4 *>(p + i * 8);
      const float4 *dr = reinterpret_cast<const float4 *>(dp + i * 8);
      const int4 ca = cr[0], cb = cr[1];
      const float4 pa = pr[0], pb = pr[1], da = dr[0], db = dr[1];
      const int cv[8] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
      const float pv[8] = {pa.x, pa.y, pa.z, pa.w, pb.x, pb.y, pb.z, pb.w};
      const float dv[8] = {da.x, da.y, da.z, da.w, db.x, db.y, db.z, db.w};
      c0 = cv[0];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int64_t j = cv[kk] >= 0 ? (int64_t)cv[kk] : i;  // empty slot: weight 0, read self
        float y0, y1, y2;
        ld3(xp, j, y0, y1, y2);
        a0 = fmaf(pv[kk], y0, a0);
        a1 = fmaf(pv[kk], y1, a1);
        a2 = fmaf(pv[kk], y2, a2);
        u0 = fmaf(dv[kk], y0, u0);
        u1 = fmaf(dv[kk], y1, u1);
        u2 = fmaf(dv[kk], y2, u2);
      }
    } else {
      const int32_t *cr = col + i * K;
      const float *pr = p + i * K;
      const float *dr = dp + i * K;
      c0 = cr[0];
      for (int kk = 0; kk < K; ++kk) {
        const int64_t j = cr[kk] >= 0 ? (int64_t)cr[kk] : i;
        const float w = cr[kk] >= 0 ? pr[kk] : 0.0f;
        const float dw = cr[kk] >= 0 ? dr[kk] : 0.0f;
        float y0, y1, y2;
        ld3(xp, j, y0, y1, y2);
        a0 = fmaf(w, y0, a0);
        a1 = fmaf(w, y1, a1);
        a2 = fmaf(w, y2, a2);
        u0 = fmaf(dw, y0, u0);
        u1 = fmaf(dw, y1, u1);
        u2 = fmaf(dw, y2, u2);
      }
    }
    st3(us, i, u0, u1, u2);
    float s0, s1, s2;
    ld3(xp, i, s0, s1, s2);
    float v0 = s0, v1 = s1, v2 = s2;
    if (c0 >= 0) {
      v0 = 0.5f * s0 + 0.5f * a0;
      v1 = 0.5f * s1 + 0.5f * a1;
      v2 = 0.5f * s2 + 0.5f * a2;
    }
    st3(xs, i, v0, v1, v2);
    if (last) {
      const float ck = coef[k];
      float o0 = ck * v0, o1 = ck * v1, o2 = ck * v2;
      for (int kk = k - 1; kk >= 0; --kk) {
        float y0, y1, y2;
        ld3(saved + (size_t)kk * S, i, y0, y1, y2);
        const float c = coef[kk];
        o0 = fmaf(c, y0, o0);
        o1 = fmaf(c, y1, o1);
        o2 = fmaf(c, y2, o2);
      }
      st3(out, i, o0, o1, o2);
    }
  }
}

// x_0 = x into saved[0] (and out = c_0 x when there is one coefficient).
__global__ __launch_bounds__(kBlock) void k_poly_first(int32_t n, int ncoef, const float *__restrict__ x,
                                                       const float *__restrict__ coef, float *__restrict__ saved,
                                                       float *__restrict__ out) {
  const float c0 = coef[0];
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < 3 * (int64_t)n; i += (int64_t)gridDim.x * kBlock) {
    const float v = x[i];
    saved[i] = v;
    if (ncoef == 1) out[i] = c0 * v;
  }
}

// ---------------------------------------------------------------- backward
// p_T[u] = p[edge[u]] / 2 for u < off[n]: the weights (with T's factor 1/2)
// in the transpose's order, so each backward step reads them contiguously.
__global__ __launch_bounds__(kBlock) void k_poly_ptrans(int32_t n, const int32_t *__restrict__ off,
                                                        const int32_t *__restrict__ tsrc, const float *__restrict__ p,
                                                        float *__restrict__ pt) {
  const int64_t E = off[n];
  if (E <= 0) return;
  // four edges per thread and round, their id loads and then their gathers
  // in flight together (indices clamped, so no load needs a branch)
  constexpr int U = 4;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t u0 = (int64_t)blockIdx.x * kBlock + threadIdx.x; u0 < E; u0 += U * stride) {
    int32_t e[U];
    float w[U];
#pragma unroll
    for (int j = 0; j < U; ++j) e[j] = tsrc[min(u0 + j * stride, E - 1)];
#pragma unroll
    for (int j = 0; j < U; ++j) w[j] = p[e[j]];
#pragma unroll
    for (int j = 0; j < U; ++j)
      if (u0 + j * stride < E) pt[u0 + j * stride] = 0.5f * w[j];
  }
}

// One backward step m (z_m in, z_{m-1} out) per point j:
//   z_{m-1}[j] = c_{m-1} g[j] + T_jj z_m[j] + sum over edges e = (i -> j) of p_T z_m[i]
// (T_jj = 1/2 for a point with edges, 1 without, read from diag, which the
// forward's weights launch stored in saved), with the sigma_g term
// <z_m[j], u_m[j]> / 2 from the saved u_m and the coefficient product
// <g[j], x_{m-1}[j]> (and <g[j], x_m[j]> at the last step, where
// z_m = c_m g).  Only the adjoint is gathered.
template <int KT>
__global__ __launch_bounds__(kBlock) void k_poly_back(int32_t n, int32_t k_rt, int m, int last, int nb, int ncoef,
                                                      const float *__restrict__ diag, const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ tsrc, const float *__restrict__ pt,
                                                      const float *__restrict__ coef, const float *__restrict__ g,
                                                      const float *__restrict__ saved, const float *__restrict__ zin,
                                                      float *__restrict__ zout, double *__restrict__ sig_part,
                                                      double *__restrict__ cpart) {
  __shared__ double s_red[8 * 3];
  const int K = KT > 0 ? KT : k_rt;
  const float cm = coef[m], cm1 = coef[m - 1];
  const size_t S = (size_t)n * 3;
  const float *xprev = saved + (size_t)(m - 1) * S;
  const float *xcur = saved + (size_t)m * S;
  const float *um = saved + (size_t)(ncoef + m - 1) * S;
  // z_{m+1} is c_m g on the last step (m = ncoef - 1), else the previous step's
  // output; <g, x_m> is needed on the last step only (yrow reads x_{m-1} again
  // otherwise, from cache)
  const float *zsrc = last ? g : zin;
  const float zs = last ? cm : 1.0f;
  const float *yrow = last ? xcur : xprev;
  // acc[0]: sigma_g term; acc[1]: <g, x_{m-1}>; acc[2]: <g, x_m> (last step only)
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
    // every load of the row is unconditional (the step's kind only picks the
    // pointers), so they are all in flight together
    float g0, g1, g2, z0, z1, z2, x0, x1, x2, y0, y1, y2, u0, u1, u2;
    ld3(g, j, g0, g1, g2);
    ld3(zsrc, j, z0, z1, z2);
    ld3(xprev, j, x0, x1, x2);
    ld3(yrow, j, y0, y1, y2);
    ld3(um, j, u0, u1, u2);
    z0 *= zs;
    z1 *= zs;
    z2 *= zs;
    acc[1] += (double)g0 * x0 + (double)g1 * x1 + (double)g2 * x2;
    const double gy = (double)g0 * y0 + (double)g1 * y1 + (double)g2 * y2;
    acc[2] += last ? gy : 0.0;
    acc[0] += 0.5 * ((double)z0 * u0 + (double)z1 * u1 + (double)z2 * u2);
    // T^T z_m at j
    const float tjj = diag[j];
    float r0 = tjj * z0, r1 = tjj * z1, r2 = tjj * z2;
    // in-edges four at a time (their ids, weights and gathers all in flight
    // together), then the rest one by one; the order of the additions is the
    // edges' order either way
    const int a = off[j], b = off[j + 1];
    int u = a;
    for (; u + 4 <= b; u += 4) {
      int64_t sr[4];
      float w[4], s[4][3];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        sr[e] = tsrc[u + e] / K;
        w[e] = pt[u + e];
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) ld3(zsrc, sr[e], s[e][0], s[e][1], s[e][2]);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        r0 = fmaf(w[e], zs * s[e][0], r0);
        r1 = fmaf(w[e], zs * s[e][1], r1);
        r2 = fmaf(w[e], zs * s[e][2], r2);
      }
    }
    for (; u < b; ++u) {
      const int64_t src = tsrc[u] / K;
      const float w = pt[u];
      float s0, s1, s2;
      ld3(zsrc, src, s0, s1, s2);
      r0 = fmaf(w, zs * s0, r0);
      r1 = fmaf(w, zs * s1, r1);
      r2 = fmaf(w, zs * s2, r2);
    }
    st3(zout, j, fmaf(cm1, g0, r0), fmaf(cm1, g1, r1), fmaf(cm1, g2, r2));
  }
  block_sum_f64<3>(acc, s_red);
  if (threadIdx.x == 0) {
    sig_part[blockIdx.x] = acc[0];
    cpart[(size_t)(m - 1) * nb + blockIdx.x] = acc[1];
    if (last) cpart[(size_t)m * nb + blockIdx.x] = acc[2];
  }
}

// One coefficient: z_0 = c_0 g and <g, x_0>.
__global__ __launch_bounds__(kBlock) void k_scale(int32_t n, const float *__restrict__ coef,
                                                  const float *__restrict__ g, const float *__restrict__ x0,
                                                  float *__restrict__ z, double *__restrict__ cpart) {
  __shared__ double s_red[8];
  const float c0 = coef[0];
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < 3 * (int64_t)n; i += (int64_t)gridDim.x * kBlock) {
    z[i] = c0 * g[i];
    acc[0] += (double)g[i] * x0[i];
  }
  block_sum_f64<1>(acc, s_red);
  if (threadIdx.x == 0) cpart[blockIdx.x] = acc[0];
}

// One block of kReduceWaves waves: wave v sums value v's nb partials (v =
// coefficient k < ncoef, then the sigma_g term of backward step m = v -
// ncoef + 1): lane l adds partials l, l + 64, ... with all its loads in
// flight together, then a shuffle tree adds the lanes; thread 0 writes the
// coefficient gradients and adds the sigma_g terms in m order.  The order of
// every sum is fixed.
constexpr int kReduceWaves = 16;
__global__ __launch_bounds__(kReduceWaves * kWave) void k_poly_reduce(int ncoef, int nb,
                                                                     const double *__restrict__ coef_part,
                                                                     const double *__restrict__ sig_part,
                                                                     float *__restrict__ grad_coef,
                                                                     double *__restrict__ grad_sigma) {
  __shared__ double s_val[2 * kMaxPoly];
  const int V = 2 * ncoef - 1;
  const int wave = threadIdx.x / kWave, lane = (int)lane_id();
  constexpr int U = 16;  // loads in flight per lane
  for (int v = wave; v < V; v += kReduceWaves) {
    const double *row = v < ncoef ? coef_part + (size_t)v * nb : sig_part + (size_t)(v - ncoef + 1) * nb;
    double acc = 0.0;
    for (int b0 = lane; b0 < nb; b0 += U * kWave) {
      double x[U];
#pragma unroll
      for (int j = 0; j < U; ++j) x[j] = row[min(b0 + j * kWave, nb - 1)];  // clamped: no branch per load
#pragma unroll
      for (int j = 0; j < U; ++j) acc += b0 + j * kWave < nb ? x[j] : 0.0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, kWave);
    if (lane == 0) s_val[v] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 0; v < ncoef; ++v)
      if (grad_coef) grad_coef[v] = (float)s_val[v];
    double total = 0.0;
    for (int v = ncoef; v < V; ++v) total += s_val[v];
    if (grad_sigma) *grad_sigma = total;
  }
}

}  // namespace

size_t transpose_workspace(int64_t n) {
  const size_t N = (size_t)(n > 0 ? n : 1);
  const size_t chunks = (N + kScanChunkLen - 1) / kScanChunkLen;
  size_t b = 0;
  auto take = [&](size_t bytes) { b += (bytes + 255) & ~(size_t)255; };
  take(N * 4);             // in-degree / fill counters
  take((chunks + 1) * 4);  // chunk sums
  return b;
}

size_t poly_workspace(int64_t n, int k, int ncoef, int nblocks) {
  const size_t N = (size_t)(n > 0 ? n : 1);
  size_t b = 0;
  auto take = [&](size_t bytes) { b += (bytes + 255) & ~(size_t)255; };
  take(N * k * 4);                     // dp (forward) or p in the transpose's order (backward)
  take((N + 1) * 4);                   // offsets (when no transpose is given)
  take(N * k * 4);                     // transposed edge ids (same)
  take(2 * N * 3 * 4);                 // z ping-pong
  take((size_t)ncoef * nblocks * 8);   // coef partials
  take((size_t)ncoef * nblocks * 8);   // sigma partials
  take(transpose_workspace(n));        // transpose scratch
  return b;
}

struct PolyBufs {
  float *aux;
  int32_t *off, *tsrc;
  float *z[2];
  double *coef_part, *sig_part;
  char *tws;
};

static PolyBufs poly_carve(char *ws, int64_t n, int k, int ncoef, int nblocks) {
  const size_t N = (size_t)(n > 0 ? n : 1);
  PolyBufs pb;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char *ptr = ws + o;
    o += (bytes + 255) & ~(size_t)255;
    return ptr;
  };
  pb.aux = (float *)take(N * k * 4);
  pb.off = (int32_t *)take((N + 1) * 4);
  pb.tsrc = (int32_t *)take(N * k * 4);
  pb.z[0] = (float *)take(N * 3 * 4);
  pb.z[1] = (float *)take(N * 3 * 4);
  pb.coef_part = (double *)take((size_t)ncoef * nblocks * 8);
  pb.sig_part = (double *)take((size_t)ncoef * nblocks * 8);
  pb.tws = take(transpose_workspace(n));
  return pb;
}

static int grid_for(int64_t items) {
  const int64_t g = (items + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g < kPolyGrid ? g : kPolyGrid));
}

hipError_t launch_transpose(int64_t n, int k, const int32_t *col, int32_t *off, int32_t *tsrc, char *ws,
                            hipStream_t s) {
  const size_t N = (size_t)(n > 0 ? n : 1);
  int32_t *cnt = (int32_t *)ws;
  int32_t *sums = (int32_t *)(ws + ((N * 4 + 255) & ~(size_t)255));
  const int chunks = (int)((N + kScanChunkLen - 1) / kScanChunkLen);
  const int G = grid_for(n);
  const int GE = grid_for(n * k);
  k_zero_i32<<<G, kBlock, 0, s>>>(cnt, n);
  k_indegree<<<GE, kBlock, 0, s>>>((int32_t)n, k, col, cnt);
  k_chunk_sums<<<chunks, kBlock, 0, s>>>((int32_t)n, cnt, sums);
  k_scan_sums<<<1, 1024, 0, s>>>(chunks, sums, off + n);
  k_chunk_apply<<<chunks, kBlock, 0, s>>>((int32_t)n, cnt, sums, off);
  k_zero_i32<<<G, kBlock, 0, s>>>(cnt, n);
  k_fill<<<GE, kBlock, 0, s>>>((int32_t)n, k, col, off, cnt, tsrc);
  k_sort_rows<<<G, kBlock, 0, s>>>((int32_t)n, off, tsrc);
  return hipGetLastError();
}

// saved: the 2 ncoef - 1 arrays [n][3] (iterates, then u_m), and for ncoef >= 2
// the forward's weights p [n][k] (from a 64-float boundary, so rows stay
// 16-byte aligned) and T's diagonal [n], which the backward reads instead of
// recomputing them.
static size_t poly_saved_p_offset(int64_t n, int ncoef) {
  const size_t iter = (size_t)(2 * ncoef - 1) * 3 * (size_t)n;
  return (iter + 63) / 64 * 64;
}
size_t poly_saved_floats(int64_t n, int k, int ncoef) {
  const size_t iter = (size_t)(2 * ncoef - 1) * 3 * (size_t)n;
  return ncoef >= 2 ? poly_saved_p_offset(n, ncoef) + (size_t)n * k + (size_t)n : iter;
}

hipError_t launch_poly_forward(int64_t n, int k, const int32_t *col, const int32_t *dist2, const float *x,
                               const float *coef, int ncoef, const double *sigma_g, float *out, float *saved,
                               char *ws, hipStream_t s) {
  PolyBufs pb = poly_carve(ws, n, k, ncoef, kPolyGrid);
  const int G = grid_for(n);
  k_poly_first<<<grid_for(3 * n), kBlock, 0, s>>>((int32_t)n, ncoef, x, coef, saved, out);
  if (ncoef == 1) return hipGetLastError();
  float *p = saved + poly_saved_p_offset(n, ncoef);
  float *diag = p + (size_t)n * k;
  if (k == 8)
    k_poly_weights<8><<<G, kBlock, 0, s>>>((int32_t)n, k, col, dist2, sigma_g, p, pb.aux, diag);
  else
    k_poly_weights<0><<<G, kBlock, 0, s>>>((int32_t)n, k, col, dist2, sigma_g, p, pb.aux, diag);
  for (int kk = 1; kk < ncoef; ++kk) {
    if (k == 8)
      k_poly_step<8><<<G, kBlock, 0, s>>>((int32_t)n, k, kk, ncoef, col, p, pb.aux, coef, saved, out);
    else
      k_poly_step<0><<<G, kBlock, 0, s>>>((int32_t)n, k, kk, ncoef, col, p, pb.aux, coef, saved, out);
  }
  return hipGetLastError();
}

hipError_t launch_poly_backward(int64_t n, int k, const int32_t *col, const int32_t *dist2, const int32_t *t_off,
                                const int32_t *t_edge, const float *saved, const float *coef, int ncoef,
                                const double *sigma_g, const float *grad_out, float *grad_x, float *grad_coef,
                                double *grad_sigma, char *ws, hipStream_t s) {
  PolyBufs pb = poly_carve(ws, n, k, ncoef, kPolyGrid);
  const int G = grid_for(n);
  if (ncoef == 1) {
    const int G3 = grid_for(3 * n);
    k_scale<<<G3, kBlock, 0, s>>>((int32_t)n, coef, grad_out, saved, grad_x, pb.coef_part);
    k_poly_reduce<<<1, kReduceWaves * kWave, 0, s>>>(1, G3, pb.coef_part, pb.sig_part, grad_coef, grad_sigma);
    return hipGetLastError();
  }
  if (!t_off) {  // no transpose given: build one in the workspace
    hipError_t e = launch_transpose(n, k, col, pb.off, pb.tsrc, pb.tws, s);
    if (e != hipSuccess) return e;
    t_off = pb.off;
    t_edge = pb.tsrc;
  }
  // the forward's weights and T's diagonal, from saved
  const float *p = saved + poly_saved_p_offset(n, ncoef);
  const float *diag = p + (size_t)n * k;
  k_poly_ptrans<<<grid_for(n * k), kBlock, 0, s>>>((int32_t)n, t_off, t_edge, p, pb.aux);
  // reverse Horner; coefficient products ride along
  const float *zin = nullptr;
  for (int m = ncoef - 1; m >= 1; --m) {
    float *zout = (m == 1) ? grad_x : pb.z[m & 1];
    if (k == 8)
      k_poly_back<8><<<G, kBlock, 0, s>>>((int32_t)n, k, m, m == ncoef - 1, G, ncoef, diag, t_off, t_edge, pb.aux,
                                          coef, grad_out, saved, zin, zout, pb.sig_part + (size_t)m * G,
                                          pb.coef_part);
    else
      k_poly_back<0><<<G, kBlock, 0, s>>>((int32_t)n, k, m, m == ncoef - 1, G, ncoef, diag, t_off, t_edge, pb.aux,
                                          coef, grad_out, saved, zin, zout, pb.sig_part + (size_t)m * G,
                                          pb.coef_part);
    zin = zout;
  }
  k_poly_reduce<<<1, kReduceWaves * kWave, 0, s>>>(ncoef, G, pb.coef_part, pb.sig_part, grad_coef, grad_sigma);
  return hipGetLastError();
}

}  // namespace fgbd
