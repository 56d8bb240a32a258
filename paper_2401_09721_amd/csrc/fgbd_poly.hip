// Polynomial graph filter and its adjoint.
//
// out = sum_{k=0}^{n-1} c_k T^k x with T = D_g^{-1} W_g of eq. 5 built from the
// graph's squared distances and a bandwidth sigma_g held in device memory
// (eq. 4), so sigma_g can be a trained parameter.  c = e_q gives eq. 5.
//
// Forward: x_0 = x, x_k = T x_{k-1}; all iterates x_0..x_{n-1} are saved.
// Backward, for L = <g, out>:
//   dL/dc_k     = <g, x_k>
//   z_{n-1} = c_{n-1} g,  z_k = c_k g + T^T z_{k+1},  dL/dx = z_0
//   dL/dsigma_g = sum_{m=1}^{n-1} <z_m, (dT/dsigma_g) x_{m-1}>, where
//     dT/dsigma_g = (1/2) dP/dsigma_g and dp_ik/dsigma_g = p_ik (a_ik - sum_k' p_ik' a_ik'),
//     a_ik = 2 (d2_ik - d2_i0) / sigma_g^3 (the row shift cancels).
// T^T uses an explicit transpose of the directed graph: for every point j
// the edges (i, k) with col_ik = j, counted with integer atomics, placed, and
// then sorted by source within each row so every sum has a fixed order.
// Scalar gradients are FP64 per-block partials summed in block order by a
// one-block kernel.  No floating-point atomics anywhere.
#include "fgbd_internal.h"

namespace fgbd {

namespace {

// Row-normalised weights from squared distances and a device bandwidth.
__global__ __launch_bounds__(kBlock) void k_poly_weights(int32_t n, int32_t K, const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ dist2,
                                                         const double *__restrict__ sigma_g,
                                                         float *__restrict__ p) {
  const double sg = *sigma_g;
  const double inv = sg > 0.0 ? 1.0 / (sg * sg) : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const int32_t *cr = col + i * K;
    const int32_t *dr = dist2 + i * K;
    const int d0 = dr[0];
    double s = 0.0;
    for (int k = 0; k < K; ++k)
      if (cr[k] >= 0) s += sg > 0.0 ? exp(-(double)(dr[k] - d0) * inv) : (dr[k] == d0 ? 1.0 : 0.0);
    const double rs = s > 0.0 ? 1.0 / s : 0.0;
    for (int k = 0; k < K; ++k) {
      double w = 0.0;
      if (cr[k] >= 0) w = sg > 0.0 ? exp(-(double)(dr[k] - d0) * inv) : (dr[k] == d0 ? 1.0 : 0.0);
      p[i * K + k] = (float)(w * rs);
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

// Exclusive scan of n int32 counts into offsets[0..n] (one block of 1024
// threads, chunks of 8 per thread with a running carry).
__global__ __launch_bounds__(1024) void k_scan_counts(int32_t n, const int32_t *__restrict__ cnt,
                                                      int32_t *__restrict__ off) {
  __shared__ uint32_t s_tmp[16];
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += 1024 * 8) {
    const int64_t i0 = base + (int64_t)threadIdx.x * 8;
    uint32_t v[8], sum = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      v[j] = (i0 + j < n) ? (uint32_t)cnt[i0 + j] : 0u;
      sum += v[j];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan(sum, s_tmp, &tot);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (i0 + j < n) off[i0 + j] = (int32_t)run;
      run += v[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) off[n] = (int32_t)carry;
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
// order independent of the atomics above.  Rows are short (about K).
__global__ __launch_bounds__(kBlock) void k_sort_rows(int32_t n, const int32_t *__restrict__ off,
                                                      int32_t *__restrict__ tsrc) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (int64_t)gridDim.x * kBlock) {
    const int a = off[j], b = off[j + 1];
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

// ---------------------------------------------------------------- forward
// x_k = T x_{k-1} (k >= 1) into saved[k]; out = c_0 x_0 + ... accumulated.
// k == 0 copies x into saved[0] and sets out = c_0 x.
__global__ __launch_bounds__(kBlock) void k_poly_step(int32_t n, int32_t K, int k, const int32_t *__restrict__ col,
                                                      const float *__restrict__ p, const float *__restrict__ x,
                                                      const float *__restrict__ coef, float *__restrict__ saved,
                                                      float *__restrict__ out) {
  const float ck = coef[k];
  const size_t S = (size_t)n * 3;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    float v[3];
    if (k == 0) {
      v[0] = x[3 * i + 0];
      v[1] = x[3 * i + 1];
      v[2] = x[3 * i + 2];
    } else {
      const float *xp = saved + (size_t)(k - 1) * S;
      const int32_t *cr = col + i * K;
      const float *pr = p + i * K;
      float a0 = 0.f, a1 = 0.f, a2 = 0.f;
      for (int kk = 0; kk < K; ++kk) {
        const int64_t j = cr[kk] >= 0 ? (int64_t)cr[kk] : i;  // empty slot: weight 0, read self
        const float w = cr[kk] >= 0 ? pr[kk] : 0.0f;
        a0 = fmaf(w, xp[3 * j + 0], a0);
        a1 = fmaf(w, xp[3 * j + 1], a1);
        a2 = fmaf(w, xp[3 * j + 2], a2);
      }
      const float s0 = xp[3 * i + 0], s1 = xp[3 * i + 1], s2 = xp[3 * i + 2];
      if (cr[0] >= 0) {
        v[0] = 0.5f * s0 + 0.5f * a0;
        v[1] = 0.5f * s1 + 0.5f * a1;
        v[2] = 0.5f * s2 + 0.5f * a2;
      } else {
        v[0] = s0;
        v[1] = s1;
        v[2] = s2;
      }
    }
    float *xs = saved + (size_t)k * S;
    xs[3 * i + 0] = v[0];
    xs[3 * i + 1] = v[1];
    xs[3 * i + 2] = v[2];
    if (k == 0) {
      out[3 * i + 0] = ck * v[0];
      out[3 * i + 1] = ck * v[1];
      out[3 * i + 2] = ck * v[2];
    } else {
      out[3 * i + 0] = fmaf(ck, v[0], out[3 * i + 0]);
      out[3 * i + 1] = fmaf(ck, v[1], out[3 * i + 1]);
      out[3 * i + 2] = fmaf(ck, v[2], out[3 * i + 2]);
    }
  }
}

// ---------------------------------------------------------------- backward
// One step m (n-1 >= m >= 1): from z_m compute z_{m-1} = c_{m-1} g + T^T z_m
// and the sigma_g term of step m, <z_m, (dT/dsigma) x_{m-1}>, as per-block
// FP64 partials.  z_m for m = n-1 is c_{n-1} g (read from g directly).
__global__ __launch_bounds__(kBlock) void k_poly_back(int32_t n, int32_t K, int m, int last,
                                                      const int32_t *__restrict__ col, const int32_t *__restrict__ dist2,
                                                      const float *__restrict__ p, const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ tsrc, const double *__restrict__ sigma_g,
                                                      const float *__restrict__ coef, const float *__restrict__ g,
                                                      const float *__restrict__ saved, const float *__restrict__ zin,
                                                      float *__restrict__ zout, double *__restrict__ part) {
  __shared__ double s_red[8];
  const double sg = *sigma_g;
  const double a_scale = sg > 0.0 ? 2.0 / (sg * sg * sg) : 0.0;
  const float cm = coef[m], cm1 = coef[m - 1];
  const float *xprev = saved + (size_t)(m - 1) * n * 3;
  double acc[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    // z_m of this point (z_{n-1} = c_{n-1} g)
    float z0, z1, z2;
    if (last) {
      z0 = cm * g[3 * i + 0];
      z1 = cm * g[3 * i + 1];
      z2 = cm * g[3 * i + 2];
    } else {
      z0 = zin[3 * i + 0];
      z1 = zin[3 * i + 1];
      z2 = zin[3 * i + 2];
    }
    // sigma_g term: (1/2) sum_k dp_ik <z_m[i], x_{m-1}[col_ik]>
    const int32_t *cr = col + i * K;
    if (cr[0] >= 0) {
      const int32_t *dr = dist2 + i * K;
      const float *pr = p + i * K;
      const int d0 = dr[0];
      double pa = 0.0;
      for (int k = 0; k < K; ++k)
        if (cr[k] >= 0) pa += (double)pr[k] * a_scale * (double)(dr[k] - d0);
      double t = 0.0;
      for (int k = 0; k < K; ++k) {
        const int j = cr[k];
        if (j >= 0) {
          const double dp = (double)pr[k] * (a_scale * (double)(dr[k] - d0) - pa);
          const double dot = (double)z0 * xprev[3 * (size_t)j + 0] + (double)z1 * xprev[3 * (size_t)j + 1] +
                             (double)z2 * xprev[3 * (size_t)j + 2];
          t += dp * dot;
        }
      }
      acc[0] += 0.5 * t;
    }
    // z_{m-1}[i] = c_{m-1} g[i] + T_ii z_m[i] + sum over in-edges (e = src*K + k) of p_e / 2 z_m[src]
    const float tii = cr[0] >= 0 ? 0.5f : 1.0f;
    float r0 = tii * z0, r1 = tii * z1, r2 = tii * z2;
    const int a = off[i], b = off[i + 1];
    for (int u = a; u < b; ++u) {
      const int e = tsrc[u];
      const int64_t src = e / K;
      const float w = 0.5f * p[e];
      float s0, s1, s2;
      if (last) {
        s0 = cm * g[3 * src + 0];
        s1 = cm * g[3 * src + 1];
        s2 = cm * g[3 * src + 2];
      } else {
        s0 = zin[3 * src + 0];
        s1 = zin[3 * src + 1];
        s2 = zin[3 * src + 2];
      }
      r0 = fmaf(w, s0, r0);
      r1 = fmaf(w, s1, r1);
      r2 = fmaf(w, s2, r2);
    }
    zout[3 * i + 0] = fmaf(cm1, g[3 * i + 0], r0);
    zout[3 * i + 1] = fmaf(cm1, g[3 * i + 1], r1);
    zout[3 * i + 2] = fmaf(cm1, g[3 * i + 2], r2);
  }
  block_sum_f64<1>(acc, s_red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// z_0 = c_0 g when there is a single coefficient.
__global__ __launch_bounds__(kBlock) void k_scale(int32_t n, const float *__restrict__ coef,
                                                  const float *__restrict__ g, float *__restrict__ z) {
  const float c0 = coef[0];
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < 3 * (int64_t)n; i += (int64_t)gridDim.x * kBlock)
    z[i] = c0 * g[i];
}

// <g, x_k> per block for every k.
__global__ __launch_bounds__(kBlock) void k_coef_grad(int32_t n, int ncoef, const float *__restrict__ g,
                                                      const float *__restrict__ saved, double *__restrict__ part) {
  __shared__ double s_buf[8];
  for (int k = 0; k < ncoef; ++k) {
    const float *xk = saved + (size_t)k * n * 3;
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < 3 * (int64_t)n; i += (int64_t)gridDim.x * kBlock)
      acc[0] += (double)g[i] * (double)xk[i];
    block_sum_f64<1>(acc, s_buf);
    if (threadIdx.x == 0) part[(size_t)k * gridDim.x + blockIdx.x] = acc[0];
  }
}

// One block: sum partials in block order.  grad_coef[k] from coef partials,
// grad_sigma from the n-1 backward-step partials.
__global__ __launch_bounds__(kBlock) void k_poly_reduce(int ncoef, int nb, const double *__restrict__ coef_part,
                                                        const double *__restrict__ sig_part,
                                                        float *__restrict__ grad_coef,
                                                        double *__restrict__ grad_sigma) {
  __shared__ double s_red[8];
  for (int k = 0; k < ncoef; ++k) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += kBlock) v[0] += coef_part[(size_t)k * nb + b];
    block_sum_f64<1>(v, s_red);
    if (threadIdx.x == 0 && grad_coef) grad_coef[k] = (float)v[0];
  }
  double total = 0.0;
  for (int m = 1; m < ncoef; ++m) {
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += kBlock) v[0] += sig_part[(size_t)m * nb + b];
    block_sum_f64<1>(v, s_red);
    total += v[0];  // valid in thread 0
  }
  if (threadIdx.x == 0 && grad_sigma) *grad_sigma = total;
}

}  // namespace

size_t poly_workspace(int64_t n, int k, int ncoef, int nblocks) {
  const size_t N = (size_t)(n > 0 ? n : 1);
  size_t b = 0;
  auto take = [&](size_t bytes) { b += (bytes + 255) & ~(size_t)255; };
  take(N * k * 4);                     // p
  take(N * 4);                         // indegree / fill counters
  take((N + 1) * 4);                   // offsets
  take(N * k * 4);                     // transposed edge ids
  take(2 * N * 3 * 4);                 // z ping-pong
  take((size_t)ncoef * nblocks * 8);   // coef partials
  take((size_t)ncoef * nblocks * 8);   // sigma partials
  return b;
}

struct PolyBufs {
  float *p;
  int32_t *cnt, *off, *tsrc;
  float *z[2];
  double *coef_part, *sig_part;
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
  pb.p = (float *)take(N * k * 4);
  pb.cnt = (int32_t *)take(N * 4);
  pb.off = (int32_t *)take((N + 1) * 4);
  pb.tsrc = (int32_t *)take(N * k * 4);
  pb.z[0] = (float *)take(N * 3 * 4);
  pb.z[1] = (float *)take(N * 3 * 4);
  pb.coef_part = (double *)take((size_t)ncoef * nblocks * 8);
  pb.sig_part = (double *)take((size_t)ncoef * nblocks * 8);
  return pb;
}

static int grid_for(int64_t items) {
  const int64_t g = (items + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g < kMaxGrid ? g : kMaxGrid));
}

hipError_t launch_poly_forward(int64_t n, int k, const int32_t *col, const int32_t *dist2, const float *x,
                               const float *coef, int ncoef, const double *sigma_g, float *out, float *saved,
                               char *ws, hipStream_t s) {
  PolyBufs pb = poly_carve(ws, n, k, ncoef, kMaxGrid);
  const int G = grid_for(n);
  k_poly_weights<<<G, kBlock, 0, s>>>((int32_t)n, k, col, dist2, sigma_g, pb.p);
  for (int kk = 0; kk < ncoef; ++kk)
    k_poly_step<<<G, kBlock, 0, s>>>((int32_t)n, k, kk, col, pb.p, x, coef, saved, out);
  return hipGetLastError();
}

hipError_t launch_poly_backward(int64_t n, int k, const int32_t *col, const int32_t *dist2, const float *saved,
                                const float *coef, int ncoef, const double *sigma_g, const float *grad_out,
                                float *grad_x, float *grad_coef, double *grad_sigma, char *ws, hipStream_t s) {
  PolyBufs pb = poly_carve(ws, n, k, ncoef, kMaxGrid);
  const int G = grid_for(n);
  const int GE = grid_for(n * k);
  k_poly_weights<<<G, kBlock, 0, s>>>((int32_t)n, k, col, dist2, sigma_g, pb.p);
  // transpose of the directed graph, rows sorted by source
  k_zero_i32<<<G, kBlock, 0, s>>>(pb.cnt, n);
  k_indegree<<<GE, kBlock, 0, s>>>((int32_t)n, k, col, pb.cnt);
  k_scan_counts<<<1, 1024, 0, s>>>((int32_t)n, pb.cnt, pb.off);
  k_zero_i32<<<G, kBlock, 0, s>>>(pb.cnt, n);
  k_fill<<<GE, kBlock, 0, s>>>((int32_t)n, k, col, pb.off, pb.cnt, pb.tsrc);
  k_sort_rows<<<G, kBlock, 0, s>>>((int32_t)n, pb.off, pb.tsrc);
  // reverse Horner
  if (ncoef == 1) {
    k_scale<<<grid_for(3 * n), kBlock, 0, s>>>((int32_t)n, coef, grad_out, grad_x);
  } else {
    const float *zin = nullptr;
    for (int m = ncoef - 1; m >= 1; --m) {
      float *zout = (m == 1) ? grad_x : pb.z[m & 1];
      k_poly_back<<<G, kBlock, 0, s>>>((int32_t)n, k, m, m == ncoef - 1, col, dist2, pb.p, pb.off, pb.tsrc, sigma_g,
                                       coef, grad_out, saved, zin, zout, pb.sig_part + (size_t)m * G);
      zin = zout;
    }
  }
  k_coef_grad<<<G, kBlock, 0, s>>>((int32_t)n, ncoef, grad_out, saved, pb.coef_part);
  // the reduce reads G partials per coefficient; coef partials are laid out [k][G]
  k_poly_reduce<<<1, kBlock, 0, s>>>(ncoef, G, pb.coef_part, pb.sig_part, grad_coef, grad_sigma);
  return hipGetLastError();
}

}  // namespace fgbd
