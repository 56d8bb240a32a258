// NE-GBP noise estimation (Sec. 2.3) and the per-point patch statistics used
// by FSLR (Sec. 2.4).
//
// k_noise works on tiles of TP points.  Each thread gathers the patch of one
// point (its colour, then its first P neighbours in row order = increasing
// distance) into LDS as three rows (one per channel) of D = P + 1 floats, and
// from its own rows computes, in FP64,
//   - the FSLR spread s_i = (sigma_R + sigma_G + sigma_B) / 3 (population
//     standard deviations over the patch), and
//   - optionally the eigenvalues of the point's 3x3 colour covariance by the
//     trigonometric closed form for symmetric 3x3 matrices (O. K. Smith,
//     "Eigenvalues of a symmetric 3x3 matrix", CACM 4(4), 1961), whose cubic
//     step runs in FP64.
// The block then accumulates the pooled patch moments over the tile from LDS:
// every thread owns a fixed set of entries of sum_rows a a^T (upper triangle,
// D(D+1)/2 entries) and of the per-channel sums, and walks a fixed set of
// rows, so all sums have a fixed order (products of two floats are exact in
// FP64).  Incomplete patches contribute zero rows and are not counted.
// Each block writes its partial sums; k_noise_solve (one block) reduces them
// in block order, forms
//   Sigma = (S2 - sum_c s1_c s1_c^T / N) / (3 N),
// finds its eigenvalues with a parallel cyclic Jacobi method (round-robin
// pair ordering, FP64), and applies the tail rule: the smallest m with
// mean(lambda_{m+1..D}) <= median(lambda_{m+1..D}); sigma_est = sqrt(mean).
#include "fgbd_internal.h"

namespace fgbd {

namespace {

__device__ void eig3_sym(double a00, double a01, double a02, double a11, double a12, double a22, double out[3]) {
  const double p1 = a01 * a01 + a02 * a02 + a12 * a12;
  double e0, e1, e2;
  if (p1 == 0.0) {
    e0 = a00;
    e1 = a11;
    e2 = a22;
  } else {
    const double q = (a00 + a11 + a22) / 3.0;
    const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
    const double p2 = b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * p1;
    const double p = sqrt(p2 / 6.0);
    const double ip = 1.0 / p;
    const double c00 = b00 * ip, c11 = b11 * ip, c22 = b22 * ip;
    const double c01 = a01 * ip, c02 = a02 * ip, c12 = a12 * ip;
    const double det = c00 * (c11 * c22 - c12 * c12) - c01 * (c01 * c22 - c12 * c02) + c02 * (c01 * c12 - c11 * c02);
    const double r = 0.5 * det;
    const double third_pi = 1.0471975511965976;  // pi / 3
    double phi;
    if (r <= -1.0)
      phi = third_pi;
    else if (r >= 1.0)
      phi = 0.0;
    else
      phi = acos(r) / 3.0;
    e0 = q + 2.0 * p * cos(phi);
    e2 = q + 2.0 * p * cos(phi + 2.0 * third_pi);
    e1 = 3.0 * q - e0 - e2;
  }
  // descending
  if (e0 < e1) { double t = e0; e0 = e1; e1 = t; }
  if (e1 < e2) { double t = e1; e1 = e2; e2 = t; }
  if (e0 < e1) { double t = e0; e0 = e1; e1 = t; }
  out[0] = e0;
  out[1] = e1;
  out[2] = e2;
}

struct NoiseArgs {
  int32_t n, K, P, D, TP;
  int32_t E2, E;       // D(D+1)/2 and E2 + 3D
  int32_t groups;      // row groups per entry
  int32_t want_eig3;
};

// Parallel cyclic Jacobi on a symmetric Dp x Dp matrix in LDS (Dp even).
__device__ void jacobi_eigs(double *A, int Dp, double *s_c, double *s_s, int *s_p, int *s_q, int *s_flag) {
  const int t = threadIdx.x;
  const int half = Dp / 2;
  for (int sweep = 0; sweep < 64; ++sweep) {
    if (t == 0) {
      double off = 0.0, dia = 0.0;
      for (int i = 0; i < Dp; ++i) {
        dia += A[i * Dp + i] * A[i * Dp + i];
        for (int j = i + 1; j < Dp; ++j) off += A[i * Dp + j] * A[i * Dp + j];
      }
      *s_flag = (off <= 1e-30 * dia) ? 1 : 0;
    }
    __syncthreads();
    if (*s_flag) break;
    __syncthreads();
    for (int round = 0; round < Dp - 1; ++round) {
      if (t < half) {
        auto pos = [&](int k) { return k == 0 ? 0 : 1 + ((k - 1 + round) % (Dp - 1)); };
        int p = pos(t), q = pos(Dp - 1 - t);
        if (p > q) { int tmp = p; p = q; q = tmp; }
        const double apq = A[p * Dp + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double tau = (A[q * Dp + q] - A[p * Dp + p]) / (2.0 * apq);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        s_p[t] = p;
        s_q[t] = q;
        s_c[t] = c;
        s_s[t] = s;
      }
      __syncthreads();
      for (int w = t; w < half * Dp; w += blockDim.x) {  // A := A J (columns p, q)
        const int pr = w / Dp, k = w % Dp;
        const int p = s_p[pr], q = s_q[pr];
        const double c = s_c[pr], s = s_s[pr];
        const double akp = A[k * Dp + p], akq = A[k * Dp + q];
        A[k * Dp + p] = c * akp - s * akq;
        A[k * Dp + q] = s * akp + c * akq;
      }
      __syncthreads();
      for (int w = t; w < half * Dp; w += blockDim.x) {  // A := J^T A (rows p, q)
        const int pr = w / Dp, k = w % Dp;
        const int p = s_p[pr], q = s_q[pr];
        const double c = s_c[pr], s = s_s[pr];
        const double apk = A[p * Dp + k], aqk = A[q * Dp + k];
        A[p * Dp + k] = c * apk - s * aqk;
        A[q * Dp + k] = s * apk + c * aqk;
      }
      __syncthreads();
      if (t < half) {  // the rotation annihilates the pair entry; drop its rounding residue
        A[s_p[t] * Dp + s_q[t]] = 0.0;
        A[s_q[t] * Dp + s_p[t]] = 0.0;
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_noise(NoiseArgs a, const int32_t *__restrict__ col,
                                                  const float *__restrict__ rgb, double *__restrict__ spread,
                                                  float *__restrict__ eig3, double *__restrict__ part) {
  extern __shared__ float s_v[];  // [3 * TP][D] patch rows of the current tile
  __shared__ uint16_t s_pair[kMaxD * (kMaxD + 1) / 2];
  __shared__ double s_red[8];

  const int t = threadIdx.x;
  const int D = a.D, P = a.P, K = a.K, TP = a.TP;
  for (int e = t; e < a.E2; e += kBlock) {
    int k = 0, rem = e;
    while (rem >= D - k) { rem -= D - k; ++k; }
    s_pair[e] = (uint16_t)((k << 8) | (k + rem));
  }
  // entry ownership: thread t owns entries e = (t % Eg) + m * 256 (m < 3) in row group t / Eg
  const int G = a.groups;
  const int Eg = (G > 1) ? a.E : kBlock;
  const int grp = (G > 1) ? t / a.E : 0;
  const bool owner = (G > 1) ? (t < G * a.E) : true;
  double acc[3] = {0.0, 0.0, 0.0};
  double count = 0.0;
  const int rows = 3 * TP;
  __syncthreads();

  const Share sh = xcd_share(a.n, TP);
  for (int64_t tbase = sh.first; tbase < sh.end; tbase += sh.step) {
    if (t < TP) {
      const int64_t i = tbase + t;
      float *r0 = s_v + (size_t)(3 * t + 0) * D;
      float *r1 = s_v + (size_t)(3 * t + 1) * D;
      float *r2 = s_v + (size_t)(3 * t + 2) * D;
      bool complete = false;
      if (i < sh.end) complete = col[i * K + (P - 1)] >= 0;
      if (complete) {
        r0[0] = rgb[3 * i + 0];
        r1[0] = rgb[3 * i + 1];
        r2[0] = rgb[3 * i + 2];
        for (int k = 0; k < P; ++k) {
          const int64_t j = col[i * K + k];
          r0[1 + k] = rgb[3 * j + 0];
          r1[1 + k] = rgb[3 * j + 1];
          r2[1 + k] = rgb[3 * j + 2];
        }
        count += 1.0;
        // per-channel mean and population variance over the patch (FP64)
        double mean[3], cov[6] = {0, 0, 0, 0, 0, 0};
        const float *rr[3] = {r0, r1, r2};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double s = 0.0;
          for (int k = 0; k < D; ++k) s += (double)rr[c][k];
          mean[c] = s / (double)D;
        }
        for (int k = 0; k < D; ++k) {
          const double d0 = (double)r0[k] - mean[0];
          const double d1 = (double)r1[k] - mean[1];
          const double d2 = (double)r2[k] - mean[2];
          cov[0] += d0 * d0;
          cov[1] += d0 * d1;
          cov[2] += d0 * d2;
          cov[3] += d1 * d1;
          cov[4] += d1 * d2;
          cov[5] += d2 * d2;
        }
        const double invD = 1.0 / (double)D;
#pragma unroll
        for (int m = 0; m < 6; ++m) cov[m] *= invD;
        spread[i] = (sqrt(cov[0]) + sqrt(cov[3]) + sqrt(cov[5])) / 3.0;
        if (a.want_eig3) {
          double ev[3];
          eig3_sym(cov[0], cov[1], cov[2], cov[3], cov[4], cov[5], ev);
          eig3[3 * i + 0] = (float)ev[0];
          eig3[3 * i + 1] = (float)ev[1];
          eig3[3 * i + 2] = (float)ev[2];
        }
      } else {
        for (int k = 0; k < D; ++k) {
          r0[k] = 0.0f;
          r1[k] = 0.0f;
          r2[k] = 0.0f;
        }
        if (i < sh.end) {
          spread[i] = __builtin_huge_val();
          if (a.want_eig3) {
            eig3[3 * i + 0] = 0.0f;
            eig3[3 * i + 1] = 0.0f;
            eig3[3 * i + 2] = 0.0f;
          }
        }
      }
    }
    __syncthreads();
    if (owner) {
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int e = (G > 1 ? t % a.E : t) + m * Eg;
        if (e < a.E && (G > 1 ? m == 0 : true)) {
          double s = acc[m];
          if (e < a.E2) {
            const int kk = s_pair[e] >> 8, ll = s_pair[e] & 255;
            for (int r = grp; r < rows; r += G) s += (double)s_v[r * D + kk] * (double)s_v[r * D + ll];
          } else {
            const int c = (e - a.E2) / D, kk = (e - a.E2) % D;
            for (int p = grp; p < TP; p += G) s += (double)s_v[(3 * p + c) * D + kk];
          }
          acc[m] = s;
        }
      }
    }
    __syncthreads();
  }

  // combine row groups (fixed order) and write this block's partial
  double *scratch = reinterpret_cast<double *>(s_v);  // >= 768 doubles available
  {
    double cv[1] = {count};
    block_sum_f64<1>(cv, s_red);
    if (t == 0) part[(size_t)blockIdx.x * (1 + a.E)] = cv[0];
  }
  scratch[3 * t + 0] = acc[0];
  scratch[3 * t + 1] = acc[1];
  scratch[3 * t + 2] = acc[2];
  __syncthreads();
  double *dst = part + (size_t)blockIdx.x * (1 + a.E) + 1;
  if (G > 1) {
    for (int e = t; e < a.E; e += kBlock) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += scratch[3 * (g * a.E + e) + 0];
      dst[e] = s;
    }
  } else {
    for (int e = t; e < a.E; e += kBlock) dst[e] = scratch[3 * (e % kBlock) + e / kBlock];
  }
}

// One block: sum the k_noise partials in block order, form Sigma, find its
// eigenvalues (parallel Jacobi, FP64) and apply the tail rule.
__global__ __launch_bounds__(kBlock) void k_noise_solve(NoiseArgs a, const double *__restrict__ part, int nb,
                                                        fgbd_result *__restrict__ res) {
  __shared__ double s_buf[1 + kMaxD * (kMaxD + 1) / 2 + 3 * kMaxD + 1 + (kMaxD + 1) * (kMaxD + 1)];
  __shared__ double s_jc[kMaxD], s_js[kMaxD];
  __shared__ int s_jp[kMaxD], s_jq[kMaxD], s_flag;
  const int t = threadIdx.x;
  const int D = a.D;
  const int stride = 1 + a.E;
  double *tot = s_buf;
  for (int e = t; e < stride; e += kBlock) {
    double s = 0.0;
#pragma unroll 16
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * stride + e];
    tot[e] = s;
  }
  __syncthreads();
  const double n_eff = tot[0];
  const int Dp = D + (D & 1);
  double *A = tot + stride + (stride & 1);  // Dp x Dp
  if (n_eff > 0.0) {
    const double *S2 = tot + 1;
    const double *S1 = tot + 1 + a.E2;
    for (int w = t; w < Dp * Dp; w += kBlock) {
      const int k = w / Dp, l = w % Dp;
      double v = 0.0;
      if (k < D && l < D) {
        const int kk = min(k, l), ll = max(k, l);
        const int e = kk * D - kk * (kk - 1) / 2 + (ll - kk);
        double m = 0.0;
        for (int c = 0; c < 3; ++c) m += S1[c * D + kk] * S1[c * D + ll];
        v = (S2[e] - m / n_eff) / (3.0 * n_eff);
      }
      A[w] = v;
    }
    __syncthreads();
    jacobi_eigs(A, Dp, s_jc, s_js, s_jp, s_jq, &s_flag);
  }
  __syncthreads();
  if (t == 0) {
    double sigma = 0.0;
    int m_star = 0;
    if (n_eff > 0.0) {
      double lam[kMaxD + 1];
      for (int k = 0; k < D; ++k) lam[k] = A[k * Dp + k];
      for (int k = 1; k < D; ++k) {  // descending insertion sort
        const double v = lam[k];
        int j = k - 1;
        while (j >= 0 && lam[j] < v) { lam[j + 1] = lam[j]; --j; }
        lam[j + 1] = v;
      }
      for (int m = 0; m < D; ++m) {
        const int cntm = D - m;
        double s = 0.0;
        for (int k = m; k < D; ++k) s += lam[k];
        const double tau = s / (double)cntm;
        const double med = (cntm & 1) ? lam[m + cntm / 2] : 0.5 * (lam[m + cntm / 2 - 1] + lam[m + cntm / 2]);
        if (tau <= med) {
          sigma = sqrt(tau > 0.0 ? tau : 0.0);
          m_star = m;
          break;
        }
      }
    }
    res->sigma_est = sigma;
    res->n_eff = (int32_t)n_eff;
    res->m = m_star;
    res->status = (res->status & ~FGBD_ST_NO_PATCH) | (n_eff > 0.0 ? 0 : FGBD_ST_NO_PATCH);
  }
}

NoiseArgs make_args(int64_t n, int k, int P, bool want_eig3) {
  NoiseArgs a;
  a.n = (int32_t)n;
  a.K = k;
  a.P = P;
  a.D = P + 1;
  a.TP = a.D <= 17 ? 256 : 128;
  a.E2 = a.D * (a.D + 1) / 2;
  a.E = a.E2 + 3 * a.D;
  a.groups = a.E <= kBlock ? kBlock / a.E : 1;
  a.want_eig3 = want_eig3;
  return a;
}

}  // namespace

hipError_t launch_noise(int64_t n, int k, int P, const int32_t *col, const float *rgb, double *spread, float *eig3,
                        double *part, int nblocks, hipStream_t stream) {
  const NoiseArgs a = make_args(n, k, P, eig3 != nullptr);
  const size_t lds = (size_t)3 * a.TP * a.D * sizeof(float);
  k_noise<<<nblocks, kBlock, lds, stream>>>(a, col, rgb, spread, eig3, part);
  return hipGetLastError();
}

hipError_t launch_noise_solve(int P, const double *part, int nblocks, fgbd_result *res, hipStream_t stream) {
  const NoiseArgs a = make_args(0, P, P, false);
  k_noise_solve<<<1, kBlock, 0, stream>>>(a, part, nblocks, res);
  return hipGetLastError();
}

}  // namespace fgbd
