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
// Every block works on one cloud and writes its partial sums; k_noise_solve
// (one block per cloud) reduces its cloud's partials in block order, forms
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
  SegArgs sa;
  int32_t K, P, D, TP;
  int32_t E2, E;       // D(D+1)/2 and E2 + 3D
  int32_t groups;      // row groups per entry
  int32_t want_eig3;
};

// Orders this wave's LDS writes before its later LDS reads (all lanes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Parallel cyclic Jacobi on a symmetric Dp x Dp matrix in LDS (Dp even), run
// by one wave.  Round-robin pairing applies Dp/2 disjoint rotations at once.
// An entry already negligible (|a_pq| <= 1e-15 |A|_F, or against its diagonal
// pair) is set to zero instead of rotated; the sweeps stop when a whole sweep
// needed no rotation (at most 64 sweeps).  Eigenvalues are then accurate to
// about 1e-15 |A|_F.
__device__ void jacobi_eigs_wave(double *A, int Dp, double *s_c, double *s_s, int *s_p, int *s_q, int *s_flag) {
  const int t = (int)lane_id();
  const int half = Dp / 2;
  // Frobenius norm (invariant under the rotations): entries below eps * |A|
  // are rounding residue and are not rotated
  double f = 0.0;
  for (int w = t; w < Dp * Dp; w += kWave) f += A[w] * A[w];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) f += __shfl_xor(f, o, kWave);
  const double tiny = 1e-15 * sqrt(f);
  for (int sweep = 0; sweep < 64; ++sweep) {
    if (t == 0) *s_flag = 0;
    wave_lds_sync();
    for (int round = 0; round < Dp - 1; ++round) {
      if (t < half) {
        auto pos = [&](int k) { return k == 0 ? 0 : 1 + ((k - 1 + round) % (Dp - 1)); };
        int p = pos(t), q = pos(Dp - 1 - t);
        if (p > q) { int tmp = p; p = q; q = tmp; }
        const double apq = A[p * Dp + q];
        const double app = A[p * Dp + p], aqq = A[q * Dp + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > tiny && fabs(apq) > 1e-16 * sqrt(fabs(app * aqq))) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          *s_flag = 1;
        }
        s_p[t] = p;
        s_q[t] = q;
        s_c[t] = c;
        s_s[t] = s;
      }
      wave_lds_sync();
      for (int w = t; w < half * Dp; w += kWave) {  // A := A J (columns p, q)
        const int pr = w / Dp, k = w % Dp;
        if (s_s[pr] == 0.0) continue;
        const int p = s_p[pr], q = s_q[pr];
        const double c = s_c[pr], s = s_s[pr];
        const double akp = A[k * Dp + p], akq = A[k * Dp + q];
        A[k * Dp + p] = c * akp - s * akq;
        A[k * Dp + q] = s * akp + c * akq;
      }
      wave_lds_sync();
      for (int w = t; w < half * Dp; w += kWave) {  // A := J^T A (rows p, q)
        const int pr = w / Dp, k = w % Dp;
        if (s_s[pr] == 0.0) continue;
        const int p = s_p[pr], q = s_q[pr];
        const double c = s_c[pr], s = s_s[pr];
        const double apk = A[p * Dp + k], aqk = A[q * Dp + k];
        A[p * Dp + k] = c * apk - s * aqk;
        A[q * Dp + k] = s * apk + c * aqk;
      }
      wave_lds_sync();
      if (t < half) {  // the rotation annihilates the pair entry; drop its rounding residue
        A[s_p[t] * Dp + s_q[t]] = 0.0;
        A[s_q[t] * Dp + s_p[t]] = 0.0;
      }
      wave_lds_sync();
    }
    const int any = *s_flag;
    wave_lds_sync();
    if (any == 0) break;
  }
}

// Per-point work of one tile slot: gather the patch into three LDS rows,
// compute the FSLR spread (and optionally the 3x3 eigenvalues) in FP64.
// PT > 0: the patch size is a compile-time constant (values in registers,
// every gather issued before any is used).
template <int PT, bool EIG3>
__device__ __forceinline__ bool patch_point(const NoiseArgs &a, int64_t i, const int32_t *__restrict__ col,
                                            const float *__restrict__ rgb, float *r0, float *r1, float *r2,
                                            double *__restrict__ spread, float *__restrict__ eig3) {
  const int D = a.D, P = a.P, K = a.K;
  if (col[i * K + (P - 1)] < 0) return false;
  double mean[3], cov[6] = {0, 0, 0, 0, 0, 0};
  if constexpr (PT > 0) {
    int cj[PT];
    if (PT % 4 == 0 && (K % 4) == 0) {
#pragma unroll
      for (int q = 0; q < PT / 4; ++q) {
        const int4 c4 = reinterpret_cast<const int4 *>(col + i * K)[q];
        cj[4 * q + 0] = c4.x;
        cj[4 * q + 1] = c4.y;
        cj[4 * q + 2] = c4.z;
        cj[4 * q + 3] = c4.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < PT; ++k) cj[k] = col[i * K + k];
    }
    float v[3][PT + 1];
    v[0][0] = rgb[3 * i + 0];
    v[1][0] = rgb[3 * i + 1];
    v[2][0] = rgb[3 * i + 2];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int64_t j = cj[k];
      v[0][1 + k] = rgb[3 * j + 0];
      v[1][1 + k] = rgb[3 * j + 1];
      v[2][1 + k] = rgb[3 * j + 2];
    }
#pragma unroll
    for (int k = 0; k <= PT; ++k) {
      r0[k] = v[0][k];
      r1[k] = v[1][k];
      r2[k] = v[2][k];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k <= PT; ++k) s += (double)v[c][k];
      mean[c] = s / (double)(PT + 1);
    }
#pragma unroll
    for (int k = 0; k <= PT; ++k) {
      const double d0 = (double)v[0][k] - mean[0];
      const double d1 = (double)v[1][k] - mean[1];
      const double d2 = (double)v[2][k] - mean[2];
      cov[0] += d0 * d0;
      cov[3] += d1 * d1;
      cov[5] += d2 * d2;
      if (EIG3) {
        cov[1] += d0 * d1;
        cov[2] += d0 * d2;
        cov[4] += d1 * d2;
      }
    }
  } else {
    r0[0] = rgb[3 * i + 0];
    r1[0] = rgb[3 * i + 1];
    r2[0] = rgb[3 * i + 2];
    for (int k = 0; k < P; ++k) {
      const int64_t j = col[i * K + k];
      r0[1 + k] = rgb[3 * j + 0];
      r1[1 + k] = rgb[3 * j + 1];
      r2[1 + k] = rgb[3 * j + 2];
    }
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
      cov[3] += d1 * d1;
      cov[5] += d2 * d2;
      if (EIG3) {
        cov[1] += d0 * d1;
        cov[2] += d0 * d2;
        cov[4] += d1 * d2;
      }
    }
  }
  const double invD = 1.0 / (double)D;
#pragma unroll
  for (int m = 0; m < 6; ++m) cov[m] *= invD;
  spread[i] = (sqrt(cov[0]) + sqrt(cov[3]) + sqrt(cov[5])) / 3.0;
  if (EIG3) {
    double ev[3];
    eig3_sym(cov[0], cov[1], cov[2], cov[3], cov[4], cov[5], ev);
    eig3[3 * i + 0] = (float)ev[0];
    eig3[3 * i + 1] = (float)ev[1];
    eig3[3 * i + 2] = (float)ev[2];
  }
  return true;
}

template <int PT, bool EIG3>
__global__ __launch_bounds__(kBlock) void k_noise(NoiseArgs a, const int32_t *__restrict__ col,
                                                  const float *__restrict__ rgb, double *__restrict__ spread,
                                                  float *__restrict__ eig3, double *__restrict__ part) {
  extern __shared__ float s_v[];  // [3 * TP][D] patch rows of the current tile
  __shared__ uint16_t s_pair[kMaxD * (kMaxD + 1) / 2];
  __shared__ double s_red[8];

  const int t = threadIdx.x;
  const int D = a.D, TP = a.TP;
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
  // entries per thread: one when the patch size is compile-time (D <= 19 gives
  // E <= 256), up to three otherwise
  constexpr int NE = PT > 0 ? 1 : 3;
  double acc[NE][4];
#pragma unroll
  for (int m = 0; m < NE; ++m) acc[m][0] = acc[m][1] = acc[m][2] = acc[m][3] = 0.0;
  double count = 0.0;
  const int rows = 3 * TP;
  __syncthreads();

  const SegBlock sb = seg_block(a.sa, kGridNoise);
  const Share sh = seg_share(sb, TP);
  for (int64_t tbase = sh.first; tbase < sh.end; tbase += sh.step) {
    if (t < TP) {
      const int64_t i = tbase + t;
      float *r0 = s_v + (size_t)(3 * t + 0) * D;
      float *r1 = s_v + (size_t)(3 * t + 1) * D;
      float *r2 = s_v + (size_t)(3 * t + 2) * D;
      bool complete = false;
      if (i < sh.end) complete = patch_point<PT, EIG3>(a, i, col, rgb, r0, r1, r2, spread, eig3);
      if (complete) {
        count += 1.0;
      } else {
        for (int k = 0; k < D; ++k) {
          r0[k] = 0.0f;
          r1[k] = 0.0f;
          r2[k] = 0.0f;
        }
        if (i < sh.end) {
          spread[i] = __builtin_huge_val();
          if (EIG3) {
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
      for (int m = 0; m < NE; ++m) {
        const int e = (G > 1 ? t % a.E : t) + m * Eg;
        if (e < a.E && (G > 1 ? m == 0 : true)) {
          // four independent accumulators over the rows keep the FP64 adds
          // from forming one long dependency chain
          double s0 = acc[m][0], s1 = acc[m][1], s2 = acc[m][2], s3 = acc[m][3];
          if (e < a.E2) {
            const int kk = s_pair[e] >> 8, ll = s_pair[e] & 255;
            int r = grp;
            for (; r + 3 * G < rows; r += 4 * G) {
              s0 += (double)s_v[r * D + kk] * (double)s_v[r * D + ll];
              s1 += (double)s_v[(r + G) * D + kk] * (double)s_v[(r + G) * D + ll];
              s2 += (double)s_v[(r + 2 * G) * D + kk] * (double)s_v[(r + 2 * G) * D + ll];
              s3 += (double)s_v[(r + 3 * G) * D + kk] * (double)s_v[(r + 3 * G) * D + ll];
            }
            for (; r < rows; r += G) s0 += (double)s_v[r * D + kk] * (double)s_v[r * D + ll];
          } else {
            const int c = (e - a.E2) / D, kk = (e - a.E2) % D;
            int p = grp;
            for (; p + 3 * G < TP; p += 4 * G) {
              s0 += (double)s_v[(3 * p + c) * D + kk];
              s1 += (double)s_v[(3 * (p + G) + c) * D + kk];
              s2 += (double)s_v[(3 * (p + 2 * G) + c) * D + kk];
              s3 += (double)s_v[(3 * (p + 3 * G) + c) * D + kk];
            }
            for (; p < TP; p += G) s0 += (double)s_v[(3 * p + c) * D + kk];
          }
          acc[m][0] = s0;
          acc[m][1] = s1;
          acc[m][2] = s2;
          acc[m][3] = s3;
        }
      }
    }
    __syncthreads();
  }

  // combine accumulators and row groups (fixed order); write this block's
  // partials entry-major: part[e * nblocks + block], entry 0 = patch count
  double *scratch = reinterpret_cast<double *>(s_v);  // >= 768 doubles available
  const int nb = gridDim.x;
  {
    double cv[1] = {count};
    block_sum_f64<1>(cv, s_red);
    if (t == 0) part[blockIdx.x] = cv[0];
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) scratch[3 * t + m] = m < NE ? (acc[m < NE ? m : 0][0] + acc[m < NE ? m : 0][1]) +
                                                                (acc[m < NE ? m : 0][2] + acc[m < NE ? m : 0][3])
                                                          : 0.0;
  __syncthreads();
  if (G > 1) {
    for (int e = t; e < a.E; e += kBlock) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += scratch[3 * (g * a.E + e) + 0];
      part[(size_t)(1 + e) * nb + blockIdx.x] = s;
    }
  } else {
    for (int e = t; e < a.E; e += kBlock) part[(size_t)(1 + e) * nb + blockIdx.x] = scratch[3 * (e % kBlock) + e / kBlock];
  }
}

// One block: sum the k_noise partials in block order, form Sigma, find its
// eigenvalues (parallel Jacobi, FP64) and apply the tail rule.
constexpr int kSolveThreads = 1024;

// One block per cloud: sum the cloud's k_noise partials (one wave per entry
// row, lanes stride the blocks, fixed shuffle tree), form Sigma, then wave 0
// alone finds its eigenvalues (Jacobi, FP64) and applies the tail rule.
__global__ __launch_bounds__(kSolveThreads) void k_noise_solve(NoiseArgs a, const double *__restrict__ part, int nb,
                                                               fgbd_result *__restrict__ res_all) {
  __shared__ double s_buf[1 + kMaxD * (kMaxD + 1) / 2 + 3 * kMaxD + 1 + (kMaxD + 1) * (kMaxD + 1)];
  __shared__ double s_jc[kMaxD], s_js[kMaxD];
  __shared__ int s_jp[kMaxD], s_jq[kMaxD], s_flag;
  __shared__ double s_lam[kMaxD + 1];
  const int t = threadIdx.x;
  const int lane = (int)lane_id();
  const int wave = t / kWave;
  const int nwaves = blockDim.x / kWave;
  const int D = a.D;
  const int stride = 1 + a.E;
  const int seg = blockIdx.x;
  fgbd_result *res = res_all + seg;
  const int f0 = a.sa.n_fixed >= 0 ? 0 : a.sa.segs->blk_first[kGridNoise][seg];
  const int nbs = (a.sa.n_fixed >= 0 ? nb : a.sa.segs->blk_first[kGridNoise][seg + 1]) - f0;
  double *tot = s_buf;
  for (int e = wave; e < stride; e += nwaves) {
    const double *row = part + (size_t)e * nb + f0;
    // nbs <= kMaxGrid: every lane's loads of the row are issued together
    double vals[kMaxGrid / kWave];
#pragma unroll
    for (int u = 0; u < kMaxGrid / kWave; ++u) {
      const int b = lane + u * kWave;
      vals[u] = b < nbs ? row[b] : 0.0;
    }
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < kMaxGrid / kWave; ++u) v += vals[u];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    if (lane == 0) tot[e] = v;
  }
  __syncthreads();
  const double n_eff = tot[0];
  const int Dp = D + (D & 1);
  double *A = tot + stride + (stride & 1);  // Dp x Dp
  if (n_eff > 0.0) {
    const double *S2 = tot + 1;
    const double *S1 = tot + 1 + a.E2;
    for (int w = t; w < Dp * Dp; w += blockDim.x) {
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
  }
  __syncthreads();
  if (wave != 0) return;  // no block barrier follows
  if (n_eff > 0.0) jacobi_eigs_wave(A, Dp, s_jc, s_js, s_jp, s_jq, &s_flag);
  if (t == 0) {
    double sigma = 0.0;
    int m_star = 0;
    if (n_eff > 0.0) {
      double *lam = s_lam;  // LDS, not a private array (would live in scratch)
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

NoiseArgs make_args(const SegArgs &sa, int k, int P, bool want_eig3) {
  NoiseArgs a;
  a.sa = sa;
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

hipError_t launch_noise(const Run &r, const int32_t *col, const float *rgb, double *spread, float *eig3) {
  const NoiseArgs a = make_args(r.sa, r.prm.k, r.pl.P, eig3 != nullptr);
  const size_t lds = (size_t)3 * a.TP * a.D * sizeof(float);
  const int nb = r.pl.grid[kGridNoise];
  double *part = r.b.noise_part;
  hipStream_t st = r.stream;
  if (a.P == 8 && eig3 == nullptr)
    k_noise<8, false><<<nb, kBlock, lds, st>>>(a, col, rgb, spread, eig3, part);
  else if (a.P == 8)
    k_noise<8, true><<<nb, kBlock, lds, st>>>(a, col, rgb, spread, eig3, part);
  else if (eig3 == nullptr)
    k_noise<0, false><<<nb, kBlock, lds, st>>>(a, col, rgb, spread, eig3, part);
  else
    k_noise<0, true><<<nb, kBlock, lds, st>>>(a, col, rgb, spread, eig3, part);
  return hipGetLastError();
}

hipError_t launch_noise_solve(const Run &r, fgbd_result *res) {
  const NoiseArgs a = make_args(r.sa, r.prm.k, r.pl.P, false);
  k_noise_solve<<<r.pl.B, kSolveThreads, 0, r.stream>>>(a, r.b.noise_part, r.pl.grid[kGridNoise], res);
  return hipGetLastError();
}

}  // namespace fgbd
