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
// Every block works on one cloud and adds its partial sums, rounded to
// multiples of 2^-12, into its cloud's int64 accumulators (integer addition:
// the totals do not depend on the order of the blocks); k_noise_solve
// (one block per cloud) sums the accumulator slots, forms
//   Sigma = (S2 - sum_c s1_c s1_c^T / N) / (3 N),
// finds its eigenvalues (FP64: Householder tridiagonalisation, then Sturm
// multisection), and applies the tail rule: the smallest m with
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
  int32_t order;       // 1: patch entries by increasing point index (generic kernel only)
  // the fused per-frame path (K = P = 8): the first filter sweep's colours
  // x1 = T y with the eq. 4 weights, computed here from the same neighbour
  // rows; the first sweep launch then only marks FSLR membership and sums
  const int32_t *dist2;
  const unsigned long long *edge_acc;
  double sigma_g_fixed;
  fgbd_result *res;  // receives sigma_g
  float *p_out;      // the weights, for the later sweeps
  float4 *x1;        // the first sweep's output buffer
  // per cloud: set when the cloud was renumbered along scan order 0 (NULL:
  // never); its graph and colours are then read from col_w, dist2_w, rgb_w
  const int32_t *relabel;
  const float *rgb_w;
  const int32_t *col_w, *dist2_w;
};

// Adds entry e of a block's patch moments into its cloud's accumulators
// (acc: the row of the block's slot in the cloud's [kNoiseSlots][E1] array).
__device__ __forceinline__ void add_moment(unsigned long long *acc, int e, double v) {
  atomicAdd(&acc[e], (unsigned long long)llrint(v * kNoiseFix));
}

// Orders this wave's LDS writes before its later LDS reads (all lanes).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Sum over the wave (every lane receives the total; fixed xor tree).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Eigenvalues of the symmetric D x D matrix in LDS (row stride ld), in two
// stages:
//  1. (one wave) Householder reduction to tridiagonal form (A is
//     overwritten): at step k the column below the diagonal, x, is mapped
//     onto alpha e_1 with H = I - beta v v^T, v = x - alpha e_1,
//     alpha = -sign(x_1)|x|, and the trailing block is updated as
//     A' - v q^T - q v^T with p = beta A' v, q = p - (beta/2)(v^T p) v (lanes
//     own rows or entries; LDS vectors).  The diagonal and off-diagonal go to
//     s_d, s_e.
//  2. (every wave, one eigenvalue at a time) Sturm-sequence multisection of
//     the tridiagonal matrix: the count of eigenvalues below x follows from
//     the signs of the pivots q_0 = d_0 - x, q_i = d_i - x - e_{i-1}^2 / q_{i-1};
//     the 64 lanes evaluate the count at 64 interior points of the bracket
//     of eigenvalue k (ascending), which keeps count(lo) <= k < count(hi) and
//     shrinks 65-fold per step; eight steps from the Gershgorin interval give
//     about 48 bits of it (eigenvalues to ~3e-15 of the norm).
// Accurate to a few ulps of the matrix norm, like any backward-stable
// symmetric eigen-solver.
__device__ void householder_wave(double *A, int D, int ld, double *s_v, double *s_p, double *s_d, double *s_e) {
  const int t = (int)lane_id();
  for (int k = 0; k + 2 < D; ++k) {
    const int m = D - k - 1;
    double *Ab = A + (size_t)(k + 1) * ld + (k + 1);  // trailing block
    const double xi = t < m ? A[(size_t)(k + 1 + t) * ld + k] : 0.0;
    const double ss = wave_sum(xi * xi);
    const double x0 = __shfl(xi, 0, kWave);
    const double alpha = ss > 0.0 ? -copysign(sqrt(ss), x0) : 0.0;
    const double vn2 = 2.0 * (ss - x0 * alpha);  // |x - alpha e_1|^2
    if (t == 0) {
      s_d[k] = A[(size_t)k * ld + k];
      s_e[k] = alpha;
    }
    if (!(vn2 > 0.0)) continue;  // uniform: x = 0, nothing to reflect
    const double beta = 2.0 / vn2;
    const double vi = t < m ? (t == 0 ? xi - alpha : xi) : 0.0;
    if (t < m) s_v[t] = vi;
    wave_lds_sync();
    double pi = 0.0;
    if (t < m) {
      for (int j = 0; j < m; ++j) pi += Ab[(size_t)t * ld + j] * s_v[j];
      pi *= beta;
    }
    const double kk = 0.5 * beta * wave_sum(vi * pi);
    if (t < m) s_p[t] = pi - kk * vi;
    wave_lds_sync();
    for (int w = t; w < m * m; w += kWave) {
      const int i = w / m, j = w % m;
      Ab[(size_t)i * ld + j] -= s_v[i] * s_p[j] + s_p[i] * s_v[j];
    }
    wave_lds_sync();
  }
  if (t == 0) {
    if (D >= 2) {
      s_d[D - 2] = A[(size_t)(D - 2) * ld + (D - 2)];
      s_e[D - 2] = A[(size_t)(D - 1) * ld + (D - 2)];
    }
    s_d[D - 1] = A[(size_t)(D - 1) * ld + (D - 1)];
  }
}

// Eigenvalue k (ascending) of the tridiagonal (s_d, s_e), by one wave.
__device__ double tridiag_eig_wave(const double *s_d, const double *s_e, int D, int k) {
  const int t = (int)lane_id();
  double glo = 1e300, ghi = -1e300, emax = 0.0;
  for (int i = t; i < D; i += kWave) {
    const double r = (i > 0 ? fabs(s_e[i - 1]) : 0.0) + (i + 1 < D ? fabs(s_e[i]) : 0.0);
    glo = fmin(glo, s_d[i] - r);
    ghi = fmax(ghi, s_d[i] + r);
    if (i + 1 < D) emax = fmax(emax, s_e[i] * s_e[i]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    glo = fmin(glo, __shfl_xor(glo, o, kWave));
    ghi = fmax(ghi, __shfl_xor(ghi, o, kWave));
    emax = fmax(emax, __shfl_xor(emax, o, kWave));
  }
  const double nrm = fmax(fabs(glo), fabs(ghi));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax) * 4.0;
  double lo = glo - (4.0 * 2.220446049250313e-16 * nrm + pivmin);
  double hi = ghi + (4.0 * 2.220446049250313e-16 * nrm + pivmin);
  for (int it = 0; it < 8; ++it) {
    const double step = (hi - lo) / (double)(kWave + 1);
    const double x = lo + step * (double)(t + 1);
    double q = s_d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    for (int i = 1; i < D; ++i) {
      // 1 / q from the hardware reciprocal and one Newton step (the count
      // needs only the sign of each pivot)
      double r = __builtin_amdgcn_rcp(q);
      r = fma(r, fma(-q, r, 1.0), r);
      q = fma(-s_e[i - 1] * s_e[i - 1], r, s_d[i] - x);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
    // the count grows with x, so the lanes with count <= k are the first j:
    // the new bracket is (x_{j-1}, x_j) with x_{-1} = lo and x_64 = hi
    const int j = (int)__popcll(__builtin_amdgcn_ballot_w64(cnt <= k));
    const double nlo = j > 0 ? lo + step * (double)j : lo;
    const double nhi = j < kWave ? lo + step * (double)(j + 1) : hi;
    lo = nlo;
    hi = nhi;
  }
  return 0.5 * (lo + hi);
}

// The same two stages for a matrix of compile-time size DT held in
// registers: every lane of the wave runs the identical Householder sequence
// on its own copy of the lower triangle (no cross-lane traffic, no LDS round
// trips between the dependent steps), so every lane ends with the same
// tridiagonal matrix.  Sums run in index order.
template <int DT>
__device__ __forceinline__ void householder_regs(double (&A)[DT][DT], double (&d)[DT], double (&e)[DT]) {
#pragma unroll
  for (int k = 0; k + 2 < DT; ++k) {
    const int m = DT - k - 1;
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < DT; ++i)
      if (i < m) ss = fma(A[k + 1 + i][k], A[k + 1 + i][k], ss);
    const double x0 = A[k + 1][k];
    const double alpha = ss > 0.0 ? -copysign(sqrt(ss), x0) : 0.0;
    const double vn2 = 2.0 * (ss - x0 * alpha);
    d[k] = A[k][k];
    e[k] = alpha;
    if (!(vn2 > 0.0)) continue;  // x = 0: nothing to reflect
    const double beta = 2.0 / vn2;
    double v[DT], q[DT];
#pragma unroll
    for (int i = 0; i < DT; ++i) v[i] = i < m ? (i == 0 ? x0 - alpha : A[k + 1 + i][k]) : 0.0;
    double vp = 0.0;
#pragma unroll
    for (int i = 0; i < DT; ++i) {
      if (i >= m) continue;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < DT; ++j) {
        if (j >= m) continue;
        const int r = k + 1 + (i > j ? i : j), c = k + 1 + (i > j ? j : i);
        s = fma(A[r][c], v[j], s);
      }
      q[i] = beta * s;  // p = beta A' v
      vp = fma(v[i], q[i], vp);
    }
    const double kk = 0.5 * beta * vp;
#pragma unroll
    for (int i = 0; i < DT; ++i)
      if (i < m) q[i] = q[i] - kk * v[i];
#pragma unroll
    for (int i = 0; i < DT; ++i)
#pragma unroll
      for (int j = 0; j < DT; ++j)
        if (i < m && j <= i) A[k + 1 + i][k + 1 + j] -= v[i] * q[j] + q[i] * v[j];
  }
  d[DT - 2] = A[DT - 2][DT - 2];
  e[DT - 2] = A[DT - 1][DT - 2];
  d[DT - 1] = A[DT - 1][DT - 1];
}

// Eigenvalues k0 .. k0 + G - 1 (ascending) of the tridiagonal (d, e) held in
// registers, by one wave split into G groups of GL = 64 / G lanes, one
// eigenvalue per group (lanes past G * GL follow the last group and take no
// part in its votes).  The multisection of tridiag_eig_wave with GL interior
// points per step, so each step shrinks a bracket (GL + 1)-fold and ITERS
// steps give at least 48 bits.  Fewer lanes per eigenvalue but fewer waves:
// the waves of a block share the CU's four SIMDs, so one wave doing three
// eigenvalues in 11 steps finishes well before three waves doing one each
// in 8 steps on the same SIMD.  Returns this lane's group's eigenvalue.
template <int DT, int G>
__device__ double tridiag_eig_groups(const double (&d)[DT], const double (&e)[DT], int k0) {
  constexpr int GL = kWave / G;
  constexpr int ITERS = GL >= 63 ? 8 : GL >= 31 ? 10 : GL >= 21 ? 11 : GL >= 15 ? 12 : 48;
  const int t = (int)lane_id();
  const int g = min(t / GL, G - 1);
  const int sub = t - g * GL;  // point of the group (GL for a spare lane)
  const int k = k0 + g;
  const uint64_t gmask = (((uint64_t)1 << GL) - 1) << (g * GL);
  double glo = 1e300, ghi = -1e300, emax = 0.0, e2[DT];
#pragma unroll
  for (int i = 0; i < DT; ++i) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < DT ? fabs(e[i]) : 0.0);
    glo = fmin(glo, d[i] - r);
    ghi = fmax(ghi, d[i] + r);
    e2[i] = e[i] * e[i];
    if (i + 1 < DT) emax = fmax(emax, e2[i]);
  }
  const double nrm = fmax(fabs(glo), fabs(ghi));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax) * 4.0;
  double lo = glo - (4.0 * 2.220446049250313e-16 * nrm + pivmin);
  double hi = ghi + (4.0 * 2.220446049250313e-16 * nrm + pivmin);
  for (int it = 0; it < ITERS; ++it) {
    const double step = (hi - lo) / (double)(GL + 1);
    const double x = lo + step * (double)(sub + 1);
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
#pragma unroll
    for (int i = 1; i < DT; ++i) {
      double r = __builtin_amdgcn_rcp(q);
      r = fma(r, fma(-q, r, 1.0), r);
      q = fma(-e2[i - 1], r, d[i] - x);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
    // the group's points with count <= k are its first j
    const int j = (int)__popcll(__builtin_amdgcn_ballot_w64(cnt <= k) & gmask);
    const double nlo = j > 0 ? lo + step * (double)j : lo;
    const double nhi = j < GL ? lo + step * (double)(j + 1) : hi;
    lo = nlo;
    hi = nhi;
  }
  return 0.5 * (lo + hi);
}

// The FSLR spread (and optionally the 3x3 eigenvalues) of one complete patch
// held in registers (channel c, entry k: the point, then its PT neighbours),
// in FP64, after writing the patch's three rows to LDS.
template <int PT, bool EIG3>
__device__ __forceinline__ void patch_stats(int64_t i, const float (&v)[3][PT + 1], float *r0, float *r1, float *r2,
                                            double *__restrict__ spread, float *__restrict__ eig3) {
  double mean[3], cov[6] = {0, 0, 0, 0, 0, 0};
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
  const double invD = 1.0 / (double)(PT + 1);
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
    patch_stats<PT, EIG3>(i, v, r0, r1, r2, spread, eig3);
    return true;
  } else {
    double mean[3], cov[6] = {0, 0, 0, 0, 0, 0};
    if (a.order == 0) {
      r0[0] = rgb[3 * i + 0];
      r1[0] = rgb[3 * i + 1];
      r2[0] = rgb[3 * i + 2];
      for (int k = 0; k < P; ++k) {
        const int64_t j = col[i * K + k];
        r0[1 + k] = rgb[3 * j + 0];
        r1[1 + k] = rgb[3 * j + 1];
        r2[1 + k] = rgb[3 * j + 2];
      }
    } else {
      // unsorted patch: member m (the point, then its P neighbours) goes to
      // the slot of its rank among the D point indices, which are distinct
      // (a row never repeats a neighbour or holds the point itself), so the
      // ranks are a permutation of 0 .. D-1
      for (int m = 0; m < D; ++m) {
        const int64_t j = m == 0 ? i : (int64_t)col[i * K + m - 1];
        int rank = (m != 0 && i < j) ? 1 : 0;
        for (int l = 0; l < P; ++l) rank += (int64_t)col[i * K + l] < j ? 1 : 0;
        r0[rank] = rgb[3 * j + 0];
        r1[rank] = rgb[3 * j + 1];
        r2[rank] = rgb[3 * j + 2];
      }
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
}

// The fused per-frame path (K = P = 8), one point: the row's neighbour
// colours are gathered once and serve both the patch (as in patch_point) and
// the first filter sweep: the row's weights from its squared distances
// (row_weights, the graph builder's arithmetic) into p, and x1 = y_i / 2 +
// sum_k p_ik y_jk / 2 with the first filter sweep's own operation order (an
// empty row keeps y_i) into the first iterate buffer, whose fourth lane the
// first sweep launch fills with the FSLR flag.  Returns whether the patch
// is complete.
__device__ __forceinline__ bool fused_point8(const NoiseArgs &a, int64_t i, const int32_t *__restrict__ col,
                                             const float *__restrict__ rgb, float *r0, float *r1, float *r2,
                                             double *__restrict__ spread, double sg, const double *s_exp) {
  int cc[8], dv[8];
  const int4 *cr = reinterpret_cast<const int4 *>(col + i * 8);
  const int4 *dr = reinterpret_cast<const int4 *>(a.dist2 + i * 8);
  const int4 c0 = cr[0], c1 = cr[1], e0 = dr[0], e1 = dr[1];
  cc[0] = c0.x; cc[1] = c0.y; cc[2] = c0.z; cc[3] = c0.w;
  cc[4] = c1.x; cc[5] = c1.y; cc[6] = c1.z; cc[7] = c1.w;
  dv[0] = e0.x; dv[1] = e0.y; dv[2] = e0.z; dv[3] = e0.w;
  dv[4] = e1.x; dv[5] = e1.y; dv[6] = e1.z; dv[7] = e1.w;
  float v[3][9];
  v[0][0] = rgb[3 * i + 0];
  v[1][0] = rgb[3 * i + 1];
  v[2][0] = rgb[3 * i + 2];
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // an empty slot reads the point itself (weight 0)
    const int64_t cj = cc[k] >= 0 ? (int64_t)cc[k] : i;
    v[0][1 + k] = rgb[3 * cj + 0];
    v[1][1 + k] = rgb[3 * cj + 1];
    v[2][1 + k] = rgb[3 * cj + 2];
  }
  float ww[8];
  row_weights<8>(cc, dv, sg, s_exp, ww);
  float4 *pr = reinterpret_cast<float4 *>(a.p_out + i * 8);
  pr[0] = make_float4(ww[0], ww[1], ww[2], ww[3]);
  pr[1] = make_float4(ww[4], ww[5], ww[6], ww[7]);
  float ar = 0.f, ag = 0.f, ab = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float w = cc[k] >= 0 ? ww[k] : 0.0f;
    ar = fmaf(w, v[0][1 + k], ar);
    ag = fmaf(w, v[1][1 + k], ag);
    ab = fmaf(w, v[2][1 + k], ab);
  }
  const float xr = v[0][0], xg = v[1][0], xb = v[2][0];
  float orr = xr, og = xg, ob = xb;
  if (cc[0] >= 0) {
    orr = 0.5f * xr + 0.5f * ar;
    og = 0.5f * xg + 0.5f * ag;
    ob = 0.5f * xb + 0.5f * ab;
  }
  a.x1[i] = make_float4(orr, og, ob, 0.0f);
  if (cc[7] < 0) return false;  // fewer than P neighbours: no patch
  patch_stats<8, false>(i, v, r0, r1, r2, spread, nullptr);
  return true;
}

template <int PT, bool EIG3>
__global__ __launch_bounds__(kBlock) void k_noise(NoiseArgs a, const int32_t *__restrict__ col,
                                                  const float *__restrict__ rgb_in, double *__restrict__ spread,
                                                  float *__restrict__ eig3, unsigned long long *__restrict__ acc_all) {
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
  // a renumbered cloud reads its graph and colours in scan-order-0 numbering
  const bool relabelled = a.relabel && a.relabel[sb.s];
  const float *__restrict__ rgb = relabelled ? a.rgb_w : rgb_in;
  if (relabelled) {
    col = a.col_w;
    a.dist2 = a.dist2_w;
  }
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

  // combine accumulators and row groups (fixed order); add this block's
  // moments into its cloud's accumulators, entry 0 = patch count
  double *scratch = reinterpret_cast<double *>(s_v);  // >= 768 doubles available
  unsigned long long *acc_c = acc_all + ((size_t)sb.s * kNoiseSlots + sb.lb % kNoiseSlots) * (1 + a.E);
  {
    double cv[1] = {count};
    block_sum_f64<1>(cv, s_red);
    if (t == 0) add_moment(acc_c, 0, cv[0]);
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
      add_moment(acc_c, 1 + e, s);
    }
  } else {
    for (int e = t; e < a.E; e += kBlock) add_moment(acc_c, 1 + e, scratch[3 * (e % kBlock) + e / kBlock]);
  }
}


// The same statistics with the tile's patch moments as one FP64 Gram matrix
// on the matrix cores.  Each patch row (one channel of one patch) becomes the
// vector of its D = 9 colour entries and three channel indicators (1 in the
// row's own channel, for complete patches only), stored in LDS as W = 12
// floats.  G = sum over rows of v v^T then holds sum a a^T (the D x D block),
// the per-channel sums (columns D .. D+2 of the first D rows) and the patch
// count (G[D][D]).  G is built from 4 x 4 sub-blocks (p, q), p <= q, of
// feature groups 4p..4p+3, with v_mfma_f64_4x4x4_4b_f64: four independent
// 4 x 4 products per instruction, each summing four rows.  In block b of an
// instruction, lane l supplies A[i][k] and B[k][j] with b = (l / 4) % 4,
// i = j = l % 4, k = l / 16 (the row), and holds C[l / 16][l % 4] (layout
// checked on the device with one-hot operands).  Per pair of row groups
// (8 rows): one instruction each for blocks (0,0), (0,1), (0,2), (1,1), and
// one for (1,2), (2,2) of both groups, so 3 instructions instead of the 2
// that a 16 x 16 product would need at six times the cost per instruction
// on this GPU (measured).  Independent accumulators, operands read from LDS
// without branches, and the partial sums added in a fixed order.  Products
// of floats are exact in FP64; the accumulation order is fixed.
template <int PT, bool EIG3, bool FUSE>
__global__ __launch_bounds__(kBlock, 4) void k_noise_mfma(NoiseArgs a, const int32_t *__restrict__ col,
                                                       const float *__restrict__ rgb_in, double *__restrict__ spread,
                                                       float *__restrict__ eig3,
                                                       unsigned long long *__restrict__ acc_all) {
  constexpr int D = PT + 1;
  constexpr int W = D + 3;  // floats per LDS row
  static_assert(W == 12, "three feature groups of four: D = 9 colours and three indicators");
  extern __shared__ float s_v[];  // [3 * TP][W] patch rows of the current tile; then the Gram sums
  const int t = threadIdx.x;
  const int TP = a.TP;
  // wave-uniform in a scalar register, so the row loop below is uniform and
  // the accumulators stay in place across its iterations
  const int wave = __builtin_amdgcn_readfirstlane(t / kWave), lane = (int)lane_id();
  const int bsel = (lane >> 2) & 3, inner = lane & 3, krow = lane >> 4;
  // instruction 1 (per row group): blocks (0,0), (0,1), (0,2), (1,1)
  const int p1 = bsel == 3 ? 1 : 0, q1 = bsel == 3 ? 1 : bsel;
  // instruction 2 (per pair of groups): blocks (1,2), (2,2) of group 2P and of group 2P + 1
  const int p2 = (bsel & 1) ? 2 : 1, g2 = bsel >> 1;
  const int fa1 = 4 * p1 + inner, fb1 = 4 * q1 + inner, fa2 = 4 * p2 + inner, fb2 = 8 + inner;
  const int pairs = 3 * TP / 8;  // pairs of four-row groups
  constexpr int kWaves = kBlock / kWave;
  double c1[4] = {0.0, 0.0, 0.0, 0.0}, c2[2] = {0.0, 0.0};

  const SegBlock sb = seg_block(a.sa, kGridNoise);
  // a renumbered cloud reads its graph and colours in scan-order-0 numbering
  const bool relabelled = a.relabel && a.relabel[sb.s];
  const float *__restrict__ rgb = relabelled ? a.rgb_w : rgb_in;
  if (relabelled) {
    col = a.col_w;
    a.dist2 = a.dist2_w;
  }
  __shared__ double s_exp[FUSE ? kExpTable : 1];
  __shared__ unsigned long long s_u[kEdgeVals];
  double sg = 0.0;
  if (FUSE) {
    static_assert(!FUSE || PT == 8, "the fused first sweep is written for K = P = 8");
    sg = cloud_sigma_g(a.edge_acc + (size_t)kEdgeSlots * kEdgeVals * sb.s, a.sigma_g_fixed, s_u);
    if (sb.lb == 0 && t == 0) a.res[sb.s].sigma_g = sg;
    fill_exp_table(sg, s_exp);
    __syncthreads();
  }
  const Share sh = seg_share(sb, TP);
  for (int64_t tbase = sh.first; tbase < sh.end; tbase += sh.step) {
    if (t < TP) {
      const int64_t i = tbase + t;
      float *r[3] = {s_v + (size_t)(3 * t + 0) * W, s_v + (size_t)(3 * t + 1) * W, s_v + (size_t)(3 * t + 2) * W};
      bool complete = false;
      if (i < sh.end)
        complete = FUSE ? fused_point8(a, i, col, rgb, r[0], r[1], r[2], spread, sg, s_exp)
                        : patch_point<PT, EIG3>(a, i, col, rgb, r[0], r[1], r[2], spread, eig3);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (!complete) {
#pragma unroll
          for (int k = 0; k < D; ++k) r[c][k] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) r[c][D + k] = (complete && k == c) ? 1.0f : 0.0f;
      }
      if (!complete && i < sh.end) {
        spread[i] = __builtin_huge_val();
        if (EIG3) {
          eig3[3 * i + 0] = 0.0f;
          eig3[3 * i + 1] = 0.0f;
          eig3[3 * i + 2] = 0.0f;
        }
      }
    }
    __syncthreads();
    // two pairs of row groups per step (P and P + kWaves), six independent
    // instructions
    for (int pp = wave; pp < pairs; pp += 2 * kWaves) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int P = pp + u * kWaves;
        if (P < pairs) {  // uniform over the wave
          const float *r0 = s_v + (size_t)(8 * P + krow) * W;  // group 2P
          const float *r1 = r0 + 4 * W;                        // group 2P + 1
          const float *r2 = r0 + (size_t)(4 * g2) * W;         // group 2P + g2
          const double a0 = r0[fa1], b0 = r0[fb1], a1 = r1[fa1], b1 = r1[fb1], a2 = r2[fa2], b2 = r2[fb2];
          c1[2 * u] = __builtin_amdgcn_mfma_f64_4x4x4f64(a0, b0, c1[2 * u], 0, 0, 0);
          c1[2 * u + 1] = __builtin_amdgcn_mfma_f64_4x4x4f64(a1, b1, c1[2 * u + 1], 0, 0, 0);
          c2[u] = __builtin_amdgcn_mfma_f64_4x4x4f64(a2, b2, c2[u], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }

  // the block's Gram matrix (16 x 16 storage, only the computed sub-blocks
  // are read), then its moments into the cloud's accumulators, entry 0 =
  // patch count.  The sums reuse the row storage (4 waves x 256 doubles fit
  // in 3 * TP * W floats).
  double(*s_g)[256] = reinterpret_cast<double(*)[256]>(s_v);
  const double tot1 = (c1[0] + c1[1]) + (c1[2] + c1[3]);
  const double tot2h = c2[0] + c2[1];
  const double tot2 = tot2h + __shfl_xor(tot2h, 8, kWave);  // the two groups' halves of (1,2), (2,2)
  s_g[wave][(4 * p1 + krow) * 16 + 4 * q1 + inner] = tot1;
  if (bsel < 2) s_g[wave][(4 * p2 + krow) * 16 + 8 + inner] = tot2;
  __syncthreads();
  const double gsum = (s_g[0][t] + s_g[1][t]) + (s_g[2][t] + s_g[3][t]);
  __syncthreads();
  s_g[0][t] = gsum;
  __syncthreads();
  unsigned long long *acc_c = acc_all + ((size_t)sb.s * kNoiseSlots + sb.lb % kNoiseSlots) * (1 + a.E);
  for (int e = t; e < 1 + a.E; e += kBlock) {
    double v;
    if (e == 0) {
      v = s_g[0][D * 16 + D];
    } else if (e - 1 < a.E2) {
      int k = 0, rem = e - 1;
      while (rem >= D - k) {
        rem -= D - k;
        ++k;
      }
      v = s_g[0][k * 16 + (k + rem)];
    } else {
      const int q = e - 1 - a.E2;
      v = s_g[0][(q % D) * 16 + D + q / D];
    }
    add_moment(acc_c, e, v);
  }
}

// One block: sum the k_noise partials in block order, form Sigma, find its
// eigenvalues (FP64) and apply the tail rule.
constexpr int kSolveThreads = 1024;
// DT > 0: one wave per SIMD (the eigenvalues go three to a wave)
template <int DT>
constexpr int solve_threads() {
  return DT > 0 ? 4 * kWave : kSolveThreads;
}
constexpr int kEigGroups = 3;  // eigenvalues per wave in the register path

// One block per cloud: sum the cloud's moment accumulators (one wave per
// entry, one lane per slot, integer shuffle sums), form Sigma, then wave 0
// alone tridiagonalises and every wave brackets eigenvalues; wave 0 applies
// the tail rule.  DT > 0: D = DT, and Sigma, the reduction and the pivots
// live in registers; DT = 0: any D, through LDS.
template <int DT>
__global__ __launch_bounds__(solve_threads<DT>()) void k_noise_solve(NoiseArgs a,
                                                                     const unsigned long long *__restrict__ acc_all,
                                                                     fgbd_result *__restrict__ res_all) {
  __shared__ double s_buf[1 + kMaxD * (kMaxD + 1) / 2 + 3 * kMaxD + 1 + (kMaxD + 1) * (kMaxD + 1)];
  __shared__ double s_v[kMaxD], s_p[kMaxD], s_d[kMaxD], s_e[kMaxD];
  __shared__ double s_lam[kMaxD + 1];
  __shared__ double s_tri[DT > 0 ? DT * (DT + 1) / 2 : 1];
  __shared__ unsigned long long s_part[solve_threads<DT>()];
  const int t = threadIdx.x;
  const int lane = (int)lane_id();
  const int wave = t / kWave;
  const int nwaves = blockDim.x / kWave;
  const int D = a.D;
  const int stride = 1 + a.E;
  const int seg = blockIdx.x;
  fgbd_result *res = res_all + seg;
  const unsigned long long *acc = acc_all + (size_t)seg * kNoiseSlots * stride;
  double *tot = s_buf;
  // Thread t sums entry t % stride over every C-th slot from t / stride
  // (C = threads per entry, up to kNoiseSlots): reads of consecutive threads
  // are consecutive entries of one slot row, all of a thread's loads are in
  // flight together, and no value crosses lanes; then the C partial sums of
  // each entry are added from LDS.  Integer sums, so the order is free.
  {
    constexpr int NT = solve_threads<DT>();
    const int C = min(NT / stride, kNoiseSlots);  // stride <= NT
    const int e = t % stride, c = t / stride;
    if (c < C) {
      constexpr int U = 16;
      unsigned long long sum = 0;
      for (int s0 = c; s0 < kNoiseSlots; s0 += U * C) {
        unsigned long long u[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
          const int sl = s0 + j * C;
          u[j] = sl < kNoiseSlots ? acc[(size_t)sl * stride + e] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) sum += u[j];
      }
      s_part[c * stride + e] = sum;
    }
    __syncthreads();
    if (t < stride) {
      unsigned long long v = 0;
      for (int cc = 0; cc < C; ++cc) v += s_part[cc * stride + t];
      tot[t] = (double)(long long)v / kNoiseFix;
    }
  }
  __syncthreads();
  const double n_eff = tot[0];
  const double *S2 = tot + 1;
  const double *S1 = tot + 1 + a.E2;
  if constexpr (DT > 0) {
    static_assert(DT <= 4 * kEigGroups, "four waves of kEigGroups eigenvalues");
    constexpr int NT = DT * (DT + 1) / 2;
    static_assert(NT <= kWave, "one lane per entry of the triangle");
    // wave 0: one lane per entry of Sigma's upper triangle (row l, column
    // k >= l, the moment order), then every lane reads the whole triangle and
    // reduces it to tridiagonal form; lane 0 publishes d, e
    if (n_eff > 0.0 && wave == 0) {
      if (lane < NT) {
        int l = 0, rem = lane;
        while (rem >= DT - l) {
          rem -= DT - l;
          ++l;
        }
        const int k = l + rem;
        double m = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) m += S1[c * DT + l] * S1[c * DT + k];
        s_tri[lane] = (S2[lane] - m / n_eff) / (3.0 * n_eff);
      }
      wave_lds_sync();
      double A[DT][DT], d[DT], e[DT];
#pragma unroll
      for (int k = 0; k < DT; ++k)
#pragma unroll
        for (int l = 0; l <= k; ++l) A[k][l] = s_tri[l * DT - l * (l - 1) / 2 + (k - l)];
      householder_regs<DT>(A, d, e);
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < DT; ++i) {
          s_d[i] = d[i];
          s_e[i] = e[i];
        }
      }
    }
    __syncthreads();
    if (n_eff > 0.0 && wave * kEigGroups < DT) {
      double d[DT], e[DT];
#pragma unroll
      for (int i = 0; i < DT; ++i) {
        d[i] = s_d[i];
        e[i] = s_e[i];
      }
      const int k0 = wave * kEigGroups;
      const double ev = tridiag_eig_groups<DT, kEigGroups>(d, e, k0);
      constexpr int GL = kWave / kEigGroups;
      const int g = lane / GL;
      if (lane % GL == 0 && g < kEigGroups && k0 + g < DT) s_lam[DT - 1 - (k0 + g)] = ev;
    }
  } else {
    const int Dp = D + (D & 1);
    double *A = tot + stride + (stride & 1);  // Dp x Dp
    if (n_eff > 0.0) {
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
    // eigenvalues: wave 0 tridiagonalises, then each wave brackets its own
    // eigenvalues (k = wave, wave + 16, ...), stored descending
    if (n_eff > 0.0 && wave == 0) householder_wave(A, D, Dp, s_v, s_p, s_d, s_e);
    __syncthreads();
    if (n_eff > 0.0) {
      for (int k = wave; k < D; k += nwaves) {
        const double ev = tridiag_eig_wave(s_d, s_e, D, k);
        if (lane == 0) s_lam[D - 1 - k] = ev;
      }
    }
  }
  __syncthreads();
  if (wave != 0) return;  // no block barrier follows
  double sigma = 0.0;
  int m_star = 0;
  if (n_eff > 0.0) {  // uniform over the wave
    // tail rule, every m at once (lane m): the smallest m whose tail mean is
    // not above the tail median
    const double *lam = s_lam;
    bool ok = false;
    double tau = 0.0;
    if (lane < D) {
      const int m = lane, cntm = D - m;
      double sm = 0.0;
      for (int k = m; k < D; ++k) sm += lam[k];
      tau = sm / (double)cntm;
      const double med = (cntm & 1) ? lam[m + cntm / 2] : 0.5 * (lam[m + cntm / 2 - 1] + lam[m + cntm / 2]);
      ok = tau <= med;
    }
    const uint64_t hits = __builtin_amdgcn_ballot_w64(ok);  // bit D-1 is always set
    m_star = hits ? (int)__builtin_ctzll(hits) : D - 1;
    const double tau_star = __shfl(tau, m_star, kWave);
    sigma = sqrt(tau_star > 0.0 ? tau_star : 0.0);
  }
  if (lane == 0) {
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
  a.dist2 = nullptr;
  a.edge_acc = nullptr;
  a.sigma_g_fixed = 0.0;
  a.order = 0;
  a.res = nullptr;
  a.p_out = nullptr;
  a.x1 = nullptr;
  a.relabel = nullptr;
  a.rgb_w = nullptr;
  a.col_w = nullptr;
  a.dist2_w = nullptr;
  return a;
}

}  // namespace

hipError_t launch_noise(const Run &r, const int32_t *col, const float *rgb, double *spread, float *eig3,
                        fgbd_result *fuse_res) {
  NoiseArgs a = make_args(r.sa, r.prm.k, r.pl.P, eig3 != nullptr);
  a.order = r.prm.patch_order;
  if (r.relabel_ok) {
    a.relabel = r.b.segs->relabel;
    a.rgb_w = r.b.rgb_w;
    a.col_w = r.b.col_w;
    a.dist2_w = r.b.dist2_w;
  }
  const bool fuse = fuse_res != nullptr;
  if (fuse) {
    if (a.P != 8 || a.K != 8 || eig3 != nullptr || a.order != 0) return hipErrorInvalidValue;
    a.dist2 = r.b.dist2;
    a.edge_acc = r.b.edge_acc;
    a.sigma_g_fixed = r.prm.sigma_g;
    a.res = fuse_res;
    a.p_out = r.b.p;
    a.x1 = r.b.xbuf;  // buffer 0: the first sweep's output
  }
  // k_noise: rows of D floats; k_noise_mfma: rows of D + 3 floats, and at
  // least the 8 KB of its final sums
  const size_t lds_rows = (size_t)3 * a.TP * a.D * sizeof(float);
  const size_t lds_mfma = (size_t)3 * a.TP * (a.D + 3) * sizeof(float);
  const size_t lds = a.P == 8 ? (lds_mfma > 8192 ? lds_mfma : 8192) : lds_rows;
  const int nb = r.pl.grid[kGridNoise];
  unsigned long long *part = r.b.noise_acc;
  hipStream_t st = r.stream;
  if (fuse)
    k_noise_mfma<8, false, true><<<nb, kBlock, lds, st>>>(a, col, rgb, spread, eig3, part);
  else if (a.P == 8 && a.order == 0 && eig3 == nullptr)
    k_noise_mfma<8, false, false><<<nb, kBlock, lds, st>>>(a, col, rgb, spread, eig3, part);
  else if (a.P == 8 && a.order == 0)
    k_noise_mfma<8, true, false><<<nb, kBlock, lds, st>>>(a, col, rgb, spread, eig3, part);
  else if (eig3 == nullptr)
    k_noise<0, false><<<nb, kBlock, lds, st>>>(a, col, rgb, spread, eig3, part);
  else
    k_noise<0, true><<<nb, kBlock, lds, st>>>(a, col, rgb, spread, eig3, part);
  return hipGetLastError();
}

hipError_t launch_noise_solve(const Run &r, fgbd_result *res) {
  const NoiseArgs a = make_args(r.sa, r.prm.k, r.pl.P, false);
  if (a.D == 9)
    k_noise_solve<9><<<r.pl.B, solve_threads<9>(), 0, r.stream>>>(a, r.b.noise_acc, res);
  else
    k_noise_solve<0><<<r.pl.B, solve_threads<0>(), 0, r.stream>>>(a, r.b.noise_acc, res);
  return hipGetLastError();
}

}  // namespace fgbd
