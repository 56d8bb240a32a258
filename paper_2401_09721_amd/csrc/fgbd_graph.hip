// Neighbour selection and edge weights of the scan-line graph (Sec. 2.2).
//
// k_merge: one thread per point i.  For each direction it looks up i's sorted
// position r (rank array from the last radix pass), reads the items at
// r-w..r+w inside the cloud's range of positions (the last pass stores each
// item's packed coordinates in place of its code, so no coordinate is
// gathered), and
// keeps the K smallest distinct (squared distance, index) pairs in a
// register-resident sorted list (packed so one integer compare orders by
// distance then index).  It writes the fixed-K CSR row, and each block adds
// its FP64 sum of edge lengths and its edge count into its cloud's exact
// integer sums for sigma_g; every block works on one cloud.
//
// k_weights: every block reads its cloud's sigma_g (the mean edge length of
// eq. 4's bandwidth rule) from those sums,
// then computes row-normalised Gaussian weights of eq. 4 in FP64 with the row's
// smallest squared distance subtracted in the exponent (same ratio, no
// underflow of the whole row), stored as float.  Squared-distance gaps are
// integers, so exp(-gap / sigma_g^2) comes from a per-block table for small
// gaps.  Both kernels are grid-stride over XCD-contiguous shares of points.
#include "fgbd_internal.h"

namespace fgbd {

namespace {

// Squared distance between two points from their packed coordinates
// (x | y << b | z << 2b, b = grid bits <= 10), the form in which the last radix
// pass stores the sorted items.  Every factor is below 2^11 in magnitude, so
// the products run on the full-rate 24-bit multiplier.
// a * b + c on the 24-bit multiplier (operands within +-2^23).  Written out
// because the compiler otherwise folds a 24-bit product and an add into a
// 64-bit multiply-add.
__device__ __forceinline__ int mad_i24(int a, int b, int c) {
  int d;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}
struct Pt {
  int x, y, z;
};
__device__ __forceinline__ Pt unpack_pt(uint32_t c, int bits) {
  return {(int)__builtin_amdgcn_ubfe(c, 0u, (uint32_t)bits), (int)__builtin_amdgcn_ubfe(c, (uint32_t)bits, (uint32_t)bits),
          (int)(c >> (2 * bits))};
}
__device__ __forceinline__ uint32_t pt_dist2(const Pt &pi, uint32_t cj, int bits) {
  const int dx = (int)__builtin_amdgcn_ubfe(cj, 0u, (uint32_t)bits) - pi.x;
  const int dy = (int)__builtin_amdgcn_ubfe(cj, (uint32_t)bits, (uint32_t)bits) - pi.y;
  const int dz = (int)(cj >> (2 * bits)) - pi.z;
  return (uint32_t)mad_i24(dx, dx, mad_i24(dy, dy, __mul24(dz, dz)));
}

template <int KM, typename Key>
__device__ __forceinline__ void topk_insert_t(Key (&lst)[KM], int K, Key c) {
  if (c >= lst[K - 1]) return;
  bool dup = false;
#pragma unroll
  for (int k = 0; k < KM; ++k) dup |= (k < K) & (lst[k] == c);
  if (dup) return;
#pragma unroll
  for (int k = KM - 1; k > 0; --k) {
    if (k < K) {
      const Key prev = lst[k - 1];
      lst[k] = prev > c ? prev : (lst[k] > c ? c : lst[k]);
    }
  }
  lst[0] = lst[0] > c ? c : lst[0];
}

// |a - b| - 1, all ones exactly when a == b (keys below 2^31 or all ones).
__device__ __forceinline__ uint32_t absdiff_m1(uint32_t a, uint32_t b) {
  uint32_t d;
  asm("v_sad_u32 %0, %1, %2, -1" : "=v"(d) : "v"(a), "v"(b));
  return d;
}

// Branch-free insertion into a sorted list of KM distinct keys (keys below
// 2^31; all ones = empty): the candidate is carried down the list, each slot
// keeping the smaller of (slot, carried) and passing the larger on, and the
// largest falls off the end.  A candidate equal to a slot is turned into the
// all-ones sentinel when it meets that slot (earlier slots are smaller, so it
// meets it before any swap), which leaves the list unchanged: the carried
// value is max(slot, carried, |slot - carried| - 1), and the third term is
// all ones only for equal keys and below the larger key otherwise.  Three
// instructions per slot.  The first K slots are then the K smallest
// distinct keys for any K <= KM.
template <int KM>
__device__ __forceinline__ void topk_insert_minmax(uint32_t (&lst)[KM], uint32_t c) {
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    const uint32_t l = lst[k];
    const uint32_t e = absdiff_m1(l, c);
    lst[k] = min(l, c);
    c = max(max(l, c), e);
  }
}

// Median of three unsigned words in one instruction (the compiler forms it
// only from patterns with constants).  Vector registers only.
__device__ __forceinline__ uint32_t med3_u32(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t d;
  asm("v_med3_u32 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

// The same insertion with one median per slot: a candidate equal to a slot
// is first turned into the all-ones sentinel (eight equality tests whose
// results combine on the scalar unit), then slot k takes the median of the
// old slots k - 1 and k and the candidate, which shifts the list up from the
// candidate's place and drops the largest.
template <int KM>
__device__ __forceinline__ void topk_insert_med3(uint32_t (&lst)[KM], uint32_t c) {
  bool dup = false;
#pragma unroll
  for (int k = 0; k < KM; ++k) dup |= lst[k] == c;
  c = dup ? ~0u : c;
  uint32_t nw[KM];
  nw[0] = min(lst[0], c);
#pragma unroll
  for (int k = 1; k < KM; ++k) nw[k] = med3_u32(lst[k - 1], c, lst[k]);
#pragma unroll
  for (int k = 0; k < KM; ++k) lst[k] = nw[k];
}

// Sorts 8 keys ascending (a 19-comparator network of depth 6).
__device__ __forceinline__ void sort8(uint32_t (&v)[8]) {
  constexpr int net[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {0, 1}, {2, 3},
                              {4, 5}, {6, 7}, {2, 4}, {3, 5}, {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
  for (int c = 0; c < 19; ++c) {
    const uint32_t x = v[net[c][0]], y = v[net[c][1]];
    v[net[c][0]] = min(x, y);
    v[net[c][1]] = max(x, y);
  }
}

// Window items r-WT..r+WT; positions outside lo..hi load a clamped position
// (branch-free, all loads in flight together) and are then marked empty.
template <int WT>
__device__ __forceinline__ void load_window(const uint64_t *__restrict__ srt, int r, int lo, int hi,
                                            uint64_t (&w)[2 * WT + 1]) {
#pragma unroll
  for (int s = 0; s <= 2 * WT; ++s) {
    const int pos = r + s - WT;
    w[s] = srt[min(max(pos, lo), hi)];
  }
#pragma unroll
  for (int s = 0; s <= 2 * WT; ++s) {
    const int pos = r + s - WT;
    if (pos < lo || pos > hi) w[s] = ~0ull;
  }
}

constexpr uint32_t kKeyD2Max = 127;  // squared-distance field of the 31-bit keys

struct MergeArgs {
  DirTable dt;
  SegArgs sa;
  int64_t stride;  // items per direction (capacity)
  int32_t window, K;
};

// Exact (64-bit key) selection for one point, runtime window over positions
// lo..hi: used for every point of a cloud of more than 2^24 points and for
// the rare point whose 32-bit selection kept a clamped distance.
template <int KM>
__device__ void select_exact(const MergeArgs &a, int i, int lo, int hi, int window,
                             const uint64_t *__restrict__ sorted, const uint32_t *__restrict__ rank,
                             uint64_t (&lst)[KM]) {
#pragma unroll
  for (int k = 0; k < KM; ++k) lst[k] = ~0ull;
  for (int d = 0; d < a.dt.num_dirs; ++d) {
    const int r = (int)rank[(size_t)d * a.stride + i];
    const uint64_t *srt = sorted + (size_t)d * a.stride;
    const Pt pi = unpack_pt((uint32_t)(srt[r] >> 32), a.dt.bits);
    const int l = max(r - window, lo);
    const int h = min(r + window, hi);
    for (int rr = l; rr <= h; ++rr) {
      if (rr == r) continue;
      const uint64_t it = srt[rr];
      topk_insert_t<KM, uint64_t>(lst, a.K, ((uint64_t)pt_dist2(pi, (uint32_t)(it >> 32), a.dt.bits) << 32) | (uint32_t)it);
    }
  }
}

// One thread per point.  WT > 0 (compile-time window, clouds of at most 2^24
// points; a block of a larger cloud takes the 64-bit selection): the
// point's ranks in all directions go to LDS in one batch of loads; each
// direction's 2*WT+1 window items (the centre gives the point's own code) are
// then loaded as one batch and consumed (prefetching the next direction's
// window would raise the register count from 83 to 109 and the occupancy from
// six to four waves per SIMD, which measured slower); candidates are 31-bit
// keys (min(d2, 127) << 24 | j - cloud start), exact whenever no kept entry has a clamped
// distance, else the point is redone with 64-bit keys.  With w = 4 each
// direction's 8 candidates are first sorted by a network: the first
// direction's (distinct points, empty list) are the list, and later ones are
// inserted in ascending order until no lane of the wave has one left that
// could enter its list.
template <int KM, int WT>
__global__ __launch_bounds__(kBlock) void k_merge(MergeArgs a, const uint64_t *__restrict__ sorted,
                                                  const uint32_t *__restrict__ rank, int32_t *__restrict__ col,
                                                  int32_t *__restrict__ dist2,
                                                  unsigned long long *__restrict__ edge_acc) {
  __shared__ double s_red[4 * 3];  // block_sum_f64<3>: three doubles per wave
  __shared__ int s_rank[WT > 0 ? kMaxDirs : 1][kBlock];
  // edge lengths sqrt(d2) of the small squared distances, each computed once
  // per block (the same correctly rounded values as computing them inline)
  __shared__ double s_sqrt[kKeyD2Max + 1];
  double acc[3] = {0.0, 0.0, 0.0};  // edge lengths, edges, far edges
  const int L = a.dt.num_dirs;
  const int K = a.K;
  const int bits = a.dt.bits;
  const int t = threadIdx.x;
  for (int v = t; v <= (int)kKeyD2Max; v += kBlock) s_sqrt[v] = sqrt((double)v);
  const SegBlock sb = seg_block(a.sa, kGridMerge);
  const int lo = (int)sb.begin, hi = (int)sb.end - 1;
  // the 31-bit keys hold a cloud-local index in 24 bits: a cloud of 2^24 or
  // more points takes the 64-bit selection (uniform over the block)
  const bool fast = sb.end - sb.begin <= (int64_t)(1 << 24);
  const uint32_t gap = (uint32_t)far_gap(sb.end - sb.begin);  // an edge spanning more indices is far
  __syncthreads();
  const Share sh = seg_share(sb, kBlock);
  for (int64_t base = sh.first; base < sh.end; base += sh.step) {
    const int i = (int)(base + t);
    if (i >= sh.end) continue;
    uint64_t lst[KM];
    if (WT > 0 && !fast) {
      select_exact<KM>(a, i, lo, hi, a.window, sorted, rank, lst);
    } else if constexpr (WT > 0) {
      // the first 8 directions' ranks load unconditionally (a direction
      // index past L - 1 re-reads the last one) so all loads are in flight
      // together; a conditional load per direction would be waited for
      // before the next is issued
      int rv[8];
#pragma unroll
      for (int d = 0; d < 8; ++d) rv[d] = (int)rank[(size_t)min(d, L - 1) * a.stride + i];
#pragma unroll
      for (int d = 0; d < 8; ++d) s_rank[d][t] = rv[d];
      for (int d = 8; d < L; ++d) s_rank[d][t] = (int)rank[(size_t)d * a.stride + i];
      uint32_t key[KM];
#pragma unroll
      for (int k = 0; k < KM; ++k) key[k] = ~0u;
      // the point's own packed coordinates (the same item in every order)
      const Pt pi = unpack_pt((uint32_t)(sorted[rv[0]] >> 32), bits);
      for (int d = 0; d < L; ++d) {
        const uint64_t *srt = sorted + (size_t)d * a.stride;
        const int r = s_rank[d][t];
        uint64_t cur[2 * WT + 1];
        uint32_t kc[2 * WT];
        // Wave-uniform: when every window of the wave lies inside the
        // cloud, the items load from one base address with no clamping and
        // no empty slots.
        if (__builtin_amdgcn_ballot_w64(r - WT < lo || r + WT > hi) == 0) {
          const uint64_t *wp = srt + (r - WT);
#pragma unroll
          for (int s = 0; s <= 2 * WT; ++s)
            if (s != WT) cur[s] = wp[s];
#pragma unroll
          for (int s = 0; s < 2 * WT; ++s) {
            const uint64_t it = cur[s < WT ? s : s + 1];
            const uint32_t d2 = pt_dist2(pi, (uint32_t)(it >> 32), bits);
            kc[s] = (min(d2, kKeyD2Max) << 24) | ((uint32_t)it - (uint32_t)lo);
          }
        } else {
          load_window<WT>(srt, r, lo, hi, cur);
#pragma unroll
          for (int s = 0; s < 2 * WT; ++s) {
            const uint64_t it = cur[s < WT ? s : s + 1];
            const uint32_t d2 = pt_dist2(pi, (uint32_t)(it >> 32), bits);
            kc[s] = it == ~0ull ? ~0u : ((min(d2, kKeyD2Max) << 24) | ((uint32_t)it - (uint32_t)lo));
          }
        }
        if constexpr (WT == 4) {
          sort8(kc);
          if (d == 0) {
#pragma unroll
            for (int k = 0; k < 8 && k < KM; ++k) key[k] = kc[k];
            continue;
          }
          // Sorted candidates: once no lane's next one is below its last
          // slot, none of the rest can enter any list (the slots only
          // decrease).
#pragma unroll
          for (int s = 0; s < 8; ++s) {
            if (__builtin_amdgcn_ballot_w64(kc[s] < key[KM - 1]) == 0) break;
            topk_insert_med3<KM>(key, kc[s]);
          }
        } else {
#pragma unroll
          for (int s = 0; s < 2 * WT; ++s) topk_insert_minmax<KM>(key, kc[s]);
        }
      }
      bool clamped = false;
#pragma unroll
      for (int k = 0; k < KM; ++k) clamped |= (k < K) & (key[k] != ~0u) & ((key[k] >> 24) == kKeyD2Max);
      if (clamped) {
        select_exact<KM>(a, i, lo, hi, WT, sorted, rank, lst);
      } else {
#pragma unroll
        for (int k = 0; k < KM; ++k)
          lst[k] = key[k] == ~0u ? ~0ull : ((uint64_t)(key[k] >> 24) << 32) | ((key[k] & 0xffffffu) + (uint32_t)lo);
      }
    } else {
      select_exact<KM>(a, i, lo, hi, a.window, sorted, rank, lst);
    }
    int cv[KM], dv[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const bool ok = lst[k] != ~0ull;
      const uint32_t d2 = (uint32_t)(lst[k] >> 32);
      cv[k] = ok ? (int32_t)(uint32_t)lst[k] : -1;

      dv[k] = ok ? (int32_t)d2 : 0;
      if (ok && k < K) {
        acc[0] += d2 <= kKeyD2Max ? s_sqrt[d2] : sqrt((double)d2);
        acc[1] += 1.0;
        acc[2] += (uint32_t)abs(cv[k] - i) > gap ? 1.0 : 0.0;
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
  block_sum_f64<3>(acc, s_red);
  if (threadIdx.x == 0) {
    unsigned long long *e = edge_acc + ((size_t)sb.s * kEdgeSlots + sb.lb % kEdgeSlots) * kEdgeVals;
    const double whole = floor(acc[0]);  // acc[0] >= 0; the fraction below is exact
    atomicAdd(&e[0], (unsigned long long)whole);
    atomicAdd(&e[1], (unsigned long long)llrint((acc[0] - whole) * kEdgeFrac));
    atomicAdd(&e[2], (unsigned long long)acc[1]);
    atomicAdd(&e[3], (unsigned long long)acc[2]);
  }
}

// Selection for grids above 2^10 (codes wider than 32 bits): the sorted items
// hold only indices, so each candidate's coordinates come from the input;
// squared distances are 64-bit and the K nearest are kept by (squared
// distance, index) in a sorted list of pairs.  One thread per point, runtime
// window.  dist2 saturates at 2^31 - 1 (FGBD_ST_DIST_CLAMPED), which only a
// neighbour more than 46340 voxels away can reach.
template <int KM>
__global__ __launch_bounds__(kBlock) void k_merge_wide(MergeArgs a, const int32_t *__restrict__ xyz,
                                                       const uint64_t *__restrict__ sorted,
                                                       const uint32_t *__restrict__ rank, int32_t *__restrict__ col,
                                                       int32_t *__restrict__ dist2,
                                                       unsigned long long *__restrict__ edge_acc,
                                                       fgbd_result *__restrict__ res) {
  __shared__ double s_red[4 * 3];
  double acc[3] = {0.0, 0.0, 0.0};  // edge lengths, edges, far edges
  const int L = a.dt.num_dirs;
  const int K = a.K;
  const SegBlock sb = seg_block(a.sa, kGridMerge);
  const int lo = (int)sb.begin, hi = (int)sb.end - 1;
  const uint32_t gap = (uint32_t)far_gap(sb.end - sb.begin);
  int clamped = 0;
  const Share sh = seg_share(sb, kBlock);
  for (int64_t base = sh.first; base < sh.end; base += sh.step) {
    const int i = (int)(base + threadIdx.x);
    if (i >= sh.end) continue;
    const int64_t px = xyz[3 * (size_t)i + 0], py = xyz[3 * (size_t)i + 1], pz = xyz[3 * (size_t)i + 2];
    uint64_t kd[KM];
    uint32_t kj[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      kd[k] = ~0ull;
      kj[k] = ~0u;
    }
    for (int d = 0; d < L; ++d) {
      const uint64_t *srt = sorted + (size_t)d * a.stride;
      const int r = (int)rank[(size_t)d * a.stride + i];
      const int l = max(r - a.window, lo), h = min(r + a.window, hi);
      for (int rr = l; rr <= h; ++rr) {
        if (rr == r) continue;
        const uint32_t j = (uint32_t)srt[rr];
        const int64_t dx = xyz[3 * (size_t)j + 0] - px, dy = xyz[3 * (size_t)j + 1] - py,
                      dz = xyz[3 * (size_t)j + 2] - pz;
        uint64_t cd = (uint64_t)(dx * dx + dy * dy + dz * dz);
        uint32_t cj = j;
        // insert (cd, cj) into the list ordered by (distance, index), once
        bool dup = false;
#pragma unroll
        for (int k = 0; k < KM; ++k) dup |= kd[k] == cd && kj[k] == cj;
        if (dup) continue;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const bool less = cd < kd[k] || (cd == kd[k] && cj < kj[k]);
          const uint64_t td = kd[k];
          const uint32_t tj = kj[k];
          kd[k] = less ? cd : td;
          kj[k] = less ? cj : tj;
          cd = less ? td : cd;
          cj = less ? tj : cj;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (k >= K) continue;
      const bool ok = kj[k] != ~0u;
      int32_t dv = 0;
      if (ok) {
        dv = kd[k] > 0x7fffffffull ? 0x7fffffff : (int32_t)kd[k];
        clamped |= kd[k] > 0x7fffffffull;
        acc[0] += sqrt((double)kd[k]);
        acc[1] += 1.0;
        acc[2] += (uint32_t)abs((int)kj[k] - i) > gap ? 1.0 : 0.0;
      }
      col[(size_t)i * K + k] = ok ? (int32_t)kj[k] : -1;
      dist2[(size_t)i * K + k] = dv;
    }
  }
  if (__builtin_amdgcn_ballot_w64(clamped != 0) != 0 && lane_id() == 0)
    atomicOr(&res[sb.s].status, FGBD_ST_DIST_CLAMPED);
  block_sum_f64<3>(acc, s_red);
  if (threadIdx.x == 0) {
    unsigned long long *e = edge_acc + ((size_t)sb.s * kEdgeSlots + sb.lb % kEdgeSlots) * kEdgeVals;
    const double whole = floor(acc[0]);
    atomicAdd(&e[0], (unsigned long long)whole);
    atomicAdd(&e[1], (unsigned long long)llrint((acc[0] - whole) * kEdgeFrac));
    atomicAdd(&e[2], (unsigned long long)acc[1]);
    atomicAdd(&e[3], (unsigned long long)acc[2]);
  }
}

// Renumbering of a cloud along scan order 0, for clouds whose kept edges
// mostly span more than far_gap input indices (an input order far from
// spatial, where every gather of the noise estimate and the sweeps would touch
// its own cache line): row r of col_w / dist2_w is the row of the point at
// position r of scan order 0, each neighbour replaced by its own position, and
// rgb_w[r] is that point's colour.  The rows keep their neighbours and their
// order (the selection broke ties by input index).  Runs on the merge grid; a
// cloud left as it is returns at once.
template <int KT>
__global__ __launch_bounds__(kBlock) void k_relabel(SegArgs sa, int32_t k_rt, Segs *__restrict__ order,
                                                    const unsigned long long *__restrict__ edge_acc,
                                                    const uint64_t *__restrict__ sorted0,
                                                    const uint32_t *__restrict__ rank0,
                                                    const int32_t *__restrict__ col, const int32_t *__restrict__ dist2,
                                                    const float *__restrict__ rgb, int32_t *__restrict__ col_w,
                                                    int32_t *__restrict__ dist2_w, float *__restrict__ rgb_w) {
  const int K = KT > 0 ? KT : k_rt;
  const SegBlock sb = seg_block(sa, kGridMerge);
  __shared__ unsigned long long s_u[kEdgeVals];
  if (threadIdx.x < kWave) {  // the cloud's edge and far-edge counts over its slots
    static_assert(kEdgeSlots == kWave, "one slot per lane");
    const unsigned long long *e = edge_acc + ((size_t)sb.s * kEdgeSlots + threadIdx.x) * kEdgeVals;
    unsigned long long all = e[2], far = e[3];
    for (int o = 32; o > 0; o >>= 1) {
      all += __shfl_xor(all, o, kWave);
      far += __shfl_xor(far, o, kWave);
    }
    if (threadIdx.x == 0) {
      s_u[0] = all;
      s_u[1] = far;
    }
  }
  __syncthreads();
  if (s_u[0] == 0 || 4ull * s_u[1] <= s_u[0]) return;  // uniform over the block
  if (sb.lb == 0 && threadIdx.x == 0) order->relabel[sb.s] = 1;
  const Share sh = seg_share(sb, kBlock);
  for (int64_t base = sh.first; base < sh.end; base += sh.step) {
    const int64_t r = base + threadIdx.x;
    if (r >= sh.end) continue;
    const int64_t i = (uint32_t)sorted0[r];  // the point at position r
    rgb_w[3 * r + 0] = rgb[3 * i + 0];
    rgb_w[3 * r + 1] = rgb[3 * i + 1];
    rgb_w[3 * r + 2] = rgb[3 * i + 2];
    if (KT == 8) {
      const int4 *cr = reinterpret_cast<const int4 *>(col + i * 8);
      const int4 *dr = reinterpret_cast<const int4 *>(dist2 + i * 8);
      const int4 c0 = cr[0], c1 = cr[1];
      int cv[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
      for (int k = 0; k < 8; ++k) cv[k] = cv[k] >= 0 ? (int)rank0[cv[k]] : -1;
      int4 *cw = reinterpret_cast<int4 *>(col_w + r * 8);
      int4 *dw = reinterpret_cast<int4 *>(dist2_w + r * 8);
      cw[0] = make_int4(cv[0], cv[1], cv[2], cv[3]);
      cw[1] = make_int4(cv[4], cv[5], cv[6], cv[7]);
      dw[0] = dr[0];
      dw[1] = dr[1];
    } else {
      for (int k = 0; k < K; ++k) {
        const int c = col[i * K + k];
        col_w[r * K + k] = c >= 0 ? (int)rank0[c] : -1;
        dist2_w[r * K + k] = dist2[i * K + k];
      }
    }
  }
}

// Runs on the merge grid: block b belongs to the same cloud as merge block b.
template <int KT>
__global__ __launch_bounds__(kBlock) void k_weights(SegArgs sa, int32_t k_rt, const int32_t *__restrict__ col,
                                                    const int32_t *__restrict__ dist2,
                                                    const unsigned long long *__restrict__ edge_acc,
                                                    double sigma_g_fixed,
                                                    fgbd_result *__restrict__ res, float *__restrict__ p) {
  __shared__ double s_red[8];
  __shared__ double s_exp[kExpTable];
  const int K = KT > 0 ? KT : k_rt;
  const SegBlock sb = seg_block(sa, kGridMerge);
  const double sg = cloud_sigma_g(edge_acc + (size_t)kEdgeSlots * kEdgeVals * sb.s, sigma_g_fixed,
                                  reinterpret_cast<unsigned long long *>(s_red));
  if (sb.lb == 0 && threadIdx.x == 0) res[sb.s].sigma_g = sg;
  fill_exp_table(sg, s_exp);
  __syncthreads();
  constexpr int KB = KT > 0 ? KT : kMaxK;
  const Share sh = seg_share(sb, kBlock);
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
    float pw[KB];
    row_weights<KB>(cv, dv, sg, s_exp, pw);
    if (KT == 8) {
      float4 *pr = reinterpret_cast<float4 *>(p + i * 8);
      pr[0] = make_float4(pw[0], pw[1], pw[2], pw[3]);
      pr[1] = make_float4(pw[4], pw[5], pw[6], pw[7]);
    } else {
#pragma unroll
      for (int k = 0; k < KB; ++k)
        if (k < K) p[i * K + k] = pw[k];
    }
  }
}

}  // namespace

hipError_t launch_merge(const Run &r, const int32_t *xyz, const uint64_t *sorted, int32_t *col, int32_t *dist2,
                        fgbd_result *res) {
  MergeArgs a;
  a.dt = r.dt;
  a.sa = r.sa;
  a.stride = r.pl.stride;
  a.window = r.prm.window;
  a.K = r.prm.k;
  const int k = r.prm.k, window = r.prm.window;
  const int nb = r.pl.grid[kGridMerge];
  const uint32_t *rank = r.b.rank;
  unsigned long long *part = r.b.edge_acc;
  hipStream_t st = r.stream;
  if (r.dt.passes > kSortPasses) {  // codes above 32 bits: items hold indices only
    if (k <= 8)
      k_merge_wide<8><<<nb, kBlock, 0, st>>>(a, xyz, sorted, rank, col, dist2, part, res);
    else if (k <= 16)
      k_merge_wide<16><<<nb, kBlock, 0, st>>>(a, xyz, sorted, rank, col, dist2, part, res);
    else
      k_merge_wide<32><<<nb, kBlock, 0, st>>>(a, xyz, sorted, rank, col, dist2, part, res);
    return hipGetLastError();
  }
  // the compile-time-window kernels take 64-bit keys for a cloud of more
  // than 2^24 points (their 31-bit keys hold a cloud-local index)
  if (k <= 8 && window == 4)
    k_merge<8, 4><<<nb, kBlock, 0, st>>>(a, sorted, rank, col, dist2, part);
  else if (k <= 8 && window == 1)
    k_merge<8, 1><<<nb, kBlock, 0, st>>>(a, sorted, rank, col, dist2, part);
  else if (k <= 8 && window == 2)
    k_merge<8, 2><<<nb, kBlock, 0, st>>>(a, sorted, rank, col, dist2, part);
  else if (k <= 8)
    k_merge<8, 0><<<nb, kBlock, 0, st>>>(a, sorted, rank, col, dist2, part);
  else if (k <= 16 && window == 4)
    k_merge<16, 4><<<nb, kBlock, 0, st>>>(a, sorted, rank, col, dist2, part);
  else if (k <= 16)
    k_merge<16, 0><<<nb, kBlock, 0, st>>>(a, sorted, rank, col, dist2, part);
  else
    k_merge<32, 0><<<nb, kBlock, 0, st>>>(a, sorted, rank, col, dist2, part);
  return hipGetLastError();
}

hipError_t launch_relabel(const Run &r, const uint64_t *sorted, const int32_t *col, const int32_t *dist2,
                          const float *rgb) {
  if (!r.relabel_ok) return hipSuccess;
  const int nb = r.pl.grid[kGridMerge];
  if (r.prm.k == 8)
    k_relabel<8><<<nb, kBlock, 0, r.stream>>>(r.sa, 8, r.b.segs, r.b.edge_acc, sorted, r.b.rank, col, dist2, rgb,
                                              r.b.col_w, r.b.dist2_w, r.b.rgb_w);
  else
    k_relabel<0><<<nb, kBlock, 0, r.stream>>>(r.sa, r.prm.k, r.b.segs, r.b.edge_acc, sorted, r.b.rank, col, dist2,
                                              rgb, r.b.col_w, r.b.dist2_w, r.b.rgb_w);
  return hipGetLastError();
}

hipError_t launch_weights(const Run &r, const int32_t *col, const int32_t *dist2, fgbd_result *res, float *p) {
  const int nb = r.pl.grid[kGridMerge];
  if (r.prm.k == 8)
    k_weights<8><<<nb, kBlock, 0, r.stream>>>(r.sa, 8, col, dist2, r.b.edge_acc, r.prm.sigma_g, res, p);
  else
    k_weights<0><<<nb, kBlock, 0, r.stream>>>(r.sa, r.prm.k, col, dist2, r.b.edge_acc, r.prm.sigma_g, res, p);
  return hipGetLastError();
}

}  // namespace fgbd
