// Scan-line codes and the LSD radix sort of Sec. 2.2 (the paper orders the
// points of each code with a radix sort).  One launch covers all L directions
// (grid.y = direction).  Items are 64-bit: code << 32 | point index, so each
// pass moves 8 bytes per item and ties (duplicate points) keep index order
// because every pass is stable.
//
// Per 8-bit digit pass (4 passes for 32-bit codes):
//   upsweep   per tile digit histogram            -> hist[dir][digit][tile]
//   scan      exclusive prefix over (digit, tile)  -> global offsets, in place
//   downsweep stable rank inside the tile (wave-level match of digits with
//             64-bit ballots, per-wave counters in LDS), stage in LDS in digit
//             order, then write runs of equal digits to their global offsets.
// Pass 0 computes the codes from the int32 coordinates on the fly; the last
// pass also writes rank[dir][index] = sorted position, which the neighbour
// search uses to find each point's place in every order.
#include "fgbd_internal.h"

namespace fgbd {

namespace {

struct SortArgs {
  DirTable dt;
  int32_t n;
  int32_t ntiles;
  int32_t shift;  // digit shift of this pass
  int32_t pass;
};

__device__ __forceinline__ uint64_t load_item(const SortArgs &a, const int32_t *__restrict__ xyz,
                                              const uint64_t *__restrict__ src, int d, int pos, int *bad) {
  if (a.pass == 0) {
    const int gx = xyz[3 * pos + 0], gy = xyz[3 * pos + 1], gz = xyz[3 * pos + 2];
    const int top = (1 << a.dt.bits) - 1;
    if ((unsigned)gx > (unsigned)top || (unsigned)gy > (unsigned)top || (unsigned)gz > (unsigned)top) *bad = 1;
    const uint32_t code = scan_code(gx, gy, gz, a.dt.d[d], a.dt.bits);
    return ((uint64_t)code << 32) | (uint32_t)pos;
  }
  return src[(size_t)d * a.n + pos];
}

__global__ __launch_bounds__(kSortThreads) void k_sort_upsweep(SortArgs a, const int32_t *__restrict__ xyz,
                                                               const uint64_t *__restrict__ src,
                                                               uint32_t *__restrict__ hist,
                                                               uint32_t *__restrict__ totals,
                                                               fgbd_result *__restrict__ res) {
  __shared__ uint32_t s_h[256];
  __shared__ uint32_t s_all[kSortPasses][256];
  const int d = blockIdx.y;
  const int tile = blockIdx.x;
  const int t = threadIdx.x;
  s_h[t] = 0;
  if (a.pass == 0) {
#pragma unroll
    for (int q = 0; q < kSortPasses; ++q) s_all[q][t] = 0;
  }
  __syncthreads();
  const int wave = t / kWave;
  const int lane = (int)lane_id();
  const int base = tile * kSortTile + wave * kWave * kSortItems + lane;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int pos = base + j * kWave;
    if (pos < a.n) {
      const uint64_t it = load_item(a, xyz, src, d, pos, &bad);
      const uint32_t digit = (uint32_t)(it >> (32 + a.shift)) & 255u;
      atomicAdd(&s_h[digit], 1u);
      if (a.pass == 0) {  // digit totals of every pass, for the offset scan
#pragma unroll
        for (int q = 1; q < kSortPasses; ++q) atomicAdd(&s_all[q][(uint32_t)(it >> (32 + 8 * q)) & 255u], 1u);
      }
    }
  }
  if (bad && d == 0) atomicOr(&res->status, FGBD_ST_COORD_RANGE);
  __syncthreads();
  hist[((size_t)d * 256 + t) * a.ntiles + tile] = s_h[t];
  if (a.pass == 0) {
    uint32_t *tot = totals + (size_t)d * kSortPasses * 256;
    if (s_h[t]) atomicAdd(&tot[t], s_h[t]);
#pragma unroll
    for (int q = 1; q < kSortPasses; ++q)
      if (s_all[q][t]) atomicAdd(&tot[q * 256 + t], s_all[q][t]);
  }
}

// Global offsets: one wave per (direction, digit) row of tile counts.  The
// row's base is the sum of the direction's totals of all smaller digits; the
// row is then scanned 64 tiles at a time with a wave prefix sum.
__global__ __launch_bounds__(256) void k_sort_scan(int ntiles, int num_dirs, int pass, uint32_t *__restrict__ hist,
                                                   const uint32_t *__restrict__ totals) {
  const int row = blockIdx.x * 4 + threadIdx.x / kWave;
  if (row >= num_dirs * 256) return;
  const int d = row / 256, digit = row % 256;
  const uint32_t lane = lane_id();
  const uint32_t *tot = totals + ((size_t)d * kSortPasses + pass) * 256;
  uint32_t b = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int dg = (int)lane + 64 * j;
    b += dg < digit ? tot[dg] : 0u;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) b += __shfl_xor(b, o, kWave);
  uint32_t carry = b;
  uint32_t *h = hist + (size_t)row * ntiles;
  for (int t0 = 0; t0 < ntiles; t0 += kWave) {
    const int tile = t0 + (int)lane;
    const uint32_t v = tile < ntiles ? h[tile] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, kWave);
      if (lane >= (uint32_t)o) x += y;
    }
    if (tile < ntiles) h[tile] = carry + x - v;
    carry += __shfl(x, kWave - 1, kWave);
  }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_downsweep(SortArgs a, const int32_t *__restrict__ xyz,
                                                                 const uint64_t *__restrict__ src,
                                                                 uint64_t *__restrict__ dst,
                                                                 const uint32_t *__restrict__ hist,
                                                                 uint32_t *__restrict__ rank) {
  __shared__ uint32_t s_wh[4][256];
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_tmp[4];
  __shared__ uint64_t s_stage[kSortTile];

  const int d = blockIdx.y;
  const int tile = blockIdx.x;
  const int t = threadIdx.x;
  const int wave = t / kWave;
  const int lane = (int)lane_id();
  const int tile0 = tile * kSortTile;
  const int valid = min(kSortTile, a.n - tile0);

  s_wh[0][t] = 0;
  s_wh[1][t] = 0;
  s_wh[2][t] = 0;
  s_wh[3][t] = 0;
  s_off[t] = hist[((size_t)d * 256 + t) * a.ntiles + tile];

  uint64_t item[kSortItems];
  const int base = tile0 + wave * kWave * kSortItems + lane;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int pos = base + j * kWave;
    item[j] = (pos < a.n) ? load_item(a, xyz, src, d, pos, &bad) : ~0ull;
  }
  __syncthreads();

  // Stable rank of each item among the equal digits of its wave: items are
  // visited in tile order (j major, lane minor within the wave).
  uint32_t rk[kSortItems];
  const uint64_t below_mask = (1ull << lane) - 1ull;
  (void)below_mask;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t digit = (uint32_t)(item[j] >> (32 + a.shift)) & 255u;
    uint64_t peers = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t vote = __builtin_amdgcn_ballot_w64((digit >> b) & 1u);
      peers &= ((digit >> b) & 1u) ? vote : ~vote;
    }
    const uint32_t before = count_below(peers);
    const uint32_t cnt = (uint32_t)__popcll(peers);
    const uint32_t cur = s_wh[wave][digit];
    rk[j] = cur + before;
    if (before == 0) s_wh[wave][digit] = cur + cnt;
  }
  __syncthreads();

  // per digit: exclusive over waves, then exclusive over digits in the tile
  {
    const uint32_t c0 = s_wh[0][t], c1 = s_wh[1][t], c2 = s_wh[2][t], c3 = s_wh[3][t];
    s_wh[0][t] = 0;
    s_wh[1][t] = c0;
    s_wh[2][t] = c0 + c1;
    s_wh[3][t] = c0 + c1 + c2;
    uint32_t total;
    s_base[t] = block_exclusive_scan_256(c0 + c1 + c2 + c3, s_tmp, &total);
  }
  __syncthreads();

#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t digit = (uint32_t)(item[j] >> (32 + a.shift)) & 255u;
    s_stage[s_base[digit] + s_wh[wave][digit] + rk[j]] = item[j];
  }
  __syncthreads();

  const bool last_pass = (a.pass == kSortPasses - 1);
  uint64_t *out = dst + (size_t)d * a.n;
  for (int s = t; s < valid; s += kSortThreads) {
    const uint64_t it = s_stage[s];
    const uint32_t digit = (uint32_t)(it >> (32 + a.shift)) & 255u;
    const uint32_t gpos = s_off[digit] + (uint32_t)s - s_base[digit];
    out[gpos] = it;
    if (last_pass) rank[(size_t)d * a.n + (uint32_t)it] = gpos;
  }
}

}  // namespace

__global__ void k_zero(uint32_t *__restrict__ p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t launch_sort(const int32_t *xyz, int64_t n, const DirTable &dt, const Plan &pl, uint64_t *items_a,
                       uint64_t *items_b, uint32_t *hist, uint32_t *totals, uint32_t *rank, fgbd_result *res,
                       hipStream_t stream, const uint64_t **sorted_out, Prof *pf) {
  SortArgs a;
  a.dt = dt;
  a.n = (int32_t)n;
  a.ntiles = pl.ntiles;
  const dim3 grid(pl.ntiles, dt.num_dirs);
  const uint64_t *src = nullptr;
  uint64_t *bufs[2] = {items_a, items_b};
  FGBD_PRE(pf, kUpsweep);
  k_zero<<<1, 256, 0, stream>>>(totals, dt.num_dirs * kSortPasses * 256);
  FGBD_POST(pf);
  for (int pass = 0; pass < kSortPasses; ++pass) {
    a.pass = pass;
    a.shift = 8 * pass;
    uint64_t *dst = bufs[pass & 1];
    FGBD_PRE(pf, kUpsweep);
    k_sort_upsweep<<<grid, kSortThreads, 0, stream>>>(a, xyz, src, hist, totals, res);
    FGBD_POST(pf);
    FGBD_PRE(pf, kScan);
    k_sort_scan<<<(dt.num_dirs * 256 + 3) / 4, 256, 0, stream>>>(pl.ntiles, dt.num_dirs, pass, hist, totals);
    FGBD_POST(pf);
    FGBD_PRE(pf, kDownsweep);
    k_sort_downsweep<<<grid, kSortThreads, 0, stream>>>(a, xyz, src, dst, hist, rank);
    FGBD_POST(pf);
    src = dst;
  }
  *sorted_out = src;
  return hipGetLastError();
}

}  // namespace fgbd
