// Scan-line codes and the radix sort of Sec. 2.2 (the paper orders the
// points of each code with a radix sort).  One launch covers all L directions
// (grid.y = direction).  Items are 64-bit: code << 32 | point index, so each
// pass moves 8 bytes per item and ties (duplicate points) keep index order
// because every pass is stable.  Codes of at most 32 bits take the top-digit
// route at the end of this file (one pass on the top 10 bits, then each
// window's buckets sorted in LDS); the LSD passes below sort wider codes.
//
// Per 8-bit digit pass (4 passes for 32-bit codes):
//   upsweep   per tile digit histogram            -> hist[dir][tile][digit]
//   scan      exclusive prefix over (digit, tile)  -> global offsets, in place
//   downsweep stable rank inside the tile (wave-level match of digits with
//             64-bit ballots, per-wave counters in LDS), stage in LDS in digit
//             order, then write runs of equal digits to their global offsets.
// Pass 0 computes the codes from the int32 coordinates on the fly; the last
// pass also writes rank[dir][index] = sorted position, which the neighbour
// search uses to find each point's place in every order, and stores each
// sorted item with the point's packed coordinates (x | y << b | z << 2b) in
// place of its code.
//
// Grids above 2^10 (b = 11..21) give codes of up to 63 bits.  Items then carry
// the code 32 bits at a time: passes 0-3 sort by the low 32 bits, pass 3
// re-keys every item with the high bits of its code (made again from the
// point's coordinates), and passes 4.. sort by those (LSD over digit groups:
// the order is by the whole code).  The last pass then stores only the index
// (packed coordinates no longer fit beside it) and the neighbour search reads
// coordinates from the input.
//
// Several clouds are sorted in the same launches, each inside its own range
// of positions: tiles never straddle two clouds, the scan runs over all tiles
// of each digit and also stores the total after the last tile, and with P the
// scanned counts of digit c, the cloud's count of c is P[next cloud's first
// tile] - P[its first tile], so each tile's output offset for digit c is
//   start[s] + (digits < c in cloud s) + (P[this tile] - P[cloud's first tile]).
#include "fgbd_internal.h"

namespace fgbd {

namespace {

struct SortArgs {
  DirTable dt;
  SegArgs sa;
  int64_t stride;     // items per direction (capacity)
  int32_t row;        // hist row length (tile capacity + 1: the row total)
  int32_t shift;      // digit shift of this pass inside the item's 32 code bits
  int32_t pass;
  int32_t passes;     // passes of the sort (4, or more for codes above 32 bits)
  int32_t fold;       // pass 0 only: the first blocks also do the call's setup
  SetupArgs su;
  int32_t *win;       // top-digit pass: the first bucket start of each local-sort window
  int32_t nwin;       // windows per direction
};

// The tile's cloud and point range; false for a tile beyond the last one.
struct TileInfo {
  int s;
  int begin, end;  // points of the tile
  int first;       // first tile of the cloud
  int next_first;  // first tile of the next cloud (= tile count after the last)
  int seg_start;   // first point of the cloud
};
__device__ __forceinline__ bool tile_info(const SortArgs &a, int tile, TileInfo &ti) {
  if (a.sa.n_fixed >= 0) {
    const int n = a.sa.n_fixed;
    if (tile * kSortTile >= n) return false;
    ti.s = 0;
    ti.first = 0;
    ti.next_first = (n + kSortTile - 1) / kSortTile;
    ti.seg_start = 0;
    ti.begin = tile * kSortTile;
    ti.end = min(ti.begin + kSortTile, n);
    return true;
  }
  const Segs *sg = a.sa.segs;
  if (tile >= sg->ntiles) return false;
  const int s = seg_lookup(sg->tile_first, a.sa.B, tile);
  ti.s = s;
  ti.first = sg->tile_first[s];
  ti.next_first = sg->tile_first[s + 1];
  ti.seg_start = sg->start[s];
  ti.begin = ti.seg_start + (tile - ti.first) * kSortTile;
  ti.end = min(ti.begin + kSortTile, (int)sg->start[s + 1]);
  return true;
}

// (direction, tile) of a block (grid.x = tiles, grid.y = directions):
// workgroups go to the 8 XCDs round robin, so block b runs on XCD b % 8; each
// XCD gets one contiguous range of the tile-major sequence (tile, direction),
// so it works on a contiguous range of tiles in every direction.  The L
// directions of one tile run back to back on one XCD, so pass 0 reads the
// tile's coordinates from memory once and from L2 after, and the runs that
// consecutive tiles write side by side for each digit meet in one L2 before
// they are written back.
__device__ __forceinline__ void xcd_tile(int &d, int &tile) {
  const int nb = (int)(gridDim.x * gridDim.y);
  const int b = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int x = b % kXcds, k = b / kXcds;
  const int g = x * (nb / kXcds) + min(x, nb % kXcds) + k;
  d = g % (int)gridDim.y;
  tile = g / (int)gridDim.y;
}

// The last pass instead gives each XCD one contiguous range of the
// direction-major sequence (direction, tile): with 8 directions each XCD
// sorts one direction, so its scattered rank writes land in one array of
// 4 bytes per point (measured slightly faster than the tile-major ranges).
__device__ __forceinline__ void xcd_tile_last(int &d, int &tile) {
  const int nb = (int)(gridDim.x * gridDim.y);
  const int b = (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int x = b % kXcds, k = b / kXcds;
  const int g = x * (nb / kXcds) + min(x, nb % kXcds) + k;
  d = g / (int)gridDim.x;
  tile = g % (int)gridDim.x;
}

__device__ __forceinline__ int num_tiles(const SortArgs &a) {
  return a.sa.n_fixed >= 0 ? (a.sa.n_fixed + kSortTile - 1) / kSortTile : a.sa.segs->ntiles;
}

// The scan-line code of one direction (the same integers as scan_code), with
// the direction's constants read once per block: inside the item loops a
// reload from the argument segment would wait on the LDS atomics too.
struct CodeGen {
  int ia, ih, im, uh, um, wm, bits;
  uint32_t oh, om;
};
__device__ __forceinline__ CodeGen code_gen(const DirTable &dt, int d) {
  const DirInfo di = dt.d[d];
  const uint32_t top = (1u << dt.bits) - 1u;
  CodeGen c;
  c.ia = di.a;
  c.ih = di.h;
  c.im = di.m;
  c.uh = di.uh;
  c.um = di.um;
  c.oh = di.uh > 0 ? (uint32_t)di.uh * top : 0u;
  c.om = di.um > 0 ? (uint32_t)di.um * top : 0u;
  c.wm = dt.bits + di.wm_extra;
  c.bits = dt.bits;
  return c;
}
__device__ __forceinline__ uint32_t gen_code(const CodeGen &c, int gx, int gy, int gz) {
  const int ga = c.ia == 0 ? gx : (c.ia == 1 ? gy : gz);
  const int gh = c.ih == 0 ? gx : (c.ih == 1 ? gy : gz);
  const int gm = c.im == 0 ? gx : (c.im == 1 ? gy : gz);
  const uint32_t eh = (uint32_t)(gh - c.uh * ga) + c.oh;
  const uint32_t em = (uint32_t)(gm - c.um * ga) + c.om;
  return (((eh << c.wm) + em) << c.bits) | (uint32_t)ga;
}

// The code's bits above 32 (codes of grids above 2^10).
__device__ __forceinline__ uint32_t gen_code_hi(const CodeGen &c, int gx, int gy, int gz) {
  const int ga = c.ia == 0 ? gx : (c.ia == 1 ? gy : gz);
  const int gh = c.ih == 0 ? gx : (c.ih == 1 ? gy : gz);
  const int gm = c.im == 0 ? gx : (c.im == 1 ? gy : gz);
  const uint64_t eh = (uint32_t)(gh - c.uh * ga) + c.oh;
  const uint64_t em = (uint32_t)(gm - c.um * ga) + c.om;
  return (uint32_t)((((eh << c.wm) + em) << c.bits | (uint32_t)ga) >> 32);
}

// The inverse of gen_code, packed as x | y << b | z << 2b (b = grid bits).
__device__ __forceinline__ uint32_t decode_packed(const CodeGen &c, uint32_t code) {
  const uint32_t top = (1u << c.bits) - 1u;
  const int ga = (int)(code & top);
  const int em = (int)((code >> c.bits) & ((1u << c.wm) - 1u));
  const int eh = (int)(code >> (c.bits + c.wm));
  const int gm = em + c.um * ga - (int)c.om;
  const int gh = eh + c.uh * ga - (int)c.oh;
  const int gx = c.ia == 0 ? ga : (c.ih == 0 ? gh : gm);
  const int gy = c.ia == 1 ? ga : (c.ih == 1 ? gh : gm);
  const int gz = c.ia == 2 ? ga : (c.ih == 2 ? gh : gm);
  return (uint32_t)gx | ((uint32_t)gy << c.bits) | ((uint32_t)gz << (2 * c.bits));
}

__device__ __forceinline__ uint64_t load_item(const SortArgs &a, const CodeGen &cg, const int32_t *__restrict__ xyz,
                                              const uint64_t *__restrict__ src, int d, int pos, int *bad) {
  if (a.pass == 0) {
    const int gx = xyz[3 * pos + 0], gy = xyz[3 * pos + 1], gz = xyz[3 * pos + 2];
    const int top = (1 << a.dt.bits) - 1;
    if ((unsigned)gx > (unsigned)top || (unsigned)gy > (unsigned)top || (unsigned)gz > (unsigned)top) *bad = 1;
    return ((uint64_t)gen_code(cg, gx, gy, gz) << 32) | (uint32_t)pos;
  }
  return src[(size_t)d * a.stride + pos];
}

// All blocks clear the first sweep's sums and the noise moment accumulators;
// block 0 builds the segment table:
// offsets clamped into a valid form (start[0] = 0, non-decreasing, at most
// n_cap), radix tiles per cloud, and each per-cloud grid's block ranges
// first(s) = floor(start[s] (G - B) / n) + s (at least one block per cloud).
__device__ __forceinline__ void setup_work(const SetupArgs &a, int block) {
  Segs *__restrict__ sg = a.sg;
  unsigned long long *__restrict__ sums1 = a.sums1;
  fgbd_result *__restrict__ res = a.res;
  __shared__ int64_t s_raw[kMaxSeg + 1];
  __shared__ int32_t s_start[kMaxSeg + 1], s_tf[kMaxSeg + 1];
  __shared__ int32_t s_bad;
  const int t = threadIdx.x;
  const int stride = a.blocks * (int)blockDim.x;
  for (int i = block * blockDim.x + t; i < 3 * a.sums_count; i += stride) sums1[i] = 0ull;
  for (int i = block * blockDim.x + t; i < a.noise_count; i += stride) a.noise_acc[i] = 0ull;
  for (int i = block * blockDim.x + t; i < a.edge_count; i += stride) a.edge_acc[i] = 0ull;
  if (block != 0) return;  // uniform over the block
  if (t < kMaxSeg) sg->relabel[t] = 0;
  const int B = a.B;
  if (t <= B) s_raw[t] = a.offsets ? a.offsets[t] : (t == 0 ? 0 : a.n_host);
  __syncthreads();
  if (t == 0) {
    int bad = s_raw[0] != 0;
    int64_t prev = 0;
    int32_t tiles = 0;
    s_start[0] = 0;
    for (int s = 1; s <= B; ++s) {
      int64_t v = s_raw[s];
      v = v < prev ? prev : v;
      v = v > a.n_cap ? a.n_cap : v;
      bad |= v != s_raw[s];
      s_start[s] = (int32_t)v;
      s_tf[s - 1] = tiles;
      tiles += (int32_t)((v - prev + kSortTile - 1) / kSortTile);
      prev = v;
    }
    s_tf[B] = tiles;
    s_bad = bad;
    sg->B = B;
    sg->n = s_start[B];
    sg->ntiles = tiles;
    sg->status = bad ? FGBD_ST_BAD_OFFSETS : 0;
    sg->sweep_barrier = 0u;
  }
  __syncthreads();
  if (t <= B) {
    sg->start[t] = s_start[t];
    sg->tile_first[t] = s_tf[t];
    const int64_t n = s_start[B];
#pragma unroll
    for (int g = 0; g < kNumGrids; ++g) {
      const int G = a.grid[g];
      sg->blk_first[g][t] = t == B ? G : (n > 0 ? (int32_t)((int64_t)s_start[t] * (G - B) / n) + t : t);
    }
  }
  if (t < B && res && a.zero_result) {
    fgbd_result *r = res + t;
    r->sigma_est = 0.0;
    r->sigma_g = 0.0;
    r->loss = 0.0;
    r->q = 0;
    r->n_fslr = 0;
    r->n_eff = 0;
    r->status = (s_bad ? FGBD_ST_BAD_OFFSETS : 0) | (a.zero_result == 2 ? FGBD_ST_NO_PATCH : 0);
    r->sweeps = 0;
    r->m = 0;
  }
}

__global__ __launch_bounds__(256) void k_setup(SetupArgs a) { setup_work(a, (int)blockIdx.x); }

// Per-tile digit counts.  Pass 0 makes the codes from the coordinates;
// later passes read only the byte array of this pass's digits that the
// previous downsweep wrote beside the items (16 digits per thread, one
// 16-byte load).  The counts go to 8 LDS sub-histograms picked by lane
// (rows 257 words apart), so lanes of one atomic instruction that share a
// digit, or a bank, mostly hit different words; the 8 are summed at the end.
__global__ __launch_bounds__(kSortThreads) void k_sort_upsweep(SortArgs a, const int32_t *__restrict__ xyz,
                                                               const uint8_t *__restrict__ digits,
                                                               uint32_t *__restrict__ hist) {
  constexpr int kSub = 8, kSubStride = 257;
  __shared__ uint32_t s_hs[kSub * kSubStride];
  if (a.fold) {  // the call's setup, by the first blocks (no other work of this launch reads it)
    const int lin = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (lin < a.su.blocks) setup_work(a.su, lin);
  }
  int d, tile;
  xcd_tile(d, tile);
  TileInfo ti;
  if (!tile_info(a, tile, ti)) return;  // uniform over the block
  const int t = threadIdx.x;
  for (int i = t; i < kSub * kSubStride; i += kSortThreads) s_hs[i] = 0;
  __syncthreads();
  uint32_t *s_h = s_hs + (lane_id() & (kSub - 1)) * kSubStride;
  if (a.pass == 0) {
    // every coordinate load of the thread is issued before the first count
    // (the LDS atomics would otherwise wait for each load in turn)
    const int wave = t / kWave;
    const int lane = (int)lane_id();
    const int base = ti.begin + wave * kWave * kSortItems + lane;
    int g[kSortItems][3];
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      const int pos = min(base + j * kWave, ti.end - 1);  // a tile holds at least one point
#pragma unroll
      for (int c = 0; c < 3; ++c) g[j][c] = xyz[3 * pos + c];
    }
    // Runs of equal digits are counted in registers and added once: with
    // the input in a raster order, the digit (low bits of the position
    // along the line) is often the same for a thread's items, and for every
    // lane of the wave, whose atomics on one word would serialise.
    const CodeGen cg = code_gen(a.dt, d);
    uint32_t run_digit = 0, run_count = 0;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      if (base + j * kWave < ti.end) {
        const uint32_t digit = gen_code(cg, g[j][0], g[j][1], g[j][2]) & 255u;
        if (run_count != 0 && digit != run_digit) {
          atomicAdd(&s_h[run_digit], run_count);
          run_count = 0;
        }
        run_digit = digit;
        ++run_count;
      }
    }
    if (run_count != 0) atomicAdd(&s_h[run_digit], run_count);
  } else {
    // tile starts are multiples of 16 inside the direction's row (clouds
    // start at any position, so only the bytes of the tile are counted)
    const uint8_t *row = digits + (size_t)d * a.stride;
    const int p0 = ti.begin + 16 * t;
    if (p0 + 16 <= ti.end && (p0 & 15) == 0) {
      const uint4 q = *reinterpret_cast<const uint4 *>(row + p0);
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
      // runs of equal digits among the 16 consecutive items add once
      uint32_t rd = w[0] & 255u, rc = 0;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const uint32_t dg = (w[j >> 2] >> (8 * (j & 3))) & 255u;
        if (dg != rd) {
          atomicAdd(&s_h[rd], rc);
          rc = 0;
        }
        rd = dg;
        ++rc;
      }
      atomicAdd(&s_h[rd], rc);
    } else {
      for (int j = 0; j < 16; ++j)
        if (p0 + j < ti.end) atomicAdd(&s_h[row[p0 + j]], 1u);
    }
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kSub; ++k) c += s_hs[k * kSubStride + t];
  hist[((size_t)d * a.row + tile) * 256 + t] = c;  // one 1 KB row per tile
}

// Exclusive prefix over tiles of every (direction, digit) count, and the
// total after the last tile (row ntiles).  The counts are stored tile-major,
// one row of BINS digits per tile, so every access is a contiguous row
// segment.  One block per (direction, 64 digits): lane = digit, the 16 waves
// split the tiles into 16 consecutive ranges; each wave sums its range with
// all loads of a chunk in flight, the waves' sums are scanned in LDS, and
// each wave writes its range's prefixes starting from the sums of the waves
// before it.
constexpr int kScanWaves = 16;
constexpr int kScanChunk = 16;  // tiles per wave per round trip
template <int BINS>
__global__ __launch_bounds__(kScanWaves * 64) void k_sort_scan(SortArgs a, uint32_t *__restrict__ hist) {
  __shared__ uint32_t s_sum[kScanWaves][kWave];
  constexpr int kGroups = BINS / kWave;
  const int d = blockIdx.x / kGroups;
  const int digit = (blockIdx.x % kGroups) * kWave + (int)lane_id();
  const int w = threadIdx.x / kWave;
  const int ntiles = num_tiles(a);
  const int per = (ntiles + kScanWaves - 1) / kScanWaves;
  const int t0 = w * per, t1 = min(t0 + per, ntiles);
  uint32_t *h = hist + (size_t)d * a.row * BINS + digit;  // h[tile * BINS]
  if (per <= kScanChunk) {  // (up to 256 tiles) one round trip: the counts stay in registers
    uint32_t v[kScanChunk];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) v[j] = t0 + j < t1 ? h[(size_t)(t0 + j) * BINS] : 0u;
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) sum += v[j];
    s_sum[w][lane_id()] = sum;
    __syncthreads();
    uint32_t run = 0, total = 0;
    for (int ww = 0; ww < kScanWaves; ++ww) {
      const uint32_t x = s_sum[ww][lane_id()];
      run += ww < w ? x : 0u;
      total += x;
    }
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      if (t0 + j < t1) h[(size_t)(t0 + j) * BINS] = run;
      run += v[j];
    }
    if (w == kScanWaves - 1) h[(size_t)ntiles * BINS] = total;
    return;
  }
  uint32_t sum = 0;
  for (int c0 = t0; c0 < t1; c0 += kScanChunk) {
    uint32_t v[kScanChunk];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) v[j] = c0 + j < t1 ? h[(size_t)(c0 + j) * BINS] : 0u;
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) sum += v[j];
  }
  s_sum[w][lane_id()] = sum;
  __syncthreads();
  uint32_t run = 0, total = 0;
  for (int ww = 0; ww < kScanWaves; ++ww) {
    const uint32_t x = s_sum[ww][lane_id()];
    run += ww < w ? x : 0u;
    total += x;
  }
  for (int c0 = t0; c0 < t1; c0 += kScanChunk) {
    uint32_t v[kScanChunk];
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) v[j] = c0 + j < t1 ? h[(size_t)(c0 + j) * BINS] : 0u;
#pragma unroll
    for (int j = 0; j < kScanChunk; ++j) {
      if (c0 + j < t1) h[(size_t)(c0 + j) * BINS] = run;
      run += v[j];
    }
  }
  if (w == kScanWaves - 1) h[(size_t)ntiles * BINS] = total;
}

// This pass's digit of an item (code << 32 | index).
__device__ __forceinline__ uint32_t digit_of(uint64_t item, int shift) {
  return __builtin_amdgcn_ubfe((uint32_t)(item >> 32), (uint32_t)shift, 8u);
}
// Bit b of x spread over the word: 0 or all ones.  Written out so the
// compiler keeps one sign-extending field extract instead of rebuilding the
// mask from compares.
__device__ __forceinline__ int32_t bit_mask(uint32_t x, int b) {
  int32_t m;
  asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(m) : "v"(x), "i"(b));
  return m;
}

// Exclusive scans of two uint32 per thread over a 256-thread block.
__device__ __forceinline__ void block_exclusive_scan2_256(uint32_t &v0, uint32_t &v1, uint32_t (*s_tmp)[4]) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x / kWave;
  uint32_t x0 = v0, x1 = v1;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y0 = __shfl_up(x0, o, kWave), y1 = __shfl_up(x1, o, kWave);
    if (lane >= (uint32_t)o) {
      x0 += y0;
      x1 += y1;
    }
  }
  if (lane == kWave - 1) {
    s_tmp[0][w] = x0;
    s_tmp[1][w] = x1;
  }
  __syncthreads();
  uint32_t b0 = 0, b1 = 0;
  for (int ww = 0; ww < w; ++ww) {
    b0 += s_tmp[0][ww];
    b1 += s_tmp[1][ww];
  }
  v0 = b0 + x0 - v0;
  v1 = b1 + x1 - v1;
}

__global__ __launch_bounds__(kSortThreads) void k_sort_downsweep(SortArgs a, const int32_t *__restrict__ xyz,
                                                                 const uint64_t *__restrict__ src,
                                                                 uint64_t *__restrict__ dst,
                                                                 const uint32_t *__restrict__ hist,
                                                                 uint8_t *__restrict__ digits,
                                                                 uint32_t *__restrict__ rank,
                                                                 fgbd_result *__restrict__ res) {
  __shared__ uint32_t s_wh[4][256];
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_tmp[2][4];
  __shared__ uint64_t s_stage[kSortTile];

  int d, tile;
  if (a.pass == a.passes - 1)
    xcd_tile_last(d, tile);
  else
    xcd_tile(d, tile);
  TileInfo ti;
  if (!tile_info(a, tile, ti)) return;  // uniform over the block
  const int t = threadIdx.x;
  const int wave = t / kWave;
  const int lane = (int)lane_id();
  const int valid = ti.end - ti.begin;

  s_wh[0][t] = 0;
  s_wh[1][t] = 0;
  s_wh[2][t] = 0;
  s_wh[3][t] = 0;
  // scanned counts of digit t: the cloud's count of t and this tile's offset
  // inside the cloud (the first cloud starts at column 0 with prefix 0)
  const uint32_t *hd = hist + (size_t)d * a.row * 256 + t;  // hd[tile * 256]: digit t of a tile row
  const uint32_t p_first = ti.first > 0 ? hd[(size_t)ti.first * 256] : 0u;
  uint32_t off_t = hd[(size_t)tile * 256] - p_first;
  uint32_t below_t = hd[(size_t)ti.next_first * 256] - p_first;  // becomes the exclusive prefix over digits

  uint64_t item[kSortItems];
  const CodeGen cg = code_gen(a.dt, d);
  const int base = ti.begin + wave * kWave * kSortItems + lane;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int pos = base + j * kWave;
    item[j] = (pos < ti.end) ? load_item(a, cg, xyz, src, d, pos, &bad) : ~0ull;
  }
  // pass 0: coordinates outside the grid (flagged once, by direction 0)
  if (bad && d == 0) atomicOr(&res[ti.s].status, FGBD_ST_COORD_RANGE);
  __syncthreads();

  // Stable rank of each item among the equal digits of its wave: items are
  // visited in tile order (j major, lane minor within the wave).  The lanes
  // holding the same digit (its peers) are those that agree with it on all 8
  // ballots: with m = bit b of the digit spread over the word (0 or all
  // ones), a lane keeps ~(vote ^ m).  Each round every lane reads the wave's
  // count of its digit over the earlier rounds, and the first lane of each
  // group of peers then adds the group's size to it.  A wave's LDS
  // operations are performed in the order they are issued, so the rounds
  // need no wait between them: the reads are waited for once, after the last
  // round, and each item's rank is that count plus its peers in lower lanes.
  uint32_t rk[kSortItems], before[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t digit = digit_of(item[j], a.shift);
    int32_t m[8];
    uint64_t vote[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      m[b] = bit_mask(digit, b);
      vote[b] = __builtin_amdgcn_ballot_w64(m[b] != 0);
    }
    uint32_t plo = ~0u, phi = ~0u;  // lanes that agree with this one in every bit
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      plo &= ~((uint32_t)vote[b] ^ (uint32_t)m[b]);
      phi &= ~((uint32_t)(vote[b] >> 32) ^ (uint32_t)m[b]);
    }
    const uint64_t peers = ((uint64_t)phi << 32) | plo;
    before[j] = count_below(peers);
    rk[j] = __hip_atomic_load(&s_wh[wave][digit], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (before[j] == 0)
      __hip_atomic_fetch_add(&s_wh[wave][digit], (uint32_t)__popcll(peers), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  }
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) rk[j] += before[j];
  __syncthreads();

  // per digit: exclusive over digits in the tile and (for the global
  // offset) over the cloud's digit totals; then each wave's start of the
  // digit in the staged tile (the tile's start of the digit plus the counts
  // of the waves before), and the global position of staged slot 0 of the
  // digit's run (its global offset minus its start in the tile, mod 2^32)
  {
    const uint32_t c0 = s_wh[0][t], c1 = s_wh[1][t], c2 = s_wh[2][t], c3 = s_wh[3][t];
    uint32_t in_tile = c0 + c1 + c2 + c3;
    block_exclusive_scan2_256(in_tile, below_t, s_tmp);
    s_wh[0][t] = in_tile;
    s_wh[1][t] = in_tile + c0;
    s_wh[2][t] = in_tile + c0 + c1;
    s_wh[3][t] = in_tile + c0 + c1 + c2;
    s_off[t] = (uint32_t)ti.seg_start + below_t + off_t - in_tile;
  }
  __syncthreads();

#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t digit = digit_of(item[j], a.shift);
    s_stage[s_wh[wave][digit] + rk[j]] = item[j];
  }
  __syncthreads();

  const bool last_pass = (a.pass == a.passes - 1);
  const bool wide = a.passes > kSortPasses;
  const bool rekey = wide && a.pass == kSortPasses - 1;  // the low 32 code bits are done
  uint64_t *out = dst + (size_t)d * a.stride;
  uint8_t *dig = digits + (size_t)d * a.stride;
  // Write-out in staged order: thread t takes slots t + 256 j, so each
  // store instruction of a wave covers 64 consecutive slots (runs of equal
  // digits go to consecutive global positions).  All slots' LDS reads are
  // issued before the first store (slots past the tile's items are read but
  // not stored).
  uint64_t st[kSortItems];
  uint32_t gp[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) st[j] = s_stage[t + j * kSortThreads];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) gp[j] = s_off[digit_of(st[j], a.shift)] + (uint32_t)(t + j * kSortThreads);
  if (last_pass) {
    // the sorted item keeps its index and carries the point's packed
    // coordinates instead of its code (the neighbour search's form); wide
    // codes keep the index only
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      if (t + j * kSortThreads < valid) {
        const uint32_t idx = (uint32_t)st[j];
        out[gp[j]] = wide ? (uint64_t)idx : ((uint64_t)decode_packed(cg, (uint32_t)(st[j] >> 32)) << 32) | idx;
        rank[(size_t)d * a.stride + idx] = gp[j];
      }
    }
  } else if (rekey) {
    // the item's key becomes the code's bits above 32
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      if (t + j * kSortThreads < valid) {
        const uint32_t idx = (uint32_t)st[j];
        const uint32_t hi =
            gen_code_hi(cg, xyz[3 * (size_t)idx + 0], xyz[3 * (size_t)idx + 1], xyz[3 * (size_t)idx + 2]);
        out[gp[j]] = ((uint64_t)hi << 32) | idx;
        dig[gp[j]] = (uint8_t)hi;  // the next pass's digit
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
      if (t + j * kSortThreads < valid) {
        out[gp[j]] = st[j];
        dig[gp[j]] = (uint8_t)(st[j] >> (40 + a.shift));  // the next pass's digit
      }
    }
  }
}


// ------------------------------------------------------------ hybrid sort
// Codes of at most 32 bits (grids up to 2^10) take a shorter route.  One
// pass on the kMsdBits most significant bits of each direction's code
// (upsweep, scan and downsweep as above, with 2^kMsdBits digits, the codes
// made from the coordinates) splits every cloud's points, stably, into
// buckets of equal top digit; the downsweep also records, from its counts,
// the first bucket start inside every window of kLocalWin sorted positions.
// k_local_sort then gives each window of a direction one block, which sorts
// the buckets that start in its window (the range from its recorded start
// to the next window's), stably, by their codes less the smallest top
// digit's base, with 8-bit LSD passes in LDS (three for the usual ranges).
// Buckets are ordered by their top digits already, so sorting a range by the
// whole code sorts each bucket and keeps the buckets in place; ties keep the
// MSD pass's order, which is the input's.  The final pass writes the sorted
// items in their final form and rank, as the last LSD pass does.  A range of
// more than kLocalCap items, of two clouds, or of keys wider than 26 bits is
// sorted by its block alone through the two item buffers: correct for any
// input, slow for a very large range (points crowded into few top digits,
// such as a plane normal to a scan axis), which the block then reports
// through a host-mapped flag so that the caller's context can choose the LSD
// passes for its next calls.

__device__ __forceinline__ int code_width(const DirTable &dt, int d) {
  const DirInfo di = dt.d[d];
  const uint32_t uh = (uint32_t)(di.uh < 0 ? -di.uh : di.uh);
  return 3 * dt.bits + (32 - __clz(uh)) + di.wm_extra;  // bit_length(0) = 0
}
__device__ __forceinline__ int msd_shift(const DirTable &dt, int d) {
  const int w = code_width(dt, d);
  return w > kMsdBits ? w - kMsdBits : 0;
}
// The top digit of a code (a field extract, so it stays below 2^kMsdBits
// even for the codes of coordinates outside the grid).
__device__ __forceinline__ uint32_t msd_digit(uint32_t code, int sh) {
  return __builtin_amdgcn_ubfe(code, (uint32_t)sh, (uint32_t)kMsdBits);
}

// Per-tile counts of the top digits, codes made from the coordinates (and
// the call's setup folded in, as in pass 0 of the LSD sort).
__global__ __launch_bounds__(kSortThreads) void k_msd_upsweep(SortArgs a, const int32_t *__restrict__ xyz,
                                                              uint32_t *__restrict__ hist) {
  constexpr int kSub = 4, kSubStride = kMsdBins + 1;
  __shared__ uint32_t s_hs[kSub * kSubStride];
  if (a.fold) {
    const int lin = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (lin < a.su.blocks) setup_work(a.su, lin);
  }
  int d, tile;
  xcd_tile(d, tile);
  // every (direction, window) entry of the window table starts empty; the
  // downsweep then writes each window's first bucket start (blocks and
  // windows pair up one to one: the grid has at least one tile per window)
  if (threadIdx.x == 0 && tile < a.nwin) a.win[(size_t)d * a.nwin + tile] = 0x7fffffff;
  TileInfo ti;
  if (!tile_info(a, tile, ti)) return;  // uniform over the block
  const int t = threadIdx.x;
  for (int i = t; i < kSub * kSubStride; i += kSortThreads) s_hs[i] = 0;
  __syncthreads();
  uint32_t *s_h = s_hs + (lane_id() & (kSub - 1)) * kSubStride;
  const int wave = t / kWave;
  const int lane = (int)lane_id();
  const int base = ti.begin + wave * kWave * kSortItems + lane;
  int g[kSortItems][3];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int pos = min(base + j * kWave, ti.end - 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) g[j][c] = xyz[3 * pos + c];
  }
  const CodeGen cg = code_gen(a.dt, d);
  const int sh = msd_shift(a.dt, d);
  uint32_t run_digit = 0, run_count = 0;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    if (base + j * kWave < ti.end) {
      const uint32_t digit = msd_digit(gen_code(cg, g[j][0], g[j][1], g[j][2]), sh);
      if (run_count != 0 && digit != run_digit) {
        atomicAdd(&s_h[run_digit], run_count);
        run_count = 0;
      }
      run_digit = digit;
      ++run_count;
    }
  }
  if (run_count != 0) atomicAdd(&s_h[run_digit], run_count);
  __syncthreads();
  uint32_t *row = hist + ((size_t)d * a.row + tile) * kMsdBins;
#pragma unroll
  for (int q = 0; q < kMsdBins / kSortThreads; ++q) {
    const int c = t + q * kSortThreads;
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < kSub; ++k) v += s_hs[k * kSubStride + c];
    row[c] = v;
  }
}

// The stable partition by top digit: the LSD downsweep's ranking with
// kMsdBits ballots, per-wave digit counts in LDS, staging in digit order and
// runs written to their offsets.  Items keep their code (code << 32 | index).
__global__ __launch_bounds__(kSortThreads) void k_msd_downsweep(SortArgs a, const int32_t *__restrict__ xyz,
                                                                uint64_t *__restrict__ dst,
                                                                const uint32_t *__restrict__ hist,
                                                                fgbd_result *__restrict__ res) {
  constexpr int kPer = kMsdBins / kSortThreads;  // digits per thread: kPer t .. kPer t + kPer - 1
  static_assert(kPer == 4, "one 16-byte count load per tile row and thread");
  __shared__ uint32_t s_wh[4][kMsdBins];
  __shared__ uint32_t s_off[kMsdBins];
  __shared__ uint32_t s_tmp[2][4];
  __shared__ uint64_t s_stage[kSortTile];

  int d, tile;
  xcd_tile(d, tile);
  TileInfo ti;
  if (!tile_info(a, tile, ti)) return;  // uniform over the block
  const int t = threadIdx.x;
  const int wave = t / kWave;
  const int lane = (int)lane_id();
  const int valid = ti.end - ti.begin;
  for (int i = t; i < 4 * kMsdBins; i += kSortThreads) (&s_wh[0][0])[i] = 0;
  // scanned counts of the thread's digits: the cloud's count and this tile's
  // offset inside the cloud
  const uint32_t *hd = hist + (size_t)d * a.row * kMsdBins + kPer * t;
  const uint4 pf = ti.first > 0 ? *reinterpret_cast<const uint4 *>(hd + (size_t)ti.first * kMsdBins)
                                : make_uint4(0u, 0u, 0u, 0u);
  const uint4 pt = *reinterpret_cast<const uint4 *>(hd + (size_t)tile * kMsdBins);
  const uint4 pn = *reinterpret_cast<const uint4 *>(hd + (size_t)ti.next_first * kMsdBins);
  const uint32_t off_q[kPer] = {pt.x - pf.x, pt.y - pf.y, pt.z - pf.z, pt.w - pf.w};
  const uint32_t below_q[kPer] = {pn.x - pf.x, pn.y - pf.y, pn.z - pf.z, pn.w - pf.w};

  uint64_t item[kSortItems];
  const CodeGen cg = code_gen(a.dt, d);
  const int sh = msd_shift(a.dt, d);
  const int base = ti.begin + wave * kWave * kSortItems + lane;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int pos = base + j * kWave;
    item[j] = (pos < ti.end) ? load_item(a, cg, xyz, nullptr, d, pos, &bad) : ~0ull;
  }
  if (bad && d == 0) atomicOr(&res[ti.s].status, FGBD_ST_COORD_RANGE);
  __syncthreads();

  // stable rank among the wave's equal digits (as in k_sort_downsweep);
  // items past the tile's end have the largest digit and come last
  uint32_t rk[kSortItems], before[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t digit = msd_digit((uint32_t)(item[j] >> 32), sh);
    int32_t m[kMsdBits];
    uint64_t vote[kMsdBits];
#pragma unroll
    for (int b = 0; b < kMsdBits; ++b) {
      m[b] = bit_mask(digit, b);
      vote[b] = __builtin_amdgcn_ballot_w64(m[b] != 0);
    }
    uint32_t plo = ~0u, phi = ~0u;
#pragma unroll
    for (int b = 0; b < kMsdBits; ++b) {
      plo &= ~((uint32_t)vote[b] ^ (uint32_t)m[b]);
      phi &= ~((uint32_t)(vote[b] >> 32) ^ (uint32_t)m[b]);
    }
    const uint64_t peers = ((uint64_t)phi << 32) | plo;
    before[j] = count_below(peers);
    rk[j] = __hip_atomic_load(&s_wh[wave][digit], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (before[j] == 0)
      __hip_atomic_fetch_add(&s_wh[wave][digit], (uint32_t)__popcll(peers), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  }
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) rk[j] += before[j];
  __syncthreads();

  // per digit: exclusive over the tile's digits and over the cloud's digit
  // totals (over the thread's kPer digits, then over the threads), each
  // wave's start of the digit in the staged tile, and the global position of
  // staged slot 0 of the digit's run
  {
    uint32_t c[4][kPer], ex_in[kPer], ex_below[kPer];
    uint32_t run_in = 0, run_below = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
#pragma unroll
      for (int w = 0; w < 4; ++w) c[w][q] = s_wh[w][kPer * t + q];
      ex_in[q] = run_in;
      run_in += c[0][q] + c[1][q] + c[2][q] + c[3][q];
      ex_below[q] = run_below;
      run_below += below_q[q];
    }
    block_exclusive_scan2_256(run_in, run_below, s_tmp);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const uint32_t e = run_in + ex_in[q];
      s_wh[0][kPer * t + q] = e;
      s_wh[1][kPer * t + q] = e + c[0][q];
      s_wh[2][kPer * t + q] = e + c[0][q] + c[1][q];
      s_wh[3][kPer * t + q] = e + c[0][q] + c[1][q] + c[2][q];
      s_off[kPer * t + q] = (uint32_t)ti.seg_start + run_below + ex_below[q] + off_q[q] - e;
    }
    // the cloud's first tile records where its buckets start: each window's
    // entry keeps the first start inside it
    if (tile == ti.first) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        if (below_q[q] > 0) {
          const int st = ti.seg_start + (int)(run_below + ex_below[q]);
          atomicMin(&a.win[(size_t)d * a.nwin + st / kLocalWin], st);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const uint32_t digit = msd_digit((uint32_t)(item[j] >> 32), sh);
    s_stage[s_wh[wave][digit] + rk[j]] = item[j];
  }
  __syncthreads();
  uint64_t *out = dst + (size_t)d * a.stride;
  uint64_t st[kSortItems];
  uint32_t gp[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) st[j] = s_stage[t + j * kSortThreads];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j)
    gp[j] = s_off[msd_digit((uint32_t)(st[j] >> 32), sh)] + (uint32_t)(t + j * kSortThreads);
  // (the offsets stay inside the direction's row for counts that agree
  // with the upsweep's; the bound only keeps a broken count from writing
  // outside it)
#pragma unroll
  for (int j = 0; j < kSortItems; ++j)
    if (t + j * kSortThreads < valid && gp[j] < (uint32_t)a.stride) out[gp[j]] = st[j];
}

constexpr int kLocalThreads = 512;
constexpr int kLocalWaves = kLocalThreads / kWave;
constexpr int kLocalItems = 16;                         // per thread, in-LDS ranges
constexpr int kLocalCap = kLocalThreads * kLocalItems;  // 8192 items
constexpr int kLocalKeyBits = 26;                       // wider relative keys take the slow path
constexpr int kSlowItems = 8;                           // per thread and chunk, slow path
static_assert(2 * kLocalThreads == kMsdBins, "two top digits per thread when the range is found");

struct LocalArgs {
  DirTable dt;
  SegArgs sa;
  int64_t stride;
  const int32_t *win;  // [L][nwin]: each window's first bucket start (0x7fffffff: none)
  int32_t nwin;
  int32_t *big;        // host-mapped flag set for a range of more than kBigRange items (NULL: none)
};

// Stable rank of an 8-bit digit among the wave's equal digits (the
// downsweep's ballot matching): returns the wave's count of the digit so far
// (an LDS read not yet waited for), sets `before` to the peers in lower
// lanes, and the first lane of each group of peers adds the group's size.
__device__ __forceinline__ uint32_t wave_rank8(uint32_t digit, uint32_t *cnt, uint32_t &before) {
  int32_t m[8];
  uint64_t vote[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    m[b] = bit_mask(digit, b);
    vote[b] = __builtin_amdgcn_ballot_w64(m[b] != 0);
  }
  uint32_t plo = ~0u, phi = ~0u;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    plo &= ~((uint32_t)vote[b] ^ (uint32_t)m[b]);
    phi &= ~((uint32_t)(vote[b] >> 32) ^ (uint32_t)m[b]);
  }
  const uint64_t peers = ((uint64_t)phi << 32) | plo;
  before = count_below(peers);
  const uint32_t r = __hip_atomic_load(&cnt[digit], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (before == 0)
    __hip_atomic_fetch_add(&cnt[digit], (uint32_t)__popcll(peers), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  return r;
}

// Exclusive prefix of v over the threads of the block (up to 16 waves);
// every thread calls it.  s_w: 16 words.
__device__ __forceinline__ uint32_t exclusive_scan_block(uint32_t v, uint32_t *s_w) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == kWave - 1) s_w[w] = x;
  __syncthreads();
  uint32_t b = 0;
  for (int ww = 0; ww < w; ++ww) b += s_w[ww];
  __syncthreads();  // s_w is free again when this returns
  return b + x - v;
}

// The cloud holding position x: the last cloud whose start is at most x.
__device__ __forceinline__ int cloud_at(const int32_t *starts, int B, int x) {
  int l = 0, h = B;  // starts[l] <= x; h == B or starts[h] > x
  while (h - l > 1) {
    const int m = (l + h) >> 1;
    if (starts[m] <= x)
      l = m;
    else
      h = m;
  }
  return l;
}

// One block per (direction, window of kLocalWin sorted positions).
__global__ __launch_bounds__(kLocalThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_local_sort(
    LocalArgs a, uint64_t *__restrict__ src, uint64_t *__restrict__ dst, uint32_t *__restrict__ rank) {
  __shared__ uint64_t s_it[kLocalCap];
  __shared__ uint32_t s_cnt[kLocalWaves][256];
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_w[16];
  __shared__ int32_t s_starts[kMaxSeg + 1];
  __shared__ int32_t s_multi;
  __shared__ unsigned long long s_max;

  // each XCD takes one contiguous range of the direction-major sequence
  int d, win;
  xcd_tile_last(d, win);
  const bool segmented = a.sa.n_fixed < 0;
  const int B = segmented ? a.sa.segs->B : 1;
  const int n_tot = segmented ? a.sa.segs->n : a.sa.n_fixed;
  const int w0 = win * kLocalWin;
  if (w0 >= n_tot) return;  // uniform over the block
  const int w1 = min(w0 + kLocalWin, n_tot);
  const int t = threadIdx.x;
  const int wave = t / kWave;
  const int lane = (int)lane_id();
  const size_t dbase = (size_t)d * a.stride;
  const uint64_t *items = src + dbase;
  const int sh = msd_shift(a.dt, d);

  // The range: buckets start at the cloud starts and, inside a cloud, where
  // the top digit changes.  The top-digit pass recorded each window's first
  // bucket start (from its counts, never from the items, which a
  // neighbouring block may be reordering): lo = this window's, hi = the
  // next one recorded after it (or the end).
  const int32_t *wrow = a.win + (size_t)d * a.nwin;
  const int lo = wrow[win];
  if (lo >= w1) return;  // no bucket starts in the window (uniform)
  int hi = n_tot;
  for (int k = win + 1; k < a.nwin; ++k) {  // uniform; nearly always one step
    const int v = wrow[k];
    if (v < n_tot) {
      hi = v;
      break;
    }
  }
  if (t == 0) {
    s_multi = 0;
    s_max = 0ull;
  }
  for (int i = t; i <= B; i += kLocalThreads) s_starts[i] = segmented ? a.sa.segs->start[i] : (i == 0 ? 0 : n_tot);
  for (int i = t; i < kLocalWaves * 256; i += kLocalThreads) (&s_cnt[0][0])[i] = 0u;  // the first pass's counts
  __syncthreads();
  for (int i = t; i <= B; i += kLocalThreads)
    if (s_starts[i] > lo && s_starts[i] < hi) s_multi = 1;
  __syncthreads();
  const bool multi = s_multi != 0;
  const int R = hi - lo;
  const uint32_t cf = (uint32_t)(items[lo] >> 32), cl = (uint32_t)(items[hi - 1] >> 32);
  const uint32_t df = msd_digit(cf, sh), dl = msd_digit(cl, sh);
  const uint32_t base = df << sh;
  const int bits = sh + (dl > df ? 32 - __clz(dl - df) : 0);
  const CodeGen cg = code_gen(a.dt, d);
  uint64_t *out = dst + dbase;

  if (!multi && R <= kLocalCap && bits <= kLocalKeyBits) {
    // ---- in LDS.  Slots: wave w holds range positions (w J + j) 64 + lane,
    // j < J, so the visiting order (wave, round, lane) is the range order.
    // The items move from pass to pass through s_it carrying the code less
    // the range's base (rel << 32 | index), so a pass's digit is one byte of
    // rel; slots past the range hold all ones, take the largest digit in
    // every pass and stay after every real item.
    const int passes = bits > 0 ? (bits + 7) / 8 : 1;  // (one pass of digit 0 copies)
    const int J = (R + kLocalThreads - 1) / kLocalThreads;  // <= kLocalItems
    uint64_t it[kLocalItems];
#pragma unroll
    for (int j = 0; j < kLocalItems; ++j) {
      const int s = (wave * J + j) * kWave + lane;
      const uint64_t v = items[lo + min(s, R - 1)];  // clamped: every load unconditional
      it[j] = (j < J && s < R) ? v - ((uint64_t)base << 32) : ~0ull;
    }
    for (int pass = 0; pass < passes; ++pass) {
      const bool last = pass == passes - 1;
      const uint32_t sft = 8u * (uint32_t)pass;
      auto digit = [&](uint64_t v) { return __builtin_amdgcn_ubfe((uint32_t)(v >> 32), sft, 8u); };
      uint32_t rk[kLocalItems], bf[kLocalItems];
#pragma unroll
      for (int j = 0; j < kLocalItems; ++j)
        if (j < J) rk[j] = wave_rank8(digit(it[j]), s_cnt[wave], bf[j]);  // (j < J is uniform)
#pragma unroll
      for (int j = 0; j < kLocalItems; ++j)
        if (j < J) rk[j] += bf[j];
      __syncthreads();
      // per digit t: the exclusive prefix over digits, then each wave's start
      // (column t is read twice rather than held in registers)
      uint32_t tot = 0;
      if (t < 256) {
#pragma unroll
        for (int w = 0; w < kLocalWaves; ++w) tot += s_cnt[w][t];
      }
      const uint32_t ex = exclusive_scan_block(tot, s_w);
      if (t < 256) {
        uint32_t run = ex;
#pragma unroll
        for (int w = 0; w < kLocalWaves; ++w) {
          const uint32_t c = s_cnt[w][t];
          s_cnt[w][t] = run;
          run += c;
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kLocalItems; ++j)
        if (j < J) s_it[s_cnt[wave][digit(it[j])] + rk[j]] = it[j];
      __syncthreads();
      if (!last) {
#pragma unroll
        for (int j = 0; j < kLocalItems; ++j)
          if (j < J) it[j] = s_it[(wave * J + j) * kWave + lane];
        for (int i = t; i < kLocalWaves * 256; i += kLocalThreads) (&s_cnt[0][0])[i] = 0u;
        __syncthreads();
      }
    }
    // write-out in sorted order, straight from LDS
    for (int i0 = 0; i0 * kLocalThreads < R; i0 += 4) {  // uniform
      uint64_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = s_it[min(t + (i0 + u) * kLocalThreads, R - 1)];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int s = t + (i0 + u) * kLocalThreads;
        const uint32_t idx = (uint32_t)v[u];
        if (s < R && idx < (uint32_t)a.stride) {  // (idx is a point of the range; the bound is a guard)
          out[lo + s] = ((uint64_t)decode_packed(cg, (uint32_t)(v[u] >> 32) + base) << 32) | idx;
          rank[dbase + idx] = (uint32_t)(lo + s);
        }
      }
    }
    return;
  }

  // ---- slow path: the block sorts its range alone, LSD over 8-bit digits of
  // the 64-bit key ((cloud - first cloud) << 32 | code) - base, in chunks of
  // kSlowItems * kLocalThreads items per round, through the two item buffers
  // (its own range of each).  An odd number of passes (a first pass of digit
  // 0, a plain stable copy, when needed) ends in dst, in the final form.
  if (a.big && R > kBigRange && t == 0) *a.big = 1;  // (only ever set to 1)
  const int c_first = cloud_at(s_starts, B, lo);
  const uint64_t base64 = (uint64_t)base;
  // the widest key of the range, for the pass count
  {
    unsigned long long mx = 0ull;
    for (int s = t; s < R; s += kLocalThreads) {
      const uint64_t it = items[lo + s];
      const int cr = multi ? cloud_at(s_starts, B, (int)(uint32_t)it) - c_first : 0;
      const uint64_t k64 = ((((uint64_t)cr) << 32) | (it >> 32)) - base64;
      mx = k64 > mx ? k64 : mx;
    }
    atomicMax(&s_max, mx);
  }
  __syncthreads();
  const unsigned long long kmax = s_max;
  int P = kmax ? (64 - __clzll(kmax) + 7) / 8 : 0;
  const int extra = (P % 2 == 0) ? 1 : 0;
  P += extra;
  for (int q = 0; q < P; ++q) {
    const uint64_t *rd = ((q & 1) == 0 ? src : dst) + dbase;
    uint64_t *wr = ((q & 1) == 0 ? dst : src) + dbase;
    const bool last = q == P - 1;
    const int shift = 8 * (q - extra);  // q < extra: the copy pass (digit 0)
    if (t < 256) s_base[t] = 0u;
    __syncthreads();
    for (int s = t; s < R; s += kLocalThreads) {
      const uint64_t it = rd[lo + s];
      const int cr = multi ? cloud_at(s_starts, B, (int)(uint32_t)it) - c_first : 0;
      const uint64_t k64 = ((((uint64_t)cr) << 32) | (it >> 32)) - base64;
      const uint32_t digit = q < extra ? 0u : (uint32_t)((k64 >> shift) & 255u);
      atomicAdd(&s_base[digit], 1u);
    }
    __syncthreads();
    const uint32_t hv = t < 256 ? s_base[t] : 0u;
    const uint32_t hex = exclusive_scan_block(hv, s_w);
    if (t < 256) s_base[t] = hex;
    __syncthreads();
    for (int c0 = 0; c0 < R; c0 += kSlowItems * kLocalThreads) {
      for (int i = t; i < kLocalWaves * 256; i += kLocalThreads) (&s_cnt[0][0])[i] = 0u;
      __syncthreads();
      uint64_t it[kSlowItems];
      uint32_t dg[kSlowItems], rk[kSlowItems], bf[kSlowItems];
#pragma unroll
      for (int j = 0; j < kSlowItems; ++j) {
        const int s = c0 + (wave * kSlowItems + j) * kWave + lane;
        it[j] = rd[lo + min(s, R - 1)];
      }
#pragma unroll
      for (int j = 0; j < kSlowItems; ++j) {
        const int s = c0 + (wave * kSlowItems + j) * kWave + lane;
        const int cr = multi ? cloud_at(s_starts, B, (int)(uint32_t)it[j]) - c_first : 0;
        const uint64_t k64 = ((((uint64_t)cr) << 32) | (it[j] >> 32)) - base64;
        dg[j] = s >= R ? 255u : (q < extra ? 0u : (uint32_t)((k64 >> shift) & 255u));
      }
#pragma unroll
      for (int j = 0; j < kSlowItems; ++j) rk[j] = wave_rank8(dg[j], s_cnt[wave], bf[j]);
#pragma unroll
      for (int j = 0; j < kSlowItems; ++j) rk[j] += bf[j];
      __syncthreads();
      uint32_t tot = 0;
      if (t < 256) {
        uint32_t run = s_base[t];
#pragma unroll
        for (int w = 0; w < kLocalWaves; ++w) {
          const uint32_t c = s_cnt[w][t];
          s_cnt[w][t] = run;
          run += c;
          tot += c;
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kSlowItems; ++j) {
        const int s = c0 + (wave * kSlowItems + j) * kWave + lane;
        const uint32_t dest = s_cnt[wave][dg[j]] + rk[j];
        if (s < R && dest < (uint32_t)R) {  // (dest < R for counts that agree; the bound is a guard)
          if (last) {
            const uint32_t idx = (uint32_t)it[j];
            wr[lo + dest] = ((uint64_t)decode_packed(cg, (uint32_t)(it[j] >> 32)) << 32) | idx;
            if (idx < (uint32_t)a.stride) rank[dbase + idx] = (uint32_t)(lo + dest);
          } else {
            wr[lo + dest] = it[j];
          }
        }
      }
      __syncthreads();
      if (t < 256) s_base[t] += tot;
    }
    __syncthreads();
  }
}

}  // namespace

SetupArgs setup_args(const Run &r, const int64_t *offsets, int64_t n_host, fgbd_result *res, int zero_result) {
  SetupArgs a;
  a.offsets = offsets;
  a.n_host = n_host;
  a.n_cap = r.pl.n_cap;
  a.B = r.pl.B;
  for (int g = 0; g < kNumGrids; ++g) a.grid[g] = r.pl.grid[g];
  a.zero_result = zero_result;
  a.sums_count = r.pl.B * kSweepSlots * kSweepParts;
  a.noise_count = r.pl.B * r.pl.E1 * kNoiseSlots;
  a.edge_count = r.pl.B * kEdgeSlots * kEdgeVals;
  const int most = 3 * a.sums_count > a.noise_count ? 3 * a.sums_count : a.noise_count;
  int blocks = (most + 256 * 8 - 1) / (256 * 8);
  a.blocks = blocks < 1 ? 1 : (blocks > 256 ? 256 : blocks);
  // the first sweep adds into sums buffer 1, the fused first launch into
  // buffers 2 (x_2) and 3 (x_1): buffers 1-3 start cleared (see launch_sweep)
  a.sums1 = r.b.sums + (size_t)a.sums_count;
  a.noise_acc = r.b.noise_acc;
  a.edge_acc = r.b.edge_acc;
  a.sg = r.b.segs;
  a.res = res;
  return a;
}

hipError_t launch_setup(const Run &r, const int64_t *offsets, int64_t n_host, fgbd_result *res, int zero_result) {
  const SetupArgs a = setup_args(r, offsets, n_host, res, zero_result);
  k_setup<<<a.blocks, 256, 0, r.stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_sort(const Run &r, const int32_t *xyz, fgbd_result *res, const uint64_t **sorted_out) {
  SortArgs a;
  a.win = nullptr;
  a.nwin = 0;
  a.dt = r.dt;
  a.sa = r.sa;
  a.stride = r.pl.stride;
  a.row = r.pl.ntiles_cap + 1;
  a.fold = 0;
  a.su = r.setup;
  const int ntiles = r.sa.n_fixed >= 0 ? (r.sa.n_fixed + kSortTile - 1) / kSortTile : r.pl.ntiles_cap;
  const dim3 grid(ntiles > 0 ? ntiles : 1, r.dt.num_dirs);
  if (r.dt.passes == kSortPasses && !r.sort_lsd) {
    // codes of at most 32 bits: the MSD pass, then the windows' local sorts
    const int64_t npos = r.sa.n_fixed >= 0 ? r.sa.n_fixed : r.pl.n_cap;
    a.nwin = (int)((npos + kLocalWin - 1) / kLocalWin);
    if (a.nwin < 1) a.nwin = 1;
    a.win = r.b.win;
    a.pass = 0;
    a.passes = 1;
    a.shift = 0;
    a.fold = r.fold_setup ? 1 : 0;
    if (a.fold && a.su.blocks > (int)(grid.x * grid.y)) a.su.blocks = (int)(grid.x * grid.y);
    FGBD_PRE(r.pf, kUpsweep);
    k_msd_upsweep<<<grid, kSortThreads, 0, r.stream>>>(a, xyz, r.b.hist);
    FGBD_POST(r.pf);
    FGBD_PRE(r.pf, kScan);
    k_sort_scan<kMsdBins><<<r.dt.num_dirs * (kMsdBins / kWave), kScanWaves * kWave, 0, r.stream>>>(a, r.b.hist);
    FGBD_POST(r.pf);
    FGBD_PRE(r.pf, kDownsweep);
    k_msd_downsweep<<<grid, kSortThreads, 0, r.stream>>>(a, xyz, r.b.items_a, r.b.hist, res);
    FGBD_POST(r.pf);
    LocalArgs la;
    la.dt = r.dt;
    la.sa = r.sa;
    la.stride = r.pl.stride;
    la.win = r.b.win;
    la.nwin = a.nwin;
    la.big = r.sort_big;
    FGBD_PRE(r.pf, kLocalSort);
    k_local_sort<<<dim3(a.nwin, r.dt.num_dirs), kLocalThreads, 0, r.stream>>>(la, r.b.items_a, r.b.items_b,
                                                                              r.b.rank);
    FGBD_POST(r.pf);
    if (r.sort_big && r.sort_ev) {
      if (hipEventRecord(r.sort_ev, r.stream) == hipSuccess)
        *r.sort_pending = true;
      else
        (void)hipGetLastError();
    }
    *sorted_out = r.b.items_b;
    return hipGetLastError();
  }
  const uint64_t *src = nullptr;
  uint64_t *bufs[2] = {r.b.items_a, r.b.items_b};
  a.passes = r.dt.passes;
  for (int pass = 0; pass < a.passes; ++pass) {
    a.pass = pass;
    a.shift = 8 * (pass % kSortPasses);
    uint64_t *dst = bufs[pass & 1];
    FGBD_PRE(r.pf, kUpsweep);
    a.fold = (pass == 0 && r.fold_setup) ? 1 : 0;
    if (a.fold && a.su.blocks > (int)(grid.x * grid.y)) a.su.blocks = (int)(grid.x * grid.y);  // clears are strided
    k_sort_upsweep<<<grid, kSortThreads, 0, r.stream>>>(a, xyz, r.b.digits, r.b.hist);
    FGBD_POST(r.pf);
    FGBD_PRE(r.pf, kScan);
    k_sort_scan<256><<<r.dt.num_dirs * 4, kScanWaves * kWave, 0, r.stream>>>(a, r.b.hist);
    FGBD_POST(r.pf);
    FGBD_PRE(r.pf, kDownsweep);
    k_sort_downsweep<<<grid, kSortThreads, 0, r.stream>>>(a, xyz, src, dst, r.b.hist, r.b.digits, r.b.rank, res);
    FGBD_POST(r.pf);
    src = dst;
  }
  *sorted_out = src;
  return hipGetLastError();
}

}  // namespace fgbd
