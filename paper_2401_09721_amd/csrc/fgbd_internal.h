// Internal declarations shared by the HIP translation units of libfgbd.
// Everything here is gfx950 (CDNA4, wave64) code; nothing is exported.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fgbd.h"

namespace fgbd {

constexpr int kWave = 64;
constexpr int kMaxDirs = 16;
constexpr int kMaxK = 32;
constexpr int kMaxD = kMaxK + 1;

// ---------------------------------------------------------------- directions
// A scan direction u (a primitive integer vector) is described by its position
// axis a (first axis with |u_a| = 1, u normalised to u_a = +1), the high and
// middle axes h = (a+2)%3, m = (a+1)%3 replaced by line invariants
// e_j = g_j - u_j g_a + max(u_j,0)(2^b-1), and the bit width of e_m.
// The code is ((e_h << wm) + e_m) << b | g_a; d0..d2 are eqs. 1-3.
struct DirInfo {
  int8_t a, h, m, uh, um, wm_extra, pad0, pad1;  // wm = bits + wm_extra
};
struct DirTable {
  DirInfo d[kMaxDirs];
  int32_t bits;
  int32_t num_dirs;
  int32_t code_bits;  // widest code of the table's first num_dirs directions
  int32_t passes;     // radix passes of 8 bits: 4 for codes of up to 32 bits, 4 + more for the bits above
};
// Codes wider than 32 bits (bits > 10): items carry 32 code bits at a time.
constexpr int kMaxCodeBits = 63;
void make_dir_table(int bits, int num_dirs, DirTable *t);

__device__ __forceinline__ uint32_t scan_code(int gx, int gy, int gz, const DirInfo &di, int bits) {
  const int g[3] = {gx, gy, gz};
  const uint32_t top = (1u << bits) - 1u;
  const int ga = g[di.a];
  const uint32_t eh = (uint32_t)(g[di.h] - di.uh * ga) + (di.uh > 0 ? (uint32_t)di.uh * top : 0u);
  const uint32_t em = (uint32_t)(g[di.m] - di.um * ga) + (di.um > 0 ? (uint32_t)di.um * top : 0u);
  const int wm = bits + di.wm_extra;
  return (((eh << wm) + em) << bits) | (uint32_t)ga;
}

__device__ __forceinline__ void scan_decode(uint32_t code, const DirInfo &di, int bits, int g[3]) {
  const uint32_t top = (1u << bits) - 1u;
  const int wm = bits + di.wm_extra;
  const int ga = (int)(code & top);
  const int em = (int)((code >> bits) & ((1u << wm) - 1u));
  const int eh = (int)(code >> (bits + wm));
  g[di.a] = ga;
  g[di.h] = eh + di.uh * ga - (di.uh > 0 ? di.uh * (int)top : 0);
  g[di.m] = em + di.um * ga - (di.um > 0 ? di.um * (int)top : 0);
}

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
// number of set bits of m below this lane
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Fixed-order block reduction of NV doubles per thread (blockDim.x == 256).
// Result valid in thread 0.  s_buf: >= 256 * NV doubles of LDS... uses a
// wave shuffle tree then a 4-entry combine, so the order never changes.
template <int NV>
__device__ __forceinline__ void block_sum_f64(double (&v)[NV], double *s_buf) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] += __shfl_down(v[j], o, kWave);
  }
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) s_buf[w * NV + j] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double acc = s_buf[j];
      for (int ww = 1; ww < nw; ++ww) acc += s_buf[ww * NV + j];
      v[j] = acc;
    }
  }
  __syncthreads();
}

// Exclusive scan of one uint32 per thread over a 256-thread block; also
// returns the block total.  s_tmp: 4 uint32 of LDS.
__device__ __forceinline__ uint32_t block_exclusive_scan_256(uint32_t v, uint32_t *s_tmp, uint32_t *total) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == kWave - 1) s_tmp[w] = x;
  __syncthreads();
  uint32_t base = 0;
  for (int ww = 0; ww < w; ++ww) base += s_tmp[ww];
  uint32_t tot = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// Exclusive scan of one uint32 per thread over a block of blockDim.x threads
// (a multiple of 64, at most 1024).  s_tmp: 16 uint32 of LDS.  Returns the
// exclusive prefix; *total receives the block total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp, uint32_t *total) {
  const uint32_t lane = lane_id();
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(x, o, kWave);
    if (lane >= (uint32_t)o) x += y;
  }
  if (lane == kWave - 1) s_tmp[w] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int ww = 0; ww < nw; ++ww) {
    const uint32_t c = s_tmp[ww];
    base += ww < w ? c : 0u;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// ------------------------------------------------------------- segments
// A call covers B clouds stored back to back; cloud s owns the points
// start[s] .. start[s+1]-1, and in every direction's sorted order it owns the
// same positions.  A setup kernel writes the table from device offsets, so a
// captured launch sequence serves any cloud sizes up to the planned capacity.
// Every block of a per-cloud grid works on one cloud only: cloud s gets blocks
// blk_first[g][s] .. blk_first[g][s+1]-1 (at least one, the rest in proportion
// to its size), and radix tiles never straddle two clouds.
constexpr int kMaxSeg = 64;
enum GridKind { kGridMerge = 0, kGridNoise = 1, kGridSweep = 2, kNumGrids = 3 };
struct Segs {
  int32_t B;
  int32_t n;       // start[B]
  int32_t ntiles;  // radix tiles in use
  int32_t status;  // FGBD_ST_BAD_OFFSETS when the offsets had to be clamped
  uint32_t sweep_barrier;  // arrival counter of the in-launch sweep loop (0 at setup)
  uint32_t pad_[3];
  int32_t start[kMaxSeg + 1];
  int32_t tile_first[kMaxSeg + 1];
  int32_t blk_first[kNumGrids][kMaxSeg + 1];
  // Per cloud: set by the relabel launch when more than a quarter of the
  // kept edges are far (the merge's counts in the edge-length sums); 0 at
  // setup.
  int32_t relabel[kMaxSeg];
};
// An edge is far when its points are more than a sixteenth of the cloud, and
// more than 4096 points, apart in the input numbering (a raster order keeps
// the neighbours of a 1M-point frame within a few thousand indices).
__host__ __device__ inline int64_t far_gap(int64_t cloud_n) {
  return cloud_n / 16 > 4096 ? cloud_n / 16 : 4096;
}

// How kernels find their cloud: n_fixed >= 0 means one cloud of n_fixed
// points known on the host (the table is not read); otherwise B clouds from
// the device table.
struct SegArgs {
  const Segs *segs;
  int32_t B;
  int32_t n_fixed;
};

// Largest s < B with first[s] <= x, for a non-decreasing table with
// first[0] = 0 (one load per lane and a ballot; all 64 lanes must be active).
__device__ __forceinline__ int seg_lookup(const int32_t *first, int B, int x) {
  if (B <= 1) return 0;
  const int l = (int)lane_id();
  const bool c = l >= 1 && l < B && first[l] <= x;
  return (int)__popcll(__builtin_amdgcn_ballot_w64(c));
}

struct SegBlock {
  int s;              // cloud
  int64_t begin, end; // its points
  int lb, nb;         // this block's index among the cloud's blocks, and their count
};
__device__ __forceinline__ SegBlock seg_block(const SegArgs &a, int grid) {
  SegBlock r;
  if (a.n_fixed >= 0) {
    r.s = 0;
    r.begin = 0;
    r.end = a.n_fixed;
    r.lb = blockIdx.x;
    r.nb = gridDim.x;
    return r;
  }
  const Segs *sg = a.segs;
  const int s = seg_lookup(sg->blk_first[grid], a.B, (int)blockIdx.x);
  r.s = s;
  r.begin = sg->start[s];
  r.end = sg->start[s + 1];
  const int f0 = sg->blk_first[grid][s];
  r.lb = (int)blockIdx.x - f0;
  r.nb = sg->blk_first[grid][s + 1] - f0;
  return r;
}

// XCD-aware work split for grid-stride kernels.  Workgroups are dispatched to
// the 8 XCDs round-robin by block index, and each XCD has its own L2; giving
// each XCD one contiguous share of a cloud's points keeps the neighbour
// gathers of spatially ordered clouds inside one L2.  The cloud's blocks are
// consecutive, so local block b works on share b % 8 (all blocks of one share
// sit on one XCD), as block b / 8 of the blocks of that share.
constexpr int kXcds = 8;
struct Share {
  int64_t begin, end;  // points of this block's XCD share
  int64_t first;       // first chunk start for this block
  int64_t step;        // chunk stride
};
__device__ __forceinline__ Share seg_share(const SegBlock &sb, int chunk) {
  const int nx = sb.nb < kXcds ? sb.nb : kXcds;
  const int x = sb.lb % nx;
  const int nbx = (sb.nb - x + nx - 1) / nx;
  const int lb = sb.lb / nx;
  const int64_t len = sb.end - sb.begin;
  Share s;
  s.begin = sb.begin + len * x / nx;
  s.end = sb.begin + len * (x + 1) / nx;
  s.first = s.begin + (int64_t)lb * chunk;
  s.step = (int64_t)nbx * chunk;
  return s;
}

// ------------------------------------------------------------ edge weights
// Eq. 4 on the integer squared distances of a CSR row: w_k = exp(-(d_k -
// d_0) / sigma_g^2) over the valid slots (d_0 is the nearest neighbour's, so
// the largest term is exactly 1 and nothing underflows), normalised to sum 1
// and rounded to float32.  The graph builder stores these weights; the fused
// per-frame path recomputes them inside the filter sweeps from the same code,
// so both obtain the same bits.  Gaps are integers: exp of the small ones
// comes from a table in LDS.
constexpr int kExpTable = 256;

// Edge lengths for sigma_g: every merge block adds its FP64 sum of edge
// lengths into integers of its cloud as the integer part and the fraction in
// units of 2^-40, and its edge count (exact integer sums in any order; each
// block's sum is rounded by at most 2^-41).  Blocks spread their atomics over
// kEdgeSlots slots (block index mod kEdgeSlots): thousands of blocks adding
// into one word serialise.
// integer part, fraction * 2^40, count, and the count of far edges (two
// points more than far_gap(cloud size) apart in the input numbering)
constexpr int kEdgeVals = 4;
constexpr int kEdgeSlots = 64;
constexpr double kEdgeFrac = 1099511627776.0;  // 2^40

// sigma_g of one cloud: the fixed value when positive, else the mean merge
// edge length from the cloud's edge sums (acc: its [kEdgeSlots][kEdgeVals]
// integers; the first wave adds the slots).  Called by every thread of the
// block; s_u: kEdgeVals integers of LDS.
__device__ __forceinline__ double cloud_sigma_g(const unsigned long long *__restrict__ acc, double fixed,
                                                unsigned long long *s_u) {
  if (fixed > 0.0) return fixed;
  static_assert(kEdgeSlots == kWave, "one slot per lane");
  if (threadIdx.x < kWave) {
    unsigned long long v[kEdgeVals];
#pragma unroll
    for (int j = 0; j < kEdgeVals; ++j) v[j] = acc[threadIdx.x * kEdgeVals + j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
      for (int j = 0; j < kEdgeVals; ++j) v[j] += __shfl_xor(v[j], o, kWave);
    }
    if (threadIdx.x < kEdgeVals) s_u[threadIdx.x] = v[threadIdx.x];
  }
  __syncthreads();
  const unsigned long long cnt = s_u[2];
  const double total = (double)s_u[0] + (double)s_u[1] / kEdgeFrac;
  __syncthreads();  // s_u may be reused
  return cnt > 0 ? total / (double)cnt : 0.0;
}

// Fills s_exp[g] = exp(-g / sigma_g^2); the caller synchronises the block.
__device__ __forceinline__ void fill_exp_table(double sg, double *s_exp) {
  const double inv = sg > 0.0 ? 1.0 / (sg * sg) : 0.0;
  for (int g = threadIdx.x; g < kExpTable; g += blockDim.x)
    s_exp[g] = sg > 0.0 ? exp(-(double)g * inv) : (g == 0 ? 1.0 : 0.0);
}

template <int KB>
__device__ __forceinline__ void row_weights(const int (&cv)[KB], const int (&dv)[KB], double sg,
                                            const double *s_exp, float (&pw)[KB]) {
  const double inv = sg > 0.0 ? 1.0 / (sg * sg) : 0.0;
  double w[KB];
  double s = 0.0;
  const int d0 = dv[0];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    w[k] = 0.0;
    if (cv[k] >= 0) {
      const int gap = dv[k] - d0;
      w[k] = gap < kExpTable ? s_exp[gap] : (sg > 0.0 ? exp(-(double)gap * inv) : 0.0);
      s += w[k];
    }
  }
  const double rs = s > 0.0 ? 1.0 / s : 0.0;
#pragma unroll
  for (int k = 0; k < KB; ++k) pw[k] = (float)(w[k] * rs);
}

// ---------------------------------------------------------------- control
// Selection state of the filter sweeps, kept in the workspace.
struct SweepCtrl {
  double sigma_est;
  double target;     // sigma_est^2
  double y2_sel;     // sum over the FSLR subset of |y|^2
  double best_loss;
  double last_energy;
  double sigma_g;    // of the cloud, when the sweeps compute the weights themselves
  int32_t n_sel;     // |S| (all points when FSLR is off or S is empty)
  int32_t use_all;
  int32_t q;         // sweeps completed
  int32_t best_q;
  int32_t in_buf;    // buffer holding x_q (3 = caller input)
  int32_t best_buf;  // buffer holding x_{best_q}
  int32_t done;
  int32_t select;    // 1: eq. 6 selection, 0: fixed q
  int32_t q_limit;   // q_max (select) or q_fixed
  int32_t fslr;      // FSLR subset in use (select and kappa > 0)
  int32_t first_pending;  // stored by the fused first launch: the sums of x_1 (in the fourth
                          // sums buffer) are still to be applied before those of x_2
  int32_t pad_;
};
// No implicit padding: a copy of the struct then splits into its fields and
// stays in registers (padding bytes inside a 16-byte chunk made the compiler
// keep the chunk in memory, which it placed in LDS at 16 bytes per thread).
static_assert(sizeof(SweepCtrl) == 6 * 8 + 12 * 4, "SweepCtrl has no implicit padding");


// ----------------------------------------------------------- workspace plan
// Capacity of a call: up to n_cap points in B clouds.  Grids and buffers are
// sized from the capacity; kernels take the actual sizes from SegArgs.
struct Plan {
  int64_t n_cap;
  int64_t stride;            // per-direction length of the sort items and ranks (n_cap rounded up to 64)
  int32_t B, L, K, P, D, TP;
  int32_t ntiles_cap;        // radix tiles: ceil(n_cap / tile) + B - 1
  int32_t grid[kNumGrids];   // blocks of the per-cloud grids (each >= B)
  int32_t E1;                // 1 + D(D+1)/2 + 3D: patch count and moment entries
  size_t off_segs, off_items_a, off_items_b, off_hist, off_rank, off_digits, off_win;
  size_t off_col, off_dist2, off_p, off_spread, off_xbuf, off_rgbw, off_colw, off_dist2w;
  size_t off_edge_acc, off_noise_acc, off_ctrl, off_sweep_sums;
  size_t total;
};

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys per tile
constexpr int kSortPasses = 4;                        // 8-bit digits of 32-bit codes
// codes of at most 32 bits: one pass on the top kMsdBits bits, then local sorts
constexpr int kMsdBits = 10;
constexpr int kMsdBins = 1 << kMsdBits;
constexpr int kLocalWin = kSortTile;  // sorted positions per local-sort window
// a range this large sorted by one block makes later eager calls on the
// context sort by LSD passes for kSortLsdCalls calls
constexpr int kBigRange = 32768;
constexpr int kSortLsdCalls = 32;

constexpr int kBlock = 256;
constexpr int kMaxGrid = 1024;  // default grid cap of the grid-stride kernels
constexpr int kGridCapMin = 64;
constexpr int kGridCapMax = 4096;       // merge and sweep grids
constexpr int kNoiseGridCapMax = 1024;  // the noise solve reduces at most this many partials per cloud
constexpr int kSweepParts = 5;  // energy sums per sweep
constexpr int kSweepSlots = 64;  // atomic slots per cloud and sum (spread to limit contention)
constexpr int kSweepMaxGrid = 1024;
// Patch moments of the noise estimate: every block adds its FP64 partial sums,
// rounded to multiples of 1 / kNoiseFix, into int64 accumulators (slot = the
// block's index in its cloud mod kNoiseSlots; slot-major, so one block's
// entries are contiguous), so the totals are exact sums of the rounded
// partials in any order.
constexpr int kNoiseSlots = 64;
constexpr double kNoiseFix = 4096.0;
constexpr int kScanThreads = 1024;

// Largest grid (blocks) of each per-cloud grid kind, and the number of
// filter sweeps enqueued as launches of their own (the rest run in one
// cooperative launch); chosen by the autotuner.
struct Tune {
  int32_t cap[kNumGrids];
  int32_t sweep_launches;
};
constexpr int kDefaultSweepLaunches = 8;
constexpr int kMaxSweepLaunches = 1024;
constexpr int kDefaultMergeGrid = 4096;  // the merge gains from more blocks than the other kernels
constexpr int kDefaultSweepGrid = 512;  // fewer, longer-running sweep blocks: less block start and sum traffic
constexpr Tune kDefaultTune = {{kDefaultMergeGrid, kMaxGrid, kDefaultSweepGrid}, kDefaultSweepLaunches};

Plan make_plan(int64_t n_cap, int B, const fgbd_params &p, const Tune &tune = kDefaultTune);

// Workspace views of a plan.
struct Bufs {
  Segs *segs;
  uint64_t *items_a, *items_b;  // [L][n_cap]
  uint32_t *hist;               // [L][ntiles_cap + 1][256]
  uint32_t *rank;               // [L][stride]
  uint8_t *digits;              // [L][stride]: the next radix pass's digit of each sorted item
  int32_t *win;                 // [L][windows]: the first bucket start in each local-sort window
  int32_t *col, *dist2;         // [n_cap][K]
  float *p;                     // [n_cap][K] weights the fused path's first sweep stores
  double *spread;               // [n_cap]
  float4 *xbuf;                 // [3][n_cap]
  // a relabelled cloud's graph and colours in scan-order-0 numbering
  float *rgb_w;                 // [n_cap][3]
  int32_t *col_w, *dist2_w;     // [n_cap][K]
  unsigned long long *edge_acc;  // [B][kEdgeSlots][kEdgeVals] edge-length sums for sigma_g
  unsigned long long *noise_acc;  // [B][kNoiseSlots][E1] fixed-point patch moments
  SweepCtrl *ctrl;              // [2][B]
  unsigned long long *sums;     // [3][B][slots][parts]
};
Bufs carve(char *ws, const Plan &pl);

// ------------------------------------------------------------- profiling
enum Kind {
  kUpsweep = 0, kScan, kDownsweep, kMerge, kWeights, kNoise, kNoiseSolve, kSweep, kFinalize, kRelabel, kLocalSort,
  kNumKinds
};
static_assert(kNumKinds == FGBD_NUM_KERNELS, "one profiling slot per kernel kind");
// Optional per-launch timing hook (events around each launch).
struct Prof {
  virtual void pre(int kind) = 0;
  virtual void post() = 0;
  virtual ~Prof() {}
};
#define FGBD_PRE(pf, kind) \
  do {                     \
    if (pf) (pf)->pre(kind); \
  } while (0)
#define FGBD_POST(pf)  \
  do {                 \
    if (pf) (pf)->post(); \
  } while (0)

// ------------------------------------------------------------- launchers
// Everything one call's launches need.  All launchers enqueue on r.stream
// and return hipSuccess or the launch error.
// The per-call setup: the segment table from device offsets (B + 1 entries)
// or from one host-known size, the clears of the first sweep's sums and of
// the moment and edge accumulators, and optionally zeroed results.
struct SetupArgs {
  const int64_t *offsets;  // device, B + 1 entries, or NULL
  int64_t n_host;          // the one cloud's size when offsets is NULL
  int64_t n_cap;
  int32_t B;
  int32_t grid[kNumGrids];
  int32_t zero_result;  // 0 leave res, 1 zero res[0..B-1], 2 zero and flag FGBD_ST_NO_PATCH
  int32_t sums_count;   // sweep sums of one buffer (uint64); buffers 1-3 are cleared
  int32_t noise_count;  // noise moment accumulators to clear (uint64)
  int32_t edge_count;   // edge-length sums to clear (uint64)
  int32_t blocks;       // blocks that share the clears
  unsigned long long *sums1, *noise_acc, *edge_acc;
  Segs *sg;
  fgbd_result *res;
};

struct Run {
  Plan pl;
  Bufs b;
  SegArgs sa;
  DirTable dt;
  fgbd_params prm;
  hipStream_t stream;
  Prof *pf;
  int32_t sweep_launches;  // sweeps enqueued as launches of their own
  // the per-frame path may relabel points into scan order 0 when the input's
  // point order is incoherent (not for graphs handed to the caller, nor for
  // index-ordered patches)
  bool relabel_ok = false;
  int32_t *hint = nullptr;  // host-mapped: the finalising launch stores each cloud's sweep count here
  // Sort route for codes of at most 32 bits: the top-digit pass and local
  // sorts unless sort_lsd.  sort_big (host-mapped, NULL: not watched): the
  // local sort sets it when a block had to sort a range of more than
  // kBigRange items alone; sort_ev is recorded after the sort, and
  // *sort_pending marks the read-back outstanding.
  bool sort_lsd = false;
  int32_t *sort_big = nullptr;
  hipEvent_t sort_ev = nullptr;
  bool *sort_pending = nullptr;
  // bound of each wait between sweeps in the in-launch sweep loop, in
  // microseconds (negative: half a second)
  int64_t wait_us = -1;
  // set: the first radix launch also does the call's setup (one cloud of
  // host-known size; saves a launch)
  bool fold_setup = false;
  SetupArgs setup;
};

// Segment table from device offsets (B+1 entries) or, with offsets == NULL,
// one cloud of n_host points; clears the first sweep's sums.  zero_result: 0 leave res, 1 zero res[0..B-1], 2 zero and flag
// FGBD_ST_NO_PATCH.
hipError_t launch_setup(const Run &r, const int64_t *offsets, int64_t n_host, fgbd_result *res, int zero_result);
SetupArgs setup_args(const Run &r, const int64_t *offsets, int64_t n_host, fgbd_result *res, int zero_result);

hipError_t launch_sort(const Run &r, const int32_t *xyz, fgbd_result *res, const uint64_t **sorted_out);

// With r.relabel_ok the merge also counts each cloud's far edges.
// xyz: the input coordinates (read by the selection for codes above 32 bits);
// res: FGBD_ST_DIST_CLAMPED is set there when a kept squared distance does not
// fit int32.
hipError_t launch_merge(const Run &r, const int32_t *xyz, const uint64_t *sorted, int32_t *col, int32_t *dist2,
                        fgbd_result *res);

// Relabelling (only when r.relabel_ok): for every cloud whose kept edges are
// mostly far apart in the input numbering, the graph (col, dist2) and the
// colours rgb renumbered along scan order 0 into r.b.col_w, dist2_w, rgb_w,
// and the cloud's relabel flag set; other clouds are left as they are.
hipError_t launch_relabel(const Run &r, const uint64_t *sorted, const int32_t *col, const int32_t *dist2,
                          const float *rgb);

// sigma_g of each cloud (the fixed value or the mean merge edge length, into
// res[s].sigma_g) and the row-normalised weights p.
hipError_t launch_weights(const Run &r, const int32_t *col, const int32_t *dist2, fgbd_result *res, float *p);

// fuse_res != NULL (K = P = 8, no eig3): the launch also derives sigma_g (into
// fuse_res) and the weights p, and writes the first filter sweep's colours
// into the first iterate buffer (see launch_sweep's pre).
hipError_t launch_noise(const Run &r, const int32_t *col, const float *rgb, double *spread, float *eig3,
                        fgbd_result *fuse_res);

// One block per cloud: sigma_est, n_eff, m and the NO_PATCH flag into res[s].
hipError_t launch_noise_solve(const Run &r, fgbd_result *res);

// Sweep number q (1-based): reads ctrl[(q-1)&1][.] and sums[(q-1)%3], writes
// ctrl[q&1][.] and sums[q%3], clears sums[(q+1)%3].  noise: per-cloud
// results holding sigma_est (select == 1).  dist2 != NULL (first sweep only):
// the weights come from the squared distances and res[s].sigma_g and are
// stored into p (which is then an output).  pre (first sweep only, K = 8):
// the noise launch already wrote the sweep's colours into the first iterate
// buffer; this launch adds the FSLR flags and the sums.
hipError_t launch_sweep(const Run &r, const int32_t *col, const float *p, const int32_t *dist2,
                        const float *rgb_in, const double *spread, const fgbd_result *noise, fgbd_result *res,
                        int select, int q_limit, int q, bool pre = false, bool merged = false);

// Whether the sweep grid of r fits on the current device at once, as the
// in-launch sweep loop below needs.
bool sweep_tail_fits(const Run &r);

// Sweeps q0..q_last in one launch whose blocks wait for each other between
// sweeps, after separate launches of sweeps 1..q0-1 (same arguments as
// launch_sweep), then the work of launch_finalize; skips the sweeps when
// every cloud's selection was done at the start of sweep q0-1.  Uses the
// segment table's barrier counter (zeroed by the setup launch of the call).
hipError_t launch_sweep_tail(const Run &r, const int32_t *col, const float *p, const float *rgb_in,
                             const double *spread, const fgbd_result *noise, fgbd_result *res, int select,
                             int q_limit, int q0, int q_last, float *rgb_out);

// r.hint != NULL: block 0 of each cloud also stores its sweep count there.
hipError_t launch_finalize(const Run &r, const float *rgb_in, int q_launches, const fgbd_result *noise,
                           float *rgb_out, fgbd_result *res);

// Polynomial filter and its adjoint (ws: at least poly_workspace bytes).
constexpr int kMaxPoly = 32;
// grid cap of the polynomial filter's grid-stride kernels; also the length
// of each of their per-block partial-sum rows
constexpr int kPolyGrid = 1024;
size_t poly_workspace(int64_t n, int k, int ncoef, int nblocks);
// floats of the saved buffer of a polynomial filter call
size_t poly_saved_floats(int64_t n, int k, int ncoef);
// Float coordinates onto the 2^bits grid (keys: 6 words of scratch) and
// colours to uint8 (fgbd_io.hip).
hipError_t launch_quantize(const float *xyz, int64_t n, int32_t bits, int32_t *out, double *frame, uint32_t *keys,
                           hipStream_t st);
hipError_t launch_round_u8(const float *x, int64_t m, uint8_t *out, hipStream_t st);
hipError_t launch_coords_f32(const int32_t *g, int64_t m, float *out, hipStream_t st);
hipError_t launch_poly_forward(int64_t n, int k, const int32_t *col, const int32_t *dist2, const float *x,
                               const float *coef, int ncoef, const double *sigma_g, float *out, float *saved,
                               char *ws, hipStream_t s);
hipError_t launch_poly_backward(int64_t n, int k, const int32_t *col, const int32_t *dist2, const int32_t *t_off,
                                const int32_t *t_edge, const float *saved, const float *coef, int ncoef,
                                const double *sigma_g, const float *grad_out, float *grad_x, float *grad_coef,
                                double *grad_sigma, char *ws, hipStream_t s);
// Transpose of a graph's directed edges (off: [n + 1], edge: [n * k]); ws:
// at least transpose_workspace(n) bytes.
size_t transpose_workspace(int64_t n);
hipError_t launch_transpose(int64_t n, int k, const int32_t *col, int32_t *off, int32_t *edge, char *ws,
                            hipStream_t s);

}  // namespace fgbd
