// Host side of the C ABI (include/fgbd.h): argument validation, workspace
// planning, and the order of launches for each call.  No call blocks the
// host; every launch goes to the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "fgbd_internal.h"

using namespace fgbd;

namespace {

thread_local char g_err[512] = "";

fgbd_status fail(fgbd_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

fgbd_status ok() {
  g_err[0] = '\0';
  return FGBD_OK;
}

// The direction table: d0..d2 are the raster codes of eqs. 1-3; the rest are
// diagonal scan lines.  Each entry is a primitive integer vector.
const int kDirVec[kMaxDirs][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0}, {0, 1, 1}, {0, 1, -1}, {1, 0, 1},
    {1, 0, -1}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}, {1, 2, 0}, {0, 1, 2}, {2, 0, 1},
};

int bit_length(int v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

struct Record {
  int kind;
  hipEvent_t a, b;
};

}  // namespace

struct fgbd_ctx_s {
  int device = 0;
  void *own = nullptr;
  size_t own_bytes = 0;
  void *user = nullptr;
  size_t user_bytes = 0;
  bool profile = false;
  Tune tune = kDefaultTune;
  std::vector<hipEvent_t> pool;
  std::vector<Record> pending;
  double ms[FGBD_NUM_KERNELS] = {0};
  int64_t launches[FGBD_NUM_KERNELS] = {0};
  // Sweep counts of recent eager calls, read back without waiting: the last
  // finalising launch stores each cloud's count into host-mapped memory and
  // an event marks it; a later call reads it once the event has completed.
  int32_t *hint_host = nullptr;  // [kMaxSeg], hipHostMalloc'ed
  int32_t *hint_dev = nullptr;   // its device address
  hipEvent_t hint_ev = nullptr;
  bool hint_failed = false;      // could not set up: no adaptation
  bool hint_pending = false;
  int hint_B = 0;
  int hint_recent[8] = {0};      // ring of the last counts read (max over clouds)
  int hint_count = 0;
  // Sort route: a host-mapped flag the local sort sets when a block sorted a
  // very large range alone (points crowded into few top code digits, such as
  // a plane normal to a scan axis), read back without waiting like the sweep
  // counts; while sort_lsd_left > 0, eager calls sort by LSD passes.
  int32_t *sort_flag_host = nullptr;
  int32_t *sort_flag_dev = nullptr;
  hipEvent_t sort_ev = nullptr;
  bool sort_failed = false;
  bool sort_pending = false;
  int sort_lsd_left = 0;
  int64_t wait_us = -1;  // fgbd_set_sweep_wait
};

namespace fgbd {

void make_dir_table(int bits, int num_dirs, DirTable *t) {
  memset(t, 0, sizeof(*t));
  t->bits = bits;
  t->num_dirs = num_dirs;
  for (int d = 0; d < num_dirs; ++d) {
    int u[3] = {kDirVec[d][0], kDirVec[d][1], kDirVec[d][2]};
    int a = 0;
    while (abs(u[a]) != 1) ++a;
    if (u[a] < 0)
      for (int j = 0; j < 3; ++j) u[j] = -u[j];
    const int h = (a + 2) % 3, m = (a + 1) % 3;
    DirInfo &di = t->d[d];
    di.a = (int8_t)a;
    di.h = (int8_t)h;
    di.m = (int8_t)m;
    di.uh = (int8_t)u[h];
    di.um = (int8_t)u[m];
    di.wm_extra = (int8_t)bit_length(abs(u[m]));
    // code = ((e_h << B_m) + e_m) << b | g_a with e_j of b + bit_length(|u_j|) bits
    const int width = (bits + bit_length(abs(u[h]))) + (bits + di.wm_extra) + bits;
    t->code_bits = width > t->code_bits ? width : t->code_bits;
  }
  t->passes = t->code_bits <= 32 ? 4 : 4 + (t->code_bits - 32 + 7) / 8;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Plan make_plan(int64_t n_cap, int B, const fgbd_params &p, const Tune &tune) {
  Plan pl;
  memset(&pl, 0, sizeof(pl));
  pl.n_cap = n_cap;
  pl.stride = ((n_cap > 0 ? n_cap : 1) + 63) / 64 * 64;  // keeps every direction's items 512-byte aligned
  pl.B = B;
  pl.L = p.num_dirs;
  pl.K = p.k;
  pl.P = p.patch > 0 ? p.patch : p.k;
  pl.D = pl.P + 1;
  pl.TP = pl.D <= 17 ? 256 : 128;
  // tiles never straddle clouds: sum over clouds of ceil(n_s / tile) is at
  // most ceil(n / tile) + B - 1
  const int64_t tiles = (n_cap + kSortTile - 1) / kSortTile + B - 1;
  pl.ntiles_cap = (int32_t)(tiles < 1 ? 1 : tiles);
  auto grid_for = [&](int64_t units, int cap) {
    int64_t g = units < 1 ? 1 : (units < cap ? units : cap);
    return (int32_t)(g < B ? B : g);
  };
  pl.grid[kGridMerge] = grid_for((n_cap + kBlock - 1) / kBlock, tune.cap[kGridMerge]);
  pl.grid[kGridSweep] = grid_for((n_cap + kBlock - 1) / kBlock, tune.cap[kGridSweep]);
  pl.grid[kGridNoise] = grid_for((n_cap + pl.TP - 1) / pl.TP, tune.cap[kGridNoise]);
  pl.E1 = 1 + pl.D * (pl.D + 1) / 2 + 3 * pl.D;
  const size_t N = (size_t)(n_cap > 0 ? n_cap : 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  pl.off_segs = take(sizeof(Segs));
  pl.off_items_a = take((size_t)pl.L * pl.stride * 8);
  pl.off_items_b = take((size_t)pl.L * pl.stride * 8);
  pl.off_hist = take((size_t)pl.L * (pl.ntiles_cap + 1) * kMsdBins * 4);  // 256 digits per tile row in LSD passes
  pl.off_rank = take((size_t)pl.L * pl.stride * 4);
  pl.off_digits = take((size_t)pl.L * pl.stride);
  pl.off_win = take((size_t)pl.L * ((N + kLocalWin - 1) / kLocalWin) * 4);
  pl.off_col = take(N * pl.K * 4);
  pl.off_dist2 = take(N * pl.K * 4);
  pl.off_p = take(N * pl.K * 4);
  pl.off_spread = take(N * 8);
  pl.off_xbuf = take(3 * N * 16);
  pl.off_rgbw = take(N * 12);
  pl.off_colw = take(N * pl.K * 4);
  pl.off_dist2w = take(N * pl.K * 4);
  pl.off_edge_acc = take((size_t)B * kEdgeSlots * kEdgeVals * 8);
  pl.off_noise_acc = take((size_t)B * pl.E1 * kNoiseSlots * 8);
  pl.off_ctrl = take((size_t)2 * B * sizeof(SweepCtrl));
  pl.off_sweep_sums = take((size_t)4 * B * kSweepSlots * kSweepParts * 8);  // 3 rotating + the fused first launch's
  pl.total = off;
  return pl;
}

Bufs carve(char *ws, const Plan &pl) {
  Bufs b;
  b.segs = (Segs *)(ws + pl.off_segs);
  b.items_a = (uint64_t *)(ws + pl.off_items_a);
  b.items_b = (uint64_t *)(ws + pl.off_items_b);
  b.hist = (uint32_t *)(ws + pl.off_hist);
  b.rank = (uint32_t *)(ws + pl.off_rank);
  b.digits = (uint8_t *)(ws + pl.off_digits);
  b.win = (int32_t *)(ws + pl.off_win);
  b.col = (int32_t *)(ws + pl.off_col);
  b.dist2 = (int32_t *)(ws + pl.off_dist2);
  b.p = (float *)(ws + pl.off_p);
  b.spread = (double *)(ws + pl.off_spread);
  b.xbuf = (float4 *)(ws + pl.off_xbuf);
  b.rgb_w = (float *)(ws + pl.off_rgbw);
  b.col_w = (int32_t *)(ws + pl.off_colw);
  b.dist2_w = (int32_t *)(ws + pl.off_dist2w);
  b.edge_acc = (unsigned long long *)(ws + pl.off_edge_acc);
  b.noise_acc = (unsigned long long *)(ws + pl.off_noise_acc);
  b.ctrl = (SweepCtrl *)(ws + pl.off_ctrl);
  b.sums = (unsigned long long *)(ws + pl.off_sweep_sums);
  return b;
}

}  // namespace fgbd

namespace {

fgbd_status check_params(const fgbd_params *p) {
  if (!p) return fail(FGBD_E_INVALID, "params is NULL");
  if (p->bits < 1) return fail(FGBD_E_INVALID, "bits must be >= 1 (got %d)", p->bits);
  if (p->bits > 21) return fail(FGBD_E_UNSUPPORTED, "bits above 21 are not supported (got %d)", p->bits);
  if (p->num_dirs < 1 || p->num_dirs > kMaxDirs)
    return fail(FGBD_E_INVALID, "num_dirs must be in 1..%d (got %d)", kMaxDirs, p->num_dirs);
  if (p->window < 1 || p->window > 64) return fail(FGBD_E_INVALID, "window must be in 1..64 (got %d)", p->window);
  if (p->k < 1 || p->k > kMaxK) return fail(FGBD_E_INVALID, "k must be in 1..%d (got %d)", kMaxK, p->k);
  if (p->patch < 0 || p->patch > p->k)
    return fail(FGBD_E_INVALID, "patch must be in 0..k (got %d with k=%d)", p->patch, p->k);
  if (p->q_max < 0 || p->q_max > 1024) return fail(FGBD_E_INVALID, "q_max must be in 0..1024 (got %d)", p->q_max);
  if (!isfinite(p->fslr_kappa)) return fail(FGBD_E_INVALID, "fslr_kappa must be finite");
  if (!isfinite(p->sigma_g)) return fail(FGBD_E_INVALID, "sigma_g must be finite");
  if (p->patch_order != 0 && p->patch_order != 1)
    return fail(FGBD_E_INVALID, "patch_order must be 0 or 1 (got %d)", p->patch_order);
  DirTable dt;
  make_dir_table(p->bits, p->num_dirs, &dt);
  if (dt.code_bits > kMaxCodeBits)
    return fail(FGBD_E_UNSUPPORTED, "bits %d with %d directions needs %d-bit scan codes (at most %d)", p->bits,
                p->num_dirs, dt.code_bits, kMaxCodeBits);
  return FGBD_OK;
}

fgbd_status check_n(int64_t n) {
  if (n < 0) return fail(FGBD_E_INVALID, "n must be >= 0 (got %lld)", (long long)n);
  if (n > (int64_t)0x7fffffff - kSortTile) return fail(FGBD_E_INVALID, "n too large (got %lld)", (long long)n);
  return FGBD_OK;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa < pb + nb && pb < pa + na;
}

struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) {
      err = hipSetDevice(dev);
      changed = err == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

fgbd_status hip_fail(hipError_t e, const char *what) {
  return fail(FGBD_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

fgbd_status get_workspace(fgbd_ctx ctx, size_t need, char **ws) {
  if (ctx->user) {
    if (ctx->user_bytes < need)
      return fail(FGBD_E_WORKSPACE, "workspace has %zu bytes, call needs %zu", ctx->user_bytes, need);
    *ws = (char *)ctx->user;
    return FGBD_OK;
  }
  if (ctx->own_bytes < need) {
    if (ctx->own) {
      hipError_t e = hipDeviceSynchronize();  // the old buffer may still be in use
      if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
      (void)hipFree(ctx->own);
      ctx->own = nullptr;
      ctx->own_bytes = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) return fail(FGBD_E_NOMEM, "hipMalloc(%zu) failed: %s", need, hipGetErrorString(e));
    ctx->own = p;
    ctx->own_bytes = need;
  }
  *ws = (char *)ctx->own;
  return FGBD_OK;
}

// ------------------------------------------------------------ profiling
// Records an event pair around every launch when the context has profiling on.
struct EventProf final : Prof {
  fgbd_ctx ctx;
  hipStream_t stream;
  int kind = -1;
  hipEvent_t a = nullptr;
  EventProf(fgbd_ctx c, hipStream_t s) : ctx(c), stream(s) {}
  hipEvent_t take() {
    if (ctx->pool.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  void pre(int k) override {
    kind = k;
    a = take();
    if (a) (void)hipEventRecord(a, stream);
  }
  void post() override {
    if (kind < 0 || !a) return;
    hipEvent_t b = take();
    if (b) {
      (void)hipEventRecord(b, stream);
      ctx->pending.push_back(Record{kind, a, b});
    }
    kind = -1;
    a = nullptr;
  }
};

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Waits for the recorded event pairs and adds their times per kernel kind.
fgbd_status drain(fgbd_ctx ctx, double *ms, int64_t *launches) {
  for (auto &r : ctx->pending) {
    HIP_TRY(hipEventSynchronize(r.b), "hipEventSynchronize");
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, r.a, r.b), "hipEventElapsedTime");
    ms[r.kind] += t;
    launches[r.kind] += 1;
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->pending.clear();
  return FGBD_OK;
}

Run make_run(fgbd_ctx ctx, const Plan &pl, char *ws, const fgbd_params &prm, int64_t n_fixed, hipStream_t s,
             Prof *pf) {
  Run r;
  r.pl = pl;
  r.b = carve(ws, pl);
  r.sa.segs = r.b.segs;
  r.sa.B = pl.B;
  r.sa.n_fixed = (int32_t)n_fixed;
  make_dir_table(prm.bits, prm.num_dirs, &r.dt);
  r.prm = prm;
  r.stream = s;
  r.pf = ctx->profile ? pf : nullptr;
  r.sweep_launches = ctx->tune.sweep_launches;
  r.wait_us = ctx->wait_us;
  return r;
}

// The sort route of an eager call (captured calls keep the top-digit sort and
// watch nothing).  A completed read-back that found a very large range sorted
// by one block switches the context to LSD passes for kSortLsdCalls calls;
// otherwise, with no read-back outstanding, the call arms the flag.
static void sort_policy(fgbd_ctx ctx, hipStream_t s, Run &r) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (ctx->sort_failed) return;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  if (cs != hipStreamCaptureStatusNone) return;
  if (!ctx->sort_flag_host) {
    void *dev = nullptr;
    if (hipHostMalloc((void **)&ctx->sort_flag_host, sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer(&dev, ctx->sort_flag_host, 0) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->sort_ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      ctx->sort_failed = true;
      return;
    }
    ctx->sort_flag_dev = (int32_t *)dev;
  }
  if (ctx->sort_pending) {
    const hipError_t q = hipEventQuery(ctx->sort_ev);
    if (q == hipSuccess) {
      if (*(volatile int32_t *)ctx->sort_flag_host) ctx->sort_lsd_left = kSortLsdCalls;
      ctx->sort_pending = false;
    } else if (q != hipErrorNotReady) {
      (void)hipGetLastError();
      ctx->sort_failed = true;
      return;
    }
  }
  if (ctx->sort_lsd_left > 0) {
    r.sort_lsd = true;
    --ctx->sort_lsd_left;
    return;
  }
  if (!ctx->sort_pending) {
    *(volatile int32_t *)ctx->sort_flag_host = 0;
    r.sort_big = ctx->sort_flag_dev;
    r.sort_ev = ctx->sort_ev;
    r.sort_pending = &ctx->sort_pending;
  }
}

// Graph construction into (col, dist2, p); sigma_g into res.  p == NULL
// stops after the merge: the sweeps then derive sigma_g and the weights.
fgbd_status run_slg(const Run &r, const int32_t *xyz, int32_t *col, int32_t *dist2, float *p, fgbd_result *res,
                    const float *rgb = nullptr) {
  const uint64_t *sorted = nullptr;
  HIP_TRY(launch_sort(r, xyz, res, &sorted), "radix sort launch");
  FGBD_PRE(r.pf, kMerge);
  HIP_TRY(launch_merge(r, xyz, sorted, col, dist2, res), "neighbour merge launch");
  FGBD_POST(r.pf);
  if (rgb && r.relabel_ok) {  // the per-frame path: renumber clouds whose input order is not spatial
    FGBD_PRE(r.pf, kRelabel);
    HIP_TRY(launch_relabel(r, sorted, col, dist2, rgb), "relabel launch");
    FGBD_POST(r.pf);
  }
  if (p == nullptr) return FGBD_OK;
  FGBD_PRE(r.pf, kWeights);
  HIP_TRY(launch_weights(r, col, dist2, res, p), "weights launch");
  FGBD_POST(r.pf);
  return FGBD_OK;
}

// fuse: the noise launch also computes the weights and the first sweep's
// colours (the fused per-frame path, K = P = 8).
fgbd_status run_noise(const Run &r, const int32_t *col, const float *rgb, double *spread, float *eig3,
                      fgbd_result *res, bool fuse = false) {
  FGBD_PRE(r.pf, kNoise);
  HIP_TRY(launch_noise(r, col, rgb, spread, eig3, fuse ? res : nullptr), "noise launch");
  FGBD_POST(r.pf);
  FGBD_PRE(r.pf, kNoiseSolve);
  HIP_TRY(launch_noise_solve(r, res), "noise solve launch");
  FGBD_POST(r.pf);
  return FGBD_OK;
}

// Sweeps and the final copy.  The first sweep's sums buffer was cleared by
// the call's setup launch.  With dist2 given, the first sweep derives sigma_g
// (into res) and the weights from the squared distances and stores the
// weights into p, which the later sweeps read.
fgbd_status run_filter(const Run &r, const int32_t *col, const float *p, const int32_t *dist2, const float *rgb_in,
                       const double *spread, const fgbd_result *noise, int select, int q_limit, float *rgb_out,
                       fgbd_result *res, bool pre = false) {
  const int sweeps = q_limit > 0 ? q_limit : 1;
  // with fixed q every sweep computes: all of them are separate launches
  const int separate = (!select || sweeps < r.sweep_launches) ? sweeps : r.sweep_launches;
  // The fused path with selection and at least two separate sweeps starts
  // with one launch for sweeps 1 and 2 (x_1 came from the noise launch).
  const bool merged = pre && select && separate >= 2 && r.prm.k == 8;
  for (int q = merged ? 2 : 1; q <= separate; ++q) {
    FGBD_PRE(r.pf, kSweep);
    HIP_TRY(launch_sweep(r, col, p, q == 1 ? dist2 : nullptr, rgb_in, spread, noise, res, select, q_limit, q,
                         pre && q == 1, merged && q == 2),
            "sweep launch");
    FGBD_POST(r.pf);
  }
  bool tail = separate < sweeps && sweep_tail_fits(r);
  if (tail) {  // the loop launch also finalises
    FGBD_PRE(r.pf, kSweep);
    const hipError_t e =
        launch_sweep_tail(r, col, p, rgb_in, spread, noise, res, select, q_limit, separate + 1, sweeps, rgb_out);
    FGBD_POST(r.pf);
    HIP_TRY(e, "sweep loop launch");
    return FGBD_OK;
  }
  for (int q = tail ? sweeps + 1 : separate + 1; q <= sweeps; ++q) {
    FGBD_PRE(r.pf, kSweep);
    HIP_TRY(launch_sweep(r, col, p, nullptr, rgb_in, spread, noise, res, select, q_limit, q), "sweep launch");
    FGBD_POST(r.pf);
  }
  FGBD_PRE(r.pf, kFinalize);
  HIP_TRY(launch_finalize(r, rgb_in, sweeps, noise, rgb_out, res), "finalize launch");
  FGBD_POST(r.pf);
  return FGBD_OK;
}

// ------------------------------------------------ no-allocation variant
// Scratch of fgbd_estimate_noise_noalloc: one fixed array in the library,
// one copy per GPU at that GPU's own address, held until the process ends.
// In host code the name `scratch` is only a stand-in for the symbol, not a
// device address: it is never passed to a kernel or a copy.  The device
// address comes from hipGetSymbolAddress, taken once per device with that
// device current, and kept in g_scratch_dev.
constexpr size_t kNoAllocBytes = FGBD_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) static unsigned char scratch[kNoAllocBytes];
constexpr int kNoAllocDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_dev[kNoAllocDevices] = {};

// The device address of this GPU's scratch array (the caller has made the
// device current).
fgbd_status scratch_address(int device, char **out) {
  if (device < 0 || device >= kNoAllocDevices)
    return fail(FGBD_E_UNSUPPORTED, "device %d: the no-allocation calls cover devices 0..%d", device,
                kNoAllocDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(FGBD_E_HIP, "scratch array has no aligned device address");
    g_scratch_dev[device] = (char *)ptr;
  }
  *out = g_scratch_dev[device];
  return FGBD_OK;
}

// The buffers the noise estimate uses (segment table, edge-length and moment
// accumulators, the sweep sums the setup launch clears) packed from offset 0;
// every other buffer of the plan is absent.
Plan noise_scratch_plan(int64_t n, const fgbd_params &p, const Tune &tune) {
  Plan pl = make_plan(n, 1, p, tune);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  pl.off_segs = take(sizeof(Segs));
  pl.off_edge_acc = take((size_t)pl.B * kEdgeSlots * kEdgeVals * 8);
  pl.off_noise_acc = take((size_t)pl.B * pl.E1 * kNoiseSlots * 8);
  pl.off_ctrl = take((size_t)2 * pl.B * sizeof(SweepCtrl));
  pl.off_sweep_sums = take((size_t)4 * pl.B * kSweepSlots * kSweepParts * 8);
  pl.total = off;
  return pl;
}

// Argument checks of fgbd_estimate_noise (shared by its no-allocation variant).
fgbd_status check_estimate_noise(fgbd_ctx ctx, const fgbd_graph *g, const float *rgb, const fgbd_params *params,
                                 const fgbd_result *res) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  fgbd_status st = check_params(params);
  if (st != FGBD_OK) return st;
  if (!g) return fail(FGBD_E_INVALID, "graph is NULL");
  if ((st = check_n(g->n)) != FGBD_OK) return st;
  if (g->k != params->k) return fail(FGBD_E_INVALID, "graph k (%d) != params k (%d)", g->k, params->k);
  if (!res) return fail(FGBD_E_INVALID, "res is NULL");
  if (g->n > 0 && (!rgb || !g->col)) return fail(FGBD_E_INVALID, "NULL colour or graph array");
  return FGBD_OK;
}

// The launches of fgbd_estimate_noise on a prepared run: the setup launch
// (segment table, cleared moment accumulators), the patch statistics and the
// noise solve.  spread: where the FSLR spreads go (never NULL).
fgbd_status run_estimate_noise(const Run &r, const fgbd_graph *g, const float *rgb, fgbd_result *res, double *spread,
                               float *eig3) {
  const int64_t n = g->n;
  if (n == 0) {
    HIP_TRY(launch_setup(r, nullptr, 0, res, 2), "setup launch");
    return ok();
  }
  // one cloud of host-known size: the kernels do not read the segment table;
  // the setup launch clears the moment accumulators
  HIP_TRY(launch_setup(r, nullptr, n, nullptr, 0), "setup launch");
  const fgbd_status st = run_noise(r, g->col, rgb, spread, eig3, res);
  return st != FGBD_OK ? st : ok();
}

}  // namespace

extern "C" {

int32_t fgbd_abi_version(void) { return FGBD_ABI_VERSION; }

const char *fgbd_last_error(void) { return g_err; }

fgbd_status fgbd_default_params(fgbd_params *p) {
  if (!p) return fail(FGBD_E_INVALID, "params is NULL");
  p->bits = 10;
  p->num_dirs = 8;
  p->window = 4;
  p->k = 8;
  p->patch = 0;
  p->q_max = 32;
  p->fslr_kappa = 2.0;
  p->sigma_g = 0.0;
  p->patch_order = 0;
  p->pad_ = 0;
  return ok();
}

fgbd_status fgbd_create(fgbd_ctx *out, int32_t hip_device) {
  if (!out) return fail(FGBD_E_INVALID, "out is NULL");
  if (hip_device < 0) return fail(FGBD_E_INVALID, "hip_device must be >= 0");
  fgbd_ctx c = new (std::nothrow) fgbd_ctx_s();
  if (!c) return fail(FGBD_E_NOMEM, "host allocation failed");
  c->device = hip_device;
  *out = c;
  return ok();
}

fgbd_status fgbd_destroy(fgbd_ctx ctx) {
  if (!ctx) return ok();
  if (ctx->own || !ctx->pool.empty() || !ctx->pending.empty() || ctx->hint_host || ctx->hint_ev ||
      ctx->sort_flag_host || ctx->sort_ev) {
    DeviceGuard g(ctx->device);
    if (ctx->hint_ev) {
      (void)hipEventSynchronize(ctx->hint_ev);
      (void)hipEventDestroy(ctx->hint_ev);
    }
    if (ctx->hint_host) (void)hipHostFree(ctx->hint_host);
    if (ctx->sort_ev) {
      (void)hipEventSynchronize(ctx->sort_ev);
      (void)hipEventDestroy(ctx->sort_ev);
    }
    if (ctx->sort_flag_host) (void)hipHostFree(ctx->sort_flag_host);
    if (ctx->own) {
      (void)hipDeviceSynchronize();
      (void)hipFree(ctx->own);
    }
    for (auto &r : ctx->pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
  }
  delete ctx;
  return ok();
}

fgbd_status fgbd_workspace_size(const fgbd_params *p, int64_t n_max, int32_t batch, size_t *bytes) {
  fgbd_status st = check_params(p);
  if (st != FGBD_OK) return st;
  if ((st = check_n(n_max)) != FGBD_OK) return st;
  if (batch < 1 || batch > kMaxSeg) return fail(FGBD_E_INVALID, "batch must be in 1..%d (got %d)", kMaxSeg, batch);
  if (!bytes) return fail(FGBD_E_INVALID, "bytes is NULL");
  // sized for the largest schedule, so any later fgbd_set_schedule fits
  const Tune widest = {{kGridCapMax, kNoiseGridCapMax, kGridCapMax}, kDefaultSweepLaunches};
  const size_t a = make_plan(n_max, batch, *p, widest).total;
  const size_t b = poly_workspace(n_max, p->k, kMaxPoly, kPolyGrid);
  *bytes = a > b ? a : b;
  return ok();
}

fgbd_status fgbd_set_workspace(fgbd_ctx ctx, void *dev, size_t bytes) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  if ((dev == nullptr) != (bytes == 0)) return fail(FGBD_E_INVALID, "dev and bytes must both be set or both zero");
  if (((uintptr_t)dev & 255) != 0) return fail(FGBD_E_INVALID, "workspace must be 256-byte aligned");
  ctx->user = dev;
  ctx->user_bytes = bytes;
  return ok();
}

fgbd_status fgbd_build_slg(fgbd_ctx ctx, const int32_t *xyz, int64_t n, const fgbd_params *params,
                           const fgbd_graph *g, fgbd_result *res, void *stream) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  fgbd_status st = check_params(params);
  if (st != FGBD_OK) return st;
  if ((st = check_n(n)) != FGBD_OK) return st;
  if (!g) return fail(FGBD_E_INVALID, "graph is NULL");
  if (g->n != n || g->k != params->k) return fail(FGBD_E_INVALID, "graph shape (%lld, %d) != (n, k)", (long long)g->n, g->k);
  if (!res) return fail(FGBD_E_INVALID, "res is NULL");
  if (n > 0 && (!xyz || !g->col || !g->dist2 || !g->p)) return fail(FGBD_E_INVALID, "NULL input or graph array");
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  const Plan pl = make_plan(n, 1, *params, ctx->tune);
  char *ws = nullptr;
  if ((st = get_workspace(ctx, pl.total, &ws)) != FGBD_OK) return st;
  EventProf ep(ctx, s);
  Run r = make_run(ctx, pl, ws, *params, n, s, &ep);
  sort_policy(ctx, s, r);
  HIP_TRY(launch_setup(r, nullptr, n, res, 1), "setup launch");
  if (n == 0) return ok();
  if ((st = run_slg(r, xyz, g->col, g->dist2, g->p, res)) != FGBD_OK) return st;
  return ok();
}

fgbd_status fgbd_estimate_noise(fgbd_ctx ctx, const fgbd_graph *g, const float *rgb, const fgbd_params *params,
                                fgbd_result *res, double *patch_spread, float *eig3, void *stream) {
  fgbd_status st = check_estimate_noise(ctx, g, rgb, params, res);
  if (st != FGBD_OK) return st;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  const Plan pl = make_plan(g->n, 1, *params, ctx->tune);
  char *ws = nullptr;
  if ((st = get_workspace(ctx, pl.total, &ws)) != FGBD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  EventProf ep(ctx, s);
  const Run r = make_run(ctx, pl, ws, *params, g->n, s, &ep);
  return run_estimate_noise(r, g, rgb, res, patch_spread ? patch_spread : r.b.spread, eig3);
}

fgbd_status fgbd_filter(fgbd_ctx ctx, const fgbd_graph *g, const float *rgb_in, const fgbd_params *params,
                        const fgbd_result *noise, const double *patch_spread, int32_t q_fixed, float *rgb_out,
                        fgbd_result *res, void *stream) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  fgbd_status st = check_params(params);
  if (st != FGBD_OK) return st;
  if (!g) return fail(FGBD_E_INVALID, "graph is NULL");
  if ((st = check_n(g->n)) != FGBD_OK) return st;
  if (g->k != params->k) return fail(FGBD_E_INVALID, "graph k (%d) != params k (%d)", g->k, params->k);
  if (!res) return fail(FGBD_E_INVALID, "res is NULL");
  const int64_t n = g->n;
  const int select = noise != nullptr;
  if (!select && (q_fixed < 0 || q_fixed > 1024)) return fail(FGBD_E_INVALID, "q_fixed must be in 0..1024");
  if (select && params->fslr_kappa > 0 && !patch_spread && n > 0)
    return fail(FGBD_E_INVALID, "patch_spread is required when FSLR is on (fslr_kappa > 0)");
  if (n > 0 && (!rgb_in || !rgb_out || !g->col || !g->p)) return fail(FGBD_E_INVALID, "NULL colour or graph array");
  if (n > 0 && overlap(rgb_in, (size_t)n * 12, rgb_out, (size_t)n * 12))
    return fail(FGBD_E_INVALID, "rgb_in and rgb_out overlap");
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  const Plan pl = make_plan(n, 1, *params, ctx->tune);
  char *ws = nullptr;
  if ((st = get_workspace(ctx, pl.total, &ws)) != FGBD_OK) return st;
  EventProf ep(ctx, s);
  const Run r = make_run(ctx, pl, ws, *params, n, s, &ep);
  HIP_TRY(launch_setup(r, nullptr, n, res, n == 0 ? 1 : 0), "setup launch");
  if (n == 0) return ok();
  const int q_limit = select ? params->q_max : q_fixed;
  if ((st = run_filter(r, g->col, g->p, nullptr, rgb_in, patch_spread, noise, select, q_limit, rgb_out, res)) !=
      FGBD_OK)
    return st;
  return ok();
}

// Separate sweep launches for an eager call: the schedule's count, lowered to
// the most sweeps any of the last eight read-back calls needed when those
// counts agree (the finalising launch then applies the last sweep's sums
// itself and finds the selection stopped), else to one more (a launch that
// finds it stopped, so the in-launch loop after it returns at once).
// Captured calls keep the schedule's count.  *hint receives where this call's finalising launch
// should store its sweep counts (NULL: no read-back requested).
static int adaptive_sweep_launches(fgbd_ctx ctx, hipStream_t s, int32_t **hint) {
  *hint = nullptr;
  const int cap = ctx->tune.sweep_launches;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone || ctx->hint_failed) return cap;
  if (!ctx->hint_host) {
    void *dev = nullptr;
    if (hipHostMalloc((void **)&ctx->hint_host, kMaxSeg * sizeof(int32_t),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer(&dev, ctx->hint_host, 0) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->hint_ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      ctx->hint_failed = true;
      return cap;
    }
    ctx->hint_dev = (int32_t *)dev;
  }
  if (ctx->hint_pending) {
    const hipError_t q = hipEventQuery(ctx->hint_ev);
    if (q == hipSuccess) {
      int m = 0;
      for (int i = 0; i < ctx->hint_B; ++i) m = ctx->hint_host[i] > m ? ctx->hint_host[i] : m;
      ctx->hint_recent[ctx->hint_count % 8] = m;
      ++ctx->hint_count;
      ctx->hint_pending = false;
    } else if (q != hipErrorNotReady) {
      (void)hipGetLastError();
      ctx->hint_failed = true;
      return cap;
    }
  }
  if (!ctx->hint_pending) *hint = ctx->hint_dev;
  if (ctx->hint_count == 0) return cap;
  int m = 0, lo = 1 << 30;
  const int k = ctx->hint_count < 8 ? ctx->hint_count : 8;
  for (int i = 0; i < k; ++i) {
    m = ctx->hint_recent[i] > m ? ctx->hint_recent[i] : m;
    lo = ctx->hint_recent[i] < lo ? ctx->hint_recent[i] : lo;
  }
  const int want = (k >= 2 && lo == m) ? m : m + 1;  // steady counts: no spare launch
  return want < 1 ? 1 : (want < cap ? want : cap);
}

// After the launches of an eager call that asked for a read-back: mark it.
static void request_hint(fgbd_ctx ctx, hipStream_t s, int B) {
  if (hipEventRecord(ctx->hint_ev, s) == hipSuccess) {
    ctx->hint_pending = true;
    ctx->hint_B = B;
  } else {
    (void)hipGetLastError();
    ctx->hint_failed = true;
  }
}

// The fused path over the call's segments (one cloud of host-known size, or
// B clouds from device offsets).  No separate weights launch: the first sweep
// derives sigma_g and turns the squared distances into the weights as it uses
// them, and stores them for the later sweeps (the noise estimate needs only
// the neighbour lists).
static fgbd_status run_denoise(const Run &r, const int32_t *xyz, const float *rgb_in, float *rgb_out,
                               fgbd_result *res) {
  fgbd_status st;
  if ((st = run_slg(r, xyz, r.b.col, r.b.dist2, nullptr, res, rgb_in)) != FGBD_OK) return st;
  if (r.prm.k == 8 && r.pl.P == 8 && r.prm.patch_order == 0) {
    // the noise launch gathers each point's row and its neighbours' colours
    // anyway: it also computes the weights and the first sweep's colours, and
    // the first sweep launch only adds the FSLR flags and the sums
    if ((st = run_noise(r, r.b.col, rgb_in, r.b.spread, nullptr, res, true)) != FGBD_OK) return st;
    return run_filter(r, r.b.col, r.b.p, nullptr, rgb_in, r.b.spread, res, 1, r.prm.q_max, rgb_out, res, true);
  }
  if ((st = run_noise(r, r.b.col, rgb_in, r.b.spread, nullptr, res)) != FGBD_OK) return st;
  return run_filter(r, r.b.col, r.b.p, r.b.dist2, rgb_in, r.b.spread, res, 1, r.prm.q_max, rgb_out, res);
}

fgbd_status fgbd_denoise(fgbd_ctx ctx, const int32_t *xyz, const float *rgb_in, int64_t n,
                         const fgbd_params *params, float *rgb_out, fgbd_result *res, void *stream) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  fgbd_status st = check_params(params);
  if (st != FGBD_OK) return st;
  if ((st = check_n(n)) != FGBD_OK) return st;
  if (!res) return fail(FGBD_E_INVALID, "res is NULL");
  if (n > 0 && (!xyz || !rgb_in || !rgb_out)) return fail(FGBD_E_INVALID, "NULL input or output array");
  if (n > 0 && overlap(rgb_in, (size_t)n * 12, rgb_out, (size_t)n * 12))
    return fail(FGBD_E_INVALID, "rgb_in and rgb_out overlap");
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  const Plan pl = make_plan(n, 1, *params, ctx->tune);
  char *ws = nullptr;
  if ((st = get_workspace(ctx, pl.total, &ws)) != FGBD_OK) return st;
  EventProf ep(ctx, s);
  Run r = make_run(ctx, pl, ws, *params, n, s, &ep);
  sort_policy(ctx, s, r);
  if (n == 0) {
    HIP_TRY(launch_setup(r, nullptr, n, res, 2), "setup launch");
    return ok();
  }
  // the first radix launch does the setup
  r.fold_setup = true;
  r.setup = setup_args(r, nullptr, n, res, 1);
  r.sweep_launches = adaptive_sweep_launches(ctx, s, &r.hint);
  r.relabel_ok = r.prm.patch_order == 0;  // index-ordered patches need the input numbering
  if ((st = run_denoise(r, xyz, rgb_in, rgb_out, res)) != FGBD_OK) return st;
  if (r.hint) request_hint(ctx, s, 1);
  return ok();
}

static fgbd_status check_batched(fgbd_ctx ctx, const int32_t *xyz, const float *rgb_in, int64_t n_total,
                                 const int64_t *offsets, int32_t batch, const fgbd_params *params,
                                 const float *rgb_out, const fgbd_result *res) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  fgbd_status st = check_params(params);
  if (st != FGBD_OK) return st;
  if ((st = check_n(n_total)) != FGBD_OK) return st;
  if (batch < 1 || batch > kMaxSeg) return fail(FGBD_E_INVALID, "batch must be in 1..%d (got %d)", kMaxSeg, batch);
  if (!offsets) return fail(FGBD_E_INVALID, "offsets is NULL");
  if (!res) return fail(FGBD_E_INVALID, "res is NULL");
  if (n_total > 0 && (!xyz || !rgb_in || !rgb_out)) return fail(FGBD_E_INVALID, "NULL input or output array");
  if (n_total > 0 && overlap(rgb_in, (size_t)n_total * 12, rgb_out, (size_t)n_total * 12))
    return fail(FGBD_E_INVALID, "rgb_in and rgb_out overlap");
  return FGBD_OK;
}

fgbd_status fgbd_denoise_batched(fgbd_ctx ctx, const int32_t *xyz, const float *rgb_in, int64_t n_total,
                                 const int64_t *offsets, int32_t batch, const fgbd_params *params, float *rgb_out,
                                 fgbd_result *res, void *stream) {
  fgbd_status st = check_batched(ctx, xyz, rgb_in, n_total, offsets, batch, params, rgb_out, res);
  if (st != FGBD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  const Plan pl = make_plan(n_total, batch, *params, ctx->tune);
  char *ws = nullptr;
  if ((st = get_workspace(ctx, pl.total, &ws)) != FGBD_OK) return st;
  EventProf ep(ctx, s);
  Run r = make_run(ctx, pl, ws, *params, -1, s, &ep);
  sort_policy(ctx, s, r);
  HIP_TRY(launch_setup(r, offsets, 0, res, n_total == 0 ? 2 : 1), "setup launch");
  if (n_total == 0) return ok();
  r.sweep_launches = adaptive_sweep_launches(ctx, s, &r.hint);
  r.relabel_ok = r.prm.patch_order == 0;  // index-ordered patches need the input numbering
  if ((st = run_denoise(r, xyz, rgb_in, rgb_out, res)) != FGBD_OK) return st;
  if (r.hint) request_hint(ctx, s, batch);
  return ok();
}

fgbd_status fgbd_denoise_batched_fixed_q(fgbd_ctx ctx, const int32_t *xyz, const float *rgb_in, int64_t n_total,
                                         const int64_t *offsets, int32_t batch, const fgbd_params *params,
                                         int32_t q_fixed, float *rgb_out, fgbd_result *res, void *stream) {
  fgbd_status st = check_batched(ctx, xyz, rgb_in, n_total, offsets, batch, params, rgb_out, res);
  if (st != FGBD_OK) return st;
  if (q_fixed < 0 || q_fixed > 1024) return fail(FGBD_E_INVALID, "q_fixed must be in 0..1024 (got %d)", q_fixed);
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  const Plan pl = make_plan(n_total, batch, *params, ctx->tune);
  char *ws = nullptr;
  if ((st = get_workspace(ctx, pl.total, &ws)) != FGBD_OK) return st;
  EventProf ep(ctx, s);
  Run r = make_run(ctx, pl, ws, *params, -1, s, &ep);
  sort_policy(ctx, s, r);
  HIP_TRY(launch_setup(r, offsets, 0, res, n_total == 0 ? 2 : 1), "setup launch");
  if (n_total == 0) return ok();
  // SLG, then q_fixed sweeps whose first derives sigma_g and the weights;
  // no noise estimate and no selection (every sweep is a launch of its own)
  r.relabel_ok = true;
  if ((st = run_slg(r, xyz, r.b.col, r.b.dist2, nullptr, res, rgb_in)) != FGBD_OK) return st;
  return run_filter(r, r.b.col, r.b.p, r.b.dist2, rgb_in, nullptr, nullptr, 0, q_fixed, rgb_out, res);
}

fgbd_status fgbd_smooth_geometry(fgbd_ctx ctx, const int32_t *xyz, int64_t n, const fgbd_params *params, int32_t q,
                                 float *xyz_out, fgbd_result *res, void *stream) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  fgbd_status st = check_params(params);
  if (st != FGBD_OK) return st;
  if ((st = check_n(n)) != FGBD_OK) return st;
  if (!res) return fail(FGBD_E_INVALID, "res is NULL");
  if (q < 0 || q > 1024) return fail(FGBD_E_INVALID, "q must be in 0..1024 (got %d)", q);
  if (n > 0 && (!xyz || !xyz_out)) return fail(FGBD_E_INVALID, "NULL input or output array");
  if (n > 0 && overlap(xyz, (size_t)n * 12, xyz_out, (size_t)n * 12))
    return fail(FGBD_E_INVALID, "xyz and xyz_out overlap");
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  const Plan pl = make_plan(n, 1, *params, ctx->tune);
  char *ws = nullptr;
  if ((st = get_workspace(ctx, pl.total, &ws)) != FGBD_OK) return st;
  EventProf ep(ctx, s);
  Run r = make_run(ctx, pl, ws, *params, n, s, &ep);
  sort_policy(ctx, s, r);
  HIP_TRY(launch_setup(r, nullptr, n, res, n == 0 ? 2 : 1), "setup launch");
  if (n == 0) return ok();
  // the coordinates become the signal in the output buffer; with a fixed q
  // the filter reads its input only in the first sweep and writes the output
  // after the last, so it runs in place
  HIP_TRY(launch_coords_f32(xyz, 3 * n, xyz_out, s), "coordinate launch");
  if ((st = run_slg(r, xyz, r.b.col, r.b.dist2, nullptr, res)) != FGBD_OK) return st;
  return run_filter(r, r.b.col, r.b.p, r.b.dist2, xyz_out, nullptr, nullptr, 0, q, xyz_out, res);
}

static fgbd_status check_schedule(const fgbd_schedule *s) {
  if (!s) return fail(FGBD_E_INVALID, "schedule is NULL");
  if (s->merge_blocks < kGridCapMin || s->merge_blocks > kGridCapMax || s->sweep_blocks < kGridCapMin ||
      s->sweep_blocks > kGridCapMax)
    return fail(FGBD_E_INVALID, "merge_blocks and sweep_blocks must be in %d..%d", kGridCapMin, kGridCapMax);
  if (s->noise_blocks < kGridCapMin || s->noise_blocks > kNoiseGridCapMax)
    return fail(FGBD_E_INVALID, "noise_blocks must be in %d..%d", kGridCapMin, kNoiseGridCapMax);
  if (s->sweep_launches < 1 || s->sweep_launches > kMaxSweepLaunches)
    return fail(FGBD_E_INVALID, "sweep_launches must be in 1..%d", kMaxSweepLaunches);
  return FGBD_OK;
}

fgbd_status fgbd_get_schedule(fgbd_ctx ctx, fgbd_schedule *out) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  if (!out) return fail(FGBD_E_INVALID, "out is NULL");
  out->merge_blocks = ctx->tune.cap[kGridMerge];
  out->noise_blocks = ctx->tune.cap[kGridNoise];
  out->sweep_blocks = ctx->tune.cap[kGridSweep];
  out->sweep_launches = ctx->tune.sweep_launches;
  return ok();
}

fgbd_status fgbd_set_schedule(fgbd_ctx ctx, const fgbd_schedule *s) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  fgbd_status st = check_schedule(s);
  if (st != FGBD_OK) return st;
  ctx->tune.cap[kGridMerge] = s->merge_blocks;
  ctx->tune.cap[kGridNoise] = s->noise_blocks;
  ctx->tune.cap[kGridSweep] = s->sweep_blocks;
  ctx->tune.sweep_launches = s->sweep_launches;
  return ok();
}

fgbd_status fgbd_autotune(fgbd_ctx ctx, const int32_t *xyz, const float *rgb_in, int64_t n_total,
                          const int64_t *offsets, int32_t batch, const fgbd_params *params, float *rgb_out,
                          fgbd_result *res, int32_t reps, fgbd_schedule *chosen, void *stream) {
  if (reps < 1 || reps > 100) return fail(FGBD_E_INVALID, "reps must be in 1..100 (got %d)", reps);
  fgbd_status st = check_batched(ctx, xyz, rgb_in, n_total, offsets, batch, params, rgb_out, res);
  if (st != FGBD_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  // the caller's pending timings go to its counters first; tuning uses its own
  st = drain(ctx, ctx->ms, ctx->launches);
  if (st != FGBD_OK) return st;
  const bool was_profiling = ctx->profile;
  ctx->profile = true;
  {  // argument checks of the batched call, and a warm-up
    double w[FGBD_NUM_KERNELS] = {0};
    int64_t wl[FGBD_NUM_KERNELS] = {0};
    st = fgbd_denoise_batched(ctx, xyz, rgb_in, n_total, offsets, batch, params, rgb_out, res, stream);
    fgbd_status st2 = drain(ctx, w, wl);
    if (st == FGBD_OK) st = st2;
    if (st != FGBD_OK) {
      ctx->profile = was_profiling;
      return st;
    }
  }
  static const int kMergeCand[] = {256, 512, 1024, 2048, 4096};
  static const int kNoiseCand[] = {256, 512, 1024};
  static const int kSweepCand[] = {256, 512, 1024, 2048, 4096};
  const int *cands[kNumGrids] = {kMergeCand, kNoiseCand, kSweepCand};
  const int ncand[kNumGrids] = {5, 3, 5};
  // kernel kinds whose time each grid kind decides
  const int kinds[kNumGrids][2] = {{kMerge, kWeights}, {kNoise, kNoiseSolve}, {kSweep, kFinalize}};
  Tune best = ctx->tune;
  for (int g = 0; g < kNumGrids && st == FGBD_OK; ++g) {
    double best_ms = 1e300;
    for (int c = 0; c < ncand[g] && st == FGBD_OK; ++c) {
      ctx->tune = best;
      ctx->tune.cap[g] = cands[g][c];
      double ms[FGBD_NUM_KERNELS] = {0};
      int64_t nl[FGBD_NUM_KERNELS] = {0};
      for (int r = 0; r <= reps && st == FGBD_OK; ++r) {  // run 0 warms up
        st = fgbd_denoise_batched(ctx, xyz, rgb_in, n_total, offsets, batch, params, rgb_out, res, stream);
        if (st == FGBD_OK && r == 0) {
          double w[FGBD_NUM_KERNELS] = {0};
          int64_t wl[FGBD_NUM_KERNELS] = {0};
          st = drain(ctx, w, wl);
        }
      }
      if (st == FGBD_OK) st = drain(ctx, ms, nl);
      const double t = ms[kinds[g][0]] + ms[kinds[g][1]];
      if (st == FGBD_OK && t < best_ms) {
        best_ms = t;
        best.cap[g] = cands[g][c];
      }
    }
  }
  // separate sweep launches: a launch costs little, so it is timed over
  // whole calls (profiling off) rather than per kernel
  ctx->profile = false;
  static const int kLaunchCand[] = {2, 4, 6, 8, 12, 16, 32};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (st == FGBD_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    st = fail(FGBD_E_HIP, "hipEventCreate failed");
  double best_ms = 1e300;
  for (int c = 0; c < 7 && st == FGBD_OK; ++c) {
    ctx->tune = best;
    ctx->tune.sweep_launches = kLaunchCand[c];
    st = fgbd_denoise_batched(ctx, xyz, rgb_in, n_total, offsets, batch, params, rgb_out, res, stream);  // warm-up
    if (st == FGBD_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(FGBD_E_HIP, "hipEventRecord failed");
    for (int r = 0; r < reps && st == FGBD_OK; ++r)
      st = fgbd_denoise_batched(ctx, xyz, rgb_in, n_total, offsets, batch, params, rgb_out, res, stream);
    float t = 0.f;
    if (st == FGBD_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      st = fail(FGBD_E_HIP, "timing the sweep launch count failed");
    if (st == FGBD_OK && t < best_ms) {
      best_ms = t;
      best.sweep_launches = kLaunchCand[c];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  ctx->tune = best;
  ctx->profile = was_profiling;
  if (st != FGBD_OK) return st;
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (chosen) (void)fgbd_get_schedule(ctx, chosen);
  return ok();
}

static fgbd_status check_poly(fgbd_ctx ctx, const fgbd_graph *g, int32_t ncoef, const double *sigma_g) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  if (!g) return fail(FGBD_E_INVALID, "graph is NULL");
  fgbd_status st = check_n(g->n);
  if (st != FGBD_OK) return st;
  if (g->k < 1 || g->k > kMaxK) return fail(FGBD_E_INVALID, "graph k must be in 1..%d", kMaxK);
  if (ncoef < 1 || ncoef > kMaxPoly) return fail(FGBD_E_INVALID, "ncoef must be in 1..%d (got %d)", kMaxPoly, ncoef);
  if (!sigma_g) return fail(FGBD_E_INVALID, "sigma_g is NULL");
  if (g->n > 0 && (!g->col || !g->dist2)) return fail(FGBD_E_INVALID, "NULL graph array");
  return FGBD_OK;
}

int64_t fgbd_poly_saved_floats(int64_t n, int32_t k, int32_t ncoef) {
  if (n < 0 || k < 1 || ncoef < 1 || ncoef > kMaxPoly) return -1;
  return (int64_t)poly_saved_floats(n, k, ncoef);
}

fgbd_status fgbd_poly_filter(fgbd_ctx ctx, const fgbd_graph *g, const float *x, const float *coef, int32_t ncoef,
                             const double *sigma_g, float *out, float *saved, void *stream) {
  fgbd_status st = check_poly(ctx, g, ncoef, sigma_g);
  if (st != FGBD_OK) return st;
  const int64_t n = g->n;
  if (n > 0 && (!x || !coef || !out || !saved)) return fail(FGBD_E_INVALID, "NULL input or output array");
  if (n > 0 && overlap(x, (size_t)n * 12, out, (size_t)n * 12)) return fail(FGBD_E_INVALID, "x and out overlap");
  if (n == 0) return ok();
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  char *ws = nullptr;
  if ((st = get_workspace(ctx, poly_workspace(n, g->k, ncoef, kPolyGrid), &ws)) != FGBD_OK) return st;
  HIP_TRY(launch_poly_forward(n, g->k, g->col, g->dist2, x, coef, ncoef, sigma_g, out, saved, ws, s),
          "poly filter launch");
  return ok();
}

fgbd_status fgbd_graph_transpose(fgbd_ctx ctx, const fgbd_graph *g, const fgbd_transpose *t, void *stream) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  if (!g || !t) return fail(FGBD_E_INVALID, "graph or transpose is NULL");
  fgbd_status st = check_n(g->n);
  if (st != FGBD_OK) return st;
  if (g->k < 1 || g->k > kMaxK) return fail(FGBD_E_INVALID, "graph k must be in 1..%d", kMaxK);
  if (t->n != g->n || t->k != g->k) return fail(FGBD_E_INVALID, "transpose shape (%lld, %d) != graph (%lld, %d)",
                                                 (long long)t->n, t->k, (long long)g->n, g->k);
  if (!t->off) return fail(FGBD_E_INVALID, "transpose off is NULL");
  if (g->n > 0 && (!g->col || !t->edge)) return fail(FGBD_E_INVALID, "NULL graph or transpose array");
  if (g->n * (int64_t)g->k > (int64_t)0x7fffffff) return fail(FGBD_E_INVALID, "n * k must be below 2^31");
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  char *ws = nullptr;
  if ((st = get_workspace(ctx, transpose_workspace(g->n), &ws)) != FGBD_OK) return st;
  HIP_TRY(launch_transpose(g->n, g->k, g->col, t->off, t->edge, ws, (hipStream_t)stream), "transpose launch");
  return ok();
}

fgbd_status fgbd_poly_filter_backward(fgbd_ctx ctx, const fgbd_graph *g, const fgbd_transpose *t, const float *saved,
                                      const float *coef, int32_t ncoef, const double *sigma_g, const float *grad_out,
                                      float *grad_x, float *grad_coef, double *grad_sigma_g, void *stream) {
  fgbd_status st = check_poly(ctx, g, ncoef, sigma_g);
  if (st != FGBD_OK) return st;
  const int64_t n = g->n;
  if (n > 0 && (!saved || !coef || !grad_out || !grad_x)) return fail(FGBD_E_INVALID, "NULL input or output array");
  if (n > 0 && overlap(grad_out, (size_t)n * 12, grad_x, (size_t)n * 12))
    return fail(FGBD_E_INVALID, "grad_out and grad_x overlap");
  if (t && (t->n != n || t->k != g->k || !t->off || (n > 0 && !t->edge)))
    return fail(FGBD_E_INVALID, "transpose does not match the graph");
  if (n * (int64_t)g->k > (int64_t)0x7fffffff) return fail(FGBD_E_INVALID, "n * k must be below 2^31");
  if (n == 0) return ok();
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  char *ws = nullptr;
  if ((st = get_workspace(ctx, poly_workspace(n, g->k, ncoef, kPolyGrid), &ws)) != FGBD_OK) return st;
  HIP_TRY(launch_poly_backward(n, g->k, g->col, g->dist2, t ? t->off : nullptr, t ? t->edge : nullptr, saved, coef,
                               ncoef, sigma_g, grad_out, grad_x, grad_coef, grad_sigma_g, ws, s),
          "poly filter backward launch");
  return ok();
}

fgbd_status fgbd_quantize(fgbd_ctx ctx, const float *xyz, int64_t n, int32_t bits, int32_t *xyz_out, double *frame,
                          void *stream) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  fgbd_status st = check_n(n);
  if (st != FGBD_OK) return st;
  if (bits < 1 || bits > 21) return fail(FGBD_E_INVALID, "bits must be in 1..21 (got %d)", bits);
  if (!frame) return fail(FGBD_E_INVALID, "frame is NULL");
  if (n > 0 && (!xyz || !xyz_out)) return fail(FGBD_E_INVALID, "NULL input or output array");
  if (n > 0 && overlap(xyz, (size_t)n * 12, xyz_out, (size_t)n * 12)) return fail(FGBD_E_INVALID, "xyz and xyz_out overlap");
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  char *ws = nullptr;
  if ((st = get_workspace(ctx, 256, &ws)) != FGBD_OK) return st;
  HIP_TRY(launch_quantize(xyz, n, bits, xyz_out, frame, (uint32_t *)ws, (hipStream_t)stream), "quantize launch");
  return ok();
}

fgbd_status fgbd_round_u8(fgbd_ctx ctx, const float *rgb, int64_t n, uint8_t *out, void *stream) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  fgbd_status st = check_n(n);
  if (st != FGBD_OK) return st;
  if (n > 0 && (!rgb || !out)) return fail(FGBD_E_INVALID, "NULL input or output array");
  if (n > 0 && overlap(rgb, (size_t)n * 12, out, (size_t)n * 3)) return fail(FGBD_E_INVALID, "rgb and out overlap");
  if (n == 0) return ok();
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  HIP_TRY(launch_round_u8(rgb, 3 * n, out, (hipStream_t)stream), "round launch");
  return ok();
}

fgbd_status fgbd_set_sweep_wait(fgbd_ctx ctx, int64_t microseconds) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  if (microseconds > 10000000) return fail(FGBD_E_INVALID, "the wait bound is at most 10 s (10000000 us)");
  ctx->wait_us = microseconds < 0 ? -1 : microseconds;
  return ok();
}

fgbd_status fgbd_profile_enable(fgbd_ctx ctx, int32_t enable) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  ctx->profile = enable != 0;
  return ok();
}

fgbd_status fgbd_profile_read(fgbd_ctx ctx, double *ms, int64_t *launches, int32_t count) {
  if (!ctx) return fail(FGBD_E_INVALID, "ctx is NULL");
  if (count < 0 || count > FGBD_NUM_KERNELS) return fail(FGBD_E_INVALID, "count must be in 0..%d", FGBD_NUM_KERNELS);
  if (count > 0 && (!ms || !launches)) return fail(FGBD_E_INVALID, "NULL output array");
  if (!ctx->pending.empty()) {
    DeviceGuard dg(ctx->device);
    if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
    fgbd_status st = drain(ctx, ctx->ms, ctx->launches);
    if (st != FGBD_OK) return st;
  }
  for (int i = 0; i < count; ++i) {
    ms[i] = ctx->ms[i];
    launches[i] = ctx->launches[i];
  }
  for (int i = 0; i < FGBD_NUM_KERNELS; ++i) {
    ctx->ms[i] = 0;
    ctx->launches[i] = 0;
  }
  return ok();
}

fgbd_status fgbd_estimate_noise_noalloc(fgbd_ctx ctx, const fgbd_graph *g, const float *rgb,
                                        const fgbd_params *params, fgbd_result *res, double *patch_spread,
                                        float *eig3, void *stream) {
  fgbd_status st = check_estimate_noise(ctx, g, rgb, params, res);
  if (st != FGBD_OK) return st;
  if (g->n > 0 && !patch_spread) return fail(FGBD_E_INVALID, "patch_spread is required by the no-allocation call");
  const Plan pl = noise_scratch_plan(g->n, *params, ctx->tune);
  if (pl.total > kNoAllocBytes)
    return fail(FGBD_E_WORKSPACE, "these parameters need %zu bytes of scratch, the array holds %zu", pl.total,
                kNoAllocBytes);
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  char *ws = nullptr;
  if ((st = scratch_address(ctx->device, &ws)) != FGBD_OK) return st;
  Run r = make_run(ctx, pl, ws, *params, g->n, (hipStream_t)stream, nullptr);
  // only the packed buffers exist
  r.b.items_a = r.b.items_b = nullptr;
  r.b.hist = r.b.rank = nullptr;
  r.b.digits = nullptr;
  r.b.win = nullptr;
  r.b.col = r.b.dist2 = nullptr;
  r.b.p = nullptr;
  r.b.spread = nullptr;
  r.b.xbuf = nullptr;
  return run_estimate_noise(r, g, rgb, res, patch_spread, eig3);
}

}  // extern "C"
