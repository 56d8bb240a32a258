/*
 * fgbd.h -- C ABI of the MI355X (gfx950) implementation of fast graph-based
 * denoising (FGBD) of point-cloud colour: Watanabe, Nonaka, Pavez, Kobayashi,
 * Ortega, "Fast graph-based denoising for point cloud color information",
 * arXiv:2401.09721.
 *
 * The per-frame path of the paper (Sec. 2.1, Fig. 1(b)) is exposed as four
 * calls that can be used one by one or fused:
 *   fgbd_build_slg       scan-line graph, Sec. 2.2, eqs. 1-4
 *   fgbd_estimate_noise  NE-GBP noise level, Sec. 2.3
 *   fgbd_filter          FSLR filter selection and the low-pass filter, Sec. 2.4,
 *                        eqs. 5-6
 *   fgbd_denoise         all four steps in one call
 *   fgbd_denoise_batched all four steps for several clouds of different sizes
 *                        in one launch sequence, sizes read from device memory
 *   fgbd_denoise_batched_fixed_q  the frames between two full ones in the
 *                        periodic mode of Sec. 4: graph and q given sweeps
 *
 * Around the path: fgbd_quantize (float coordinates onto the voxel grid),
 * fgbd_round_u8 (colours to 8 bits), fgbd_smooth_geometry (the same graph and
 * filter applied to the coordinates), fgbd_poly_filter and its adjoint (a
 * polynomial in the filter operator with a trainable bandwidth), and the
 * schedule, workspace and timing calls.
 *
 * Conventions shared by every call
 *   - Every pointer named in a call is a DEVICE pointer on the context's GPU
 *     unless its comment says "host".  Arrays are dense, row-major, with no
 *     padding: coordinates int32 [n][3] (x, y, z), colours float32 [n][3]
 *     (R, G, B) on the 0..255 scale.  The caller owns every input and output
 *     buffer; the context owns only its workspace.
 *   - Every call validates its arguments on the host and returns a status
 *     before enqueuing anything.  On success all work is enqueued
 *     asynchronously on `stream` (a hipStream_t; NULL is the default stream)
 *     and the call returns without waiting, so a sequence of calls can be
 *     captured in a HIP graph.  Values that steer control flow (sigma_est, q)
 *     stay in device memory, in an fgbd_result the caller provides.
 *   - A call allocates device memory only when no workspace has been set with
 *     fgbd_set_workspace and the context's own workspace is too small.
 *   - Errors never throw across the ABI; the message of the last failing call
 *     on this thread is available from fgbd_last_error().
 *   - Results are deterministic: the same inputs and parameters give bitwise
 *     identical outputs on the same device (no floating-point atomics).
 *   - Calls on one context must not overlap in time (they share the
 *     workspace); use one context per concurrent stream.
 *   - A context adapts its launch schedule to what its recent eager calls
 *     found, read back without waiting: the number of sweep launches, and
 *     the radix sort's route (a call whose points crowd into few top code
 *     digits, such as a large plane normal to a scan axis, makes the next
 *     calls sort by LSD passes for a while).  Either route gives the same
 *     result; only the time differs.  Calls under stream capture keep the
 *     default schedule.
 */
#ifndef FGBD_H_
#define FGBD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGBD_ABI_VERSION 9

/* Largest number of clouds in one fgbd_denoise_batched call. */
#define FGBD_MAX_BATCH 64

typedef enum {
  FGBD_OK = 0,
  FGBD_E_INVALID = -1,     /* bad argument (null pointer, size or parameter out of range) */
  FGBD_E_NOMEM = -2,       /* device allocation of the workspace failed                   */
  FGBD_E_HIP = -3,         /* a HIP runtime call failed (message names it)                 */
  FGBD_E_WORKSPACE = -4,   /* the workspace set with fgbd_set_workspace is too small      */
  FGBD_E_UNSUPPORTED = -5  /* valid but not supported by this build (e.g. codes above 63 bits) */
} fgbd_status;

/* Device-detected conditions, OR-ed into fgbd_result.status. */
#define FGBD_ST_COORD_RANGE 1 /* a coordinate was outside 0 .. 2^bits - 1 (graph undefined)  */
#define FGBD_ST_NO_PATCH 2    /* no point had P neighbours: sigma_est set to 0 (Sec. 2.3)    */
#define FGBD_ST_BAD_OFFSETS 4 /* batched offsets did not start at 0, decreased, or exceeded
                                 n_total: they were clamped into range before use           */
#define FGBD_ST_DIST_CLAMPED 32 /* a kept neighbour's squared distance exceeded 2^31 - 1 (grids above
                                 2^15, neighbours more than 46340 voxels apart): its dist2 entry
                                 holds 2^31 - 1 and the weights see that value               */
#define FGBD_ST_RELABELED 16  /* information, not an error: the input's point order was far from
                                 any spatial order (most points adjacent along scan line 0 lie
                                 far apart in the input), so the graph was built with the input
                                 numbering as always, then the noise estimate and the sweeps
                                 ran with the points renumbered along scan order 0 and the
                                 output was put back in the input order (same results up to
                                 the rounding order of the patch-moment block sums)           */
#define FGBD_ST_SWEEP_STALL 8 /* the sweeps run inside one launch waited longer than their
                                 bound (half a second by default, fgbd_set_sweep_wait) for
                                 each other (the GPU was shared with work that kept blocks
                                 from starting): the selection did not finish.  Every
                                 point of rgb_out is still written, with either its input
                                 colour or its filtered one, and q, loss, n_fslr and
                                 sweeps of the result are not valid                          */

/* Parameters of one run.  fgbd_default_params gives the values used for 1M-point
 * frames (b = 10, L = 8, w = 4, K = 8). */
typedef struct {
  int32_t bits;       /* b: coordinates lie in 0 .. 2^b - 1 (Sec. 2.2); 1..21, as long as every scan
                         code of the first num_dirs directions fits 63 bits (3b bits for the axis
                         directions, 3b + 1 for (1,1,0)-type diagonals, 3b + 2 for the rest): b <= 20
                         with all 16 directions, b = 21 with the three axis directions.  Codes above
                         32 bits (b > 10) take more radix passes and a slower neighbour selection. */
  int32_t num_dirs;   /* L: scan directions 1..16; the first three are eqs. 1-3, the rest diagonal
                         lines (Sec. 2.2 mentions them as an alternative)                          */
  int32_t window;     /* w >= 1: candidates are the w predecessors and w successors in each scan
                         order (the paper connects consecutive points: w = 1); w <= 64              */
  int32_t k;          /* K: neighbours kept per point, the first K candidates by (squared distance,
                         index); 1..32.  Paper mode L = 3, w = 1, K = 6 keeps all candidates.      */
  int32_t patch;      /* P: NE-GBP patch = the point plus its P nearest neighbours (D = P + 1
                         entries, Sec. 2.3); 0 means K; 1..K                                       */
  int32_t q_max;      /* largest number of filter sweeps tried by the selection (eq. 6); 0..1024  */
  double fslr_kappa;  /* FSLR excludes points whose patch spread exceeds kappa * sigma_est
                         (kappa = 2 in Sec. 2.4); <= 0 disables FSLR (all points used)            */
  double sigma_g;     /* Gaussian bandwidth of eq. 4; <= 0 means the mean edge length (Sec. 2.2) */
  int32_t patch_order; /* order of the D entries of a patch vector (Sec. 2.3): 0 = the point, then
                         its neighbours by increasing distance (the method); 1 = the same points
                         by increasing point index, the unsorted patch of the "NE-GBP w/o sort"
                         ablation (Sec. 3, noise estimation).  1 runs a slower generic kernel.   */
  int32_t pad_;       /* set to 0 */
} fgbd_params;

/* A fixed-K neighbour graph in device memory (CSR with K slots per row).
 * Row i lists its neighbours in increasing (squared distance, index) order;
 * unused slots have col = -1, dist2 = 0, p = 0.  p[i][k] is the row-normalised
 * weight w_ik / deg_i of eq. 4, so (T x)_i = x_i / 2 + sum_k p[i][k] x[col[i][k]] / 2
 * is the filter operator D_g^{-1} W_g of eq. 5. */
typedef struct {
  int32_t *col;   /* device int32 [n][k] */
  int32_t *dist2; /* device int32 [n][k], exact integer squared distances */
  float *p;       /* device float32 [n][k] */
  int64_t n;
  int32_t k;
  int32_t pad_;
} fgbd_graph;

/* Per-frame results, written to DEVICE memory by the calls (48 bytes). */
typedef struct {
  double sigma_est; /* NE-GBP noise level on the 0..255 scale (Sec. 2.3)           */
  double sigma_g;   /* bandwidth used in eq. 4                                     */
  double loss;      /* |sigma_est^2 - E(q)| at the selected q (eq. 6)              */
  int32_t q;        /* number of filter sweeps applied (selected or fixed)         */
  int32_t n_fslr;   /* points entering eq. 6 after FSLR (Sec. 2.4)                 */
  int32_t n_eff;    /* points with a complete patch (entered the covariance)       */
  int32_t status;   /* FGBD_ST_* bits                                              */
  int32_t sweeps;   /* filter sweeps computed before the selection stopped        */
  int32_t m;        /* index m of the first eigenvalue in the noise tail (Sec. 2.3) */
} fgbd_result;

typedef struct fgbd_ctx_s *fgbd_ctx;

/* ABI version compiled into the library (FGBD_ABI_VERSION). */
int32_t fgbd_abi_version(void);

/* Fill *p with the defaults: bits 10, num_dirs 8, window 4, k 8, patch 0 (= k),
 * q_max 32, fslr_kappa 2.0, sigma_g 0 (mean edge length), patch_order 0.  p: host. */
fgbd_status fgbd_default_params(fgbd_params *p);

/* Create a context bound to HIP device `hip_device`.  No device memory is
 * touched until the first compute call.  out: host. */
fgbd_status fgbd_create(fgbd_ctx *out, int32_t hip_device);

/* Free the context and any workspace it allocated itself.  NULL is allowed. */
fgbd_status fgbd_destroy(fgbd_ctx ctx);

/* Device workspace in bytes that a call needs for up to n_max points in
 * `batch` clouds: batch = 1 covers fgbd_denoise and every single-cloud call,
 * batch = B covers fgbd_denoise_batched with B clouds totalling at most n_max
 * points (1 <= batch <= FGBD_MAX_BATCH).  p, bytes: host. */
fgbd_status fgbd_workspace_size(const fgbd_params *p, int64_t n_max, int32_t batch, size_t *bytes);

/* Hand the context a caller-owned device buffer (256-byte aligned) to use as
 * its workspace; afterwards no call allocates.  dev = NULL, bytes = 0 returns
 * to self-allocation.  The buffer must outlive every call that uses it. */
fgbd_status fgbd_set_workspace(fgbd_ctx ctx, void *dev, size_t bytes);

/* Scan-line graph (Sec. 2.2).  For each of the first L directions, every
 * point gets a scan-line code (eqs. 1-3; the diagonal directions replace two
 * coordinates by line invariants); the codes are sorted by an LSD radix sort
 * (equal codes keep index order); the w points before and after each point
 * in every sorted order are its candidates; the first K distinct candidates by
 * (squared distance, index) form its row.  Then sigma_g (params->sigma_g, or
 * the mean Euclidean length of all edges) and the weights of eq. 4.
 *   xyz: int32 [n][3];  n >= 0, n < 2^31;  g->col/dist2/p: outputs with n*k
 *   slots each (g->n == n, g->k == params->k);  res: sigma_g and status are
 *   written, every other field is zeroed. */
fgbd_status fgbd_build_slg(fgbd_ctx ctx, const int32_t *xyz, int64_t n, const fgbd_params *params,
                           const fgbd_graph *g, fgbd_result *res, void *stream);

/* NE-GBP (Sec. 2.3).  Patches of D = P + 1 entries per colour channel (the
 * point, then its first P neighbours in row order, i.e. by distance) from
 * every point with at least P neighbours; their covariance, pooled over the
 * channels with each channel's mean removed; its eigenvalues in FP64; the
 * noise level sqrt(tau) from the smallest m with tau_m <= median of the tail
 * lambda_{m+1..D}, where tau_m is the tail mean.
 *   g: graph from fgbd_build_slg;  rgb: float32 [n][3];
 *   res: sigma_est, n_eff written, status bit FGBD_ST_NO_PATCH set or cleared;
 *   patch_spread: optional output double [n], the FSLR spread
 *     (sigma_R + sigma_G + sigma_B) / 3 of each patch (Sec. 2.4; +inf for an
 *     incomplete patch), needed by fgbd_filter when FSLR is on;
 *   eig3: optional output float32 [n][3], eigenvalues (descending) of each
 *     point's 3x3 colour covariance over its patch, a diagnostic whose diagonal
 *     the FSLR spread uses; 0 for incomplete patches. */
fgbd_status fgbd_estimate_noise(fgbd_ctx ctx, const fgbd_graph *g, const float *rgb, const fgbd_params *params,
                                fgbd_result *res, double *patch_spread, float *eig3, void *stream);

/* fgbd_estimate_noise for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, checks, launches and results (bit for bit) as
 * fgbd_estimate_noise, except:
 *   - its scratch (segment table, patch-moment and edge-length accumulators)
 *     is one fixed array of FGBD_NOALLOC_SCRATCH_BYTES inside the library,
 *     one copy per GPU, held from the library's load until the process ends;
 *     the context's workspace is neither used nor allocated, and the call
 *     allocates nothing (no device memory, no events: per-kernel timing is
 *     off for it).  Each call clears the accumulators it uses before use.
 *   - patch_spread is required when n > 0 (there is no workspace to hold the
 *     spreads otherwise).
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents: calls that overlap in time on one GPU (other streams,
 *     contexts or threads) race on it and give wrong results; serialise them.
 *   - FGBD_E_WORKSPACE if the parameters need more scratch than the array
 *     holds (the need depends on the patch size only and is at most about
 *     350 KB, for k = patch = 32); FGBD_E_UNSUPPORTED for devices >= 64. */
#define FGBD_NOALLOC_SCRATCH_BYTES (512 * 1024)
fgbd_status fgbd_estimate_noise_noalloc(fgbd_ctx ctx, const fgbd_graph *g, const float *rgb,
                                        const fgbd_params *params, fgbd_result *res, double *patch_spread,
                                        float *eig3, void *stream);

/* Filter selection (FSLR, Sec. 2.4, eq. 6) and the low-pass filter (eq. 5).
 * With `noise` non-NULL: x_0 = rgb_in, x_q = T x_{q-1}; E(q) is the mean over
 * the FSLR subset and the channels of y^2 - x_q^2; sweeps stop at the first q
 * with E(q) >= sigma_est^2 (or q_max) and the q in 0..that minimising
 * |sigma_est^2 - E(q)| (ties to the smaller q) is applied.  The subset is the
 * points whose patch_spread is <= fslr_kappa * sigma_est (all points when
 * fslr_kappa <= 0 or the subset is empty).  With `noise` NULL: exactly
 * q_fixed sweeps (q_fixed >= 0), no selection.
 *   rgb_in, rgb_out: float32 [n][3], must not overlap;
 *   noise: device fgbd_result holding sigma_est (may equal res);
 *   patch_spread: double [n] from fgbd_estimate_noise, required when noise is
 *     non-NULL and fslr_kappa > 0;
 *   res: q, n_fslr, loss written and sigma_est copied from noise. */
fgbd_status fgbd_filter(fgbd_ctx ctx, const fgbd_graph *g, const float *rgb_in, const fgbd_params *params,
                        const fgbd_result *noise, const double *patch_spread, int32_t q_fixed, float *rgb_out,
                        fgbd_result *res, void *stream);

/* The whole per-frame path of Fig. 1(b): build_slg, estimate_noise and filter
 * with selection, with every intermediate in the workspace.
 *   xyz: int32 [n][3]; rgb_in, rgb_out: float32 [n][3] (must not overlap);
 *   res: every field written. */
fgbd_status fgbd_denoise(fgbd_ctx ctx, const int32_t *xyz, const float *rgb_in, int64_t n,
                         const fgbd_params *params, float *rgb_out, fgbd_result *res, void *stream);

/* The per-frame path for B clouds stored back to back, each denoised on its
 * own (own graph, sigma_g, sigma_est, FSLR subset and q, exactly as
 * fgbd_denoise would on that cloud alone, up to rounding order), in one
 * launch sequence whose grids are sized from n_total and B only: the cloud
 * sizes are read from device memory, so one captured sequence serves any
 * sizes up to n_total (streaming frames of varying size: B = 1).
 *   xyz: int32 [n_total][3]; rgb_in, rgb_out: float32 [n_total][3] (must not
 *   overlap);  offsets: device int64 [batch + 1]: cloud s owns the points
 *   offsets[s] .. offsets[s+1]-1.  offsets[0] must be 0, the entries
 *   non-decreasing and offsets[batch] <= n_total; otherwise each entry is
 *   clamped into that form and FGBD_ST_BAD_OFFSETS is set in every result.
 *   Points from offsets[batch] on are left untouched.
 *   1 <= batch <= FGBD_MAX_BATCH;  res: device fgbd_result [batch], every
 *   field written.  Neighbours never cross clouds. */
fgbd_status fgbd_denoise_batched(fgbd_ctx ctx, const int32_t *xyz, const float *rgb_in, int64_t n_total,
                                 const int64_t *offsets, int32_t batch, const fgbd_params *params, float *rgb_out,
                                 fgbd_result *res, void *stream);

/* The periodic mode of the per-frame path (Sec. 4: noise estimation and
 * filter selection run once every few frames, the frames in between reuse
 * the last selected q): fgbd_denoise_batched without the noise estimate and
 * the selection, filtering every cloud with q_fixed sweeps of eq. 5 on its
 * own graph (its own sigma_g and weights).  Same arguments and layout as
 * fgbd_denoise_batched, plus
 *   q_fixed: 0..1024 (the caller passes the q of the last full frame; 0
 *     returns the input colours);
 *   res: sigma_g, q = sweeps = q_fixed written; sigma_est, n_eff, m, n_fslr
 *     and loss are 0.
 * Errors as fgbd_denoise_batched, and FGBD_E_INVALID for q_fixed out of range. */
fgbd_status fgbd_denoise_batched_fixed_q(fgbd_ctx ctx, const int32_t *xyz, const float *rgb_in, int64_t n_total,
                                         const int64_t *offsets, int32_t batch, const fgbd_params *params,
                                         int32_t q_fixed, float *rgb_out, fgbd_result *res, void *stream);

/* Launch schedule of the per-cloud kernels: the largest grid, in blocks of
 * 256 threads, of (merge_blocks) the neighbour merge and edge weights,
 * (noise_blocks) the patch statistics and (sweep_blocks) the filter sweeps
 * and finalise; and (sweep_launches) how many of the up to q_max filter
 * sweeps of eq. 6 are enqueued as launches of their own.  The sweeps after
 * those run in one launch whose blocks wait for each other between sweeps
 * (the grid is sized to be resident on the device at once), which returns at
 * once when every cloud's selection has already finished (a launch that
 * finds the selection finished still costs about two microseconds; waiting
 * for all blocks costs far more than a launch boundary, so the count should
 * cover the sweeps a workload usually needs).  When the sweep grid cannot be
 * resident on the device at once, every sweep is a launch of its own.
 * Defaults 4096, 1024, 512 and 8.  A schedule changes no result beyond the
 * rounding order of FP64 sums (block partials); it is a property of the
 * context and applies to every later call on it.  Valid ranges:
 * merge_blocks and sweep_blocks 64..4096, noise_blocks 64..1024,
 * sweep_launches 1..1024. */
typedef struct {
  int32_t merge_blocks;
  int32_t noise_blocks;
  int32_t sweep_blocks;
  int32_t sweep_launches;
} fgbd_schedule;

/* out, s: host. */
fgbd_status fgbd_get_schedule(fgbd_ctx ctx, fgbd_schedule *out);
fgbd_status fgbd_set_schedule(fgbd_ctx ctx, const fgbd_schedule *s);

/* Autotuner of the launch schedule.  Runs fgbd_denoise_batched on the given
 * inputs (same arguments and rules as that call; the outputs hold the last
 * run) under candidate grid sizes, one kernel group at a time (merge and
 * weights, then patch statistics and the noise solve, then sweeps and
 * finalise), `reps` timed
 * runs per candidate after one warm-up, times every kernel with HIP events,
 * then times whole calls for each candidate count of separate sweep
 * launches, and keeps the fastest schedule in the context.  Blocks the host until the runs
 * finish, so it must not be captured; tune once per workload shape, then
 * capture or stream.  The caller's own profiling counters are kept.
 * reps: 1..100;  chosen: optional host output of the selected schedule. */
fgbd_status fgbd_autotune(fgbd_ctx ctx, const int32_t *xyz, const float *rgb_in, int64_t n_total,
                          const int64_t *offsets, int32_t batch, const fgbd_params *params, float *rgb_out,
                          fgbd_result *res, int32_t reps, fgbd_schedule *chosen, void *stream);

/* Polynomial graph filter, the differentiable generalisation of eq. 5:
 *   out = sum_{k=0}^{ncoef-1} coef[k] T^k x,
 * with T = D_g^{-1} W_g (eq. 5) whose weights (eq. 4) are recomputed from
 * g->dist2 and the bandwidth *sigma_g (so sigma_g may be a trained parameter;
 * g->p is not used).  coef = e_q reproduces fgbd_filter with q_fixed = q.
 *   g: col and dist2 of a graph from fgbd_build_slg;  x, out: float32 [n][3]
 *   (must not overlap);  coef: device float32 [ncoef], 1 <= ncoef <= 32;
 *   sigma_g: device double (one value, > 0);  saved: output float32 buffer of
 *   fgbd_poly_saved_floats(n, k, ncoef) floats that the backward call needs:
 *   [2 ncoef - 1][n][3], the iterates x_0..x_{ncoef-1}, then u_1..u_{ncoef-1}
 *   with u_m = 2 (dT/dsigma_g) x_{m-1} (formed from the neighbour values the
 *   sweep gathers); for ncoef >= 2 then, from the next multiple of 64 floats,
 *   the weights p [n][k] and T's diagonal [n] the forward used. */
fgbd_status fgbd_poly_filter(fgbd_ctx ctx, const fgbd_graph *g, const float *x, const float *coef, int32_t ncoef,
                             const double *sigma_g, float *out, float *saved, void *stream);

/* Floats of fgbd_poly_filter's saved buffer for n points, k neighbours per
 * row and ncoef coefficients; -1 for n < 0, k < 1 or ncoef outside 1..32.
 * Host only. */
int64_t fgbd_poly_saved_floats(int64_t n, int32_t k, int32_t ncoef);

/* Transpose of a graph's directed edges, the structure the adjoint of eq. 5
 * pulls along (T^T).  For every point j, the ids e = i * k + slot of the
 * edges with col[i][slot] == j, in increasing order:
 *   edge[off[j]] .. edge[off[j + 1] - 1],  off[0] = 0, off[n] = edges.
 * The graph is fixed while a filter's coefficients and bandwidth are fitted,
 * so the transpose is built once (fgbd_graph_transpose) and passed to every
 * backward call.  Caller-owned device arrays. */
typedef struct {
  int32_t *off;  /* device int32 [n + 1] */
  int32_t *edge; /* device int32 [n * k] (the first off[n] entries are used) */
  int64_t n;
  int32_t k;
  int32_t pad_;
} fgbd_transpose;

/* Build t from the graph's col (t->n == g->n, t->k == g->k, n * k < 2^31).
 * Deterministic (rows are sorted after their atomic placement).  Uses the
 * context workspace (4 bytes per point).  Errors: FGBD_E_INVALID for NULL
 * pointers or mismatched shapes. */
fgbd_status fgbd_graph_transpose(fgbd_ctx ctx, const fgbd_graph *g, const fgbd_transpose *t, void *stream);

/* Hand-written adjoint of fgbd_poly_filter for L = <grad_out, out>:
 *   grad_x = z_0 with z_{ncoef-1} = c_{ncoef-1} grad_out and
 *            z_k = c_k grad_out + T^T z_{k+1} (T^T along the transpose t);
 *   grad_coef[k] = <grad_out, x_k>;
 *   grad_sigma_g = sum_{m>=1} <z_m, (dT/dsigma_g) x_{m-1}>.
 *   t: the graph's transpose from fgbd_graph_transpose, or NULL to build one
 *   in the workspace for this call;
 *   saved: the buffer written by fgbd_poly_filter with the same g, coef,
 *   ncoef and sigma_g (its weights are used, not recomputed);  grad_out, grad_x: float32 [n][3] (must not overlap);
 *   grad_coef: optional device float32 [ncoef];  grad_sigma_g: optional device
 *   double.  Scalar gradients are reduced in a fixed order (deterministic). */
fgbd_status fgbd_poly_filter_backward(fgbd_ctx ctx, const fgbd_graph *g, const fgbd_transpose *t, const float *saved,
                                      const float *coef, int32_t ncoef, const double *sigma_g, const float *grad_out,
                                      float *grad_x, float *grad_coef, double *grad_sigma_g, void *stream);

/* Float coordinates onto the 2^bits integer grid that the scan-line graph
 * takes (Sec. 2.2 assumes voxelised integer coordinates).  One scale for the
 * three axes keeps the shape:
 *   lo_c = min_i x_ic, ext = max over c of (max_i x_ic - lo_c), s = 2^bits / ext
 *   (s = 0 when ext = 0), g_ic = min(floor((x_ic - lo_c) * s), 2^bits - 1),
 * evaluated in FP64 with IEEE division, so the codes are exact.  Points that
 * share a voxel are all kept (the graph links them at distance 0).  NaN
 * coordinates take no part in the bounds and map to 0; an infinite one makes
 * s = 0 (every code 0).
 *   xyz:     device float32 [n][3], read only.
 *   bits:    1..21 (the per-frame calls take the same range, see fgbd_params).
 *   xyz_out: device int32 [n][3], written; must not overlap xyz.
 *   frame:   device double[4], written: lo_x, lo_y, lo_z, s, so a voxel g maps
 *            back to lo + (g + 1/2) / s.  lo is NaN on an axis with no finite
 *            value (and for n = 0).
 * Uses 32 bytes of the context workspace.  Errors: FGBD_E_INVALID for a NULL
 * pointer, bits out of range, n < 0 or overlapping buffers. */
fgbd_status fgbd_quantize(fgbd_ctx ctx, const float *xyz, int64_t n, int32_t bits, int32_t *xyz_out, double *frame,
                          void *stream);

/* Colours to 8 bits after filtering: out = clip(round_half_even(rgb), 0, 255),
 * NaN to 0 (the filter output is neither rounded nor clipped).
 *   rgb: device float32 [n][3]; out: device uint8 [n][3], must not overlap rgb.
 * Errors: FGBD_E_INVALID for a NULL pointer, n < 0 or overlapping buffers. */
fgbd_status fgbd_round_u8(fgbd_ctx ctx, const float *rgb, int64_t n, uint8_t *out, void *stream);

/* Geometry smoothing with the same graph and filter (the paper names applying
 * them to coordinates as the next step, Secs. 1 and 4): the scan-line graph
 * of the integer coordinates and its eq. 4 weights (Sec. 2.2), then q sweeps
 * of eq. 5 applied to the coordinates themselves as a three-channel signal.
 * No noise estimate and no selection: q is the caller's.
 *   xyz:     device int32 [n][3] in 0 .. 2^bits - 1 (as for fgbd_denoise).
 *   q:       0..1024 sweeps (0 returns the coordinates as float).
 *   xyz_out: device float32 [n][3], written; must not overlap xyz.
 *   res:     device fgbd_result: sigma_g, q and status are set.
 * Uses the context workspace like fgbd_denoise.  Errors: FGBD_E_INVALID for
 * NULL pointers, bad parameters, q out of range or overlapping buffers. */
fgbd_status fgbd_smooth_geometry(fgbd_ctx ctx, const int32_t *xyz, int64_t n, const fgbd_params *params, int32_t q,
                                 float *xyz_out, fgbd_result *res, void *stream);

/* Bound of each wait between two sweeps in the launch that runs the sweeps
 * after the separate ones (see fgbd_schedule), in microseconds; negative
 * restores the default of half a second.  A wait that reaches the bound ends
 * that launch with FGBD_ST_SWEEP_STALL in the cloud's result instead of
 * waiting on (FGBD_ST_SWEEP_STALL describes the output then).  0 gives up at
 * the first wait that is not already over, which lets a test drive that path
 * from the host.  A property of the context, for every later call.
 * Errors: FGBD_E_INVALID for a NULL ctx or a bound above 10 s. */
fgbd_status fgbd_set_sweep_wait(fgbd_ctx ctx, int64_t microseconds);

/* Message for the last non-OK status returned on the calling thread ("" if
 * none).  Valid until the next call on this thread. */
const char *fgbd_last_error(void);

/* Kernel timing for measurement.  When enabled, the compute calls record a
 * HIP event pair on their stream around every kernel launch;
 * fgbd_profile_read waits for the work recorded so far and returns, per kernel
 * kind, the summed milliseconds and the number of launches, then clears the
 * counters.  Kinds:
 *   0 radix upsweep (digit counts; pass 0 also makes the codes), 1 radix scan,
 *   2 radix downsweep (stable scatter), 3 neighbour merge, 4 edge weights,
 *   5 patch statistics, 6 noise eigen-solve, 7 filter sweep, 8 finalise,
 *   9 renumbering of clouds stored in no spatial order, 10 local sort of the
 *   buckets left by the top-digit pass (codes of at most 32 bits, which sort
 *   with one top-digit pass of kinds 0-2 and this launch instead of four
 *   LSD passes).
 * The event records add a little time of their own between launches.
 * ms, launches: host arrays of `count` entries (count <= FGBD_NUM_KERNELS). */
#define FGBD_NUM_KERNELS 11
fgbd_status fgbd_profile_enable(fgbd_ctx ctx, int32_t enable);
fgbd_status fgbd_profile_read(fgbd_ctx ctx, double *ms, int64_t *launches, int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* FGBD_H_ */
