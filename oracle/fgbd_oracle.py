"""FP64 CPU oracle of the FGBD per-frame path (test infrastructure only).

Watanabe et al., "Fast graph-based denoising for point cloud color information"
(arXiv:2401.09721).  Each function states the passage it follows.  Integer steps
are exact int64; floating point is float64 throughout.  Where the paper is
silent or ambiguous the reading taken is stated in the docstring (readings R1..R13
below; the same list is kept with the design notes).

Readings
  R1  directions: the paper fixes three raster codes (eqs. 1-3) and says diagonal
      scan lines were also tried (Sec. 2.2).  A scan direction is a primitive
      integer vector u; ``DIRECTIONS`` lists sixteen, the first three being
      eqs. 1-3; a run uses the first L.  Each point's candidates are the ``w``
      predecessors and successors in each scan order (the paper: w = 1, L = 3).
  R2  ties: equal keys (duplicate points) are ordered by original index; the K
      kept neighbours are the first K candidates by (squared distance, index).
  R3  sigma_g is the mean Euclidean length over all directed graph edges (one
      global value), so long line-wrap edges get negligible weight (Sec. 2.2).
  R4  patches hold one colour channel each: D = P + 1 entries (the point, then
      its P nearest neighbours in CSR order, i.e. distance order, Sec. 2.3);
      the three channels are pooled in one D x D covariance with each channel's
      mean removed, normalised by the number of patches.
  R5  the eigenvalue-tail mean uses 1/(D - m), the number of terms.
  R6  m is the smallest value at which the tail mean is not above the tail
      median (the loop "increase m while tau > median"); sigma_est = sqrt(tau).
  R7  eq. 6 over colour sums all three channels and divides by 3|S|; the FSLR
      subset only restricts that sum, never the filtering.
  R8  q: sweep q = 1, 2, ... until the first q_c with E(q_c) >= sigma_est^2 (or
      q_max); q* minimises |sigma_est^2 - E(q)| over 0..q_c, ties to smaller q.
  R9  FSLR standard deviations are population (1/D) values over the patch; a
      point with spread equal to 2 sigma_est stays in the subset.
  R10 rows with fewer than P neighbours are left out of the covariance and the
      subset; a row with no neighbour is the identity row of the filter.  An
      empty subset, or kappa <= 0, means all points.
  R11 the output is not clipped or rounded.
  R12 several results can be correct only at floating-point near-ties of q or m.
  R13 the "w/o sort" patch of the noise-estimation ablation (Sec. 3) holds the
      same D points as the sorted one (the point and its first P neighbours), in
      increasing point index: the order the points have in the input, which is
      what an unsorted patch keeps.
  R14 sigma_g = 0 (every edge of length 0, i.e. duplicate points only) takes
      eq. 4 at its limit sigma_g -> 0+: a row's weight is shared evenly by its
      entries at the row's smallest distance.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "DIRECTIONS",
    "quantize",
    "round_u8",
    "smooth_geometry",
    "direction_frame",
    "scan_keys",
    "scan_orders",
    "slg_candidates",
    "slg_graph",
    "knn_bruteforce",
    "bandwidth",
    "edge_weights",
    "filter_step",
    "filter_power",
    "patch_matrix",
    "patch_covariance",
    "sigma_from_eigenvalues",
    "estimate_noise",
    "patch_spread",
    "patch_colour_eigs",
    "fslr_subset",
    "select_filter",
    "denoise",
    "default_params",
    "transpose_apply",
    "poly_filter",
    "poly_filter_grads",
]

#: Scan directions (R1).  d0..d2 reproduce eqs. 1-3 exactly.
DIRECTIONS = (
    (1, 0, 0), (0, 1, 0), (0, 0, 1),
    (1, 1, 0), (1, -1, 0), (0, 1, 1), (0, 1, -1), (1, 0, 1), (1, 0, -1),
    (1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1),
    (1, 2, 0), (0, 1, 2), (2, 0, 1),
)


def default_params(**kw) -> dict:
    """Parameters of one run: bits b, directions L, window w, neighbours K,
    patch size P (0 means K), q_max, FSLR factor kappa (2 in Sec. 2.4), and a
    fixed sigma_g (<= 0: mean edge length, Sec. 2.2), and the patch order
    (0: by distance, Sec. 2.3; 1: by point index, R13)."""
    p = dict(bits=10, num_dirs=8, window=4, k=8, patch=0, q_max=32, fslr_kappa=2.0, sigma_g=0.0, patch_order=0)
    p.update(kw)
    return p


# ---------------------------------------------------------------------------
# Sec. 2.2: scan-line graph
# ---------------------------------------------------------------------------

def direction_frame(u):
    """Axes of the scan code for direction u (R1).

    The position axis ``a`` is the first axis with |u_a| = 1 (u is negated if
    needed so that u_a = +1).  The remaining axes, high ``h`` = (a+2) mod 3 and
    middle ``m`` = (a+1) mod 3, are replaced by the line invariants
    e_j = g_j - u_j g_a + max(u_j, 0)(2^b - 1), which are constant along a line
    of direction u and non-negative.  Returns (a, h, m, u) with u normalised."""
    u = np.asarray(u, np.int64)
    a = int(np.flatnonzero(np.abs(u) == 1)[0])
    if u[a] < 0:
        u = -u
    return a, (a + 2) % 3, (a + 1) % 3, u


def scan_keys(xyz, bits: int, num_dirs: int) -> np.ndarray:
    """Scan-line codes C_{i,l} (eqs. 1-3 and R1), int64 [L, N].

    code = ((e_h * 2^{B_m}) + e_m) * 2^b + g_a, where B_j is the bit width of
    e_j: b plus the bit length of |u_j|.  For the axis directions this is
    2^{2b} g_h + 2^b g_m + g_a, i.e. eq. 1 (z, y, x), eq. 2 (x, z, y), eq. 3 (y, x, z)."""
    g = np.asarray(xyz, np.int64)
    top = (1 << bits) - 1
    keys = np.empty((num_dirs, g.shape[0]), np.int64)
    for d in range(num_dirs):
        a, h, m, u = direction_frame(DIRECTIONS[d])
        e_h = g[:, h] - u[h] * g[:, a] + max(int(u[h]), 0) * top
        e_m = g[:, m] - u[m] * g[:, a] + max(int(u[m]), 0) * top
        width_m = bits + int(abs(int(u[m]))).bit_length()
        keys[d] = ((e_h << width_m) + e_m) * (1 << bits) + g[:, a]
    return keys


def scan_orders(keys: np.ndarray) -> np.ndarray:
    """Sorted order of the points by each code (the radix sort of Sec. 2.2):
    a stable ascending sort, so equal codes keep ascending index (R2).  [L, N]."""
    return np.stack([np.argsort(k, kind="stable") for k in keys]) if keys.shape[1] else keys.copy()


def slg_candidates(orders: np.ndarray, window: int) -> np.ndarray:
    """Candidate neighbours (Sec. 2.2 and R1): for the point at sorted position r
    of each direction, the points at r-w..r-1 and r+1..r+w, crossing line ends
    (the paper keeps line-wrap links).  int64 [N, 2wL], -1 where r+s is outside
    0..N-1."""
    L, n = orders.shape
    cols = []
    for d in range(L):
        rank = np.empty(n, np.int64)
        rank[orders[d]] = np.arange(n)
        for s in list(range(-window, 0)) + list(range(1, window + 1)):
            r = rank + s
            ok = (r >= 0) & (r < n)
            cols.append(np.where(ok, orders[d][np.clip(r, 0, max(n - 1, 0))], -1))
    return np.stack(cols, axis=1) if cols else np.zeros((n, 0), np.int64)


def _keep_nearest(xyz, cand: np.ndarray, k: int):
    """Union of candidate sets, ordered by (squared distance, index), first k kept;
    the rest padded with col = -1, dist2 = 0 (R2)."""
    g = np.asarray(xyz, np.int64)
    n = g.shape[0]
    big = np.iinfo(np.int64).max
    if cand.shape[1] == 0:
        return np.full((n, k), -1, np.int64), np.zeros((n, k), np.int64)
    valid = cand >= 0
    j = np.where(valid, cand, 0)
    diff = g[j] - g[:, None, :]
    d2 = np.sum(diff * diff, axis=2)
    comp = np.where(valid, d2 * (n + 1) + j, big)
    comp.sort(axis=1)
    dup = np.zeros_like(valid)
    dup[:, 1:] = comp[:, 1:] == comp[:, :-1]
    comp[dup] = big
    comp.sort(axis=1)
    if comp.shape[1] < k:
        comp = np.concatenate([comp, np.full((n, k - comp.shape[1]), big, np.int64)], axis=1)
    comp = comp[:, :k]
    keep = comp != big
    col = np.where(keep, comp % (n + 1), -1)
    dist2 = np.where(keep, comp // (n + 1), 0)
    return col, dist2


def slg_graph(xyz, bits: int, num_dirs: int, window: int, k: int):
    """Scan-line graph (Sec. 2.2, R1, R2): codes, stable sort per direction,
    +-w candidates per sorted order, union, and the first K by (dist2, index).
    Returns (col int64 [N,K] with -1 padding, dist2 int64 [N,K])."""
    keys = scan_keys(xyz, bits, num_dirs)
    orders = scan_orders(keys)
    return _keep_nearest(xyz, slg_candidates(orders, window), k)


def knn_bruteforce(xyz, k: int):
    """Exact K nearest neighbours by brute force (the textbook definition the
    scan-line graph reduces to when the window covers every point, Sec. 2.2):
    for each point i, every other point j ordered by (squared distance, index)
    with a lexicographic sort, the first K kept, the rest of the row padded with
    col = -1 and dist2 = 0.  Written independently of the scan-line graph's own
    selection so that each checks the other.  O(N^2 log N); small clouds only."""
    g = np.asarray(xyz, np.int64)
    n = g.shape[0]
    col = np.full((n, k), -1, np.int64)
    dist2 = np.zeros((n, k), np.int64)
    for i in range(n):
        others = np.array([j for j in range(n) if j != i], np.int64)
        if others.size == 0:
            continue
        d2 = np.sum((g[others] - g[i]) ** 2, axis=1)
        order = np.lexsort((others, d2))  # primary key d2, then the index
        take = order[:k]
        col[i, :take.size] = others[take]
        dist2[i, :take.size] = d2[take]
    return col, dist2


def bandwidth(col, dist2) -> float:
    """sigma_g of eq. 4: the mean Euclidean edge length over all directed edges
    of the graph (Sec. 2.2, R3).  0 for a graph without edges."""
    valid = np.asarray(col) >= 0
    if not valid.any():
        return 0.0
    return float(np.mean(np.sqrt(np.asarray(dist2, np.float64)[valid])))


def edge_weights(col, dist2, sigma_g: float) -> np.ndarray:
    """Row-normalised Gaussian weights p_ik = w_ik / deg_i with
    w_ij = exp(-|g_i - g_j|^2 / sigma_g^2) (eq. 4), written with the row's
    smallest squared distance subtracted in the exponent, which leaves the
    ratio unchanged.  Padding entries get 0.  With sigma_g = 0 (R14) the weight
    is 1 at the smallest distance and 0 elsewhere before normalisation."""
    col = np.asarray(col)
    d2 = np.asarray(dist2, np.float64)
    valid = col >= 0
    d0 = d2[:, :1]
    delta = d2 - d0
    if sigma_g > 0:
        w = np.exp(-delta / (sigma_g * sigma_g))
    else:
        w = (delta == 0).astype(np.float64)
    w = np.where(valid, w, 0.0)
    s = w.sum(axis=1, keepdims=True)
    return np.divide(w, s, out=np.zeros_like(w), where=s > 0)


def filter_step(col, p, x):
    """One application of T = D_g^{-1} W_g with W_g = D + W and D_g = 2D
    (eq. 5), i.e. (Tx)_i = x_i / 2 + (1/2) sum_k p_ik x_{col_ik}; a row with no
    neighbour is the identity (R10).  x is [N] or [N, C]."""
    col = np.asarray(col)
    x = np.asarray(x, np.float64)
    valid = col >= 0
    j = np.where(valid, col, 0)
    pe = np.where(valid, p, 0.0)
    if x.ndim == 1:
        nb = np.sum(pe * x[j], axis=1)
    else:
        nb = np.einsum("nk,nkc->nc", pe, x[j])
    out = 0.5 * x + 0.5 * nb
    empty = ~valid[:, 0] if col.shape[1] else np.ones(col.shape[0], bool)
    out[empty] = x[empty]
    return out


def filter_power(col, p, x, q: int):
    """f_out = (D_g^{-1} W_g)^q f_in (eq. 5)."""
    for _ in range(q):
        x = filter_step(col, p, x)
    return np.asarray(x, np.float64)


# ---------------------------------------------------------------------------
# Sec. 2.3: noise estimation using graph-based patches (NE-GBP)
# ---------------------------------------------------------------------------

def _patch_size(col, patch: int) -> int:
    k = np.asarray(col).shape[1]
    return k if patch <= 0 else patch


def patch_matrix(col, y, patch: int = 0, order: int = 0):
    """Graph-based patches (Sec. 2.3, R4, R10): for every point whose row has at
    least P neighbours, the patch of each channel is its own value followed by
    the values of its first P neighbours in CSR order (increasing distance,
    index tie-break).  ``order = 1`` lists the same D points by increasing
    point index instead (R13).  Returns (complete mask [N], A [N_eff, D, 3])."""
    col = np.asarray(col)
    P = _patch_size(col, patch)
    y = np.asarray(y, np.float64)
    if P > col.shape[1]:
        raise ValueError("patch size exceeds K")
    complete = col[:, P - 1] >= 0 if P > 0 else np.ones(col.shape[0], bool)
    idx = np.concatenate([np.arange(col.shape[0])[:, None], col[:, :P]], axis=1)[complete]
    if order:
        idx = np.sort(idx, axis=1)
    return complete, y[idx]


def patch_covariance(col, y, patch: int = 0, order: int = 0):
    """Sigma = (1/N) sum_i (a_i - mu)(a_i - mu)^T with mu the mean patch
    (Sec. 2.3), pooled over the three channels with each channel's own mean
    removed (R4): Sigma = (1/(3 N_eff)) sum_c sum_i (a_i^c - mu^c)(a_i^c - mu^c)^T.
    Returns (Sigma [D,D], N_eff)."""
    complete, A = patch_matrix(col, y, patch, order)
    n_eff, D = A.shape[0], A.shape[1]
    if n_eff == 0:
        return np.zeros((D, D)), 0
    sigma = np.zeros((D, D))
    for c in range(3):
        a = A[:, :, c]
        dev = a - a.mean(axis=0)
        sigma += dev.T @ dev
    return sigma / (3.0 * n_eff), n_eff


def sigma_from_eigenvalues(lam):
    """Noise level from the eigenvalues of Sigma (Sec. 2.3, R5, R6).

    With lambda_1 >= ... >= lambda_D, tau_m = (1/(D-m)) sum_{k>m} lambda_k and
    med_m the median of lambda_{m+1..D}; m* is the smallest m with
    tau_m <= med_m and sigma_est = sqrt(max(tau_m*, 0)).  Returns (sigma_est, m*)."""
    lam = np.sort(np.asarray(lam, np.float64))[::-1]
    D = lam.size
    for m in range(D):
        tail = lam[m:]
        tau = float(np.mean(tail))
        med = float(np.median(tail))
        if tau <= med:
            return math.sqrt(max(tau, 0.0)), m
    return 0.0, D  # D == 0


def estimate_noise(col, y, patch: int = 0, order: int = 0) -> dict:
    """NE-GBP (Sec. 2.3): patch covariance, its eigenvalues (LAPACK symmetric
    solver), and the tail rule.  No complete patch gives sigma_est = 0.
    ``order`` as in patch_matrix."""
    sigma, n_eff = patch_covariance(col, y, patch, order)
    if n_eff == 0:
        return dict(sigma_est=0.0, m=0, eigvals=np.zeros(sigma.shape[0]), cov=sigma, n_eff=0)
    lam = np.linalg.eigvalsh(sigma)[::-1]
    s, m = sigma_from_eigenvalues(lam)
    return dict(sigma_est=s, m=m, eigvals=lam, cov=sigma, n_eff=n_eff)


# ---------------------------------------------------------------------------
# Sec. 2.4: filter selection with limited region (FSLR) and low-pass filter
# ---------------------------------------------------------------------------

def patch_spread(col, y, patch: int = 0) -> np.ndarray:
    """s_i = (sigma_R(i) + sigma_G(i) + sigma_B(i)) / 3, the mean of the
    per-channel population standard deviations over patch a_i (Sec. 2.4, R9).
    +inf for incomplete rows, which never enter the subset (R10)."""
    complete, A = patch_matrix(col, y, patch)
    s = np.full(np.asarray(col).shape[0], np.inf)
    if A.shape[0]:
        mean = A.mean(axis=1, keepdims=True)
        std = np.sqrt(np.mean((A - mean) ** 2, axis=1))  # [N_eff, 3]
        s[complete] = (std[:, 0] + std[:, 1] + std[:, 2]) / 3.0
    return s


def patch_colour_eigs(col, y, patch: int = 0) -> np.ndarray:
    """Eigenvalues (descending) of each point's 3x3 colour covariance over its
    patch, C_i = (1/D) sum_{j in patch} (f_j - fbar)(f_j - fbar)^T, whose
    diagonal holds the FSLR variances (Sec. 2.4).  Zero rows for incomplete
    patches.  [N, 3]."""
    complete, A = patch_matrix(col, y, patch)
    out = np.zeros((np.asarray(col).shape[0], 3))
    if A.shape[0]:
        dev = A - A.mean(axis=1, keepdims=True)
        C = np.einsum("ndi,ndj->nij", dev, dev) / A.shape[1]
        out[complete] = np.linalg.eigvalsh(C)[:, ::-1]
    return out


def fslr_subset(spread, sigma_est: float, kappa: float) -> np.ndarray:
    """FSLR (Sec. 2.4): keep the points whose patch spread is not above
    kappa * sigma_est (kappa = 2 in the paper).  kappa <= 0, or an empty subset,
    gives all points (R10)."""
    spread = np.asarray(spread)
    if kappa <= 0:
        return np.ones(spread.shape[0], bool)
    keep = spread <= kappa * sigma_est
    if not keep.any():
        return np.ones(spread.shape[0], bool)
    return keep


def select_filter(col, p, y, sigma_est: float, subset, q_max: int) -> dict:
    """Integer filter selection (Sec. 2.4, eq. 6, R7, R8).

    E(q) = (1/(3|S|)) sum_{i in S} sum_c (y_ic^2 - x_q,ic^2) with x_q = T^q y.
    Sweeps run until the first q_c with E(q_c) >= sigma_est^2 or until q_max;
    q* minimises |sigma_est^2 - E(q)| over 0..q_c (E(0) = 0), ties to the smaller q.
    Returns dict(q, loss, energies, out=x_{q*}, q_stop)."""
    y = np.asarray(y, np.float64)
    S = np.asarray(subset, bool)
    nS = int(S.sum())
    target = sigma_est * sigma_est
    y2 = float(np.sum(y[S] ** 2))
    energies = [0.0]
    best_q, best_loss, best_x = 0, abs(target), y
    x = y
    q_stop = 0
    for q in range(1, q_max + 1):
        x = filter_step(col, p, x)
        e = (y2 - float(np.sum(x[S] ** 2))) / (3.0 * nS) if nS else 0.0
        energies.append(e)
        loss = abs(target - e)
        if loss < best_loss:
            best_q, best_loss, best_x = q, loss, x
        q_stop = q
        if e >= target:
            break
    return dict(q=best_q, loss=best_loss, energies=np.array(energies), out=best_x, q_stop=q_stop)


def denoise(xyz, rgb, params: dict | None = None, q_fixed: int | None = None) -> dict:
    """The four steps of Fig. 1(b) / Sec. 2.1: SLG, NE-GBP, FSLR and the
    low-pass filter.  ``q_fixed`` skips selection and applies eq. 5 that many
    times.  Returns dict(out [N,3] float64, sigma_est, sigma_g, q, n_fslr, n_eff,
    status, col, dist2, p, spread, energies, m)."""
    prm = default_params(**(params or {}))
    g = np.asarray(xyz, np.int64)
    y = np.asarray(rgb, np.float64)
    n = g.shape[0]
    status = 0
    if n and (g.min() < 0 or g.max() >= (1 << prm["bits"])):
        status |= 1
    col, dist2 = slg_graph(g, prm["bits"], prm["num_dirs"], prm["window"], prm["k"])
    sg = prm["sigma_g"] if prm["sigma_g"] > 0 else bandwidth(col, dist2)
    p = edge_weights(col, dist2, sg)
    ne = estimate_noise(col, y, prm["patch"], prm["patch_order"])
    if ne["n_eff"] == 0:
        status |= 2
    spread = patch_spread(col, y, prm["patch"])
    if q_fixed is not None:
        out = filter_power(col, p, y, q_fixed)
        return dict(out=out, sigma_est=ne["sigma_est"], sigma_g=sg, q=q_fixed, n_fslr=n, n_eff=ne["n_eff"],
                    status=status, col=col, dist2=dist2, p=p, spread=spread, energies=None, m=ne["m"])
    S = fslr_subset(spread, ne["sigma_est"], prm["fslr_kappa"])
    sel = select_filter(col, p, y, ne["sigma_est"], S, prm["q_max"])
    return dict(out=sel["out"], sigma_est=ne["sigma_est"], sigma_g=sg, q=sel["q"], n_fslr=int(S.sum()),
                n_eff=ne["n_eff"], status=status, col=col, dist2=dist2, p=p, spread=spread,
                energies=sel["energies"], loss=sel["loss"], m=ne["m"], eigvals=ne["eigvals"])


# ---------------------------------------------------------------------------
# Steps on either side of the path: float coordinates onto the grid that
# Sec. 2.2 assumes, and filtered colours back to 8 bits
# ---------------------------------------------------------------------------

def quantize(xyz, bits: int):
    """Float coordinates to b-bit voxel codes with one scale for all axes
    (Sec. 2.2 takes integer coordinates): lo_c = min x_c, ext = the largest
    axis range, s = 2^b / ext (0 when ext = 0), g = min(floor((x - lo) s),
    2^b - 1), in FP64.  NaN coordinates are left out of the bounds and map to
    0.  Returns (int32 [N,3], (lo [3], s))."""
    x = np.asarray(xyz, np.float32).astype(np.float64)
    n = x.shape[0]
    lo = np.full(3, np.nan)
    ext = 0.0
    for c in range(3):
        finite = x[:, c][~np.isnan(x[:, c])]
        if finite.size:
            lo[c] = finite.min()
            ext = max(ext, finite.max() - lo[c])
    cells = float(2 ** bits)
    s = cells / ext if ext > 0 else 0.0
    g = np.zeros((n, 3), np.int64)
    with np.errstate(invalid="ignore"):
        v = (x - lo[None, :]) * s
        ok = v >= 0
        g[ok] = np.minimum(np.floor(np.minimum(v[ok], cells)), cells - 1).astype(np.int64)
    return g.astype(np.int32), (lo, s)


def smooth_geometry(xyz, q: int, params: dict | None = None) -> dict:
    """The scan-line graph and eq. 4 weights of the coordinates (Sec. 2.2), then
    q applications of eq. 5 to the coordinates as the signal.  Returns
    dict(out [N,3] float64, sigma_g, col, p)."""
    prm = default_params(**(params or {}))
    g = np.asarray(xyz, np.int64)
    col, dist2 = slg_graph(g, prm["bits"], prm["num_dirs"], prm["window"], prm["k"])
    sg = prm["sigma_g"] if prm["sigma_g"] > 0 else bandwidth(col, dist2)
    p = edge_weights(col, dist2, sg)
    return dict(out=filter_power(col, p, g.astype(np.float64), q), sigma_g=sg, col=col, p=p)


def round_u8(rgb):
    """Colours to uint8: round half to even, clip to 0..255, NaN to 0."""
    v = np.rint(np.asarray(rgb, np.float32))
    out = np.zeros(v.shape, np.uint8)
    ok = v >= 0
    out[ok] = np.minimum(v[ok], 255).astype(np.uint8)
    return out


# ---------------------------------------------------------------------------
# Polynomial graph filter and its gradients (generalises eq. 5: c = e_q)
# ---------------------------------------------------------------------------

def transpose_apply(col, p, z):
    """T^T z for the (directed) filter operator of eq. 5: the diagonal part
    (1/2, or 1 for an identity row) plus a scatter of (p_ik / 2) z_i onto
    col_ik.  z is [N] or [N, C]."""
    col = np.asarray(col)
    z = np.asarray(z, np.float64)
    zz = z[:, None] if z.ndim == 1 else z
    valid = col >= 0
    empty = ~valid[:, 0] if col.shape[1] else np.ones(col.shape[0], bool)
    out = np.where(empty[:, None], zz, 0.5 * zz)
    rows, ks = np.nonzero(valid & ~empty[:, None])
    np.add.at(out, col[rows, ks], 0.5 * np.asarray(p)[rows, ks][:, None] * zz[rows])
    return out[:, 0] if z.ndim == 1 else out


def poly_filter(col, dist2, x, coef, sigma_g: float):
    """out = sum_k c_k T^k x with T built from eq. 4 weights at bandwidth sigma_g
    and eq. 5's self loops (c = e_q reproduces eq. 5)."""
    p = edge_weights(col, dist2, sigma_g)
    xk = np.asarray(x, np.float64)
    out = coef[0] * xk
    for c in coef[1:]:
        xk = filter_step(col, p, xk)
        out = out + c * xk
    return out


def poly_filter_grads(col, dist2, x, coef, sigma_g: float, grad_out):
    """Gradients of <grad_out, poly_filter(...)> with respect to x, the
    coefficients and sigma_g, by reverse-mode automatic differentiation of the
    plain forward definition in float64 (PyTorch CPU autograd).  Returns
    (grad_x [N,3], grad_coef [n], grad_sigma_g)."""
    import torch

    col_t = torch.as_tensor(np.asarray(col), dtype=torch.int64)
    d2 = torch.as_tensor(np.asarray(dist2), dtype=torch.float64)
    xt = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
    ct = torch.tensor(np.asarray(coef, np.float64), requires_grad=True)
    st = torch.tensor(float(sigma_g), dtype=torch.float64, requires_grad=True)
    valid = col_t >= 0
    j = torch.where(valid, col_t, torch.zeros_like(col_t))
    w = torch.exp(-(d2 - d2[:, :1]) / (st * st)) * valid
    s = w.sum(dim=1, keepdim=True)
    p = w / torch.where(s > 0, s, torch.ones_like(s))
    empty = ~valid[:, 0]
    xk = xt
    out = ct[0] * xk
    for k in range(1, ct.shape[0]):
        nb = torch.einsum("nk,nkc->nc", p, xk[j])
        nxt = 0.5 * xk + 0.5 * nb
        xk = torch.where(empty[:, None], xk, nxt)
        out = out + ct[k] * xk
    g = torch.as_tensor(np.asarray(grad_out, np.float64))
    (out * g).sum().backward()
    # with one coefficient the output c_0 x does not involve T, so d/dsigma_g = 0
    gs = float(st.grad) if st.grad is not None else 0.0
    return xt.grad.numpy(), ct.grad.numpy(), gs
