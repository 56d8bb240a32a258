"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.

Bars: the graph (col, dist2) is bit-exact; sigma_g and the FSLR spreads agree to
FP64 rounding; sigma_est and every filtered colour are within 1e-3 on the 0..255
scale; q is equal unless the oracle's own losses at the two values are within the
FP32 sweep error (then the output is checked at the GPU's q).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2401_09721_amd import fgbd, synth  # noqa: E402

pytestmark = pytest.mark.gpu

from gpu_helpers import COLOUR_TOL, compare_denoise, dev, oracle_params  # noqa: E402


def gpu_graph(xyz, prm):
    g = fgbd.build_slg(dev(xyz, torch.int32), prm)
    torch.cuda.synchronize()
    return g, g.col.cpu().numpy(), g.dist2.cpu().numpy(), g.p.cpu().numpy(), fgbd.read_result(g.result)


def check_graph(xyz, prm):
    g, col, d2, p, res = gpu_graph(xyz, prm)
    ocol, od2 = O.slg_graph(xyz, prm.bits, prm.num_dirs, prm.window, prm.k)
    assert np.array_equal(col, ocol), "col differs"
    assert np.array_equal(d2, od2), "dist2 differs"
    sg = prm.sigma_g if prm.sigma_g > 0 else O.bandwidth(ocol, od2)
    assert math.isclose(res["sigma_g"], sg, rel_tol=1e-12, abs_tol=1e-300)
    op = O.edge_weights(ocol, od2, sg)
    assert np.allclose(p, op, rtol=0, atol=2e-7)
    return g, ocol, od2, op, sg


def check_denoise(xyz, rgb, prm, ores=None):
    out, res = fgbd.denoise(dev(xyz, torch.int32), dev(rgb, torch.float32), prm)
    torch.cuda.synchronize()
    return compare_denoise(out.cpu().numpy(), fgbd.read_result(res), xyz, rgb, prm, ores)


# ------------------------------------------------------------------ graph

@pytest.mark.parametrize("L,w,K", [(8, 4, 8), (3, 1, 6), (16, 4, 8), (8, 2, 16), (4, 8, 32), (1, 1, 1), (12, 3, 5)])
def test_slg_bitexact_tiny(L, w, K):
    c = synth.tiny_cloud(0)
    check_graph(c.xyz, fgbd.default_params(bits=8, num_dirs=L, window=w, k=K))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 4095, 4096, 4097, 9000])
def test_slg_ragged_sizes_with_duplicates(n):
    rng = np.random.default_rng(n)
    g = rng.integers(0, 32, size=(n, 3))
    if n > 4:
        g[rng.integers(0, n, size=n // 5)] = g[0]  # duplicate points
    check_graph(g.astype(np.int32), fgbd.default_params(bits=5, num_dirs=8, window=4, k=8))


def test_slg_full_window_is_exact_knn():
    rng = np.random.default_rng(7)
    g = rng.integers(0, 16, size=(300, 3)).astype(np.int32)
    _, col, d2, _, _ = gpu_graph(g, fgbd.default_params(bits=4, num_dirs=3, window=64, k=8))
    # w = 64 < N - 1 here, so compare with the oracle at the same window, and
    # separately the oracle's full-window graph with brute-force KNN
    ocol, od2 = O.slg_graph(g, 4, 3, 64, 8)
    assert np.array_equal(col, ocol) and np.array_equal(d2, od2)
    small = g[:60]
    _, col, d2, _, _ = gpu_graph(small, fgbd.default_params(bits=4, num_dirs=3, window=59, k=8))
    bcol, bd2 = O.knn_bruteforce(small, 8)
    assert np.array_equal(col, bcol) and np.array_equal(d2, bd2)


def test_slg_all_directions_b10_extremes():
    # corners and edges of the 2^10 cube exercise the widest codes (32 bits)
    rng = np.random.default_rng(3)
    g = rng.choice([0, 1, 2, 1021, 1022, 1023], size=(5000, 3)).astype(np.int32)
    check_graph(g, fgbd.default_params(bits=10, num_dirs=16, window=2, k=8))


def test_slg_plane_normal_to_a_scan_axis():
    # 25,600 points on the plane z = 500 share one top code digit in the scan
    # orders whose high axis is z: a bucket far beyond one block's LDS, which
    # the local sort then takes alone through the item buffers; the other
    # orders and the scattered points take the in-LDS passes
    rng = np.random.default_rng(11)
    xs, ys = np.meshgrid(np.arange(300, 460), np.arange(200, 360), indexing="ij")
    plane = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, 500)], axis=1)
    extra = rng.integers(0, 1024, size=(3000, 3))
    g = np.concatenate([plane, extra])[rng.permutation(plane.shape[0] + 3000)].astype(np.int32)
    check_graph(g, fgbd.default_params(bits=10, num_dirs=8, window=4, k=8))


def test_sort_route_after_a_large_plane():
    # 90,000 points on the plane z = 500: in the orders whose high axis is z
    # they form ranges far larger than a block sorts quickly alone.  The first
    # call flags that; once its read-back has completed, calls on the same
    # context sort by LSD passes (no local-sort launch) and give the same graph.
    xs, ys = np.meshgrid(np.arange(200, 500), np.arange(100, 400), indexing="ij")
    plane = np.stack([xs.ravel(), ys.ravel(), np.full(xs.size, 500)], axis=1)
    rng = np.random.default_rng(12)
    g = np.concatenate([plane, rng.integers(0, 1024, size=(5000, 3))]).astype(np.int32)
    prm = fgbd.default_params(bits=10, num_dirs=8, window=4, k=8)
    ctx = fgbd.Context("cuda")
    x = dev(g, torch.int32)
    ctx.profile(True)
    first = fgbd.build_slg(x, prm, ctx=ctx)
    torch.cuda.synchronize()
    p1 = ctx.profile_read()
    second = fgbd.build_slg(x, prm, ctx=ctx)
    torch.cuda.synchronize()
    p2 = ctx.profile_read()
    ctx.profile(False)
    assert p1["local_sort"][1] == 1 and p1["radix_downsweep"][1] == 1
    assert p2["local_sort"][1] == 0 and p2["radix_downsweep"][1] == 4
    ocol, od2 = O.slg_graph(g, prm.bits, prm.num_dirs, prm.window, prm.k)
    for gr in (first, second):
        assert np.array_equal(gr.col.cpu().numpy(), ocol)
        assert np.array_equal(gr.dist2.cpu().numpy(), od2)
    ctx.close()


def test_fixed_sigma_g():
    c = synth.tiny_cloud(0)
    check_graph(c.xyz, fgbd.default_params(bits=8, sigma_g=2.5))


def test_coordinate_out_of_range_flagged():
    g = np.array([[0, 0, 0], [1, 0, 0], [1024, 0, 0], [2, 1, 0]], np.int32)
    with pytest.warns(RuntimeWarning, match="outside"):
        _, _, _, _, res = gpu_graph(g, fgbd.default_params(bits=10))
    assert res["status"] & fgbd.FGBD_ST_COORD_RANGE


# ------------------------------------------------------------------ noise

@pytest.mark.parametrize("sigma", [10.0, 20.0, 30.0])
@pytest.mark.parametrize("P", [0, 4])
def test_noise_estimate_tiny(sigma, P):
    c = synth.tiny_cloud(0, sigma=sigma)
    prm = fgbd.default_params(bits=8, patch=P)
    g, ocol, od2, op, sg = check_graph(c.xyz, prm)
    res, spread, eig3 = fgbd.estimate_noise(g, dev(c.noisy, torch.float32), prm, want_eig3=True)
    torch.cuda.synchronize()
    r = fgbd.read_result(res)
    ne = O.estimate_noise(ocol, c.noisy, P)
    assert abs(r["sigma_est"] - ne["sigma_est"]) <= COLOUR_TOL
    assert abs(r["sigma_est"] - ne["sigma_est"]) <= 1e-9 * ne["sigma_est"]
    assert r["n_eff"] == ne["n_eff"]
    os_ = O.patch_spread(ocol, c.noisy, P)
    gs = spread.cpu().numpy()
    fin = np.isfinite(os_)
    assert np.array_equal(np.isfinite(gs), fin)
    assert np.allclose(gs[fin], os_[fin], rtol=1e-12, atol=1e-12)
    oe = O.patch_colour_eigs(ocol, c.noisy, P)
    ge = eig3.cpu().numpy()
    scale = np.maximum(oe[:, :1], 1.0)
    assert np.all(np.abs(ge - oe) <= 1e-5 * scale + 1e-4)


@pytest.mark.parametrize("shuffle", [False, True])
@pytest.mark.parametrize("P", [0, 3])
def test_noise_estimate_unsorted_patch(shuffle, P):
    # the "w/o sort" ablation: patch entries by point index (generic kernel,
    # also for P = K = 8, where the sorted patch takes the MFMA kernel)
    c = synth.random_shapes_cloud(7, bits=8, target=12000, shuffle=shuffle)
    prm = fgbd.default_params(bits=8, patch=P, patch_order=1)
    g, ocol, od2, op, sg = check_graph(c.xyz, prm)
    res, spread, _ = fgbd.estimate_noise(g, dev(c.noisy, torch.float32), prm)
    torch.cuda.synchronize()
    r = fgbd.read_result(res)
    ne = O.estimate_noise(ocol, c.noisy, P, order=1)
    assert abs(r["sigma_est"] - ne["sigma_est"]) <= 1e-9 * ne["sigma_est"]
    assert r["n_eff"] == ne["n_eff"] and r["m"] == ne["m"]
    # the spread does not depend on the order
    os_ = O.patch_spread(ocol, c.noisy, P)
    gs = spread.cpu().numpy()
    fin = np.isfinite(os_)
    assert np.allclose(gs[fin], os_[fin], rtol=1e-12, atol=1e-12)


def test_noise_constant_and_pure_noise():
    c = synth.tiny_cloud(0)
    prm = fgbd.default_params(bits=8)
    const = np.tile(np.array([[10.0, 128.0, 250.0]], np.float32), (c.n, 1))
    out, r, _ = check_denoise(c.xyz, const, prm)
    assert r["sigma_est"] == 0.0 and r["q"] == 0
    assert np.array_equal(out, const)
    rng = np.random.default_rng(1)
    noise = (128.0 + rng.normal(0, 25.0, size=(c.n, 3))).astype(np.float32)
    out, r, _ = check_denoise(c.xyz, noise, prm)
    assert abs(r["sigma_est"] - 25.0) < 0.75


def test_noise_eigen_d3_and_d33():
    # D = 3 (P = 2) and the largest supported patch D = 33 (K = P = 32)
    c = synth.tiny_cloud(0)
    for k, P in [(8, 2), (32, 32), (16, 11)]:
        prm = fgbd.default_params(bits=8, k=k, patch=P)
        check_denoise(c.xyz, c.noisy, prm)


# ------------------------------------------------------------------ filter

@pytest.mark.parametrize("q", [0, 1, 3, 7])
def test_fixed_q_filter(q):
    c = synth.tiny_cloud(0)
    prm = fgbd.default_params(bits=8)
    g, ocol, od2, op, sg = check_graph(c.xyz, prm)
    out, res = fgbd.filter(g, dev(c.noisy, torch.float32), prm, q_fixed=q)
    torch.cuda.synchronize()
    ref = O.filter_power(ocol, op, c.noisy, q)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= COLOUR_TOL
    assert fgbd.read_result(res)["q"] == q


def test_split_calls_equal_fused():
    c = synth.tiny_cloud(0)
    prm = fgbd.default_params(bits=8)
    xyz, rgb = dev(c.xyz, torch.int32), dev(c.noisy, torch.float32)
    g = fgbd.build_slg(xyz, prm)
    res, spread, _ = fgbd.estimate_noise(g, rgb, prm)
    out1, res1 = fgbd.filter(g, rgb, prm, noise=res, spread=spread)
    out2, res2 = fgbd.denoise(xyz, rgb, prm)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)
    r1, r2 = fgbd.read_result(res1), fgbd.read_result(res2)
    assert r1["q"] == r2["q"] and r1["n_fslr"] == r2["n_fslr"] and r1["sigma_est"] == r2["sigma_est"]


# ------------------------------------------------------------------ end to end

@pytest.mark.parametrize("sigma", [10.0, 20.0, 30.0])
def test_denoise_tiny(sigma):
    c = synth.tiny_cloud(0, sigma=sigma)
    out, r, o = check_denoise(c.xyz, c.noisy, fgbd.default_params(bits=8))
    clean = c.clean.astype(np.float64)
    assert np.mean((out - clean) ** 2) < np.mean((c.noisy - clean) ** 2)


@pytest.mark.parametrize("kw", [dict(num_dirs=3, window=1, k=6), dict(fslr_kappa=0.0), dict(fslr_kappa=0.5),
                                dict(q_max=1), dict(q_max=0), dict(num_dirs=16, k=12, patch=6),
                                dict(patch_order=1), dict(patch_order=1, k=12, patch=5),
                                dict(num_dirs=3, window=1, k=6, patch_order=1)])
def test_denoise_variants(kw):
    c = synth.tiny_cloud(0)
    check_denoise(c.xyz, c.noisy, fgbd.default_params(bits=8, **kw))


@pytest.mark.parametrize("order", [0, 1])
def test_denoise_shuffled_order(order):
    c = synth.random_shapes_cloud(5, bits=8, target=12000, shuffle=True)
    check_denoise(c.xyz, c.noisy, fgbd.default_params(bits=8, patch_order=order))


@pytest.mark.parametrize("n", [0, 1, 2, 9, 4097])
def test_denoise_edge_sizes(n):
    rng = np.random.default_rng(n + 100)
    g = rng.integers(0, 64, size=(n, 3)).astype(np.int32)
    rgb = rng.uniform(0, 255, size=(n, 3)).astype(np.float32)
    out, r, o = check_denoise(g, rgb, fgbd.default_params(bits=6))
    if n <= 8:
        assert r["status"] & fgbd.FGBD_ST_NO_PATCH
        assert r["sigma_est"] == 0.0


def test_all_duplicates():
    g = np.tile(np.array([[5, 6, 7]], np.int32), (40, 1))
    rng = np.random.default_rng(0)
    rgb = rng.uniform(0, 255, size=(40, 3)).astype(np.float32)
    check_denoise(g, rgb, fgbd.default_params(bits=4))


def test_deterministic_repeat():
    c = synth.tiny_cloud(0)
    prm = fgbd.default_params(bits=8)
    xyz, rgb = dev(c.xyz, torch.int32), dev(c.noisy, torch.float32)
    a, ra = fgbd.denoise(xyz, rgb, prm)
    b, rb = fgbd.denoise(xyz, rgb, prm)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(ra, rb)


@pytest.fixture(scope="module")
def large_cloud():
    return synth.body_cloud(1000, sigma=20.0)


def test_denoise_large_frame(large_cloud):
    """The 1M-point frame of the benchmark, in the benchmark's configuration."""
    c = large_cloud
    out, r, o = check_denoise(c.xyz, c.noisy, fgbd.default_params())
    assert r["n_eff"] == c.n
    g, col, d2, p, _ = gpu_graph(c.xyz, fgbd.default_params())
    assert np.array_equal(col, o["col"]) and np.array_equal(d2, o["dist2"])


# ------------------------------------------------------- polynomial filter

def _poly_case(seed, ncoef=8):
    c = synth.tiny_cloud(0)
    prm = fgbd.default_params(bits=8)
    g = fgbd.build_slg(dev(c.xyz, torch.int32), prm)
    rng = np.random.default_rng(seed)
    coef = rng.uniform(-0.5, 1.0, size=ncoef)
    sg = 1.7
    go = rng.standard_normal((c.n, 3))
    return c, g, coef, sg, go


@pytest.mark.parametrize("ncoef", [1, 2, 8])
def test_poly_filter_forward_and_adjoint(ncoef):
    c, g, coef, sg, go = _poly_case(ncoef, ncoef)
    x = dev(c.noisy, torch.float32)
    ct = dev(coef, torch.float32)
    st = torch.tensor(sg, dtype=torch.float64, device="cuda")
    out, saved = fgbd.poly_filter(g, x, ct, st)
    gx, gc, gs = fgbd.poly_filter_backward(g, saved, ct, st, dev(go, torch.float32))
    torch.cuda.synchronize()
    col, d2 = g.col.cpu().numpy(), g.dist2.cpu().numpy()
    coef32 = coef.astype(np.float32).astype(np.float64)
    ref = O.poly_filter(col, d2, c.noisy, coef32, sg)
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= COLOUR_TOL
    rx, rc, rs = O.poly_filter_grads(col, d2, c.noisy, coef32, sg, go.astype(np.float32))
    gxn = gx.cpu().numpy()
    assert np.max(np.abs(gxn - rx)) <= 1e-3 * max(1.0, np.max(np.abs(rx)))
    assert np.allclose(gc.cpu().numpy(), rc, rtol=1e-3, atol=1e-3 * np.max(np.abs(rc)))
    assert math.isclose(float(gs), rs, rel_tol=1e-3, abs_tol=1e-3 * max(1.0, abs(rs)))


def test_graph_transpose_matches_numpy():
    """fgbd_graph_transpose: for every point the ids of the edges pointing at
    it, ascending, against a numpy construction."""
    for prm in (fgbd.default_params(bits=8), fgbd.default_params(bits=8, k=5, num_dirs=3, window=1)):
        c = synth.tiny_cloud(0)
        g = fgbd.build_slg(dev(c.xyz, torch.int32), prm)
        off, edge = fgbd.graph_transpose(g)
        torch.cuda.synchronize()
        col = g.col.cpu().numpy().ravel()
        e = np.nonzero(col >= 0)[0]
        tgt = col[e]
        order = np.lexsort((e, tgt))
        exp_off = np.concatenate([[0], np.cumsum(np.bincount(tgt, minlength=g.n))])
        off = off.cpu().numpy()
        assert np.array_equal(off, exp_off)
        assert np.array_equal(edge.cpu().numpy()[:off[-1]], e[order])


def test_poly_backward_given_or_built_transpose_same_bits():
    """The backward with the graph's cached transpose, with one built inside
    the call, and twice in a row: bit-identical (fixed-order sums)."""
    c, g, coef, sg, go = _poly_case(5)
    x = dev(c.noisy, torch.float32)
    ct = dev(coef, torch.float32)
    st = torch.tensor(sg, dtype=torch.float64, device="cuda")
    _, saved = fgbd.poly_filter(g, x, ct, st)
    gt = dev(go, torch.float32)
    a = fgbd.poly_filter_backward(g, saved, ct, st, gt)
    b = fgbd.poly_filter_backward(g, saved, ct, st, gt, transpose=False)
    c2 = fgbd.poly_filter_backward(g, saved, ct, st, gt)
    torch.cuda.synchronize()
    for u, v in ((a, b), (a, c2)):
        for s, t in zip(u, v):
            assert torch.equal(s, t)


def test_poly_filter_e_q_is_eq5():
    c, g, _, _, _ = _poly_case(0)
    prm = fgbd.default_params(bits=8)
    x = dev(c.noisy, torch.float32)
    sg = fgbd.read_result(g.result)["sigma_g"]
    st = torch.tensor(sg, dtype=torch.float64, device="cuda")
    for q in (0, 3):
        coef = torch.zeros(5, dtype=torch.float32, device="cuda")
        coef[q] = 1.0
        out, _ = fgbd.poly_filter(g, x, coef, st)
        ref, _ = fgbd.filter(g, x, prm, q_fixed=q)
        torch.cuda.synchronize()
        assert torch.max(torch.abs(out - ref)).item() <= 1e-4


def test_poly_autograd_function():
    c, g, coef, sg, go = _poly_case(3)
    x = dev(c.noisy, torch.float32).requires_grad_(True)
    ct = dev(coef, torch.float32).requires_grad_(True)
    st = torch.tensor(sg, dtype=torch.float64, device="cuda", requires_grad=True)
    out = fgbd.poly_filter_autograd(x, ct, st, g)
    (out * dev(go, torch.float32)).sum().backward()
    torch.cuda.synchronize()
    col, d2 = g.col.cpu().numpy(), g.dist2.cpu().numpy()
    rx, rc, rs = O.poly_filter_grads(col, d2, c.noisy, coef.astype(np.float32), sg, go.astype(np.float32))
    assert np.max(np.abs(x.grad.cpu().numpy() - rx)) <= 1e-3 * max(1.0, np.max(np.abs(rx)))
    assert np.allclose(ct.grad.cpu().numpy(), rc, rtol=1e-3, atol=1e-3 * np.max(np.abs(rc)))
    assert math.isclose(float(st.grad), rs, rel_tol=1e-3)
