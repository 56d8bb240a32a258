"""The per-frame path on inputs whose point order is far from spatial.

When more than a quarter of a cloud's kept edges join points that lie far
apart in the input numbering (more than a sixteenth of the cloud and more
than 4096 indices), the path renumbers that cloud along scan order 0 after
the graph is built (the selection still breaks ties by input index), runs the
noise estimate and the sweeps in that numbering and writes the output back in
input order; the cloud's result carries FGBD_ST_RELABELED.  Every case is checked against the oracle
on the input as given, to the usual bars (colours within 1e-3, sigma_est
within 1e-3, sigma_g to FP64 rounding, q equal or a near-tie).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2401_09721_amd import fgbd, synth  # noqa: E402

pytestmark = pytest.mark.gpu

from gpu_helpers import COLOUR_TOL, compare_denoise, dev, oracle_params  # noqa: E402


def _run(xyz, rgb, prm):
    out, res = fgbd.denoise(dev(xyz, torch.int32), dev(rgb, torch.float32), prm)
    torch.cuda.synchronize()
    r = fgbd.read_result(res)
    compare_denoise(out.cpu().numpy(), r, xyz, rgb, prm)
    return r


def test_shuffled_cloud_is_relabelled_raster_is_not():
    c = synth.random_shapes_cloud(11, bits=8, target=15000)
    prm = fgbd.default_params(bits=8)
    r = _run(c.xyz, c.noisy, prm)
    assert not r["status"] & fgbd.FGBD_ST_RELABELED
    perm = np.random.default_rng(3).permutation(c.n)
    r2 = _run(c.xyz[perm], c.noisy[perm], prm)
    assert r2["status"] & fgbd.FGBD_ST_RELABELED


@pytest.mark.parametrize("L,w,K,P", [(3, 1, 6, 0), (8, 2, 12, 6), (4, 4, 5, 5)])
def test_relabelled_variants(L, w, K, P):
    """Other graphs and the generic (non-fused) noise and sweep kernels."""
    c = synth.random_shapes_cloud(12, bits=8, target=16000, shuffle=True)
    r = _run(c.xyz, c.noisy, fgbd.default_params(bits=8, num_dirs=L, window=w, k=K, patch=P))
    assert r["status"] & fgbd.FGBD_ST_RELABELED


def test_index_ordered_patch_is_never_relabelled():
    """The unsorted-patch ablation orders patch entries by input index, so it
    keeps the input numbering."""
    c = synth.random_shapes_cloud(13, bits=8, target=9000, shuffle=True)
    r = _run(c.xyz, c.noisy, fgbd.default_params(bits=8, patch_order=1))
    assert not r["status"] & fgbd.FGBD_ST_RELABELED


def test_relabelled_large_frame():
    """The 1M-point frame in a random order."""
    c = synth.body_cloud(synth.config_seed(1), target=1_000_000, sigma=20.0)
    perm = np.random.default_rng(20240117).permutation(c.n)
    r = _run(c.xyz[perm], c.noisy[perm], fgbd.default_params())
    assert r["status"] & fgbd.FGBD_ST_RELABELED


def test_relabelled_batch_and_fixed_q():
    """A batch of two shuffled clouds and one raster cloud, and a shuffled
    cloud of 3000 points (below the 4096-index gap: never renumbered): the
    full call and the periodic mode's fixed-q call, each cloud against the
    oracle on it alone; only the shuffled large clouds are renumbered."""
    clouds = [synth.random_shapes_cloud(20, bits=8, target=16000, shuffle=True),
              synth.random_shapes_cloud(21, bits=8, target=12000),
              synth.random_shapes_cloud(22, bits=8, target=20000, shuffle=True),
              synth.random_shapes_cloud(23, bits=8, target=3000, shuffle=True)]
    expect = [True, False, True, False]
    prm = fgbd.default_params(bits=8)
    offs = np.concatenate([[0], np.cumsum([c.n for c in clouds])]).astype(np.int64)
    xyz = dev(np.concatenate([c.xyz for c in clouds]), torch.int32)
    rgb = dev(np.concatenate([c.noisy for c in clouds]), torch.float32)
    off = dev(offs, torch.int64)
    out, res = fgbd.denoise_batched(xyz, rgb, off, prm)
    outq, resq = fgbd.denoise_batched_fixed_q(xyz, rgb, off, 3, prm)
    torch.cuda.synchronize()
    out, outq = out.cpu().numpy(), outq.cpu().numpy()
    recs, recq = fgbd.read_results(res), fgbd.read_results(resq)
    for s, c in enumerate(clouds):
        assert bool(recs[s]["status"] & fgbd.FGBD_ST_RELABELED) == expect[s]
        assert bool(recq[s]["status"] & fgbd.FGBD_ST_RELABELED) == expect[s]
        compare_denoise(out[offs[s]:offs[s + 1]], recs[s], c.xyz, c.noisy, prm)
        ores = O.denoise(c.xyz, c.noisy, oracle_params(prm), q_fixed=3)
        assert np.max(np.abs(outq[offs[s]:offs[s + 1]] - ores["out"])) <= COLOUR_TOL
        # a cloud in a batch gets what it gets alone
        o1, r1 = fgbd.denoise(dev(c.xyz, torch.int32), dev(c.noisy, torch.float32), prm)
        torch.cuda.synchronize()
        assert fgbd.read_result(r1)["status"] == recs[s]["status"]
        assert np.max(np.abs(o1.cpu().numpy() - out[offs[s]:offs[s + 1]])) <= 1e-4


def test_captured_call_follows_each_frames_order():
    """One capture replayed on a raster frame and on a shuffled one: the
    renumbering is decided on the device per replay, and every replay equals
    an eager call bit for bit."""
    prm = fgbd.default_params(bits=8)
    c = synth.random_shapes_cloud(31, bits=8, target=16000)
    perm = np.random.default_rng(5).permutation(c.n)
    cap = c.n
    ctx = fgbd.Context("cuda")
    ctx.reserve(prm, cap, 1)
    xyz_s = torch.zeros((cap, 3), dtype=torch.int32, device="cuda")
    rgb_s = torch.zeros((cap, 3), dtype=torch.float32, device="cuda")
    off_s = torch.tensor([0, cap], dtype=torch.int64, device="cuda")
    out_s = torch.zeros((cap, 3), dtype=torch.float32, device="cuda")
    res_s = fgbd.new_result("cuda", 1)
    xyz_s.copy_(dev(c.xyz, torch.int32))
    rgb_s.copy_(dev(c.noisy, torch.float32))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fgbd.denoise_batched(xyz_s, rgb_s, off_s, prm, ctx=ctx, out=out_s, res=res_s)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        fgbd.denoise_batched(xyz_s, rgb_s, off_s, prm, ctx=ctx, out=out_s, res=res_s)
    torch.cuda.synchronize()
    for xyz, rgb, relabel in ((c.xyz[perm], c.noisy[perm], True), (c.xyz, c.noisy, False),
                              (c.xyz[perm], c.noisy[perm], True)):
        xyz_s.copy_(dev(xyz, torch.int32))
        rgb_s.copy_(dev(rgb, torch.float32))
        graph.replay()
        torch.cuda.synchronize()
        got, got_r = out_s.cpu().numpy().copy(), fgbd.read_results(res_s)[0]
        ref_out, ref_res = fgbd.denoise_batched(xyz_s, rgb_s, off_s, prm, ctx=ctx)
        torch.cuda.synchronize()
        assert np.array_equal(got, ref_out.cpu().numpy())
        assert got_r == fgbd.read_results(ref_res)[0]
        assert bool(got_r["status"] & fgbd.FGBD_ST_RELABELED) == relabel
        compare_denoise(got, got_r, xyz, rgb, prm)
    ctx.close()
