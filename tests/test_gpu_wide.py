"""Grids above 2^10 (b = 11..21): scan codes wider than 32 bits.

The radix sort then runs extra passes over the code's upper bits and the
selection reads candidate coordinates from the input with 64-bit squared
distances.  The graph must equal the oracle's bit for bit (dist2 saturates at
2^31 - 1, flagged FGBD_ST_DIST_CLAMPED, for neighbours more than 46340 voxels
apart), and the denoised colours stay within 1e-3 of the oracle's.  Clouds: the
tiny cloud's shapes scaled onto the large grid with seeded jitter and placed
near its middle, so codes use their upper bits.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2401_09721_amd import fgbd, synth  # noqa: E402

pytestmark = pytest.mark.gpu

from gpu_helpers import compare_denoise, dev  # noqa: E402

I32MAX = (1 << 31) - 1


def wide_cloud(bits, seed=40, target=6000):
    c8 = synth.random_shapes_cloud(seed, bits=8, target=target)
    rng = np.random.default_rng(seed + bits)
    s = 1 << (bits - 8)
    xyz = c8.xyz.astype(np.int64) * s + rng.integers(0, max(s // 2, 1), size=c8.xyz.shape)
    xyz = xyz + ((1 << bits) - 1 - xyz.max(0)) // 2
    assert xyz.min() >= 0 and xyz.max() < (1 << bits)
    return xyz.astype(np.int32), c8.noisy


@pytest.mark.parametrize("bits,L,K", [(11, 8, 8), (12, 8, 8), (16, 8, 8), (16, 12, 16), (20, 16, 8), (21, 3, 6),
                                      (20, 9, 32)])
def test_wide_graph_bitexact(bits, L, K):
    xyz, _ = wide_cloud(bits)
    prm = fgbd.default_params(bits=bits, num_dirs=L, k=K)
    g = fgbd.build_slg(dev(xyz, torch.int32), prm)
    torch.cuda.synchronize()
    ocol, od2 = O.slg_graph(xyz, bits, L, prm.window, K)
    assert np.array_equal(g.col.cpu().numpy(), ocol)
    assert np.array_equal(g.dist2.cpu().numpy(), np.minimum(od2, I32MAX))
    r = fgbd.read_result(g.result)
    assert bool(r["status"] & fgbd.FGBD_ST_DIST_CLAMPED) == bool(od2.max() > I32MAX)


@pytest.mark.parametrize("bits", [12, 16])
def test_wide_denoise_matches_oracle(bits):
    xyz, rgb = wide_cloud(bits, seed=41, target=9000)
    out, res = fgbd.denoise(dev(xyz, torch.int32), dev(rgb, torch.float32), fgbd.default_params(bits=bits))
    torch.cuda.synchronize()
    compare_denoise(out.cpu().numpy(), fgbd.read_result(res), xyz, rgb, fgbd.default_params(bits=bits))


def test_wide_batched_with_a_narrow_sized_cloud():
    """A batch on a 2^16 grid: a scaled cloud and a small one, each against
    the oracle alone."""
    a, ra = wide_cloud(16, seed=42, target=7000)
    b8 = synth.random_shapes_cloud(43, bits=8, target=3000)
    clouds = [(a, ra), (b8.xyz, b8.noisy)]
    prm = fgbd.default_params(bits=16)
    offs = np.concatenate([[0], np.cumsum([len(c[0]) for c in clouds])]).astype(np.int64)
    out, res = fgbd.denoise_batched(dev(np.concatenate([c[0] for c in clouds]), torch.int32),
                                    dev(np.concatenate([c[1] for c in clouds]), torch.float32),
                                    dev(offs, torch.int64), prm)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    recs = fgbd.read_results(res)
    for s, (xyz, rgb) in enumerate(clouds):
        compare_denoise(out[offs[s]:offs[s + 1]], recs[s], xyz, rgb, prm)


def test_quantized_float_capture_at_16_bits():
    """Float coordinates quantised onto a 2^16 grid, then the whole path."""
    c = synth.tiny_cloud(0)
    rng = np.random.default_rng(7)
    xf = (c.xyz.astype(np.float64) * 0.37 + rng.uniform(0, 0.3, c.xyz.shape)).astype(np.float32)
    g, frame = fgbd.quantize(dev(xf, torch.float32), 16)
    torch.cuda.synchronize()
    gq = g.cpu().numpy()
    assert np.array_equal(gq, O.quantize(xf, 16)[0])
    prm = fgbd.default_params(bits=16)
    out, res = fgbd.denoise(g, dev(c.noisy, torch.float32), prm)
    torch.cuda.synchronize()
    compare_denoise(out.cpu().numpy(), fgbd.read_result(res), gq, c.noisy, prm)


def test_far_points_clamp_dist2():
    top = (1 << 21) - 1
    xyz = np.array([[0, 0, 0], [top, 0, 0], [0, top, top], [5, 5, 5]], np.int32)
    prm = fgbd.default_params(bits=21, num_dirs=3, window=3, k=3)
    g = fgbd.build_slg(dev(xyz, torch.int32), prm)
    torch.cuda.synchronize()
    ocol, od2 = O.slg_graph(xyz, 21, 3, 3, 3)
    assert np.array_equal(g.col.cpu().numpy(), ocol)
    assert np.array_equal(g.dist2.cpu().numpy(), np.minimum(od2, I32MAX))
    assert fgbd.read_result(g.result)["status"] & fgbd.FGBD_ST_DIST_CLAMPED
