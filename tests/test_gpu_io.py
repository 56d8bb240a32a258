"""The steps on either side of the path: float coordinates onto the voxel grid
(fgbd_quantize) and filtered colours to 8 bits (fgbd_round_u8), bit-exact
against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_2401_09721_amd import fgbd, synth  # noqa: E402

from gpu_helpers import compare_denoise, dev  # noqa: E402

pytestmark = pytest.mark.gpu


def check_quantize(x, bits):
    g, frame = fgbd.quantize(dev(x, torch.float32), bits)
    og, (lo, s) = O.quantize(x, bits)
    assert np.array_equal(g.cpu().numpy(), og)
    f = frame.cpu().numpy()
    assert f[3] == s
    assert np.array_equal(f[:3], lo, equal_nan=True)
    return og


@pytest.mark.parametrize("n,bits", [(0, 10), (1, 10), (2, 1), (1000, 7), (300_001, 10), (65_537, 21)])
def test_quantize_matches_oracle(n, bits):
    rng = np.random.default_rng(n + bits)
    x = rng.normal(0.0, 1.0, size=(n, 3)).astype(np.float32) * np.float32([3.0, 1.0, 0.5]) + np.float32(-12.0)
    check_quantize(x, bits)


def test_quantize_degenerate_and_nan():
    check_quantize(np.full((777, 3), 2.5, np.float32), 10)
    x = np.random.default_rng(1).uniform(-1, 1, size=(5000, 3)).astype(np.float32)
    x[::7, 1] = np.nan
    x[3, :] = np.nan
    g = check_quantize(x, 9)
    assert (g[::7, 1] == 0).all()


def test_quantized_capture_denoises_like_the_oracle():
    # a voxel capture seen as floats (voxel centres plus sub-voxel jitter),
    # quantised back to the grid and run through the whole path
    c = synth.random_shapes_cloud(9, bits=8, target=12000)
    rng = np.random.default_rng(2)
    xf = (c.xyz + rng.uniform(0.05, 0.95, size=c.xyz.shape)).astype(np.float32) * np.float32(0.01)
    g = check_quantize(xf, 8)
    prm = fgbd.default_params(bits=8)
    xyz = dev(g, torch.int32)
    rgb = dev(c.noisy, torch.float32)
    out, res = fgbd.denoise(xyz, rgb, prm)
    torch.cuda.synchronize()
    compare_denoise(out.cpu().numpy(), fgbd.read_result(res), g, c.noisy, prm)


@pytest.mark.parametrize("n", [0, 1, 5, 100_003])
def test_round_u8_matches_oracle(n):
    rng = np.random.default_rng(n)
    v = rng.uniform(-20.0, 275.0, size=(n, 3)).astype(np.float32)
    if n >= 5:
        v.flat[:12] = [0.5, 1.5, 2.5, -0.5, 254.5, 255.5, np.nan, np.inf, -np.inf, 127.5, 128.5, 3.4999998][: min(12, v.size)]
        v[n // 2:] = np.round(v[n // 2:] * 2) / 2  # many exact halves
    out = fgbd.round_u8(dev(v, torch.float32))
    assert out.dtype == torch.uint8 and tuple(out.shape) == (n, 3)
    assert np.array_equal(out.cpu().numpy(), O.round_u8(v))


@pytest.mark.parametrize("q", [0, 1, 4])
@pytest.mark.parametrize("kind", ["tiny", "shapes"])
def test_smooth_geometry_matches_oracle(q, kind):
    c = synth.tiny_cloud(0) if kind == "tiny" else synth.random_shapes_cloud(8, bits=8, target=20000, shuffle=True)
    prm = fgbd.default_params(bits=8)
    out, res = fgbd.smooth_geometry(dev(c.xyz, torch.int32), q, prm)
    torch.cuda.synchronize()
    r = fgbd.read_result(res)
    o = O.smooth_geometry(c.xyz, q, dict(bits=8))
    assert r["q"] == q
    assert abs(r["sigma_g"] - o["sigma_g"]) <= 1e-12 * o["sigma_g"]
    # FP32 sweeps on coordinates below 2^8: a few units in the last place per sweep
    tol = 2.0 ** 8 * 2.0 ** -20 * (q + 2)
    err = float(np.max(np.abs(out.cpu().numpy() - o["out"])))
    assert err <= tol, f"max coordinate error {err} > {tol}"


@pytest.mark.parametrize("n", [0, 1, 2, 9, 4097])
def test_smooth_geometry_edge_sizes(n):
    rng = np.random.default_rng(n + 100)
    g = rng.integers(0, 64, size=(n, 3)).astype(np.int32)
    prm = fgbd.default_params(bits=6)
    out, res = fgbd.smooth_geometry(dev(g, torch.int32), 2, prm)
    torch.cuda.synchronize()
    r = fgbd.read_result(res)
    o = O.smooth_geometry(g, 2, dict(bits=6))
    assert tuple(out.shape) == (n, 3)
    assert abs(r["sigma_g"] - o["sigma_g"]) <= 1e-12 * max(o["sigma_g"], 1.0)
    if n:
        err = float(np.max(np.abs(out.cpu().numpy() - o["out"])))
        assert err <= 2.0 ** 6 * 2.0 ** -20 * 4
