"""Seeded synthetic point clouds with noisy colour (inputs only).

The paper evaluates on voxelised human-body captures of about one million points
with 8-bit colour and additive Gaussian colour noise of standard deviation 10, 20
or 30 (Sec. 3.1, "Datasets").  Those captures are not available here, so every
input is generated from a seed with the same structure:

* geometry: thin shells of rotated ellipsoids and planar rectangles on a 2^b
  integer voxel grid.  A voxel is occupied when it contains at least one point of
  a dense regular sampling of a surface (sample spacing below half a voxel), and
  duplicates are removed, so the cloud is a one-voxel-thick shell like a
  voxelised capture (Sec. 2.2 assumes integer coordinates).  Points are returned
  in lexicographic (x, y, z) order, the order a voxeliser typically emits;
* colour: per channel, 128 plus a sum of four random low-frequency 3-D
  sinusoids (frequencies in cycles per 256 voxels, so the texture scale is the
  same on 2^8 and 2^10 grids), rounded and clipped to 0..255;
* patterned colour (quality measurements only): the smooth colour plus a
  constant random offset per cubic cell, which adds sharp colour edges;
* noise: i.i.d. Gaussian of a given sigma added to the clean colour and clipped
  to 0..255, kept in float32 without rounding.

This module holds none of the denoising arithmetic.  It is shared by the CPU
oracle tests, the GPU tests and the benchmark so that both sides see identical
inputs.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Cloud",
    "ellipsoid_shell",
    "plane_shell",
    "procedural_colour",
    "add_noise",
    "tiny_cloud",
    "body_cloud",
    "random_shapes_cloud",
    "moved_body_frame",
    "config_seed",
]

_SPACING = 0.4  # surface sample spacing in voxels


@dataclasses.dataclass
class Cloud:
    """One synthetic frame.  ``xyz`` int32 [N,3]; ``clean`` uint8 [N,3];
    ``noisy`` float32 [N,3] on the 0..255 scale; ``sigma`` the injected noise."""

    xyz: np.ndarray
    clean: np.ndarray
    noisy: np.ndarray
    sigma: float
    bits: int
    seed: int

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


def config_seed(config: int, cloud: int = 0, frame: int = 0) -> int:
    """Seed convention: config index x 1000 + cloud index x 100 + frame index."""
    return config * 1000 + cloud * 100 + frame


def _random_rotation(rng: np.random.Generator, max_angle: float | None = None) -> np.ndarray:
    """Uniform random rotation (QR of a Gaussian matrix), or a rotation about a
    random axis by an angle uniform in [0, max_angle] when ``max_angle`` is set."""
    if max_angle is None:
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        q = q * np.sign(np.diag(r))
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        return q
    axis = rng.standard_normal(3)
    axis /= np.linalg.norm(axis)
    ang = rng.uniform(0.0, max_angle)
    kx = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * kx + (1 - math.cos(ang)) * (kx @ kx)


def ellipsoid_shell(center, radii, rot, spacing: float = _SPACING) -> np.ndarray:
    """Sample points on the ellipsoid {c + R diag(r) s : |s| = 1} with neighbouring
    samples at most ``spacing`` voxels apart; returns float64 [M,3]."""
    center = np.asarray(center, np.float64)
    radii = np.asarray(radii, np.float64)
    rmax = float(radii.max())
    n_theta = max(2, int(math.ceil(math.pi * rmax / spacing)) + 1)
    theta = np.linspace(0.0, math.pi, n_theta)
    n_phi = np.maximum(1, np.ceil(2 * math.pi * rmax * np.sin(theta) / spacing).astype(np.int64))
    ring = np.repeat(np.arange(n_theta), n_phi)
    start = np.cumsum(n_phi) - n_phi
    k = np.arange(ring.size) - np.repeat(start, n_phi)
    phi = 2 * math.pi * k / np.repeat(n_phi, n_phi)
    th = theta[ring]
    s = np.stack([np.sin(th) * np.cos(phi), np.sin(th) * np.sin(phi), np.cos(th)], axis=1)
    return center + (s * radii) @ np.asarray(rot, np.float64).T


def plane_shell(center, half_extent, rot, spacing: float = _SPACING) -> np.ndarray:
    """Sample a planar rectangle with half extents (a, b) along the first two
    columns of ``rot``, centred at ``center``; returns float64 [M,3]."""
    center = np.asarray(center, np.float64)
    rot = np.asarray(rot, np.float64)
    a, b = float(half_extent[0]), float(half_extent[1])
    na = max(2, int(math.ceil(2 * a / spacing)) + 1)
    nb = max(2, int(math.ceil(2 * b / spacing)) + 1)
    u, v = np.meshgrid(np.linspace(-a, a, na), np.linspace(-b, b, nb), indexing="ij")
    return center + np.outer(u.ravel(), rot[:, 0]) + np.outer(v.ravel(), rot[:, 1])


def _voxelise(samples: list[np.ndarray], bits: int) -> np.ndarray:
    """Occupied voxels (floor of the samples) inside [0, 2^bits)^3, deduplicated,
    in lexicographic (x, y, z) order; int32 [N,3]."""
    side = 1 << bits
    keys = []
    for s in samples:
        v = np.floor(s).astype(np.int64)
        ok = np.all((v >= 0) & (v < side), axis=1)
        v = v[ok]
        keys.append(np.unique((v[:, 0] << (2 * bits)) | (v[:, 1] << bits) | v[:, 2]))
    key = np.unique(np.concatenate(keys)) if keys else np.zeros(0, np.int64)
    mask = side - 1
    return np.stack([key >> (2 * bits), (key >> bits) & mask, key & mask], axis=1).astype(np.int32)


def procedural_colour(xyz: np.ndarray, rng: np.random.Generator, terms: int = 4) -> np.ndarray:
    """uint8 [N,3]: per channel round(128 + sum_k A_k sin(2 pi <nu_k, g>/256 + phi_k))
    clipped to 0..255, with A_k ~ U[16, 31.75], nu_k in {-8..8}^3 minus 0."""
    g = xyz.astype(np.float64)
    out = np.empty((xyz.shape[0], 3), np.float64)
    for c in range(3):
        acc = np.full(xyz.shape[0], 128.0)
        for _ in range(terms):
            amp = rng.uniform(16.0, 31.75)
            while True:
                nu = rng.integers(-8, 9, size=3)
                if np.any(nu != 0):
                    break
            ph = rng.uniform(0.0, 2 * math.pi)
            acc += amp * np.sin(2 * math.pi * (g @ nu) / 256.0 + ph)
        out[:, c] = acc
    return np.clip(np.rint(out), 0, 255).astype(np.uint8)


def add_noise(clean: np.ndarray, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """float32(clip(clean + N(0, sigma^2), 0, 255)), no rounding."""
    noisy = clean.astype(np.float64) + rng.normal(0.0, sigma, size=clean.shape)
    return np.clip(noisy, 0.0, 255.0).astype(np.float32)


def _shapes_to_cloud(shapes, scale: float, bits: int) -> np.ndarray:
    side = float(1 << bits)
    mid = side / 2.0
    samples = []
    for kind, c, ext, rot in shapes:
        c = mid + (np.asarray(c) * side - mid) * scale
        ext = np.asarray(ext) * side * scale
        if kind == "e":
            samples.append(ellipsoid_shell(c, ext, rot))
        else:
            samples.append(plane_shell(c, ext, rot))
    return _voxelise(samples, bits)


def _fit_scale(shapes, bits: int, target: int | None):
    """Scale the shapes about the grid centre so the voxel count is within 1.5 %
    of ``target`` (count grows roughly with the square of the scale).  Returns
    (xyz, scale)."""
    scale = 1.0
    xyz = _shapes_to_cloud(shapes, scale, bits)
    if target is None or xyz.shape[0] == 0:
        return xyz, scale
    for _ in range(6):
        n = xyz.shape[0]
        if abs(n - target) <= 0.015 * target:
            break
        scale *= math.sqrt(target / n)
        xyz = _shapes_to_cloud(shapes, scale, bits)
    return xyz, scale


def _finish(xyz, bits, sigma, seed, rng, shuffle=False) -> Cloud:
    if shuffle:
        xyz = xyz[rng.permutation(xyz.shape[0])]
    clean = procedural_colour(xyz, rng)
    noisy = add_noise(clean, sigma, rng)
    return Cloud(np.ascontiguousarray(xyz, np.int32), clean, noisy, float(sigma), bits, seed)


def random_shapes_cloud(seed: int, bits: int = 8, n_ellipsoids: int = 3, target: int | None = 16000,
                        sigma: float = 20.0, shuffle: bool = False) -> Cloud:
    """Union of ``n_ellipsoids`` randomly rotated ellipsoid shells with seeded
    centres and radii (fractions of the grid side), scaled to about ``target``
    points."""
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(n_ellipsoids):
        c = rng.uniform(0.3, 0.7, size=3)
        r = rng.uniform(0.1, 0.28, size=3)
        shapes.append(("e", c, r, _random_rotation(rng)))
    xyz, _ = _fit_scale(shapes, bits, target)
    return _finish(xyz, bits, sigma, seed, rng, shuffle)


def tiny_cloud(seed: int = 0, sigma: float = 20.0) -> Cloud:
    """About 16k points on a 2^8 grid from 3 random ellipsoids, sigma 20."""
    return random_shapes_cloud(seed, bits=8, n_ellipsoids=3, target=16000, sigma=sigma)


def _body_shapes(rng: np.random.Generator, pose: np.ndarray | None = None, shift=None):
    """Six ellipsoids (torso, head, neck, two upper arms, hips) and two planes,
    in grid fractions, each jittered by the seed; y is the vertical axis."""
    j = lambda s: 1.0 + rng.uniform(-s, s)  # noqa: E731
    parts = [
        ("e", (0.50, 0.52, 0.50), (0.17 * j(.05), 0.22 * j(.05), 0.10 * j(.05))),  # torso
        ("e", (0.50, 0.86, 0.50), (0.07 * j(.05), 0.085 * j(.05), 0.08 * j(.05))),  # head
        ("e", (0.50, 0.75, 0.50), (0.04 * j(.05), 0.06 * j(.05), 0.04 * j(.05))),  # neck
        ("e", (0.27, 0.55, 0.50), (0.045 * j(.05), 0.17 * j(.05), 0.045 * j(.05))),  # left arm
        ("e", (0.73, 0.55, 0.50), (0.045 * j(.05), 0.17 * j(.05), 0.045 * j(.05))),  # right arm
        ("e", (0.50, 0.28, 0.50), (0.16 * j(.05), 0.10 * j(.05), 0.10 * j(.05))),  # hips
    ]
    shapes = []
    for kind, c, r in parts:
        c = np.asarray(c) + rng.uniform(-0.01, 0.01, size=3)
        shapes.append((kind, c, np.asarray(r), _random_rotation(rng, max_angle=0.15)))
    for _ in range(2):
        c = np.array([rng.uniform(0.35, 0.65), rng.uniform(0.3, 0.7), rng.uniform(0.62, 0.70)])
        shapes.append(("p", c, np.array([rng.uniform(0.08, 0.14), rng.uniform(0.10, 0.18)]),
                       _random_rotation(rng, max_angle=0.5)))
    if pose is not None:
        mid = np.full(3, 0.5)
        moved = []
        for kind, c, ext, rot in shapes:
            moved.append((kind, mid + pose @ (c - mid) + shift, ext, pose @ rot))
        shapes = moved
    return shapes


def body_cloud(seed: int = 1000, bits: int = 10, target: int | None = 1_000_000, sigma: float = 20.0,
               shuffle: bool = False) -> Cloud:
    """Upper-body-like shell: 6 ellipsoids plus 2 planes on a 2^bits grid,
    about ``target`` points."""
    rng = np.random.default_rng(seed)
    shapes = _body_shapes(rng)
    xyz, _ = _fit_scale(shapes, bits, target)
    return _finish(xyz, bits, sigma, seed, rng, shuffle)


def patched_body_cloud(seed: int = 1000, bits: int = 10, target: int | None = 1_000_000, sigma: float = 20.0,
                       cell: int = 32, amp: float = 48.0) -> Cloud:
    """body_cloud's geometry and smooth colour plus a constant offset per cubic
    cell of ``cell`` voxels (U[-amp, amp] per cell and channel), rounded and
    clipped to 0..255.  The offsets put sharp colour edges on the cell faces,
    like printed patterns on clothing, which the smooth texture alone lacks."""
    rng = np.random.default_rng(seed)
    shapes = _body_shapes(rng)
    xyz, _ = _fit_scale(shapes, bits, target)
    xyz = np.ascontiguousarray(xyz, np.int32)
    clean = procedural_colour(xyz, rng).astype(np.float64)
    g = -(-(1 << bits) // cell)
    c = xyz.astype(np.int64) // cell
    offs = rng.uniform(-amp, amp, size=(g * g * g, 3))
    clean = np.clip(np.rint(clean + offs[(c[:, 0] * g + c[:, 1]) * g + c[:, 2]]), 0, 255).astype(np.uint8)
    noisy = add_noise(clean, sigma, rng)
    return Cloud(xyz, clean, noisy, float(sigma), bits, seed)


def moved_body_frame(seed: int, frame: int, bits: int = 10, target: int = 1_000_000,
                     sigma: float = 20.0, scale: float | None = None):
    """Frame ``frame`` of a sequence: the body of ``seed`` rigidly moved by
    ``frame`` seeded small steps (each a rotation about a random axis by up to 1
    degree and a translation of up to 2 voxels per axis), re-voxelised, with the
    colour texture fixed by the seed and fresh noise per frame.  The shape scale
    is fitted once on frame 0 (pass it back in as ``scale`` to skip the fit).
    Returns (cloud, scale)."""
    rng = np.random.default_rng(seed)
    base_state = rng.bit_generator.state
    shapes = _body_shapes(rng)
    if scale is None:
        _, scale = _fit_scale(shapes, bits, target)
    motion = np.random.default_rng(seed + 7)
    pose = np.eye(3)
    shift = np.zeros(3)
    side = float(1 << bits)
    for _ in range(frame):
        r = _random_rotation(motion, max_angle=math.radians(1.0))
        t = motion.uniform(-2.0, 2.0, size=3) / side
        pose = r @ pose
        shift = r @ shift + t
    rng.bit_generator.state = base_state
    shapes = _body_shapes(rng, pose=pose, shift=shift)
    xyz = _shapes_to_cloud(shapes, scale, bits)
    clean = procedural_colour(xyz, np.random.default_rng(seed + 11))
    noisy = add_noise(clean, sigma, np.random.default_rng(seed * 1000 + 13 + frame))
    cloud = Cloud(np.ascontiguousarray(xyz, np.int32), clean, noisy, float(sigma), bits, seed + frame)
    return cloud, scale


def batched_specs(seed: int = 2000, count: int = 8, lo: int = 200_000, hi: int = 1_200_000,
                  sigma_lo: float = 5.0, sigma_hi: float = 35.0) -> list[dict]:
    """Arguments of ``body_cloud`` for a batch of independently seeded clouds
    whose sizes are uniform in [lo, hi] and noise levels uniform in
    [sigma_lo, sigma_hi]."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi + 1, size=count)
    sigmas = rng.uniform(sigma_lo, sigma_hi, size=count)
    return [dict(seed=seed + 100 * (s + 1), target=int(sizes[s]), sigma=float(sigmas[s])) for s in range(count)]
