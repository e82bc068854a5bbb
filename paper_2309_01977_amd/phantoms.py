"""Seeded synthetic SPECT workloads: phantoms, attenuation maps, Poisson data.

This module is the only one that both the HIP library's tests and the FP64
oracle use.  It holds no part of the reconstruction method: it voxelises
analytic shapes (cylinders, spheres, ellipsoids) by 4 x 4 x 4 supersampling,
and draws Poisson counts for an expected projection that the caller computes
with whichever projector it is checking.

The workloads stand in for the paper's SPECT data (Section 3.1 and Appendix A:
Lu-177 acquisitions with 128-bin projections at 0.48 cm, 60 to 120 angles,
OSEM with 6 or 8 subsets), which are not available here.

Conventions (shared with the library and the oracle):
  object arrays have shape (N, N, Nz), index [i][j][k] = (x, y, z), z fastest;
  voxel (i, j, k) is centred at ((i - c) dx, (j - c) dx, (k - cz) dx) cm with
  c = (N - 1) / 2 and cz = (Nz - 1) / 2; projections have shape (A, N, Nz).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

MASTER_SEED = 230901977


@dataclass
class Workload:
    """One reconstruction problem: geometry, OSEM schedule and data recipe."""
    name: str
    n: int
    nz: int
    n_angles: int
    voxel_cm: float = 0.48
    psf_a: float = 0.03
    psf_b: float = 0.1
    psf_nsigma: float = 4.0
    with_mu: bool = True
    n_iters: int = 4
    n_subsets: int = 8
    total_counts: float = 5e6
    seed_index: int = 1

    @property
    def object_shape(self) -> Tuple[int, int, int]:
        return (self.n, self.n, self.nz)

    @property
    def proj_shape(self) -> Tuple[int, int, int]:
        return (self.n_angles, self.n, self.nz)

    @property
    def voxel_angles(self) -> int:
        return self.n * self.n * self.nz * self.n_angles


# The two single-reconstruction workloads: a small 64^3 case without
# attenuation, and the 128^3, 120-angle case with attenuation.
C1 = Workload("osem_64cube_60ang", n=64, nz=64, n_angles=60, with_mu=False, n_iters=2,
              n_subsets=6, total_counts=1e6, seed_index=0)
C2 = Workload("osem_128cube_120ang_att", n=128, nz=128, n_angles=120, with_mu=True, n_iters=4,
              n_subsets=8, total_counts=5e6, seed_index=1)


# BSREM with the relative difference prior on the 128^3 data (the paper's
# examples run 40 iterations of 6 subsets with beta = 0.3, gamma = 2; here
# 40 iterations of the 8 subsets of the 120-angle acquisition).
C6 = Workload("bsrem_rdp_128cube_120ang_att", n=128, nz=128, n_angles=120, with_mu=True, n_iters=40,
              n_subsets=8, total_counts=5e6, seed_index=1)
RDP_BETA = 0.3
RDP_GAMMA = 2.0


# The differentiable-projector workload: a batch of 8 torso phantoms at the
# 128^3, 120-angle geometry; 10 unrolled OSEM subiterations (8 subsets) from
# a uniform image, loss = mean squared error to each phantom.
C4 = Workload("unrolled_osem_128cube_120ang_b8", n=128, nz=128, n_angles=120, with_mu=True,
              n_iters=1, n_subsets=8, total_counts=5e6, seed_index=3)
C4_BATCH = 8
C4_STEPS = 10


# The serving workload: requests drawn from three acquisition classes (the
# 64^3 and 128^3 workloads above and a 192 x 192 x 160 volume with 128
# angles), arriving as a Poisson stream of 20 requests per second.
C5_LARGE = Workload("osem_192x160_128ang_att", n=192, nz=160, n_angles=128, with_mu=True, n_iters=4,
                    n_subsets=8, total_counts=8e6, seed_index=4)
C5_RATE = 20.0


# The batched workload: 32 reconstructions of uneven sizes (transverse 64 to
# 192 voxels, 64 to 160 axial slices, 60 to 128 angles), each a torso phantom
# with its attenuation map, 4 iterations x 8 subsets.
C3_COUNT = 32


def c3_workloads(count: int = C3_COUNT) -> List[Workload]:
    """Seeded geometries of the batched workload (member i uses phantom and
    noise streams of its own, see member_rngs)."""
    rng, _ = rngs(2)
    out = []
    for i in range(count):
        n = int(rng.choice([64, 96, 128, 160, 192]))
        nz = 160 if n == 192 else int(rng.choice(np.arange(64, min(n, 160) + 1, 16)))
        a = int(rng.choice(np.arange(60, 129, 4)))
        out.append(Workload(f"batch_member_{i}_{n}x{n}x{nz}x{a}", n=n, nz=nz, n_angles=a, with_mu=True,
                            n_iters=4, n_subsets=8, total_counts=float(rng.uniform(1e6, 5e6)), seed_index=2))
    return out


def member_rngs(i: int) -> Tuple[np.random.Generator, np.random.Generator]:
    """(phantom rng, noise rng) of batched member i."""
    child = np.random.SeedSequence(MASTER_SEED).spawn(5)[2].spawn(C3_COUNT + 1)[i + 1]
    a, b = child.spawn(2)
    return np.random.default_rng(a), np.random.default_rng(b)


def make_member_phantom(w: Workload, i: int, ss: int = 2):
    """(f_true, mu) float32 torso phantom of batched member i, scaled to its grid."""
    rng, _ = member_rngs(i)
    act, mu_shapes = _torso(rng, (w.n * w.voxel_cm) / 61.44, n_spheres=10)
    f = voxelise(act, w.n, w.nz, w.voxel_cm, ss).astype(np.float32)
    mu = voxelise(mu_shapes, w.n, w.nz, w.voxel_cm, ss).astype(np.float32)
    return f, mu


def rngs(seed_index: int) -> Tuple[np.random.Generator, np.random.Generator]:
    """(phantom rng, noise rng) for workload ``seed_index``."""
    child = np.random.SeedSequence(MASTER_SEED).spawn(5)[seed_index]
    a, b = child.spawn(2)
    return np.random.default_rng(a), np.random.default_rng(b)


# ---------------------------------------------------------------- shapes ----

@dataclass
class Shape:
    kind: str                  # "cylinder" (axis along z), "sphere", "ellipsoid"
    centre: Tuple[float, float, float]
    size: Tuple[float, ...]    # cylinder (radius, half_length); sphere (r,); ellipsoid (a, b, c)
    value: float


def _inside(shape: Shape, x, y, z):
    cx, cy, cz = shape.centre
    if shape.kind == "cylinder":
        r, h = shape.size
        return ((x - cx) ** 2 + (y - cy) ** 2 <= r * r) & (np.abs(z - cz) <= h)
    if shape.kind == "sphere":
        (r,) = shape.size
        return (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 <= r * r
    if shape.kind == "ellipsoid":
        a, b, c = shape.size
        return ((x - cx) / a) ** 2 + ((y - cy) / b) ** 2 + ((z - cz) / c) ** 2 <= 1.0
    raise ValueError(shape.kind)


def _half_extent(shape: Shape):
    if shape.kind == "cylinder":
        r, h = shape.size
        return (r, r, h)
    if shape.kind == "sphere":
        return (shape.size[0],) * 3
    return tuple(shape.size)


def voxelise(shapes: Sequence[Shape], n: int, nz: int, voxel_cm: float, ss: int = 4) -> np.ndarray:
    """Painter's-order voxelisation (later shapes replace earlier ones) with
    ss^3 sub-samples per voxel; returns float64 (n, n, nz)."""
    c, cz = 0.5 * (n - 1), 0.5 * (nz - 1)
    acc = np.zeros((n, n, nz))
    offs = (np.arange(ss) + 0.5) / ss - 0.5
    for ox in offs:
        for oy in offs:
            for oz in offs:
                xs = (np.arange(n) - c + ox) * voxel_cm
                ys = (np.arange(n) - c + oy) * voxel_cm
                zs = (np.arange(nz) - cz + oz) * voxel_cm
                lab = np.zeros((n, n, nz))
                for sh in shapes:
                    ex = _half_extent(sh)
                    lo, hi = [], []
                    for ax, coords in enumerate((xs, ys, zs)):
                        lo.append(int(np.searchsorted(coords, sh.centre[ax] - ex[ax], "left")))
                        hi.append(int(np.searchsorted(coords, sh.centre[ax] + ex[ax], "right")))
                    if any(h <= l for l, h in zip(lo, hi)):
                        continue
                    X = xs[lo[0]:hi[0], None, None]
                    Y = ys[None, lo[1]:hi[1], None]
                    Z = zs[None, None, lo[2]:hi[2]]
                    m = _inside(sh, X, Y, Z)
                    view = lab[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
                    view[m] = sh.value
                acc += lab
    return acc / ss ** 3


# ------------------------------------------------------------- phantoms ----

def c1_shapes() -> List[Shape]:
    """Uniform cylinder (r 12 cm, |z| <= 12 cm, activity 1) with three hot
    spheres (r 1, 2, 3 cm, activity 8) 6 cm off-axis at azimuths 90, 210, 330."""
    shapes = [Shape("cylinder", (0.0, 0.0, 0.0), (12.0, 12.0), 1.0)]
    for r, az in zip((1.0, 2.0, 3.0), (90.0, 210.0, 330.0)):
        t = np.deg2rad(az)
        shapes.append(Shape("sphere", (6.0 * np.cos(t), 6.0 * np.sin(t), 0.0), (r,), 8.0))
    return shapes


def _torso(rng: np.random.Generator, scale: float = 1.0, n_spheres: int = 20):
    """Water cylinder (r 20, |z| <= 25 cm), bone rod, two lung ellipsoids and
    random hot spheres fully inside the cylinder; lengths scaled by ``scale``.
    Returns (activity shapes, attenuation shapes)."""
    R, H = 20.0 * scale, 25.0 * scale
    lungs = [Shape("ellipsoid", (sx * 8.0 * scale, 4.0 * scale, 8.0 * scale),
                   (4.5 * scale, 6.0 * scale, 10.0 * scale), 0.2) for sx in (-1.0, 1.0)]
    act = [Shape("cylinder", (0.0, 0.0, 0.0), (R, H), 1.0)] + lungs
    for _ in range(n_spheres):
        r = rng.uniform(1.0, 3.0) * scale
        while True:
            x, y = rng.uniform(-R, R, size=2)
            if np.hypot(x, y) + r <= R:
                break
        z = rng.uniform(-H + r, H - r)
        act.append(Shape("sphere", (x, y, z), (r,), 8.0))
    mu = [Shape("cylinder", (0.0, 0.0, 0.0), (R, H), 0.15),
          Shape("cylinder", (0.0, -10.0 * scale, 0.0), (1.5 * scale, 1e9), 0.25)]
    mu += [Shape(s.kind, s.centre, s.size, 0.04) for s in lungs]
    return act, mu


def make_phantom(w: Workload, ss: int = 4):
    """(f_true, mu or None) as float32 arrays for workload ``w``."""
    rng, _ = rngs(w.seed_index)
    if w.seed_index == 0:
        act = c1_shapes()
        mu_shapes = None
    else:
        scale = (w.n * w.voxel_cm) / 61.44
        act, mu_shapes = _torso(rng, scale)
    f = voxelise(act, w.n, w.nz, w.voxel_cm, ss).astype(np.float32)
    mu = None
    if w.with_mu:
        if mu_shapes is None:
            _, mu_shapes = _torso(rng, (w.n * w.voxel_cm) / 61.44, n_spheres=0)
        mu = voxelise(mu_shapes, w.n, w.nz, w.voxel_cm, ss).astype(np.float32)
    return f, mu


def make_phantom_batch(w: Workload, batch: int, ss: int = 4):
    """``batch`` different torso phantoms for the geometry of ``w``:
    (f_true, mu), each float32 of shape (batch, N, N, Nz)."""
    rng, _ = rngs(w.seed_index)
    scale = (w.n * w.voxel_cm) / 61.44
    fs, mus = [], []
    for _ in range(batch):
        act, mu_shapes = _torso(rng, scale)
        fs.append(voxelise(act, w.n, w.nz, w.voxel_cm, ss).astype(np.float32))
        mus.append(voxelise(mu_shapes, w.n, w.nz, w.voxel_cm, ss).astype(np.float32))
    return np.stack(fs), np.stack(mus)


def random_object(shape, rng: np.random.Generator, signed: bool = False) -> np.ndarray:
    """Seeded random test volume (uniform in [0, 1) or [-1, 1))."""
    a = rng.random(shape)
    if signed:
        a = 2 * a - 1
    return a.astype(np.float32)


def random_mu(shape, rng: np.random.Generator, scale: float = 0.2) -> np.ndarray:
    """Seeded random non-negative attenuation map in [0, scale) cm^-1."""
    return (scale * rng.random(shape)).astype(np.float32)


def poisson_counts(expected: np.ndarray, total_counts: float,
                   rng: np.random.Generator) -> np.ndarray:
    """Scale an expected projection to ``total_counts`` and draw Poisson counts."""
    e = np.asarray(expected, dtype=np.float64)
    lam = e * (total_counts / e.sum())
    return rng.poisson(np.maximum(lam, 0)).astype(np.float32)
