"""Input recipes: brain-slice / brain-volume phantoms, smooth random warps,
tumour-like lesions and initial momenta, all seeded.

Every array is built in float64 with ``numpy.random.default_rng(seed)`` and
handed out as float32 C-contiguous arrays, last axis = x (contiguous).
Smoothing uses ``scipy.ndimage.gaussian_filter`` and warping uses
``scipy.ndimage.map_coordinates(order=1, mode='nearest')``; neither is the
method's own kernel or interpolation code.

Workloads
---------
``c1``  2-D 64x64 disk -> shifted disk + blob, T=10, sigma=3, rho=0.5 (forward only).
``c2``  2-D 240x240 phantom -> warped phantom + lesion, T=20, sigma=5,
        rho in {1.0, 0.5, 0.1}.
``c3``  64 ragged 2-D pairs, H and W drawn independently from
        {96, 128, 192, 240, 320}, rho_i ~ U[0.05, 1], sigma_i ~ U[2, 6], T=20.
``c4``  3-D 160x192x160 phantom, T=15, sigma=4, rho=0.3.
``c5``  16 ragged 3-D volumes from {96^3, 128^3, 128x160x128, 160x192x160},
        rho_i ~ U[0.1, 1], sigma=4, T=15.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
from scipy import ndimage

SIZES_2D: Tuple[int, ...] = (96, 128, 192, 240, 320)
SHAPES_3D: Tuple[Tuple[int, int, int], ...] = (
    (96, 96, 96),
    (128, 128, 128),
    (128, 160, 128),
    (160, 192, 160),
)
LAMBDA = 0.01
P0_KINDS = ("zero", "random", "realistic")

# The "realistic" momentum is smooth Gaussian-filtered noise (filter width
# REALISTIC_SMOOTHING) scaled to REALISTIC_AMPLITUDE * sigma / REALISTIC_SIGMA_REF.
# The amplitude was chosen once, by shooting every pair of the ragged 2-D batch
# and several 3-D volumes, as about the largest for which every trajectory
# stays bounded: the residual term rho z builds steep intensity gradients out
# of a large z, and those feed the velocity back. Feet then sit off the grid
# everywhere, a few tenths of a pixel per step (up to ~0.6 px in 2-D).
REALISTIC_AMPLITUDE = {2: 25.0, 3: 25.0}
REALISTIC_SIGMA_REF = {2: 5.0, 3: 4.0}
REALISTIC_SMOOTHING = {2: 16.0, 3: 12.0}
# Same idea for the small test shapes (smoothing scaled to the extent).
SMALL_AMPLITUDE = {2: 8.0, 3: 8.0}
# Large-step regime of a batched workload: its pairs at T = LARGE_STEP_T with
# rho = 0 (LDDMM, whose transport keeps the image in range) and the realistic
# momentum scaled by LARGE_STEP_SCALE. Measured on the 2-D batch: median step
# 1.4 px (5-95 % 0.8-2.4 px, 71 % of steps in [1, 2) px, 12 % beyond); on the
# 3-D batch: median 1.2 voxel (5-95 % 0.6-1.8, 70 % of steps >= 1 voxel).
LARGE_STEP_T = 5
LARGE_STEP_SCALE = 16.0


@dataclass
class Pair:
    """One registration problem: source S, target J, initial momentum p0."""

    source: np.ndarray
    target: np.ndarray
    p0: np.ndarray
    rho: float
    sigma: float
    lam: float = LAMBDA
    meta: dict = field(default_factory=dict)

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(self.source.shape)

    @property
    def ndim(self) -> int:
        return self.source.ndim

    @property
    def size(self) -> int:
        return int(self.source.size)


@dataclass
class Workload:
    name: str
    pairs: List[Pair]
    T: int

    @property
    def voxel_steps(self) -> int:
        return sum(p.size for p in self.pairs) * self.T


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _grid(shape: Sequence[int]) -> List[np.ndarray]:
    return np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")


def gradient_noise(shape: Sequence[int], spacing: float, rng: np.random.Generator) -> np.ndarray:
    """Perlin-style gradient noise: seeded unit gradients on a lattice of the
    given spacing, quintic fade 6t^5 - 15t^4 + 10t^3, normalised to max |.| = 1."""
    d = len(shape)
    nodes = [int(np.ceil((n - 1) / spacing)) + 2 for n in shape]
    g = rng.standard_normal((d,) + tuple(nodes))
    g /= np.linalg.norm(g, axis=0, keepdims=True)
    coords = [c / spacing for c in _grid(shape)]
    base = [np.floor(c).astype(np.int64) for c in coords]
    frac = [c - b for c, b in zip(coords, base)]

    def fade(t):
        return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)

    faded = [fade(f) for f in frac]
    out = np.zeros(tuple(shape))
    for corner in itertools.product((0, 1), repeat=d):
        idx = tuple(b + c for b, c in zip(base, corner))
        dot = sum(g[a][idx] * (frac[a] - corner[a]) for a in range(d))
        wgt = np.ones(tuple(shape))
        for a in range(d):
            wgt = wgt * (faded[a] if corner[a] else 1.0 - faded[a])
        out += wgt * dot
    m = np.abs(out).max()
    return out / m if m > 0 else out


# Normalised semi-axes (per array axis) and intensities of the nested shells.
_SHELLS_2D = (((0.90, 0.80), 0.2), ((0.70, 0.60), 0.5), ((0.38, 0.30), 0.8))
_SHELLS_3D = (((0.80, 0.90, 0.80), 0.2), ((0.60, 0.70, 0.60), 0.5), ((0.30, 0.38, 0.30), 0.8))


def _normalised_coords(shape: Sequence[int]) -> List[np.ndarray]:
    return [(c - (n - 1) / 2.0) / (n / 2.0) for c, n in zip(_grid(shape), shape)]


def _inside(coords: List[np.ndarray], axes: Sequence[float]) -> np.ndarray:
    return sum((c / a) ** 2 for c, a in zip(coords, axes)) <= 1.0


def phantom(shape: Sequence[int], rng: np.random.Generator, noise_amp: float = 0.05,
            noise_spacing: Optional[float] = None) -> np.ndarray:
    """Brain-slice (2-D) or brain-volume (3-D) phantom: nested ellipses /
    ellipsoids at 0.2 / 0.5 / 0.8 (inner shells override), blurred with a
    1-pixel Gaussian, plus gradient noise masked to the outer shell."""
    d = len(shape)
    shells = _SHELLS_2D if d == 2 else _SHELLS_3D
    coords = _normalised_coords(shape)
    img = np.zeros(tuple(shape))
    for axes, val in shells:
        img[_inside(coords, axes)] = val
    img = ndimage.gaussian_filter(img, 1.0, mode="constant")
    if noise_spacing is None:
        noise_spacing = max(shape) / 8.0 if d == 2 else 20.0
    outer = _inside(coords, shells[0][0])
    img += noise_amp * gradient_noise(shape, noise_spacing, rng) * outer
    return img


def smooth_warp(shape: Sequence[int], sigma: float, max_disp: float,
                rng: np.random.Generator) -> np.ndarray:
    """Random smooth displacement u [d, *shape]: Gaussian-filtered N(0,1)
    per component, rescaled so that max_q |u(q)| = max_disp."""
    u = np.stack([ndimage.gaussian_filter(rng.standard_normal(tuple(shape)), sigma)
                  for _ in shape])
    return u * (max_disp / np.sqrt((u ** 2).sum(0)).max())


def warp_image(img: np.ndarray, u: np.ndarray) -> np.ndarray:
    """J(q) = img(q + u(q)), clamped linear interpolation (SciPy)."""
    coords = np.stack([c + du for c, du in zip(_grid(img.shape), u)])
    return ndimage.map_coordinates(img, coords, order=1, mode="nearest")


def lesion_mask(shape: Sequence[int], centre: Sequence[float], semi_axes: Sequence[float]) -> np.ndarray:
    """Soft ellipse / ellipsoid indicator (blurred by a 1-pixel Gaussian)."""
    grid = _grid(shape)
    ind = sum(((g - c) / s) ** 2 for g, c, s in zip(grid, centre, semi_axes)) <= 1.0
    return np.clip(ndimage.gaussian_filter(ind.astype(np.float64), 1.0, mode="constant"), 0.0, 1.0)


def _lesion_centre(shape: Sequence[int], rng: np.random.Generator) -> List[float]:
    """Seeded point well inside the middle shell (normalised radius <= 0.55)."""
    d = len(shape)
    mid = (_SHELLS_2D if d == 2 else _SHELLS_3D)[1][0]
    while True:
        x = rng.uniform(-1.0, 1.0, size=d)
        if np.sum(x ** 2) <= 1.0:
            break
    return [(n - 1) / 2.0 + 0.55 * xi * a * n / 2.0 for xi, a, n in zip(x, mid, shape)]


def make_p0(kind: str, shape: Sequence[int], rng: np.random.Generator,
            sigma: Optional[float] = None) -> np.ndarray:
    """Initial momentum: "zero", "random" (iid N(0, 0.01^2)) or "realistic"
    (smooth Gaussian-filtered noise, amplitude proportional to the kernel
    width ``sigma``)."""
    d = len(shape)
    if kind == "zero":
        return np.zeros(tuple(shape))
    if kind == "random":
        return rng.normal(0.0, 0.01, size=tuple(shape))
    if kind == "realistic":
        s = REALISTIC_SIGMA_REF[d] if sigma is None else float(sigma)
        n = ndimage.gaussian_filter(rng.standard_normal(tuple(shape)), REALISTIC_SMOOTHING[d])
        return REALISTIC_AMPLITUDE[d] * (s / REALISTIC_SIGMA_REF[d]) * n / np.abs(n).max()
    raise ValueError(f"unknown p0 kind {kind!r}")


def disk_pair(seed: int = 1, p0_kind: str = "random", size: int = 64) -> Pair:
    """Smooth disk (radius 20 px, intensity 1, 1-px blur) -> the same disk shifted
    4 px along x plus a Gaussian blob (amplitude 0.8, sigma 4 px) inside it."""
    rng = np.random.default_rng(seed)
    yy, xx = _grid((size, size))
    c = size / 2.0

    def disk(cy, cx):
        ind = ((yy - cy) ** 2 + (xx - cx) ** 2 <= 20.0 ** 2).astype(np.float64)
        return ndimage.gaussian_filter(ind, 1.0, mode="constant")

    S = disk(c, c)
    J = disk(c, c + 4.0) + 0.8 * np.exp(-((yy - c) ** 2 + (xx - c - 4.0) ** 2) / (2 * 4.0 ** 2))
    p0 = make_p0(p0_kind, (size, size), rng)
    return Pair(_f32(S), _f32(J), _f32(p0), rho=float(np.float32(0.5)),
                sigma=float(np.float32(3.0)), meta={"seed": seed, "p0": p0_kind})


def ripple_case(size: int = 64, amplitude: float = 100.0):
    """Stand-in for the paper's scheme comparison (Results, Fig. 1: a shot from
    an LDDMM momentum toward a 'C' picture): a sharp disk (radius 0.3 size,
    1-px blur) as source, the disk with a notch cut on its right side as the
    'C' target, and an initial momentum concentrated on the part of the disk
    edge that must move, amplitude * (S - J) (rho = 0 is intended)."""
    yy, xx = _grid((size, size))
    c = (size - 1) / 2.0
    r = 0.3 * size
    disk = ((yy - c) ** 2 + (xx - c) ** 2 <= r ** 2).astype(np.float64)
    notch = ((np.abs(yy - c) <= 0.12 * size) & (xx >= c)).astype(np.float64)
    S = ndimage.gaussian_filter(disk, 1.0, mode="constant")
    J = ndimage.gaussian_filter(disk * (1.0 - notch), 1.0, mode="constant")
    p0 = amplitude * (S - J)
    return _f32(S), _f32(J), _f32(p0)


def phantom_pair(shape: Sequence[int], seed: int, rho: float, sigma: float,
                 p0_kind: str = "realistic", warp_sigma: Optional[float] = None,
                 max_disp: Optional[float] = None) -> Pair:
    """Phantom -> phantom warped by a random smooth field, with a lesion inserted.

    2-D: warp sigma 20 px, max 6 px, lesion semi-axes 11 x 7.5 px (y, x).
    3-D: warp sigma 15 vox, max 5 vox, lesion semi-axes ~12 vox (+-15 %)."""
    rng = np.random.default_rng(seed)
    d = len(shape)
    if warp_sigma is None:
        warp_sigma = 20.0 if d == 2 else 15.0
    if max_disp is None:
        max_disp = 6.0 if d == 2 else 5.0
    S = phantom(shape, rng)
    u = smooth_warp(shape, warp_sigma, max_disp, rng)
    J = warp_image(S, u)
    centre = _lesion_centre(shape, rng)
    if d == 2:
        semi = (11.0, 7.5)
    else:
        semi = tuple(12.0 * (1.0 + rng.uniform(-0.15, 0.15)) for _ in range(3))
    mask = lesion_mask(shape, centre, semi)
    J = J * (1.0 - mask) + 1.0 * mask
    p0 = make_p0(p0_kind, shape, rng, sigma)
    return Pair(_f32(S), _f32(J), _f32(p0), rho=float(np.float32(rho)),
                sigma=float(np.float32(sigma)),
                meta={"seed": seed, "p0": p0_kind, "shape": tuple(shape)})


def small_pair(shape: Sequence[int], seed: int, rho: float = 0.5, sigma: float = 2.0,
               p0_kind: str = "realistic", lam: float = LAMBDA,
               amplitude: Optional[float] = None) -> Pair:
    """A phantom pair at a small, arbitrary shape (test sizes), with warps and
    lesion scaled to the extent; the realistic momentum has amplitude
    ``amplitude`` (default SMALL_AMPLITUDE)."""
    d = len(shape)
    ext = min(shape)
    pair = phantom_pair(shape, seed, rho, sigma, p0_kind="zero",
                        warp_sigma=max(ext / 8.0, 1.5), max_disp=max(ext / 24.0, 0.5))
    rng = np.random.default_rng(seed + 7919)
    if p0_kind == "realistic":
        n = ndimage.gaussian_filter(rng.standard_normal(tuple(shape)), max(ext / 16.0, 1.0))
        amp = SMALL_AMPLITUDE[d] if amplitude is None else amplitude
        p0 = amp * n / np.abs(n).max()
    else:
        p0 = make_p0(p0_kind, shape, rng)
    pair.p0 = _f32(p0)
    pair.lam = lam
    pair.meta["p0"] = p0_kind
    return pair


def _c3_pair(i: int, p0_kind: str) -> Pair:
    rng = np.random.default_rng(3000 + i)
    H = int(rng.choice(SIZES_2D))
    W = int(rng.choice(SIZES_2D))
    r = float(rng.uniform(0.05, 1.0))
    s = float(rng.uniform(2.0, 6.0))
    return phantom_pair((H, W), 3000 + i + 100000, r, s, p0_kind)


def _c5_shape(i: int) -> Tuple[Tuple[int, int, int], float]:
    rng = np.random.default_rng(5000 + i)
    shp = SHAPES_3D[int(rng.integers(len(SHAPES_3D)))]
    return shp, float(rng.uniform(0.1, 1.0))


def _c5_pair(i: int, p0_kind: str) -> Pair:
    shp, r = _c5_shape(i)
    return phantom_pair(shp, 5000 + i + 100000, r, 4.0, p0_kind)


def workload_pair(name: str, i: int, p0_kind: str = "realistic") -> Pair:
    """Pair i of a batched workload ("c3" or "c5"), generated alone (the same
    arrays as workload(name).pairs[i])."""
    name = name.lower()
    if name == "c3":
        return _c3_pair(i, p0_kind)
    if name == "c5":
        return _c5_pair(i, p0_kind)
    raise ValueError(f"workload {name!r} has no per-pair generator")


def c5_shape_classes(n_pairs: int = 16) -> dict:
    """{shape: index of its first volume} over the 3-D batch (shapes only,
    no arrays are generated)."""
    out = {}
    for i in range(n_pairs):
        shp = _c5_shape(i)[0]
        out.setdefault(shp, i)
    return out


def large_step(w: "Workload") -> "Workload":
    """The large-step regime of a workload generated with the realistic
    momentum: same images, p0 scaled by LARGE_STEP_SCALE, rho = 0,
    T = LARGE_STEP_T (feet move one to a few pixels per step)."""
    pairs = [Pair(p.source, p.target, _f32(p.p0.astype(np.float64) * LARGE_STEP_SCALE), rho=0.0, sigma=p.sigma,
                  lam=p.lam, meta=dict(p.meta, p0="large-step")) for p in w.pairs]
    return Workload(w.name + "-large-step", pairs, LARGE_STEP_T)


def workload(name: str, p0_kind: str = "realistic", n_pairs: Optional[int] = None,
             rho: Optional[float] = None) -> Workload:
    """The named workload (see the module docstring)."""
    name = name.lower()
    if name == "c1":
        return Workload("c1", [disk_pair(1, "random" if p0_kind == "realistic" else p0_kind)], 10)
    if name == "c2":
        r = 0.5 if rho is None else rho
        return Workload("c2", [phantom_pair((240, 240), 2, r, 5.0, p0_kind)], 20)
    if name == "c3":
        pairs = [_c3_pair(i, p0_kind) for i in range(64 if n_pairs is None else n_pairs)]
        return Workload("c3", pairs, 20)
    if name == "c4":
        return Workload("c4", [phantom_pair((160, 192, 160), 4, 0.3, 4.0, p0_kind)], 15)
    if name == "c5":
        pairs = [_c5_pair(i, p0_kind) for i in range(16 if n_pairs is None else n_pairs)]
        return Workload("c5", pairs, 15)
    raise ValueError(f"unknown workload {name!r}")
