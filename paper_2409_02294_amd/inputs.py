"""Seeded synthetic mass densities for the free-space potential solve.

This module only produces inputs: sums of Gaussian blobs (optionally with
uniform noise) sampled at cell centres of a unit box. It performs no step of
the potential solve itself, so the CPU oracle, the GPU tests and the
benchmark can all draw from it without sharing any of the method's arithmetic.

Conventions
-----------
* Arrays are C-ordered ``[z][y][x]`` (x fastest), float64.
* Cell ``i`` along an axis has its centre at ``origin + (i + 1/2) * dx``.
* A blob with centre ``c``, width ``sigma`` and mass ``m`` contributes
  ``m / ((2 pi)^(3/2) sigma^3) * exp(-|x - c|^2 / (2 sigma^2))``.
  It is evaluated inside a box of +-``cutoff`` sigma around ``c`` (default 7,
  where the profile has fallen below 2.3e-11 of its peak) and is zero outside;
  that truncation is part of the input definition.

The paper benchmarks its solver on nested-grid potentials of an
astrophysical code whose test densities it does not publish; these blob
fields stand in for them (random masses of compact and extended structure).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

__all__ = [
    "BlobSet",
    "draw_blobs",
    "blob_density",
    "make_density",
    "WORKLOADS",
    "workload_density",
    "batched_workload",
    "nested_workload",
]


@dataclasses.dataclass(frozen=True)
class BlobSet:
    """Blob parameters: ``centres`` (n,3) as (x,y,z), ``sigmas`` (n,), ``masses`` (n,)."""

    centres: np.ndarray
    sigmas: np.ndarray
    masses: np.ndarray

    def __len__(self) -> int:
        return int(self.sigmas.shape[0])


def draw_blobs(rng: np.random.Generator, nblobs: int,
               centre: Tuple[float, float] = (0.1, 0.9),
               sigma: Tuple[float, float] = (0.01, 0.05),
               mass: Tuple[float, float] = (0.5, 2.0)) -> BlobSet:
    """Draw ``nblobs`` blobs: centres, then widths, then masses (fixed order)."""
    c = rng.uniform(centre[0], centre[1], size=(nblobs, 3))
    s = rng.uniform(sigma[0], sigma[1], size=nblobs)
    m = rng.uniform(mass[0], mass[1], size=nblobs)
    return BlobSet(c, s, m)


def blob_density(n: int, blobs: BlobSet, dx: float | None = None,
                 origin: Sequence[float] = (0.0, 0.0, 0.0),
                 cutoff: float = 7.0) -> np.ndarray:
    """Sample the blob sum on an ``n^3`` cell-centred grid (float64, [z][y][x])."""
    if dx is None:
        dx = 1.0 / n
    rho = np.zeros((n, n, n), dtype=np.float64)
    ox, oy, oz = (float(o) for o in origin)
    for (cx, cy, cz), s, m in zip(blobs.centres, blobs.sigmas, blobs.masses):
        amp = m / ((2.0 * math.pi) ** 1.5 * s ** 3)
        sl = []
        prof = []
        for c, o in ((cz, oz), (cy, oy), (cx, ox)):
            lo = max(0, int(math.floor((c - cutoff * s - o) / dx - 0.5)))
            hi = min(n, int(math.ceil((c + cutoff * s - o) / dx - 0.5)) + 1)
            if hi <= lo:
                break
            xs = o + (np.arange(lo, hi, dtype=np.float64) + 0.5) * dx
            sl.append(slice(lo, hi))
            prof.append(np.exp(-((xs - c) ** 2) / (2.0 * s * s)))
        if len(sl) != 3:
            continue
        ez, ey, ex = prof
        rho[sl[0], sl[1], sl[2]] += amp * (ez[:, None, None] * (ey[None, :, None] * ex[None, None, :]))
    return rho


def make_density(n: int, nblobs: int, seed: int,
                 centre: Tuple[float, float] = (0.1, 0.9),
                 sigma: Tuple[float, float] = (0.01, 0.05),
                 mass: Tuple[float, float] = (0.5, 2.0),
                 noise: float = 0.0) -> np.ndarray:
    """Blob density on the unit box, plus ``U[0, noise * peak]`` per cell if ``noise > 0``.

    Draw order from ``numpy.random.default_rng(seed)``: blobs (see
    :func:`draw_blobs`), then one uniform per cell in C order for the noise.
    """
    rng = np.random.default_rng(seed)
    blobs = draw_blobs(rng, nblobs, centre, sigma, mass)
    rho = blob_density(n, blobs)
    if noise > 0.0:
        peak = float(rho.max())
        rho += rng.uniform(0.0, 1.0, size=rho.shape) * (noise * peak)
    return rho


# The named single-solve workloads.  Sizes, blob counts and widths follow the
# configurations the solver is measured on; ``seed`` values are fixed.
WORKLOADS: Dict[str, dict] = {
    # 32^3 cells (dx = 1/32), padded to 64^3; 3 blobs near the centre.
    "blobs32": dict(n=32, nblobs=3, seed=1001, centre=(0.3, 0.7), sigma=(0.03, 0.08), noise=0.0),
    # 256^3 padded to 512^3; 64 compact blobs plus noise at 1e-3 of the peak.
    "blobs256": dict(n=256, nblobs=64, seed=1002, centre=(0.1, 0.9), sigma=(0.01, 0.05), noise=1e-3),
    # 512^3 padded to 1024^3; 256 compact blobs plus noise at 1e-3 of the peak.
    "blobs512": dict(n=512, nblobs=256, seed=1003, centre=(0.1, 0.9), sigma=(0.01, 0.05), noise=1e-3),
}


def workload_density(name: str) -> np.ndarray:
    w = dict(WORKLOADS[name])
    n = w.pop("n")
    return make_density(n, **w)


def batched_workload(count: int = 96, seed: int = 4000,
                     sizes: Sequence[int] = (32, 48, 64, 96, 128)) -> List[np.ndarray]:
    """``count`` independent densities of uneven sizes.

    Sizes are i.i.d. uniform over ``sizes`` from ``default_rng(seed)``; solve
    ``i`` then uses ``default_rng(seed + i)`` for its blob count (uniform over
    4..32) and its blobs (widths U[0.03, 0.08], centres U[0.1, 0.9]^3).
    """
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    out = []
    for i, n in enumerate(ns):
        r = np.random.default_rng(seed + i)
        nb = int(r.integers(4, 33))
        blobs = draw_blobs(r, nb, centre=(0.1, 0.9), sigma=(0.03, 0.08))
        out.append(blob_density(int(n), blobs))
    return out


def blob_density_torch(n: int, blobs: BlobSet, dx: float | None = None,
                       origin: Sequence[float] = (0.0, 0.0, 0.0), cutoff: float = 7.0,
                       out=None, device="cuda"):
    """:func:`blob_density` evaluated with torch on ``device`` in float64 (same
    formula, cell ranges and truncation), for workloads too large to build on
    the host; ``out`` (a float32 or float64 tensor) receives the result."""
    import torch
    if dx is None:
        dx = 1.0 / n
    rho = torch.zeros((n, n, n), dtype=torch.float64, device=device)
    ox, oy, oz = (float(o) for o in origin)
    for (cx, cy, cz), s, m in zip(blobs.centres, blobs.sigmas, blobs.masses):
        amp = m / ((2.0 * math.pi) ** 1.5 * s ** 3)
        sl, prof = [], []
        for c, o in ((cz, oz), (cy, oy), (cx, ox)):
            lo = max(0, int(math.floor((c - cutoff * s - o) / dx - 0.5)))
            hi = min(n, int(math.ceil((c + cutoff * s - o) / dx - 0.5)) + 1)
            if hi <= lo:
                break
            xs = o + (torch.arange(lo, hi, dtype=torch.float64, device=device) + 0.5) * dx
            sl.append(slice(lo, hi))
            prof.append(torch.exp(-((xs - c) ** 2) / (2.0 * s * s)))
        if len(sl) != 3:
            continue
        ez, ey, ex = prof
        rho[sl[0], sl[1], sl[2]] += amp * (ez[:, None, None] * (ey[None, :, None] * ex[None, None, :]))
    if out is not None:
        out.copy_(rho)
        return out
    return rho


def nested_workload(steps: int, coarse_n: int = 384, fine_n: int = 128, levels: int = 2,
                    nblobs: int = 32, seed: int = 5000, vmax: float = 1e-3):
    """Blob parameters and level geometry for a drifting-blob time sequence.

    Returns ``(geometry, blob_sets)``: ``geometry`` is a list of
    ``(n, dx, origin)`` per level (the coarse unit box first, then concentric
    boxes refined by 2 per level around the initial mass centroid) and
    ``blob_sets[t]`` is the :class:`BlobSet` at step ``t``.  Blobs move by a
    fixed per-step velocity drawn from ``U[-vmax, vmax]^3`` and reflect off
    the walls of ``[0.1, 0.9]^3``.
    """
    rng = np.random.default_rng(seed)
    b0 = draw_blobs(rng, nblobs, centre=(0.1, 0.9), sigma=(0.01, 0.05))
    vel = rng.uniform(-vmax, vmax, size=(nblobs, 3))
    centroid = (b0.centres * b0.masses[:, None]).sum(0) / b0.masses.sum()
    geometry = [(coarse_n, 1.0 / coarse_n, (0.0, 0.0, 0.0))]
    dx = 1.0 / coarse_n
    for _ in range(levels):
        dx = dx / 2.0
        side = fine_n * dx
        geometry.append((fine_n, dx, tuple(float(c - side / 2.0) for c in centroid)))
    sets = []
    pos = b0.centres.copy()
    v = vel.copy()
    for _ in range(steps):
        sets.append(BlobSet(pos.copy(), b0.sigmas, b0.masses))
        pos = pos + v
        lo, hi = 0.1, 0.9
        over = pos > hi
        pos[over] = 2 * hi - pos[over]
        v[over] = -v[over]
        under = pos < lo
        pos[under] = 2 * lo - pos[under]
        v[under] = -v[under]
    return geometry, sets
