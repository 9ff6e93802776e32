"""Counter-based random numbers and seeded log-normal conductivity fields.

Every random value is a pure function of (seed, counter), so the field does not
depend on thread order, chunking or the machine that draws it.

* ``splitmix64``: the SplitMix64 output function of Steele, Lea and Flood
  ("Fast splittable pseudorandom number generators", OOPSLA 2014), evaluated at
  state ``seed + (counter + 1) * 0x9E3779B97F4A7C15``.
* ``uniform01``: the top 53 bits of a SplitMix64 word, offset by half an ulp so
  the value lies strictly inside (0, 1).
* ``std_normal``: the Box-Muller transform of two such uniforms (counters 2c,
  2c+1 give normal number c).
* ``gaussian_field``: iid normals on a padded box, smoothed by a separable
  Gaussian kernel exp(-2 t^2 / l^2) per axis (covariance exp(-sum (r/l)^2)),
  cropped to the grid and normalised to zero sample mean, unit sample std.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counter: np.ndarray) -> np.ndarray:
    """SplitMix64 output for ``counter`` (uint64 array) under ``seed``."""
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counter: np.ndarray) -> np.ndarray:
    """Uniform doubles strictly inside (0, 1) from the top 53 bits."""
    z = splitmix64(seed, counter)
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * (1.0 / 9007199254740992.0)


def std_normal(seed: int, start: int, count: int) -> np.ndarray:
    """Standard normals number ``start .. start+count-1`` (Box-Muller)."""
    idx = np.arange(start, start + count, dtype=np.uint64)
    u1 = uniform01(seed, np.uint64(2) * idx)
    u2 = uniform01(seed, np.uint64(2) * idx + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def _kernel(ell: float) -> np.ndarray:
    r = int(math.ceil(3.0 * ell))
    t = np.arange(-r, r + 1, dtype=np.float64)
    return np.exp(-2.0 * t * t / (ell * ell))


def gaussian_field(n: tuple[int, int, int], ell: tuple[float, float, float], seed: int,
                   chunk: int = 1 << 24) -> np.ndarray:
    """Zero-mean unit-variance correlated field on an (nx, ny, nz) grid.

    Returned as a flat float64 array in x-fastest order c = i + nx*(j + ny*k).
    The correlation lengths ``ell`` are in cells (x, y, z).
    """
    from scipy.ndimage import correlate1d

    nx, ny, nz = n
    kx, ky, kz = (_kernel(e) for e in ell)
    rx, ry, rz = (len(k) // 2 for k in (kx, ky, kz))
    px, py, pz = nx + 2 * rx, ny + 2 * ry, nz + 2 * rz
    total = px * py * pz
    xi = np.empty(total, dtype=np.float64)
    for s in range(0, total, chunk):
        e = min(total, s + chunk)
        xi[s:e] = std_normal(seed, s, e - s)
    xi = xi.reshape(pz, py, px)
    # Filter one axis at a time and crop its padding right away (only the
    # fully supported interior is kept, so the boundary mode never matters).
    xi = correlate1d(xi, kx, axis=2, mode="constant")[:, :, rx:rx + nx]
    xi = correlate1d(xi, ky, axis=1, mode="constant")[:, ry:ry + ny, :]
    xi = correlate1d(xi, kz, axis=0, mode="constant")[rz:rz + nz, :, :]
    z = np.ascontiguousarray(xi).reshape(-1)
    z = z - z.mean()
    sd = z.std()
    if sd > 0:
        z = z / sd
    return z


def lognormal_ks(n: tuple[int, int, int], ks0: float, sigma: float,
                 ell: tuple[float, float, float], seed: int) -> np.ndarray:
    """K_s = ks0 * exp(sigma * Z) with Z from :func:`gaussian_field`."""
    if sigma == 0.0:
        return np.full(n[0] * n[1] * n[2], ks0, dtype=np.float64)
    return ks0 * np.exp(sigma * gaussian_field(n, ell, seed))
