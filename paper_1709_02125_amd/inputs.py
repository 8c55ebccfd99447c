"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module holds only random-number generation and input layout: none of the
stencil method's arithmetic lives here, so both sides can use it without
sharing any part of the computation.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), with a double formed from the top 53 bits.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
SEED = 1709


class SplitMix64:
    """Counter-based 64-bit generator; state advances by the golden-ratio gamma."""

    def __init__(self, seed: int = SEED):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def next_double(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def splitmix64_array(seed: int, n: int) -> np.ndarray:
    """n doubles in [0, 1) from SplitMix64(seed), vectorised (same stream as
    repeated next_double())."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed) + k * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


# ---------------------------------------------------------------- hydro (2D/3D)
HYDRO_BACKGROUND = (0.2, 1.0)   # density, specific internal energy
HYDRO_BLOB = (1.0, 2.5)
HYDRO_NBLOBS = 16


def hydro_boxes(n: tuple, nblobs: int = HYDRO_NBLOBS, seed: int = SEED):
    """Seeded boxes in cell units: per box and axis a side drawn uniformly in
    [0.05, 0.25] of the axis length (at least one cell), then a lower corner
    uniform in [0, n - side]. Returns a list of tuples (lo0, hi0, lo1, hi1, ...)."""
    g = SplitMix64(seed)
    boxes = []
    for _ in range(nblobs):
        b = []
        for na in n:
            side = max(1, int((0.05 + 0.2 * g.next_double()) * na))
            side = min(side, na)
            lo = int(g.next_double() * (na - side + 1))
            b += [lo, lo + side]
        boxes.append(tuple(b))
    return boxes


def hydro_initial_state(n: tuple, nblobs: int = HYDRO_NBLOBS, seed: int = SEED):
    """Interior density and energy, shape n[::-1] (row-major, x fastest):
    a uniform background with seeded boxes of the blob state."""
    shape = tuple(reversed(n))
    rho = np.full(shape, HYDRO_BACKGROUND[0])
    ene = np.full(shape, HYDRO_BACKGROUND[1])
    for b in hydro_boxes(n, nblobs, seed):
        sl = tuple(slice(b[2 * a], b[2 * a + 1]) for a in reversed(range(len(n))))
        rho[sl] = HYDRO_BLOB[0]
        ene[sl] = HYDRO_BLOB[1]
    return rho, ene


def mirror_symmetrise(a: np.ndarray, axis: int) -> np.ndarray:
    """Make an interior cell array symmetric about the domain mid-plane of `axis`
    (numpy axis) by taking the element-wise max with its reflection."""
    return np.maximum(a, np.flip(a, axis=axis))


# ------------------------------------------------------ Taylor-Green vortex
TGV_MACH = 0.1
TGV_GAMMA = 1.4
TGV_PERTURB = 1e-3


def tgv_initial_state(n: int, perturb: float = TGV_PERTURB, seed: int = SEED):
    """Taylor-Green vortex on [0, 2 pi]^3 at cell centres, arrays indexed
    [z, y, x]: u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = p0 + (cos 2x + cos 2y)(cos 2z + 2)/16 with p0 = 1/(gamma M^2), uniform
    temperature (rho = p / p0); then u, v, w each get perturb * (2 r - 1) with
    r from SplitMix64(seed), u's n^3 draws first, then v's, then w's."""
    h = 2.0 * np.pi / n
    c = (np.arange(n) + 0.5) * h
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    p0 = 1.0 / (TGV_GAMMA * TGV_MACH * TGV_MACH)
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    rho = p / p0
    if perturb:
        r = splitmix64_array(seed, 3 * n ** 3).reshape(3, n, n, n)
        u = u + perturb * (2.0 * r[0] - 1.0)
        v = v + perturb * (2.0 * r[1] - 1.0)
        w = w + perturb * (2.0 * r[2] - 1.0)
    return rho, u, v, w, p
