"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module draws the random quantities of a workload and nothing else: it
does not propagate waves, form probes or evaluate the loss.  Both sides of
every parity check read their inputs from here, rounded once to the storage
precision of the GPU path (complex64 / float32), so a comparison measures
only the arithmetic of the implementation under test.

Specimens stand in for the crystals of the paper's simulation study
(Table 1), whose structures and simulator are not available: every slice is a
pure-phase transmission t = exp(i * kappa * V) with V a sum of Gaussian atoms
of width 0.3 A on a jittered square lattice.  The lattice origin is drawn
anew for every slice, so slices differ.
"""
from __future__ import annotations

import math

import numpy as np

from .configs import Geometry

KAPPA = 0.5          # phase (rad) per unit of potential amplitude
SIGMA_R = 0.3        # Gaussian atom radius (A)
JITTER = 0.1         # lattice position jitter, standard deviation (A)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def atom_potential(h: int, w: int, dx: float, atoms: np.ndarray, amps: np.ndarray,
                   sigma: float = SIGMA_R) -> np.ndarray:
    """V[y, x] = sum_a A_a exp(-|r - r_a|^2 / (2 sigma^2)) with minimum-image distances."""
    v = np.zeros((h, w), dtype=np.float64)
    rad = int(math.ceil(5.0 * sigma / dx))
    offs = np.arange(-rad, rad + 1)
    for (ya, xa), a in zip(atoms, amps):
        cy, cx = int(round(ya / dx)), int(round(xa / dx))
        iy = (cy + offs) % h
        ix = (cx + offs) % w
        dyv = (cy + offs) * dx - ya
        dxv = (cx + offs) * dx - xa
        g = np.exp(-(dyv[:, None] ** 2 + dxv[None, :] ** 2) / (2.0 * sigma * sigma))
        v[np.ix_(iy, ix)] += a * g
    return v


def specimen(geo: Geometry, seed: int | None = None, lattice: float | None = None,
             vacancy: float = 0.0, n_species: int | None = None) -> np.ndarray:
    """Potentials V of shape (M, H, W), float64, for a seeded lattice specimen."""
    rng = rng_for(geo.seed if seed is None else seed)
    a = geo.lattice if lattice is None else lattice
    ns = geo.n_species if n_species is None else n_species
    ly, lx = geo.obj_h * geo.pixel_size, geo.obj_w * geo.pixel_size
    out = np.empty((geo.n_slices, geo.obj_h, geo.obj_w), dtype=np.float64)
    for m in range(geo.n_slices):
        y0, x0 = rng.uniform(0.0, a, size=2)
        ys = np.arange(y0, ly, a)
        xs = np.arange(x0, lx, a)
        pts = np.stack(np.meshgrid(ys, xs, indexing="ij"), axis=-1).reshape(-1, 2)
        pts = pts + rng.normal(0.0, JITTER, size=pts.shape)
        amps = rng.uniform(0.5, 1.5, size=len(pts))
        if ns == 2:
            heavy = rng.random(len(pts)) < 0.5
            amps = np.where(heavy, 2.0 * amps, amps)
        if vacancy > 0.0:
            keep = rng.random(len(pts)) >= vacancy
            pts, amps = pts[keep], amps[keep]
        pts[:, 0] %= ly
        pts[:, 1] %= lx
        out[m] = atom_potential(geo.obj_h, geo.obj_w, geo.pixel_size, pts, amps)
    return out


def transmissions(v: np.ndarray, kappa: float = KAPPA) -> np.ndarray:
    """Pure-phase slices t = exp(i kappa V), rounded to complex64."""
    return np.exp(1j * kappa * v).astype(np.complex64)


def poisson_counts(intensity: np.ndarray, dose: float, seed: int) -> np.ndarray:
    """Counts ~ Pois(dose * I / N^2) per pixel, returned rescaled as counts * N^2 / dose (float32).

    With a unit-norm probe and pure-phase slices every pattern sums to N^2, so
    the expected number of electrons per pattern is `dose`.  dose <= 0 returns
    the intensities unchanged.
    """
    intensity = np.asarray(intensity)
    if dose <= 0:
        return intensity.astype(np.float32)
    n2 = intensity.shape[-1] * intensity.shape[-2]
    rng = rng_for(seed)
    lam = np.clip(intensity.astype(np.float64), 0.0, None) * (dose / n2)
    return (rng.poisson(lam) * (n2 / dose)).astype(np.float32)


def complex_directions(shape, count: int, seed: int) -> np.ndarray:
    """`count` complex Gaussian directions with unit per-pixel variance (complex128)."""
    rng = rng_for(seed)
    d = rng.standard_normal((count,) + tuple(shape)) + 1j * rng.standard_normal((count,) + tuple(shape))
    return d / math.sqrt(2.0)


def complex_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """A seeded complex Gaussian field rounded to complex64 (generic, non unit-modulus input)."""
    rng = rng_for(seed)
    z = rng.standard_normal(tuple(shape)) + 1j * rng.standard_normal(tuple(shape))
    return (scale * z / math.sqrt(2.0)).astype(np.complex64)


def unit_phase_field(shape, seed: int, max_phase: float = 0.7) -> np.ndarray:
    """Seeded pure-phase field exp(i phi), phi ~ U[0, max_phase), complex64."""
    rng = rng_for(seed)
    return np.exp(1j * rng.uniform(0.0, max_phase, size=tuple(shape))).astype(np.complex64)


def random_positions(n_pos: int, span_y: float, span_x: float, seed: int, origin=(0.0, 0.0)) -> np.ndarray:
    """Uniformly random window corners (y, x) in [origin, origin + span), float64."""
    rng = rng_for(seed)
    p = np.empty((n_pos, 2), dtype=np.float64)
    p[:, 0] = origin[0] + rng.uniform(0.0, span_y, size=n_pos)
    p[:, 1] = origin[1] + rng.uniform(0.0, span_x, size=n_pos)
    return p
