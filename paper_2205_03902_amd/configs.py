"""Workload geometries for the five synthetic experiments.

Every length is in Angstrom, every angle in radians.  The geometry follows the
paper's problem statement (Sec. 2.1): an N x N probe window, M slices with
Fresnel gaps dz between them, a raster of S scan positions, wavelength lambda
and a circular aperture of semi-angle alpha.  The object is H x W pixels and is
treated as periodic (Sec. 1.3, "indices are wrapped around"); the paper's own
full-field model is the special case H = W = N.

The raster origin centres the scan inside the object:
    origin = floor(((H - N) - (n_scan - 1) * step) / 2)
and a window that reaches past the object edge wraps around.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Geometry:
    name: str
    n: int                 # probe window / detector side N
    obj_h: int             # object height H (pixels)
    obj_w: int             # object width W (pixels)
    n_slices: int          # M
    dz: float              # gap between consecutive slices (A)
    pixel_size: float      # real-space sampling (A)
    wavelength: float      # electron wavelength (A)
    alpha: float           # aperture semi-angle (rad)
    defocus: float         # probe defocus (A)
    scan: Tuple[int, int]  # raster shape (rows, cols)
    step_px: float         # raster step in pixels
    dose: float            # electrons per pattern; 0 means noise free
    iterations: int        # layer-wise sweeps T
    n_species: int = 1     # 1 or 2 (the heavy species has twice the amplitude)
    lattice: float = 3.9   # square lattice constant (A)
    seed: int = 0          # specimen seed; noise uses seed + 1, directions seed + 2

    @property
    def n_pos(self) -> int:
        return self.scan[0] * self.scan[1]

    def positions(self) -> np.ndarray:
        """Window top-left corners (y, x) in object pixels, row-major raster, float64."""
        ny, nx = self.scan
        oy = math.floor(((self.obj_h - self.n) - (ny - 1) * self.step_px) / 2)
        ox = math.floor(((self.obj_w - self.n) - (nx - 1) * self.step_px) / 2)
        yy = oy + self.step_px * np.arange(ny, dtype=np.float64)
        xx = ox + self.step_px * np.arange(nx, dtype=np.float64)
        pos = np.empty((ny * nx, 2), dtype=np.float64)
        pos[:, 0] = np.repeat(yy, nx)
        pos[:, 1] = np.tile(xx, ny)
        return pos

    def gaps(self) -> np.ndarray:
        """The M - 1 Fresnel distances between consecutive slices."""
        return np.full(max(self.n_slices - 1, 0), self.dz, dtype=np.float64)

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)


# Wavelength quoted for the 60 kV workloads.
LAMBDA_60KV = 0.0487

CFG0 = Geometry("cfg0_64px_2slices_64pos", n=64, obj_h=96, obj_w=96, n_slices=2, dz=2.0,
                pixel_size=0.2, wavelength=LAMBDA_60KV, alpha=0.020, defocus=50.0,
                scan=(8, 8), step_px=5.0, dose=1e5, iterations=50, n_species=1, seed=0)
CFG1 = Geometry("cfg1_128px_6slices_1024pos", n=128, obj_h=320, obj_w=320, n_slices=6, dz=2.0,
                pixel_size=0.2, wavelength=LAMBDA_60KV, alpha=0.020, defocus=200.0,
                scan=(32, 32), step_px=2.5, dose=1e5, iterations=20, n_species=2, seed=10)
CFG2 = Geometry("cfg2_256px_10slices_4096pos", n=256, obj_h=512, obj_w=512, n_slices=10, dz=1.5,
                pixel_size=0.2, wavelength=LAMBDA_60KV, alpha=0.020, defocus=200.0,
                scan=(64, 64), step_px=4.0, dose=0.0, iterations=1, n_species=2, seed=20)
CFG3 = CFG1.replace(name="cfg3_learned_init_cfg1_geometry", seed=30)
CFG4 = Geometry("cfg4_256px_12slices_16384pos", n=256, obj_h=1024, obj_w=1024, n_slices=12, dz=2.0,
                pixel_size=0.2, wavelength=LAMBDA_60KV, alpha=0.020, defocus=200.0,
                scan=(128, 128), step_px=6.0, dose=1e5, iterations=30, n_species=2, seed=40)

CONFIGS = {0: CFG0, 1: CFG1, 2: CFG2, 3: CFG3, 4: CFG4}


def small(n: int = 32, obj: int = 48, n_slices: int = 3, scan=(3, 3), step_px: float = 3.5,
          seed: int = 1234, defocus: float = 30.0, dose: float = 0.0) -> Geometry:
    """A tiny geometry for tests: several windows, wrap-around, fractional steps."""
    return Geometry(f"small_{n}px", n=n, obj_h=obj, obj_w=obj, n_slices=n_slices, dz=2.0,
                    pixel_size=0.2, wavelength=LAMBDA_60KV, alpha=0.030, defocus=defocus,
                    scan=scan, step_px=step_px, dose=dose, iterations=5, n_species=2, seed=seed)
