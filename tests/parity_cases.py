"""Seeded parity cases shared by the GPU tests: every input comes from the input
generator or from the oracle, rounded once to the GPU storage precision."""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle
from paper_2205_03902_amd import configs, synth


@dataclasses.dataclass
class Case:
    geo: configs.Geometry
    model: oracle.Model
    probe: np.ndarray      # complex64
    truth: np.ndarray      # complex64 (M, H, W)
    measured: np.ndarray   # float32 (S, N, N)
    start: np.ndarray      # complex64 (M, H, W), the iterate the gradients are taken at


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def make_case(geo: configs.Geometry, positions=None, start_phase: float = 0.3, dose=None) -> Case:
    pos = geo.positions() if positions is None else np.asarray(positions, dtype=np.float64)
    md = oracle.Model.from_geometry(geo, positions=pos)
    probe = oracle.probe(geo.n, geo.pixel_size, geo.wavelength, geo.alpha, geo.defocus).astype(np.complex64)
    truth = synth.transmissions(synth.specimen(geo))
    inten = md.forward(probe, truth)
    d = geo.dose if dose is None else dose
    measured = synth.poisson_counts(inten, d, geo.seed + 1)
    start = synth.unit_phase_field(truth.shape, geo.seed + 3, start_phase)
    return Case(geo, md, probe, truth, measured, start)


def small_geometry(n: int, n_slices: int = 3, seed: int = 11):
    """Several windows with fractional steps and wrap-around (negative corners)."""
    obj = n + n // 2
    return configs.small(n=n, obj=obj, n_slices=n_slices, scan=(3, 3), step_px=n / 8 + 0.5, seed=seed,
                         defocus=25.0)


def small_positions(geo: configs.Geometry) -> np.ndarray:
    pos = geo.positions()
    pos[0] = (-3.5, -2.0)                          # wraps through the top-left corner
    pos[-1] = (geo.obj_h - 2.0, geo.obj_w - 5.25)  # wraps through the bottom-right corner
    return pos
