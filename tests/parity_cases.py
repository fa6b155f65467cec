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


@dataclasses.dataclass
class FullRun:
    """An oracle reconstruction stored under tests/golden/ (see the script that writes it)."""
    sweeps: int
    defocus_factor: float
    final_loss: float
    slice_error_to_truth: float
    probe_rel_error_to_truth: float
    spread_probe_change: float   # the oracle's own spread: its run from the unrounded probe
    spread_final_loss: float
    spread_slice_error: float
    spread_probe_error: float
    losses: np.ndarray      # the loss before every step
    rows: np.ndarray        # sampled object rows and columns
    cols: np.ndarray
    slices: np.ndarray      # complex128 (M, len(rows), len(cols)): the final slices there
    probe_stride: int
    probe: np.ndarray       # complex128 (N / stride, N / stride): the final probe, every stride-th pixel


def read_full_run(path: str, n_slices: int) -> FullRun:
    with open(path) as f:
        lines = [ln for ln in f.read().splitlines() if ln and not ln.startswith("#")]
    it = iter(lines)
    vals = {}

    def block(count):
        return np.array([[float(t) for t in next(it).split()] for _ in range(count)])

    for ln in it:
        key, arg = ln.split()
        if key == "losses":
            vals[key] = block(int(arg))[:, 0]
        elif key in ("slice_rows", "slice_cols"):
            vals[key] = np.array([int(t) for t in next(it).split()])
            assert len(vals[key]) == int(arg)
        elif key in ("slices", "probe"):
            b = block(int(arg))
            vals[key] = b[:, 0] + 1j * b[:, 1]
        else:
            vals[key] = float(arg)
    rows, cols = vals["slice_rows"], vals["slice_cols"]
    stride = int(vals["probe_stride"])
    side = int(round(np.sqrt(len(vals["probe"]))))
    return FullRun(int(vals["sweeps"]), vals["defocus_factor"], vals["final_loss"], vals["slice_error_to_truth"],
                   vals["probe_rel_error_to_truth"], vals["spread_probe_change"], vals["spread_final_loss"],
                   vals["spread_slice_error"], vals["spread_probe_error"], vals["losses"], rows, cols,
                   vals["slices"].reshape(n_slices, len(rows), len(cols)), stride, vals["probe"].reshape(side, side))
