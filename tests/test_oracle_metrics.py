"""Pins of the reconstruction-error reference (oracle/metrics.py): the ambiguities it removes,
a closed form for an orthogonal perturbation, a brute-force search over the complex scale,
and the mask."""
import numpy as np
import pytest

from oracle import metrics
from paper_2205_03902_amd import synth


def _ref(shape=(3, 24, 20), seed=1):
    return synth.complex_field(shape, seed).astype(np.complex128)


def test_scaled_and_phase_shifted_copies_have_zero_error():
    ref = _ref()
    est = ref * np.array([0.5 * np.exp(0.7j), 2.0 * np.exp(-2.1j), 1.3j])[:, None, None]
    errs, mean = metrics.reconstruction_error(est, ref)
    assert np.all(errs < 1e-14) and mean < 1e-14


def test_orthogonal_perturbation_has_its_closed_form():
    ref = _ref((1, 16, 16))
    d = synth.complex_field((1, 16, 16), 9).astype(np.complex128)
    d -= np.vdot(ref, d) / np.vdot(ref, ref) * ref          # <ref, d> = 0
    errs, _ = metrics.reconstruction_error(ref + d, ref)
    r2, d2 = np.vdot(ref, ref).real, np.vdot(d, d).real
    assert abs(errs[0] - np.sqrt(d2 / (r2 + d2))) < 1e-13


def test_least_squares_scale_beats_every_scale_on_a_grid():
    ref = _ref((1, 12, 12), 3)
    est = ref + 0.4 * synth.complex_field((1, 12, 12), 4)
    err, _ = metrics.reconstruction_error(est, ref)
    grid = [a * np.exp(1j * p) for a in np.linspace(0.2, 2.0, 91) for p in np.linspace(-np.pi, np.pi, 181)]
    best = min(np.linalg.norm(g * est - ref) for g in grid) / np.linalg.norm(ref)
    assert err[0] <= best + 1e-12 and best - err[0] < 2e-3


def test_mask_excludes_pixels_and_zero_estimate_is_error_one():
    ref = _ref((2, 10, 10), 5)
    est = ref.copy()
    mask = np.zeros((10, 10), dtype=np.float32)
    mask[2:8, 3:9] = 1.0
    est[:, 0, 0] += 100.0                                   # outside the mask
    errs, _ = metrics.reconstruction_error(est, ref, mask)
    assert np.all(errs < 1e-14)
    errs, mean = metrics.reconstruction_error(np.zeros_like(ref), ref)
    assert np.all(errs == 1.0) and mean == 1.0
