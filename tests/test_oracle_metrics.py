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


def test_translated_copies_are_aligned_back():
    """Every slice translated together (periodically) by s: the aligned error is zero at d = -s, and
    with a per-slice complex scale as well; max_shift = 0 is the unaligned metric."""
    ref = _ref((3, 24, 20), 7)
    for s in [(3, -2), (-4, 4), (0, 1)]:
        est = np.roll(ref, s, axis=(1, 2)) * np.array([0.8j, 1.5 * np.exp(0.3j), -1.1])[:, None, None]
        errs, mean, d = metrics.reconstruction_error_aligned(est, ref, max_shift=4)
        assert d == (-s[0], -s[1])
        assert np.all(errs < 1e-14) and mean < 1e-14
        e0, m0 = metrics.reconstruction_error(est, ref)
        assert m0 > 0.5                                            # unaligned, the copy looks wrong
        e1, m1, d1 = metrics.reconstruction_error_aligned(est, ref, max_shift=0)
        assert d1 == (0, 0) and m1 == m0 and np.array_equal(e1, e0)


def test_aligned_error_of_a_noisy_translated_copy_is_the_noise_error():
    """A translated copy plus a perturbation orthogonal to the reference: the best translation is the
    true one and its error is the closed form of the perturbation alone."""
    ref = _ref((1, 16, 16), 11)
    d = 0.2 * synth.complex_field((1, 16, 16), 12).astype(np.complex128)
    d -= np.vdot(ref, d) / np.vdot(ref, ref) * ref
    est = np.roll(ref + d, (2, -3), axis=(1, 2))
    errs, mean, sh = metrics.reconstruction_error_aligned(est, ref, max_shift=3)
    r2, d2 = np.vdot(ref, ref).real, np.vdot(d, d).real
    assert sh == (-2, 3)
    assert abs(errs[0] - np.sqrt(d2 / (r2 + d2))) < 1e-13


def test_alignment_uses_the_mask_of_the_reference_frame():
    ref = _ref((2, 12, 12), 13)
    mask = np.zeros((12, 12), dtype=np.float32)
    mask[3:9, 2:10] = 1.0
    est = np.roll(ref, (1, 1), axis=(1, 2))
    est[:, 0, 0] = 50.0                  # lands at (0 - 1, 0 - 1) mod 12 = (11, 11) after alignment: unmasked
    errs, mean, sh = metrics.reconstruction_error_aligned(est, ref, mask, max_shift=2)
    assert sh == (-1, -1) and mean < 1e-14
