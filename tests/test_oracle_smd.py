"""Pins of the sparse-matrix-decomposition reference (oracle/smd.py, Algorithm 2) at tiny N:
the dense full-field matrices against the FFT-based multislice oracle, finite differences of
the matrix step, the least-squares lambda, and fixed points and descent of the decomposition."""
import numpy as np
import pytest

from oracle import smd

N, M = 8, 3
DX, LAM = 0.2, 0.0487


def _setup(orc, seed=0):
    rng = np.random.default_rng(seed)
    pos = np.array([[0, 0], [2, 3], [5, 1], [7, 6], [3, 7], [6, 4]], dtype=float)
    dz = np.array([2.0, 3.0])
    gs = [smd.propagator_matrix(orc.propagator(N, DX, LAM, d)) for d in dz]
    truth = np.exp(1j * rng.uniform(0, 0.8, (M, N, N))) * rng.uniform(0.9, 1.1, (M, N, N))
    probe = orc.probe(N, DX, LAM, 0.08, 10.0)
    md = orc.Model(N, N, N, M, pos, dz, DX, LAM)
    return rng, pos, dz, gs, truth, probe, md


def test_dense_full_field_model_equals_the_fft_multislice(orc):
    rng, pos, dz, gs, truth, probe, md = _setup(orc)
    a = smd.compose(truth, gs)
    p = smd.probe_matrix(probe, pos)
    inten = np.abs(smd.dft2_matrix(N) @ a @ p) ** 2                 # (N^2, S)
    ref = md.forward(probe, truth)                                   # (S, N, N)
    assert np.abs(inten.T.reshape(len(pos), N, N) - ref).max() < 1e-12 * ref.max()


def test_prefix_times_slice_times_suffix_is_the_whole_matrix(orc):
    rng, pos, dz, gs, truth, probe, md = _setup(orc)
    a = smd.compose(truth, gs)
    for l in range(M):
        r, s = smd.prefix_suffix(truth, gs, l)
        assert np.abs(r @ np.diag(truth[l].reshape(-1)) @ s - a).max() < 1e-12


def test_matrix_step_is_a_gradient_step_and_descends(orc):
    rng, pos, dz, gs, truth, probe, md = _setup(orc)
    p = smd.probe_matrix(probe, pos)
    meas = (np.abs(smd.dft2_matrix(N) @ smd.compose(truth, gs) @ p) ** 2)
    a0 = smd.compose(np.exp(1j * rng.uniform(0, 0.3, (M, N, N))), gs)
    a1, losses = smd.estimate_a(a0, p, meas, 1)
    mu = 1.0 / (N * N * np.linalg.norm(p, 2) ** 2)
    g = (a0 - a1) / mu
    d = rng.standard_normal(a0.shape) + 1j * rng.standard_normal(a0.shape)
    eps = 1e-6
    fd = (smd.matrix_loss(a0 + eps * d, p, meas) - smd.matrix_loss(a0 - eps * d, p, meas)) / (2 * eps)
    assert abs(fd - np.vdot(g, d).real) < 1e-6 * abs(fd)
    _, hist = smd.estimate_a(a0, p, meas, 20)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))


def test_lambda_is_the_least_squares_scale(orc):
    rng, pos, dz, gs, truth, probe, md = _setup(orc)
    a_hat = smd.compose(truth, gs) * (0.7 - 0.2j) + 1e-3 * rng.standard_normal((N * N, N * N))
    start = truth * np.exp(0.1j * rng.standard_normal(truth.shape))
    start = np.stack([smd.project(s.reshape(-1)).reshape(N, N) for s in start])
    sl, lam, at = smd.decompose_pass(a_hat, start, 1.0 + 0j, gs)
    res = np.linalg.norm(a_hat - lam * at)
    for dl in (1e-3, -1e-3, 1e-3j, -1e-3j):
        assert np.linalg.norm(a_hat - (lam + dl) * at) > res


def test_prox_step_bound_dominates_the_spectral_norms(orc):
    rng, pos, dz, gs, truth, probe, md = _setup(orc)
    peak = [np.abs(truth[m]).max() for m in range(M)]
    for l in range(M):
        r, s = smd.prefix_suffix(truth, gs, l)
        bound = np.prod([peak[m] for m in range(M) if m != l])
        assert np.linalg.norm(r, 2) * np.linalg.norm(s, 2) <= bound * (1 + 1e-12)


def test_normalised_truth_is_a_fixed_point_and_perturbed_starts_descend(orc):
    rng, pos, dz, gs, truth, probe, md = _setup(orc)
    unit = np.stack([smd.project(s.reshape(-1)).reshape(N, N) for s in truth])
    scale = np.prod([np.linalg.norm(s) for s in truth])
    a_hat = smd.compose(truth, gs)
    sl, lam, _ = smd.decompose_pass(a_hat, unit, scale + 0j, gs)
    assert np.abs(sl - unit).max() < 1e-10 and abs(lam - scale) < 1e-10 * scale
    x = np.stack([smd.project(s.reshape(-1)).reshape(N, N)
                  for s in truth * np.exp(0.2j * rng.standard_normal(truth.shape))])
    lam = 1.0 + 0j
    res = []
    for _ in range(6):
        x, lam, at = smd.decompose_pass(a_hat, x, lam, gs)
        res.append(np.linalg.norm(a_hat - lam * at))
    assert res[-1] < 0.5 * res[0], res


def test_algorithm2_improves_the_data_fit(orc):
    rng, pos, dz, gs, truth, probe, md = _setup(orc)
    p = smd.probe_matrix(probe, pos)
    meas = np.abs(smd.dft2_matrix(N) @ smd.compose(truth, gs) @ p) ** 2
    start = np.ones((M, N, N), complex)
    out, lam, hist = smd.algorithm2(probe, pos, meas, start, gs, iterations=4, a_steps=5)
    final = smd.matrix_loss(smd.compose(out, gs), p, meas)
    assert final < hist[0]
