"""Pins for the oracle's forward multislice model (Sec. 2.1) and its matrix form (Sec. 2.2)."""
import numpy as np
import pytest

from paper_2205_03902_amd import configs, synth


def _model(orc, n, obj, m, pos, dz=2.0, dx=0.2, lam=0.0487):
    return orc.Model(n, obj, obj, m, np.asarray(pos, float), np.full(max(m - 1, 1), dz), dx, lam)


def _probe(orc, n, defocus=20.0):
    return orc.probe(n, 0.2, 0.0487, 0.03, defocus)


def test_free_space_gives_probe_diffraction(orc):
    """t = 1: |F G P^s| = |F P^s| = |F P| for every position and every gap."""
    n, obj, m = 32, 40, 3
    pos = [[0, 0], [3.5, 7.25], [-2, 39], [10.5, 0.5]]
    md = _model(orc, n, obj, m, pos, dz=7.0)
    p = _probe(orc, n)
    inten = md.forward(p, np.ones((m, obj, obj), complex))
    ref = np.abs(np.fft.fft2(p)) ** 2
    for s in range(len(pos)):
        assert np.abs(inten[s] - ref).max() < 1e-12 * ref.max()


def test_pure_phase_conserves_norm(orc):
    n, obj, m = 32, 48, 4
    geo = configs.small(n=n, obj=obj, n_slices=m)
    sl = np.exp(1j * synth.KAPPA * synth.specimen(geo))   # exactly unit modulus in FP64
    md = orc.Model.from_geometry(geo)
    p = _probe(orc, n)
    inten = md.forward(p, sl)
    # sum_k I_k = N^2 ||E_M||^2 = N^2 ||P||^2 = N^2 (Parseval, unitary G, |t| = 1)
    assert np.abs(inten.sum(axis=(1, 2)) - n * n).max() < 1e-10 * n * n


def test_single_slice_is_ptychography(orc):
    """M = 1: I^s = |F(P^s o X_1)|^2, the single multiplicative model."""
    n, obj = 16, 24
    rng = np.random.default_rng(3)
    t = rng.standard_normal((1, obj, obj)) + 1j * rng.standard_normal((1, obj, obj))
    pos = [[2, 5], [20, 21]]
    md = _model(orc, n, obj, 1, pos)
    p = _probe(orc, n)
    inten = md.forward(p, t)
    for s, (py, px) in enumerate(pos):
        iy = (py + np.arange(n)) % obj
        ix = (px + np.arange(n)) % obj
        patch = t[0][np.ix_(iy, ix)]
        assert np.abs(inten[s] - np.abs(np.fft.fft2(p * patch)) ** 2).max() < 1e-11


def _dense_forward(p, slices, hs, shifts):
    """The paper's matrix model I = |F_2D A_M P|^2 (eq. measurement FAP) with
    A_M = O_M prod G_m O_m (eq. exit_wave_mslices), built element by element."""
    n = p.shape[0]
    f1 = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    f2 = np.kron(f1, f1)                         # 2D DFT on vec() in row-major order
    f2inv = np.conj(f2) / (n * n)
    a = np.diag(slices[0].reshape(-1))
    for m in range(1, len(slices)):
        g = f2inv @ np.diag(hs[m - 1].reshape(-1)) @ f2
        a = np.diag(slices[m].reshape(-1)) @ g @ a
    cols = [np.roll(p, s, axis=(0, 1)).reshape(-1) for s in shifts]   # p^s_{x,y} = p_{x-xs, y-ys}
    pm = np.stack(cols, axis=1)
    return np.abs(f2 @ a @ pm) ** 2, a @ pm


@pytest.mark.parametrize("n", [4, 8])
def test_dense_matrix_model_equals_fft_chain(orc, n):
    m = 3
    rng = np.random.default_rng(n)
    sl = rng.standard_normal((m, n, n)) + 1j * rng.standard_normal((m, n, n))
    p = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    shifts = [(0, 0), (1, 2), (n - 1, 3), (2, n - 1)]
    dz = [1.5, 3.0]
    hs = [orc.propagator(n, 0.2, 0.0487, d) for d in dz]
    dense_i, dense_e = _dense_forward(p, sl, hs, shifts)
    md = orc.Model(n, n, n, m, np.array(shifts, float), np.array(dz), 0.2, 0.0487)
    inten, ew = md.forward(p, sl, exit_waves=True)
    for s, sh in enumerate(shifts):
        assert np.abs(inten[s].reshape(-1) - dense_i[:, s]).max() < 1e-10 * dense_i.max()
        # the window model's exit wave is the paper's exit wave seen from the window corner
        paper_e = dense_e[:, s].reshape(n, n)
        assert np.abs(np.roll(ew[s], sh, axis=(0, 1)) - paper_e).max() < 1e-10 * np.abs(paper_e).max()


def test_wraparound_and_translation_invariance(orc):
    n, obj, m = 16, 24, 2
    rng = np.random.default_rng(5)
    sl = np.exp(1j * rng.uniform(0, 1, (m, obj, obj)))
    p = _probe(orc, n)
    pos = np.array([[1.5, 2.0], [20.0, 19.5]])
    i0 = _model(orc, n, obj, m, pos).forward(p, sl)
    # positions are taken modulo the object size
    i1 = _model(orc, n, obj, m, pos + np.array([obj, -2 * obj])).forward(p, sl)
    assert np.abs(i0 - i1).max() < 1e-12
    # moving every slice and every position by the same integer vector changes nothing
    d = (5, -3)
    sl2 = np.roll(sl, d, axis=(1, 2))
    i2 = _model(orc, n, obj, m, pos + np.array(d)).forward(p, sl2)
    assert np.abs(i0 - i2).max() < 1e-12


def test_ambiguities_leave_intensities_unchanged(orc):
    """Global phases of slices and probe (Sec. 5.3.3) and slice scalings with
    prod alpha_m = 1 (Sec. 3.4) do not change the measurements."""
    n, obj, m = 16, 20, 3
    rng = np.random.default_rng(6)
    sl = np.exp(1j * rng.uniform(0, 1, (m, obj, obj)))
    p = _probe(orc, n)
    md = _model(orc, n, obj, m, [[0, 0], [2.5, 3.5], [7, 1]])
    i0 = md.forward(p, sl)
    alphas = np.array([2.0 * np.exp(0.3j), 0.25 * np.exp(-1.1j), 2.0 * np.exp(0.8j)])
    assert abs(np.prod(np.abs(alphas)) - 1) < 1e-15
    i1 = md.forward(p * np.exp(0.7j), sl * alphas[:, None, None])
    assert np.abs(i0 - i1).max() < 1e-12 * i0.max()
