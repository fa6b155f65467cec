"""Pins of the oracle's scan-position gradient (row f4: positions that deviate from the raster,
Sec. 6) against central differences of the oracle loss, an independent real-variable
derivation for one slice with numpy's FFT, Parseval's closed form of the curvature bound,
and the behaviour at and near the true positions."""
import numpy as np
import pytest

N, OBJ, DX, LAM = 16, 24, 0.2, 0.0487
POS = np.array([[0.3, 0.6], [3.5, 2.25], [-3.7, 17.4], [9.2, 9.55], [14.45, -1.8]])


def _setup(orc, m=3, seed=0, pos=POS):
    rng = np.random.default_rng(seed)
    dz = np.array([2.0, 3.0, 1.5][: m - 1])
    truth = np.exp(1j * rng.uniform(0, 0.8, (m, OBJ, OBJ))) * rng.uniform(0.9, 1.1, (m, OBJ, OBJ))
    p = orc.probe(N, DX, LAM, 0.03, 15.0)
    md = orc.Model(N, OBJ, OBJ, m, pos, dz, DX, LAM)
    return md, p, truth, dz


def _loss_at(orc, pos, dz, m, p, slices, meas):
    return orc.Model(N, OBJ, OBJ, m, pos, dz, DX, LAM).loss(p, slices, meas)


def test_position_gradient_matches_central_differences(orc):
    md, p, truth, dz = _setup(orc)
    meas = md.forward(p, truth)
    start = truth * np.exp(0.15j * np.random.default_rng(4).standard_normal(truth.shape))
    loss, g, _ = md.position_grad(p, start, meas)
    assert abs(loss - md.loss(p, start, meas)) < 1e-12 * loss
    eps = 1e-4                       # every fraction stays inside (0, 1): no change of patch origin
    for s in range(len(POS)):
        for a in range(2):
            vals = []
            for h in (eps, 2 * eps):
                up, dn = POS.copy(), POS.copy()
                up[s, a] += h
                dn[s, a] -= h
                vals.append((_loss_at(orc, up, dz, 3, p, start, meas) - _loss_at(orc, dn, dz, 3, p, start, meas))
                            / (2 * h))
            fd = (4 * vals[0] - vals[1]) / 3   # Richardson: O(h^4)
            assert abs(fd - g[s, a]) <= 1e-6 * max(abs(g[s, a]), 1e-3 * loss), (s, a, fd, g[s, a])


def test_single_slice_gradient_equals_the_real_chain_rule(orc):
    """M = 1: Psi = FFT(T o P(f)), L = sum (sqrt(I) - |Psi|)^2, so
    dL/df = -2 sum (sqrt(I) - |Psi|) Re(conj(Psi) dPsi/df) / |Psi| with dPsi/df = FFT(T o dP/df)."""
    md, p, truth, dz = _setup(orc, m=1)
    meas = md.forward(p, truth * 1.05 * np.exp(0.2j))[:, ::-1, :].copy()   # any non-negative data
    start = truth[:1]
    _, g, _ = md.position_grad(p, start, meas)
    k = np.fft.fftfreq(N, 1.0 / N)
    spec = np.fft.fft2(p)
    for s, (py, px) in enumerate(POS):
        iy, ix = int(np.floor(py)), int(np.floor(px))
        fy, fx = py - iy, px - ix
        ramp = np.exp(-2j * np.pi * (k[:, None] * fy + k[None, :] * fx) / N)
        ps = np.fft.ifft2(spec * ramp)
        rows = (iy + np.arange(N)) % OBJ
        cols = (ix + np.arange(N)) % OBJ
        t = start[0][np.ix_(rows, cols)]
        psi = np.fft.fft2(t * ps)
        amp = np.abs(psi)
        for a, kk in enumerate((k[:, None] * np.ones((1, N)), np.ones((N, 1)) * k[None, :])):
            dps = np.fft.ifft2(spec * ramp * (-2j * np.pi * kk / N))
            dpsi = np.fft.fft2(t * dps)
            ref = -2 * np.sum((np.sqrt(meas[s]) - amp) * (np.conj(psi) * dpsi).real / amp)
            assert abs(ref - g[s, a]) < 1e-9 * np.abs(g).max(), (s, a, ref, g[s, a])


def test_curvature_bound_is_parsevals_closed_form(orc):
    md, p, truth, dz = _setup(orc)
    meas = md.forward(p, truth)
    _, _, c = md.position_grad(p, truth, meas)
    k = np.fft.fftfreq(N, 1.0 / N)
    power = np.abs(np.fft.fft2(p)) ** 2 / N ** 2                 # Parseval, unnormalised DFT
    dpy = np.sum(power * (2 * np.pi * k[:, None] / N) ** 2)
    dpx = np.sum(power * (2 * np.pi * k[None, :] / N) ** 2)
    tprod = np.prod([np.abs(truth[m]).max() ** 2 for m in range(truth.shape[0])])
    for s in range(len(POS)):                                     # independent of the shift
        assert abs(c[s, 0] - 2 * N * N * tprod * dpy) < 1e-10 * c[s, 0]
        assert abs(c[s, 1] - 2 * N * N * tprod * dpx) < 1e-10 * c[s, 1]


def test_gradient_vanishes_at_the_true_positions_and_steps_move_back(orc):
    md, p, truth, dz = _setup(orc)
    meas = md.forward(p, truth)
    loss, g, _ = md.position_grad(p, truth, meas)
    assert loss < 1e-20 * meas.sum() and np.abs(g).max() < 1e-9
    # positions displaced by up to 0.15 px: the majorised steps -g / c never raise the loss and
    # bring the positions back towards the truth (slowly: the bound ignores that only the
    # amplitude part of dPsi/df changes the amplitude loss)
    off = np.random.default_rng(7).uniform(-0.15, 0.15, POS.shape)   # fractions stay in (0, 1)
    pos = POS + off
    losses = []
    for _ in range(20):
        mdp = orc.Model(N, OBJ, OBJ, 3, pos, dz, DX, LAM)
        loss, g, c = mdp.position_grad(p, truth, meas)
        losses.append(loss)
        pos = pos - g / c
    assert all(b <= a * (1 + 1e-9) for a, b in zip(losses, losses[1:])), losses
    assert np.abs(pos - POS).max() < 0.7 * np.abs(off).max()
