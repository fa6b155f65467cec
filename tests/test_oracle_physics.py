"""Pins for the oracle's physics: wavelength (Sec. 5.3.2), Fresnel propagator
(eq. fresnel_element), probe (Sec. 2.1, Fig. 3 caption) and the sub-pixel shift."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_wavelength_printed_values(orc):
    rows = np.loadtxt(os.path.join(GOLDEN, "wavelength.txt"))
    for volts, lam, tol in rows:
        assert abs(orc.wavelength(volts) - lam) <= tol, (volts, orc.wavelength(volts), lam)


def test_wavelength_nonrelativistic_limit(orc):
    # for eU << m c^2 the formula reduces to the de Broglie wavelength h / sqrt(2 m e U)
    h, m, e = 6.62607015e-34, 9.1093837015e-31, 1.602176634e-19
    for volts in (1.0, 10.0):
        ref = h / np.sqrt(2 * m * e * volts) * 1e10
        assert abs(orc.wavelength(volts) / ref - 1) < 1e-5


def test_propagator_unit_modulus_and_identity(orc):
    h = orc.propagator(64, 0.2, 0.0487, 2.0)
    assert np.abs(np.abs(h) - 1).max() < 1e-14
    h0 = orc.propagator(64, 0.2, 0.0487, 0.0)
    assert np.abs(h0 - 1).max() == 0.0


def test_propagator_closed_form_value(orc):
    n, dx, lam, dz = 32, 0.2, 0.0487, 2.0
    h = orc.propagator(n, dx, lam, dz)
    ky, kx = 3, n - 5                     # q = 3/(N dx), -5/(N dx)
    qy, qx = 3 / (n * dx), -5 / (n * dx)
    ref = np.exp(-1j * np.pi * dz * lam * (qy ** 2 + qx ** 2))
    assert abs(h[ky, kx] - ref) < 1e-14
    # the Nyquist bin uses q = -N/2 / (N dx)
    qn = -0.5 / dx
    assert abs(h[n // 2, 0] - np.exp(-1j * np.pi * dz * lam * qn ** 2)) < 1e-14


def test_propagator_tilt_term(orc):
    n, dx, lam, dz, ty, tx = 16, 0.2, 0.0487, 3.0, 0.01, -0.02
    h = orc.propagator(n, dx, lam, dz, ty, tx)
    q = np.fft.fftfreq(n, dx)
    ref = np.exp(-1j * np.pi * dz * lam * ((q[:, None] ** 2 + q[None, :] ** 2)
                                           + 2 * (q[None, :] * np.sin(tx) / lam + q[:, None] * np.sin(ty) / lam)))
    assert np.abs(h - ref).max() < 1e-13


def test_propagator_semigroup_and_unitary(orc):
    n, dx, lam = 32, 0.2, 0.0487
    ha, hb, hab = (orc.propagator(n, dx, lam, d) for d in (1.5, 2.5, 4.0))
    assert np.abs(ha * hb - hab).max() < 1e-13
    # G_a G_b = G_{a+b} and G unitary, applied to a field with the oracle's FFT
    x = np.random.default_rng(0).standard_normal((n, n)) + 0j

    def g(field, h):
        return orc.fft2d(orc.fft2d(field) * h, +1) / (n * n)

    assert np.abs(g(g(x, ha), hb) - g(x, hab)).max() < 1e-12
    assert abs(np.linalg.norm(g(x, ha)) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)


def _probe_by_definition(n, dx, lam, alpha, defocus):
    """Inverse DFT of the aperture written out as a sum over the disk (no FFT)."""
    q = np.fft.fftfreq(n, dx)
    kk = np.fft.fftfreq(n) * n
    out = np.zeros((n, n), complex)
    y = np.arange(n)[:, None]
    x = np.arange(n)[None, :]
    for iy in range(n):
        for ix in range(n):
            q2 = q[iy] ** 2 + q[ix] ** 2
            if lam * np.sqrt(q2) <= alpha:
                a = np.exp(-1j * np.pi * defocus * lam * q2)
                out += a * np.exp(2j * np.pi * (kk[iy] * (y - n // 2) + kk[ix] * (x - n // 2)) / n)
    return out / np.sqrt(np.sum(np.abs(out) ** 2))


@pytest.mark.parametrize("defocus", [0.0, 50.0])
def test_probe_matches_definition(orc, defocus):
    n, dx, lam, alpha = 32, 0.2, 0.0487, 0.03
    p = orc.probe(n, dx, lam, alpha, defocus)
    ref = _probe_by_definition(n, dx, lam, alpha, defocus)
    assert np.abs(p - ref).max() < 1e-13
    assert abs(np.sum(np.abs(p) ** 2) - 1) < 1e-13


def test_probe_in_focus_is_centred_real_airy(orc):
    from scipy.special import j1
    n, dx, lam, alpha = 128, 0.2, 0.0487, 0.02
    p = orc.probe(n, dx, lam, alpha, 0.0)
    assert np.abs(p.imag).max() < 1e-12 * np.abs(p).max()
    assert np.unravel_index(np.argmax(np.abs(p)), p.shape) == (n // 2, n // 2)
    # close to the continuous Airy pattern 2 J1(2 pi qmax r) / (2 pi qmax r) (Sec. 2.1)
    qmax = alpha / lam
    y, x = np.mgrid[0:n, 0:n]
    r = np.hypot(y - n // 2, x - n // 2) * dx
    arg = 2 * np.pi * qmax * np.where(r == 0, 1e-12, r)
    airy = 2 * j1(arg) / arg
    c = np.vdot(airy, p.real).real / (np.linalg.norm(airy) * np.linalg.norm(p.real))
    assert c > 0.99


def test_shift_integer_is_roll_and_adjoint(orc):
    n = 16
    rng = np.random.default_rng(1)
    p = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    # p_{y - 1, x - 1}: the phase ramp with an integer shift is a cyclic roll
    s = orc.shift(p, 1.0, 1.0)
    assert np.abs(s - np.roll(p, (1, 1), axis=(0, 1))).max() < 1e-12
    assert np.array_equal(orc.shift(p, 0.0, 0.0), p)
    a = orc.shift(p, 0.5, 0.25)
    b = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    assert abs(np.vdot(b, a) - np.vdot(orc.unshift(b, 0.5, 0.25), p)) < 1e-11
    assert abs(np.linalg.norm(a) - np.linalg.norm(p)) < 1e-12 * np.linalg.norm(p)
    assert np.abs(orc.unshift(a, 0.5, 0.25) - p).max() < 1e-12
    # two half-pixel shifts compose to a one-pixel roll (the Nyquist bin uses k = -N/2)
    h2 = orc.shift(orc.shift(p, 0.5, 0.0), 0.5, 0.0)
    assert np.abs(h2 - np.roll(p, 1, axis=0)).max() < 1e-12


def test_aberrated_probe_with_defocus_only_is_the_probe(orc):
    a = orc.probe_aberrated(32, 0.2, 0.0487, 0.03, 40.0)
    b = orc.probe(32, 0.2, 0.0487, 0.03, 40.0)
    assert np.abs(a - b).max() < 1e-13


def test_aberrated_probe_is_the_disk_sum_of_its_definition(orc):
    """Brute-force inverse DFT over the aperture (no FFT) with the aberration phase
    chi = pi lam C1 q^2 + pi lam A1 q^2 cos 2(phi - phi_A1) + pi/2 lam^3 C3 q^4."""
    n, dx, lam, alpha = 16, 0.2, 0.0487, 0.05
    c1, a1, pa, c3 = 30.0, 12.0, 0.4, 2.0e5
    got = orc.probe_aberrated(n, dx, lam, alpha, c1, a1, pa, c3)
    k = np.fft.fftfreq(n) * n
    want = np.zeros((n, n), complex)
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for iy in range(n):
        for ix in range(n):
            qy, qx = k[iy] / (n * dx), k[ix] / (n * dx)
            q = np.hypot(qy, qx)
            if lam * q > alpha:
                continue
            chi = (np.pi * lam * c1 * q * q + np.pi * lam * a1 * q * q * np.cos(2 * (np.arctan2(qy, qx) - pa))
                   + 0.5 * np.pi * lam ** 3 * c3 * q ** 4)
            want += np.exp(-1j * chi) * (-1.0) ** (iy + ix) * np.exp(2j * np.pi * (k[iy] * yy + k[ix] * xx) / n)
    want /= np.linalg.norm(want)
    assert np.abs(got - want).max() < 1e-12


def test_astigmatism_rotation_and_spherical_symmetry(orc):
    n, dx, lam, alpha = 32, 0.2, 0.0487, 0.03
    a = orc.probe_aberrated(n, dx, lam, alpha, 20.0, 15.0, 0.3)
    b = orc.probe_aberrated(n, dx, lam, alpha, 20.0, -15.0, 0.3 + np.pi / 2)
    assert np.abs(a - b).max() < 1e-12
    s = orc.probe_aberrated(n, dx, lam, alpha, 20.0, 0.0, 0.0, 5.0e5)
    assert np.abs(s - s.T).max() < 1e-12          # rotationally symmetric aberrations
    assert np.abs(a - a.T).max() > 1e-3           # astigmatism is not
