"""Pins for the oracle's amplitude-loss gradients (Sec. 3.2) and single-layer
measurement matrix Q_l (eqs. Opt_Prob_Single_Layer to Opt_Prob_Single_Layer_Matrix)."""
import numpy as np
import pytest

from paper_2205_03902_amd import synth


def _setup(orc, n=16, obj=24, m=3, seed=0, noise=True):
    rng = np.random.default_rng(seed)
    pos = np.array([[0.0, 0.0], [3.5, 2.25], [-3.0, 17.5], [9.0, 9.5], [14.5, -1.0]])
    md = orc.Model(n, obj, obj, m, pos, np.array([2.0, 3.0, 1.5][: m - 1]), 0.2, 0.0487)
    truth = np.exp(1j * rng.uniform(0, 0.8, (m, obj, obj)))
    p = orc.probe(n, 0.2, 0.0487, 0.03, 15.0)
    meas = md.forward(p, truth)
    if noise:
        meas = synth.poisson_counts(meas, 1e4, seed + 1).astype(np.float64)
    start = np.exp(1j * rng.uniform(0, 0.3, (m, obj, obj))) * rng.uniform(0.8, 1.2, (m, obj, obj))
    return md, p, truth, meas, start


def _fd(f, x, d, eps):
    return (f(x + eps * d) - f(x - eps * d)) / (2 * eps)


def test_slice_and_probe_gradients_match_central_differences(orc):
    md, p, _truth, meas, start = _setup(orc)
    loss, gs, gp, _ = md.loss_grad(p, start, meas)
    dirs = synth.complex_directions(start.shape, 6, seed=2)
    for d in dirs:
        fd = _fd(lambda x: md.loss(p, x, meas), start, d, 1e-5)
        an = 2 * np.vdot(gs, d).real          # dL = 2 Re <dL/dconj z, dz>
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * loss), (fd, an)
    pdirs = synth.complex_directions(p.shape, 6, seed=3)
    for d in pdirs:
        fd = _fd(lambda x: md.loss(x, start, meas), p, d * 0.01, 1e-5)
        an = 2 * np.vdot(gp, d * 0.01).real
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * loss), (fd, an)


def test_layer_mode_matches_full_gradient(orc):
    md, p, _truth, meas, start = _setup(orc)
    loss, gs, _, _ = md.loss_grad(p, start, meas, want_probe=False)
    for layer in range(md.n_slices):
        l2, g_l, _, ov = md.loss_grad(p, start, meas, layer=layer, want_probe=False, want_overlap=True)
        assert abs(l2 - loss) < 1e-12 * loss
        assert np.abs(g_l - gs[layer]).max() < 1e-12 * np.abs(gs[layer]).max()
        assert ov.min() >= 0.0


def test_gradient_vanishes_at_noise_free_truth(orc):
    md, p, truth, meas, _ = _setup(orc, noise=False)
    loss, gs, gp, _ = md.loss_grad(p, truth, meas)
    assert loss < 1e-20 * meas.sum()
    assert np.abs(gs).max() < 1e-9 and np.abs(gp).max() < 1e-9


def test_subset_loss_is_sum_over_positions(orc):
    md, p, _truth, meas, start = _setup(orc)
    parts = [md.loss(p, start, meas, subset=[s]) for s in range(md.n_pos)]
    assert abs(sum(parts) - md.loss(p, start, meas)) < 1e-12 * sum(parts)
    _, _, gp_all, _ = md.loss_grad(p, start, meas, want_slices=False)
    gsum = sum(md.loss_grad(p, start, meas, subset=[s], want_slices=False)[2] for s in range(md.n_pos))
    assert np.abs(gsum - gp_all).max() < 1e-12 * np.abs(gp_all).max()


# ---------------------------------------------------------------------------
# Dense single-layer matrices at tiny size, written from the paper's definitions.

def _dense_parts(orc, n, obj, slices, probe, pos, dz):
    f1 = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    f2 = np.kron(f1, f1)
    f2inv = np.conj(f2) / (n * n)
    gs = [f2inv @ np.diag(orc.propagator(n, 0.2, 0.0487, d).reshape(-1)) @ f2 for d in dz]
    out = []
    for py, px in pos:
        iy, ix = int(np.floor(py)), int(np.floor(px))
        ps = orc.shift(probe, py - iy, px - ix).reshape(-1)
        # E_s: the N^2 x HW extraction of the window (indices wrap around)
        e = np.zeros((n * n, obj * obj))
        for i in range(n):
            for j in range(n):
                e[i * n + j, ((iy + i) % obj) * obj + (ix + j) % obj] = 1.0
        o = [np.diag(e @ slices[m].reshape(-1)) for m in range(len(slices))]
        out.append((ps, e, o))
    return f2, gs, out


def _dense_q(f2, gs, parts, layer):
    blocks = []
    for ps, e, o in parts:
        s_vec = ps
        for m in range(layer):                       # S_l p^s = G_{l-1} O_{l-1} ... G_1 O_1 p^s
            s_vec = gs[m] @ (o[m] @ s_vec)
        r = np.eye(len(ps), dtype=complex)
        for m in range(layer + 1, len(o)):           # R_l = O_M G_{M-1} ... O_{l+1} G_l
            r = o[m] @ gs[m - 1] @ r
        blocks.append(f2 @ r @ np.diag(s_vec) @ e)
    return np.vstack(blocks)


@pytest.mark.parametrize("layer", [0, 1, 2])
def test_layer_gradient_equals_dense_amplitude_flow(orc, layer):
    n, obj, m = 4, 6, 3
    rng = np.random.default_rng(10 + layer)
    pos = np.array([[0.0, 0.0], [1.5, 2.0], [4.0, 5.5], [5.0, 1.0]])
    dz = [2.0, 3.0]
    sl = rng.standard_normal((m, obj, obj)) + 1j * rng.standard_normal((m, obj, obj))
    probe = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    meas = rng.uniform(0, 4, (len(pos), n, n))
    md = orc.Model(n, obj, obj, m, pos, np.array(dz), 0.2, 0.0487)
    f2, gs, parts = _dense_parts(orc, n, obj, sl, probe, pos, dz)
    q = _dense_q(f2, gs, parts, layer)
    z = sl[layer].reshape(-1)
    qz = q @ z
    y = meas.reshape(-1)
    phase = np.where(np.abs(qz) == 0, 0, qz / np.where(np.abs(qz) == 0, 1, np.abs(qz)))
    grad = np.conj(q.T) @ (qz - phase * np.sqrt(y))          # Sec. 3.2
    loss = np.sum((np.sqrt(y) - np.abs(qz)) ** 2)
    l2, g_l, _, _ = md.loss_grad(probe, sl, meas, layer=layer, want_probe=False)
    assert abs(l2 - loss) < 1e-10 * loss
    assert np.abs(g_l.reshape(-1) - grad).max() < 1e-10 * np.abs(grad).max()


@pytest.mark.parametrize("layer", [0, 1, 2])
def test_step_size_equals_inverse_spectral_norm_for_unit_slices(orc, layer):
    """For unit-modulus slices after layer l, ||Q_l||^2 = N^2 max_pixel sum_s |psi_l^s|^2
    and the oracle's step is exactly ||Q_l||^{-2} (Sec. 3.2); otherwise it is a lower bound."""
    n, obj, m = 4, 6, 3
    rng = np.random.default_rng(20 + layer)
    pos = np.array([[0.0, 0.0], [1.5, 2.0], [4.0, 5.5]])
    dz = [2.0, 3.0]
    sl = np.exp(1j * rng.uniform(0, 2, (m, obj, obj)))
    sl[0] *= rng.uniform(0.5, 1.5, (obj, obj))          # slices before l may be anything
    probe = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    meas = rng.uniform(0, 4, (len(pos), n, n))
    md = orc.Model(n, obj, obj, m, pos, np.array(dz), 0.2, 0.0487)
    f2, gs, parts = _dense_parts(orc, n, obj, sl, probe, pos, dz)
    qn2 = np.linalg.norm(_dense_q(f2, gs, parts, layer), 2) ** 2
    _, _, mu = md.layer_step(probe, sl, meas, layer, 1)
    assert abs(mu * qn2 - 1) < 1e-10        # the slices after l all have unit modulus
    # with a non-unit slice after l the step is still <= ||Q_l||^{-2}
    sl2 = sl.copy()
    sl2[m - 1] *= rng.uniform(0.2, 1.3, (obj, obj))
    f2, gs, parts = _dense_parts(orc, n, obj, sl2, probe, pos, dz)
    qn2b = np.linalg.norm(_dense_q(f2, gs, parts, layer), 2) ** 2
    _, _, mu2 = md.layer_step(probe, sl2, meas, layer, 1)
    assert mu2 * qn2b <= 1 + 1e-12


# ---------------------------------------------------------------------------
# The probe's measurement matrix Q_p (Sec. 3.5): Psi^s = F O_M G_{M-1} ... G_1 O_1 Sh_s p, Sh_s the
# sub-pixel shift of the probe (a phase ramp on its spectrum), stacked over the positions of a subset.

def _dense_shift(n, fy, fx):
    """N^2 x N^2 sub-pixel shift: F^{-1} diag(exp(-2 pi i (k_y f_y + k_x f_x) / N)) F, k signed with the
    Nyquist bin at -N/2, written from the definition (no library FFT)."""
    k = np.array([i if i < n // 2 else i - n for i in range(n)], dtype=float)
    f1 = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    f2 = np.kron(f1, f1)
    ramp = np.exp(-2j * np.pi * (np.add.outer(k * fy, k * fx)) / n).reshape(-1)
    return (np.conj(f2) / (n * n)) @ np.diag(ramp) @ f2


def _dense_qp(orc, n, obj, slices, pos, dz, subset):
    f1 = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    f2 = np.kron(f1, f1)
    gs = [(np.conj(f2) / (n * n)) @ np.diag(orc.propagator(n, 0.2, 0.0487, d).reshape(-1)) @ f2 for d in dz]
    blocks = []
    for s in subset:
        py, px = pos[s]
        iy, ix = int(np.floor(py)), int(np.floor(px))
        idx = np.array([((iy + i) % obj) * obj + (ix + j) % obj for i in range(n) for j in range(n)])
        r = np.diag(slices[0].reshape(-1)[idx])
        for m in range(1, len(slices)):
            r = np.diag(slices[m].reshape(-1)[idx]) @ gs[m - 1] @ r
        blocks.append(f2 @ r @ _dense_shift(n, py - iy, px - ix))
    return np.vstack(blocks)


@pytest.mark.parametrize("subset", [None, [2], [0, 3, 4]])
def test_probe_step_size_equals_inverse_spectral_norm_for_unit_slices(orc, subset):
    """For unit-modulus slices Q_p^H Q_p = N^2 |subset| I, so the probe step
    mu_p = 1 / (N^2 |subset| prod_m max|t_m|^2) is exactly ||Q_p||^{-2} (Sec. 3.2 step rule applied to the
    probe step of Sec. 3.5); with a slice of non-unit modulus it is smaller than ||Q_p||^{-2}."""
    n, obj, m = 4, 6, 3
    rng = np.random.default_rng(40 + (0 if subset is None else len(subset)))
    pos = np.array([[0.0, 0.0], [1.5, 2.0], [4.0, 5.5], [5.25, 1.0], [2.0, 3.75]])
    dz = [2.0, 3.0]
    sub = list(range(len(pos))) if subset is None else subset
    sl = np.exp(1j * rng.uniform(0, 2, (m, obj, obj)))
    probe = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    meas = rng.uniform(0, 4, (len(pos), n, n))
    md = orc.Model(n, obj, obj, m, pos, np.array(dz), 0.2, 0.0487)
    qn2 = np.linalg.norm(_dense_qp(orc, n, obj, sl, pos, dz, sub), 2) ** 2
    assert abs(qn2 / (n * n * len(sub)) - 1) < 1e-12
    _, _, mu = md.probe_step(probe, sl, meas, subset, 1)
    assert abs(mu * qn2 - 1) < 1e-10
    sl2 = sl.copy()
    sl2[1] *= rng.uniform(0.2, 1.3, (obj, obj))
    qn2b = np.linalg.norm(_dense_qp(orc, n, obj, sl2, pos, dz, sub), 2) ** 2
    _, _, mu2 = md.probe_step(probe, sl2, meas, subset, 1)
    assert mu2 * qn2b <= 1 + 1e-12
    assert mu2 * qn2b < 0.999          # strictly below: the bound is not tight here


def test_probe_gradient_equals_dense_amplitude_flow(orc):
    """dL/d conj(p) = Q_p^H (Q_p p - sqrt(y) o phase(Q_p p)) (Sec. 3.2, Sec. 3.5), with sub-pixel shifts
    and general complex slices."""
    n, obj, m = 4, 6, 3
    rng = np.random.default_rng(50)
    pos = np.array([[0.0, 0.0], [1.5, 2.0], [4.0, 5.5], [5.25, 1.0]])
    dz = [2.0, 3.0]
    sl = rng.standard_normal((m, obj, obj)) + 1j * rng.standard_normal((m, obj, obj))
    probe = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    meas = rng.uniform(0, 4, (len(pos), n, n))
    md = orc.Model(n, obj, obj, m, pos, np.array(dz), 0.2, 0.0487)
    for sub in ([0, 1, 2, 3], [1, 3]):
        q = _dense_qp(orc, n, obj, sl, pos, dz, sub)
        qz = q @ probe.reshape(-1)
        y = meas[sub].reshape(-1)
        phase = qz / np.abs(qz)
        grad = np.conj(q.T) @ (qz - phase * np.sqrt(y))
        loss = np.sum((np.sqrt(y) - np.abs(qz)) ** 2)
        l2, _, gp, _ = md.loss_grad(probe, sl, meas, subset=sub, want_slices=False)
        assert abs(l2 - loss) < 1e-10 * loss
        assert np.abs(gp.reshape(-1) - grad).max() < 1e-10 * np.abs(grad).max()
