"""Pins of the oracle's Poisson objective (the outlook of Sec. 6: maximum likelihood for
low-dose data).  The deviance L = sum |Psi|^2 - I + I log(I / |Psi|^2) is the negative
log-likelihood of the counts up to a constant; its differences between two iterates are
checked against scipy's Poisson log-pmf, its gradient by central differences and by the dense
single-layer matrix of eq. (Opt_Prob_Single_Layer_Matrix) at N = 4."""
import numpy as np
import pytest
import scipy.stats

from paper_2205_03902_amd import synth

from test_oracle_gradients import _dense_parts, _dense_q, _fd

DOSE = 1e3


def _setup(orc, n=16, obj=24, m=3, seed=0, objective=1):
    rng = np.random.default_rng(seed)
    pos = np.array([[0.0, 0.0], [3.5, 2.25], [-3.0, 17.5], [9.0, 9.5], [14.5, -1.0]])
    md = orc.Model(n, obj, obj, m, pos, np.array([2.0, 3.0, 1.5][: m - 1]), 0.2, 0.0487, objective=objective)
    truth = np.exp(1j * rng.uniform(0, 0.8, (m, obj, obj)))
    p = orc.probe(n, 0.2, 0.0487, 0.03, 15.0)
    clean = md.forward(p, truth)
    meas = synth.poisson_counts(clean, DOSE, seed + 1).astype(np.float64)
    start = np.exp(1j * rng.uniform(0, 0.3, (m, obj, obj))) * rng.uniform(0.8, 1.2, (m, obj, obj))
    return md, p, truth, clean, meas, start


def test_deviance_differences_are_poisson_log_likelihood_differences(orc):
    md, p, truth, _, meas, start = _setup(orc)
    n2 = md.n * md.n
    scale = DOSE / n2
    counts = np.rint(meas * scale)
    assert np.allclose(counts, meas * scale)
    meas = counts / scale                     # the exact counts on both sides (float32 storage removed)

    def nll(slices):
        lam = md.forward(p, slices) * scale
        return -scipy.stats.poisson.logpmf(counts, lam).sum()

    d1, d2 = md.loss(p, start, meas), md.loss(p, truth, meas)
    assert abs(scale * (d1 - d2) - (nll(start) - nll(truth))) < 1e-8 * abs(nll(start) - nll(truth))


def test_deviance_is_nonnegative_and_vanishes_on_noise_free_data(orc):
    md, p, truth, clean, meas, start = _setup(orc)
    assert md.loss(p, start, meas) > 0 and md.loss(p, truth, meas) > 0
    loss, gs, gp, _ = md.loss_grad(p, truth, clean)
    assert abs(loss) < 1e-9 * clean.sum()
    assert np.abs(gs).max() < 1e-8 and np.abs(gp).max() < 1e-8


def _fd_richardson(f, x, d, eps):
    """Central difference extrapolated from steps eps and eps / 2 (error O(eps^4)): the deviance
    bends sharply at dark pixels, where I / |Psi|^2 is large."""
    return (4 * _fd(f, x, d, eps / 2) - _fd(f, x, d, eps)) / 3


def test_poisson_gradients_match_central_differences(orc):
    md, p, _truth, _, meas, start = _setup(orc)
    loss, gs, gp, _ = md.loss_grad(p, start, meas)
    for d in synth.complex_directions(start.shape, 5, seed=4):
        fd = _fd_richardson(lambda x: md.loss(p, x, meas), start, d, 2e-5)
        an = 2 * np.vdot(gs, d).real
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * loss), (fd, an)
    for d in synth.complex_directions(p.shape, 5, seed=5):
        fd = _fd_richardson(lambda x: md.loss(x, start, meas), p, d * 0.01, 2e-5)
        an = 2 * np.vdot(gp, d * 0.01).real
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * loss), (fd, an)


@pytest.mark.parametrize("layer", [0, 2])
def test_poisson_layer_gradient_equals_the_dense_matrix_form(orc, layer):
    n, obj, m = 4, 6, 3
    rng = np.random.default_rng(30 + layer)
    pos = np.array([[0.0, 0.0], [1.5, 2.0], [4.0, 5.5], [5.0, 1.0]])
    dz = [2.0, 3.0]
    sl = rng.standard_normal((m, obj, obj)) + 1j * rng.standard_normal((m, obj, obj))
    probe = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    meas = rng.uniform(0, 4, (len(pos), n, n))
    md = orc.Model(n, obj, obj, m, pos, np.array(dz), 0.2, 0.0487, objective=1)
    f2, gs, parts = _dense_parts(orc, n, obj, sl, probe, pos, dz)
    q = _dense_q(f2, gs, parts, layer)
    qz = q @ sl[layer].reshape(-1)
    y = meas.reshape(-1)
    a2 = np.abs(qz) ** 2
    loss = np.sum(a2 - y + y * np.log(y / a2))
    grad = np.conj(q.T) @ (qz * (1 - y / a2))
    l2, g_l, _, _ = md.loss_grad(probe, sl, meas, layer=layer, want_probe=False)
    assert abs(l2 - loss) < 1e-10 * loss
    assert np.abs(g_l.reshape(-1) - grad).max() < 1e-10 * np.abs(grad).max()


def test_poisson_step_is_half_the_amplitude_step_and_descends_near_the_data(orc):
    md, p, truth, _, meas, _ = _setup(orc)
    amp = orc.Model(md.n, md.obj_h, md.obj_w, md.n_slices, md.positions, md.dz, 0.2, 0.0487, objective=0)
    start = truth * np.exp(0.05j * np.random.default_rng(9).standard_normal(truth.shape))
    for layer in range(md.n_slices):
        _, _, mu_p = md.layer_step(p, start, meas, layer, 1)
        _, _, mu_a = amp.layer_step(p, start, meas, layer, 1)
        assert mu_p == pytest.approx(0.5 * mu_a, rel=1e-14)
    x = start.copy()
    losses = []
    for sweep in range(3):
        for layer in range(md.n_slices):
            x, l, _ = md.layer_step(p, x, meas, layer, 1)
            losses.append(l)
    assert all(b <= a for a, b in zip(losses, losses[1:])), losses
