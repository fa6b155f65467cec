"""Pins for the oracle's Algorithm 1 (layer-wise estimation) and probe step (Sec. 3.3, 3.5).

Monotone descent: with u = Qz, |u| >= Re(conj(phi) u) for the current phase phi, so
f(z') <= ||Q z' - sqrt(y) o phi||^2 =: g(z') with g(z) = f(z); a gradient step on the
quadratic g with mu <= ||Q||^{-2} does not increase g, hence the loss never increases
after a layer step or a probe step."""
import numpy as np

from paper_2205_03902_amd import configs, synth


def _small(orc, seed=0, dose=1e4):
    geo = configs.small(n=16, obj=24, n_slices=3, scan=(3, 3), step_px=3.5, seed=seed)
    md = orc.Model.from_geometry(geo)
    truth = np.exp(1j * synth.KAPPA * synth.specimen(geo))
    p = orc.probe(geo.n, geo.pixel_size, geo.wavelength, geo.alpha, geo.defocus)
    meas = synth.poisson_counts(md.forward(p, truth), dose, seed + 1).astype(np.float64)
    return geo, md, truth, p, meas


def test_layer_and_probe_steps_never_increase_the_loss(orc):
    geo, md, truth, p, meas = _small(orc)
    sl = np.ones_like(truth)
    p0 = orc.probe(geo.n, geo.pixel_size, geo.wavelength, geo.alpha, 1.3 * geo.defocus)
    hist = []
    for _ in range(4):
        for layer in range(geo.n_slices):
            sl, loss, mu = md.layer_step(p0, sl, meas, layer, 2)
            hist.append(loss)
            assert mu > 0
        p0, loss, mu = md.probe_step(p0, sl, meas, None, 2)
        hist.append(loss)
    hist.append(md.loss(p0, sl, meas))
    d = np.diff(hist)
    assert (d <= 1e-12 * hist[0]).all(), hist
    assert hist[-1] < 0.9 * hist[0]


def test_layer_step_is_one_amplitude_flow_step(orc):
    """o_l <- o_l - mu * grad, mu = 1 / (N^2 prod_{m>l} max|t_m|^2 max W_l)."""
    geo, md, truth, p, meas = _small(orc)
    sl = np.ones_like(truth) * 1.1
    sl[2] *= np.exp(0.1j)
    layer = 1
    loss, g, _, w = md.loss_grad(p, sl, meas, layer=layer, want_probe=False, want_overlap=True)
    mu = 1.0 / (geo.n ** 2 * 1.21 * w.max())
    new, l2, mu2 = md.layer_step(p, sl, meas, layer, 1)
    assert abs(mu2 / mu - 1) < 1e-13 and abs(l2 - loss) < 1e-12 * loss
    ref = sl.copy()
    ref[layer] -= mu * g
    assert np.abs(new - ref).max() < 1e-14
    # Gauss-Seidel: only slice l moves
    assert np.array_equal(new[0], sl[0]) and np.array_equal(new[2], sl[2])


def test_probe_step_size_and_subset(orc):
    geo, md, truth, p, meas = _small(orc)
    sub = [0, 4, 8]
    loss, _, gp, _ = md.loss_grad(p, truth, meas, subset=sub, want_slices=False)
    newp, l2, mu = md.probe_step(p, truth, meas, sub, 1)
    prod = np.prod([np.max(np.abs(t) ** 2) for t in truth])
    assert abs(mu * geo.n ** 2 * len(sub) * prod - 1) < 1e-12
    assert np.abs(newp - (p - mu * gp)).max() < 1e-15


def test_truth_is_a_fixed_point_without_noise(orc):
    geo, md, truth, p, _ = _small(orc)
    meas = md.forward(p, truth)
    sl, loss, _ = md.layer_step(p, truth, meas, 1, 1)
    assert loss < 1e-20 * meas.sum()
    assert np.abs(sl - truth).max() < 1e-12


def test_config0_fifty_sweeps_reduce_the_loss(orc):
    geo = configs.CFG0
    md = orc.Model.from_geometry(geo)
    truth = synth.transmissions(synth.specimen(geo)).astype(np.complex128)
    p = orc.probe(geo.n, geo.pixel_size, geo.wavelength, geo.alpha, geo.defocus)
    meas = synth.poisson_counts(md.forward(p, truth), geo.dose, geo.seed + 1).astype(np.float64)
    l0 = md.loss(p, np.ones_like(truth), meas)
    sl, _, hist = orc.layerwise(md, p, np.ones_like(truth), meas, sweeps=geo.iterations)
    lf = md.loss(p, sl, meas)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    assert lf < 0.5 * l0


def test_full_step_is_every_layer_step_taken_from_the_same_iterate(orc):
    """The full-gradient (Jacobi) step moves each slice exactly as a layer step of Algorithm 1
    started from the same slices would; with one slice it is the layer step."""
    import numpy as np
    from paper_2205_03902_amd import synth
    rng = np.random.default_rng(3)
    n, obj, m = 16, 24, 3
    pos = np.array([[0.0, 0.0], [3.5, 2.25], [-3.0, 17.5], [9.0, 9.5]])
    for objective in (0, 1):
        md = orc.Model(n, obj, obj, m, pos, np.array([2.0, 1.5]), 0.2, 0.0487, objective=objective)
        p = orc.probe(n, 0.2, 0.0487, 0.03, 15.0)
        truth = np.exp(1j * rng.uniform(0, 0.8, (m, obj, obj)))
        meas = synth.poisson_counts(md.forward(p, truth), 1e4, 4).astype(np.float64)
        start = np.exp(1j * rng.uniform(0, 0.3, (m, obj, obj))) * rng.uniform(0.9, 1.1, (m, obj, obj))
        new, loss, mu = md.full_step(p, start, meas)
        assert loss == md.loss(p, start, meas)
        for layer in range(m):
            ls, ll, lmu = md.layer_step(p, start, meas, layer, 1)
            assert lmu == mu[layer]
            assert np.array_equal(new[layer], ls[layer])
    one = orc.Model(n, obj, obj, 1, pos, np.zeros(1), 0.2, 0.0487)
    meas1 = one.forward(p, truth[:1])
    a, la, ma = one.full_step(p, start[:1], meas1)
    b, lb, mb = one.layer_step(p, start[:1], meas1, 0, 1)
    assert np.array_equal(a, b) and la == lb and ma[0] == mb
    # a step scale multiplies every step size
    md = orc.Model(n, obj, obj, m, pos, np.array([2.0, 1.5]), 0.2, 0.0487)
    meas = md.forward(p, truth)
    full, _, mu1 = md.full_step(p, start, meas)
    half, _, mu2 = md.full_step(p, start, meas, step_scale=0.5)
    assert np.allclose(mu2, 0.5 * mu1, rtol=1e-15)
    assert np.allclose(half - start, 0.5 * (full - start), rtol=0, atol=1e-13)
