"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (relative L2): exit waves and intensities 1e-5, gradients 1e-4; the loss
and step sizes 1e-5.  The GPU computes in FP32 complex with FP64 loss and
step-size reductions, so these bars leave a margin of 10-100x over its
rounding error after the chained FFTs.
"""
import numpy as np
import pytest

from parity_cases import make_case, rel, small_geometry, small_positions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FWD = 1e-5
TOL_GRAD = 1e-4


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _plan(case, dev, budget=0):
    from paper_2205_03902_amd import abi
    # every wave stored: a budget then splits the positions into batches
    return abi.Plan.from_geometry(case.geo, positions=case.model.positions, budget_bytes=budget, device=dev,
                                  checkpoint_every=1)


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


_CASES = {}


def case_for(n):
    if n not in _CASES:
        g = small_geometry(n)
        print(f"[case] n={n} obj={g.obj_h} M={g.n_slices} S={g.n_pos}", flush=True)
        _CASES[n] = make_case(g, positions=small_positions(g))
    return _CASES[n]


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_make_probe(dev, n):
    import oracle
    c = case_for(n)
    plan = _plan(c, dev)
    for defocus in (0.0, c.geo.defocus):
        p = plan.make_probe(c.geo.alpha, defocus).cpu().numpy()
        ref = oracle.probe(n, c.geo.pixel_size, c.geo.wavelength, c.geo.alpha, defocus)
        assert rel(p, ref) < 2e-6, (n, defocus, rel(p, ref))


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_forward(dev, n):
    c = case_for(n)
    plan = _plan(c, dev)
    inten, ew = plan.forward(_t(c.probe, dev), _t(c.start, dev), exit_waves=True)
    ref_i, ref_e = c.model.forward(c.probe, c.start, exit_waves=True)
    ei, ee = rel(inten.cpu().numpy(), ref_i), rel(ew.cpu().numpy(), ref_e)
    print(f"n={n} forward rel L2: intensity {ei:.2e} exit {ee:.2e}")
    assert ei < TOL_FWD and ee < TOL_FWD


@pytest.mark.parametrize("n", [16, 32, 64, 128])
def test_adjoint(dev, n):
    c = case_for(n)
    plan = _plan(c, dev)
    loss, gs, gp = plan.adjoint(_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev))
    ref_l, ref_gs, ref_gp, _ = c.model.loss_grad(c.probe, c.start, c.measured)
    el = abs(loss.item() - ref_l) / ref_l
    egs, egp = rel(gs.cpu().numpy(), ref_gs), rel(gp.cpu().numpy(), ref_gp)
    print(f"n={n} adjoint: loss {el:.2e} grad slices {egs:.2e} grad probe {egp:.2e}")
    assert el < TOL_FWD and egs < TOL_GRAD and egp < TOL_GRAD


@pytest.mark.parametrize("n,layer", [(32, 0), (32, 1), (32, 2), (128, 1)])
def test_layer_step(dev, n, layer):
    c = case_for(n)
    plan = _plan(c, dev)
    s_t = _t(c.start, dev)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    plan.layer_step(layer, 2, _t(c.probe, dev), s_t, _t(c.measured, dev), loss=out[0:1], mu=out[1:2])
    ref_s, ref_l, ref_mu = c.model.layer_step(c.probe, c.start, c.measured, layer, 2)
    got = s_t.cpu().numpy()
    el, emu = abs(out[0].item() - ref_l) / ref_l, abs(out[1].item() - ref_mu) / ref_mu
    es = rel(got, ref_s)
    ed = rel(got - c.start, ref_s - c.start)
    print(f"n={n} layer {layer}: loss {el:.2e} mu {emu:.2e} slices {es:.2e} step {ed:.2e}")
    assert el < TOL_FWD and emu < TOL_FWD and es < TOL_FWD and ed < 10 * TOL_GRAD
    others = [m for m in range(c.geo.n_slices) if m != layer]
    assert np.array_equal(got[others], c.start[others])


@pytest.mark.parametrize("n", [32, 64])
def test_algorithm1_sweeps_match_the_oracle(dev, n):
    """Two sweeps of Algorithm 1 through the Python driver (every layer in order, Gauss-Seidel,
    then a probe step) against the oracle's driver: the loss of every step within 1e-5, and
    the slices and probe after the 2 (M + 1) chained steps within 1e-4 (each step adds about
    1e-6 of FP32 rounding to its iterate, and later steps carry the earlier ones)."""
    import oracle
    from paper_2205_03902_amd import layerwise
    c = case_for(n)
    plan = _plan(c, dev)
    p0 = (c.probe * np.exp(0.05j)).astype(np.complex64)
    p_t, s_t = _t(p0, dev), _t(c.start, dev)
    hist = layerwise.reconstruct(plan, p_t, s_t, _t(c.measured, dev), sweeps=2, k_steps=1, probe_steps=1)
    ref_s, ref_p, ref_h = oracle.layerwise(c.model, p0, c.start, c.measured, sweeps=2, k_steps=1, probe_steps=1)
    assert hist.kind == ([f"layer{m}" for m in range(c.geo.n_slices)] + ["probe"]) * 2
    assert len(ref_h) == len(hist.loss)
    el = max(abs(a - b) / b for a, b in zip(hist.loss, ref_h))
    es, ep = rel(s_t.cpu().numpy(), ref_s), rel(p_t.cpu().numpy(), ref_p)
    print(f"n={n}: losses {el:.2e} slices {es:.2e} probe {ep:.2e}")
    assert all(b2 <= b1 for b1, b2 in zip(hist.loss, hist.loss[1:])), hist.loss
    assert el < TOL_FWD and es < TOL_GRAD and ep < TOL_GRAD


@pytest.mark.parametrize("subset", [None, [0, 4, 8], [4]])
def test_probe_step(dev, subset):
    c = case_for(32)
    plan = _plan(c, dev)
    p0 = (c.probe * np.exp(0.05j)).astype(np.complex64)
    p_t = _t(p0, dev)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    plan.probe_step(2, p_t, _t(c.start, dev), _t(c.measured, dev), subset=subset, loss=out[0:1], mu=out[1:2])
    ref_p, ref_l, ref_mu = c.model.probe_step(p0, c.start, c.measured, subset, 2)
    got = p_t.cpu().numpy()
    # a single position is solved almost exactly by one step (Q_p is N x a unitary map
    # for unit-modulus slices), so the loss is measured against the starting loss
    scale = c.model.loss(p0, c.start, c.measured, subset=subset)
    el, emu = abs(out[0].item() - ref_l) / scale, abs(out[1].item() - ref_mu) / ref_mu
    ep, ed = rel(got, ref_p), rel(got - p0, ref_p - p0)
    print(f"probe step subset={subset}: loss {el:.2e} mu {emu:.2e} probe {ep:.2e} step {ed:.2e}")
    assert el < TOL_FWD and emu < TOL_FWD and ep < TOL_FWD and ed < 10 * TOL_GRAD


def test_batching_and_repeats_are_bitwise_identical(dev):
    c = case_for(32)
    from paper_2205_03902_amd import abi
    full = _plan(c, dev)
    ws = full.workspace.numel()
    n2 = c.geo.n ** 2
    per_position = c.geo.n_slices * n2 * 8 + n2 * 8 + n2 * 4 + 8
    small = _plan(c, dev, budget=ws - 6 * per_position)   # a few positions per batch
    assert 1 < small.batch < full.batch == c.geo.n_pos
    args = (_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev))
    l1, g1, p1 = full.adjoint(*args)
    l1b, g1b, p1b = full.adjoint(*args)
    l2, g2, p2 = small.adjoint(*args)
    # one plan reproduces itself bit for bit (fixed reduction order, no atomics)
    assert torch.equal(g1, g1b) and torch.equal(p1, p1b) and l1.item() == l1b.item()
    # another batch size regroups the FP32 sums: equal up to rounding
    assert rel(g2.cpu().numpy(), g1.cpu().numpy()) < 1e-6 and rel(p2.cpu().numpy(), p1.cpu().numpy()) < 1e-6
    assert abs(l1.item() - l2.item()) <= 1e-12 * l1.item()
    i1 = full.forward(args[0], args[1])
    i2 = small.forward(args[0], args[1])
    assert torch.equal(i1, i2)
    del abi


def test_autograd_function_matches_oracle(dev):
    from paper_2205_03902_amd.autograd import amplitude_loss
    c = case_for(32)
    plan = _plan(c, dev)
    p_t = _t(c.probe, dev).requires_grad_(True)
    s_t = _t(c.start, dev).requires_grad_(True)
    loss = amplitude_loss(plan, p_t, s_t, _t(c.measured, dev))
    (3.0 * loss).backward()
    ref_l, ref_gs, ref_gp, _ = c.model.loss_grad(c.probe, c.start, c.measured)
    assert abs(loss.item() - ref_l) / ref_l < TOL_FWD
    # torch's complex gradient of a real loss is 2 dL/d conj(z)
    assert rel(s_t.grad.cpu().numpy(), 6.0 * ref_gs) < TOL_GRAD
    assert rel(p_t.grad.cpu().numpy(), 6.0 * ref_gp) < TOL_GRAD


def test_gpu_gradient_matches_oracle_finite_differences(dev):
    from paper_2205_03902_amd import synth
    c = case_for(32)
    plan = _plan(c, dev)
    _, gs, gp = plan.adjoint(_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev))
    gs, gp = gs.cpu().numpy().astype(np.complex128), gp.cpu().numpy().astype(np.complex128)
    start = c.start.astype(np.complex128)
    probe = c.probe.astype(np.complex128)
    dirs = synth.complex_directions(start.shape, 6, seed=c.geo.seed + 2)
    pdirs = synth.complex_directions(probe.shape, 6, seed=c.geo.seed + 5) * 0.01
    # The amplitude loss bends sharply at dark detector pixels: a step of 1e-3 along a
    # unit-variance direction leaves a truncation error near 1e-3 even after Richardson
    # extrapolation, while 1e-5 brings it below 1e-9 with FP64 rounding still ~1e-9.
    eps = 1e-5

    def fd(f, x, d):
        # Richardson-extrapolated central difference, O(eps^4)
        d1 = (f(x + eps * d) - f(x - eps * d)) / (2 * eps)
        d2 = (f(x + 0.5 * eps * d) - f(x - 0.5 * eps * d)) / eps
        return (4 * d2 - d1) / 3

    for d in dirs:
        ref = fd(lambda x: c.model.loss(probe, x, c.measured), start, d)
        got = 2 * np.vdot(gs, d).real
        assert abs(got - ref) <= TOL_GRAD * abs(ref), (got, ref)
    for d in pdirs:
        ref = fd(lambda x: c.model.loss(x, start, c.measured), probe, d)
        got = 2 * np.vdot(gp, d).real
        assert abs(got - ref) <= TOL_GRAD * abs(ref), (got, ref)


def test_zero_far_field_follows_the_zero_phase_rule(dev):
    """Psi = 0 everywhere (zero probe): residual = Psi = 0, so every gradient is exactly 0
    and the loss is the total measured intensity (Sec. 3.2)."""
    c = case_for(16)
    plan = _plan(c, dev)
    zero = np.zeros_like(c.probe)
    loss, gs, gp = plan.adjoint(_t(zero, dev), _t(c.start, dev), _t(c.measured, dev))
    assert torch.count_nonzero(gs).item() == 0 and torch.count_nonzero(gp).item() == 0
    ref = float(np.sum(c.measured.astype(np.float64)))
    assert abs(loss.item() - ref) <= 1e-12 * ref


@pytest.mark.parametrize("lines", [False, True])
@pytest.mark.parametrize("kind", ["single_slice", "one_position", "object_equals_window"])
def test_edge_geometries(dev, kind, lines):
    """On the default path (the fused kernel at these sizes) and forced onto the line kernels."""
    from paper_2205_03902_amd import abi, configs
    if kind == "single_slice":
        g = configs.small(n=32, obj=40, n_slices=1, scan=(2, 2), step_px=5.5, seed=3)
        pos = None
    elif kind == "one_position":
        g = configs.small(n=64, obj=64, n_slices=4, scan=(1, 1), step_px=0.0, seed=4)
        pos = np.array([[17.25, -40.5]])
    else:
        # H = W = N: the paper's full-field periodic model, every window wraps
        g = configs.small(n=32, obj=32, n_slices=3, scan=(3, 3), step_px=7.0, seed=5)
        pos = None
    c = make_case(g, positions=pos)
    plan = _plan(c, dev)
    if lines:
        plan.set_path(abi.MS_PATH_LINES)
    print(f"[case] edge geometry {kind}, {'line' if lines else 'default'} path", flush=True)
    inten = plan.forward(_t(c.probe, dev), _t(c.start, dev))
    loss, gs, gp = plan.adjoint(_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev))
    ref_i = c.model.forward(c.probe, c.start)
    ref_l, ref_gs, ref_gp, _ = c.model.loss_grad(c.probe, c.start, c.measured)
    assert rel(inten.cpu().numpy(), ref_i) < TOL_FWD
    assert abs(loss.item() - ref_l) / ref_l < TOL_FWD
    assert rel(gs.cpu().numpy(), ref_gs) < TOL_GRAD and rel(gp.cpu().numpy(), ref_gp) < TOL_GRAD


@pytest.mark.parametrize("n", [32, 128, 256])
def test_make_probe_with_aberrations(dev, n):
    """Astigmatism and spherical aberration on top of defocus (ms_make_probe_aberrated)."""
    import oracle
    from paper_2205_03902_amd import abi, configs
    g = configs.small(n=n, obj=n + n // 2, n_slices=2)
    plan = abi.Plan.from_geometry(g, device=dev)
    got = plan.make_probe_aberrated(0.02, 120.0, 25.0, 0.7, 4.0e5).cpu().numpy()
    ref = oracle.probe_aberrated(n, g.pixel_size, g.wavelength, 0.02, 120.0, 25.0, 0.7, 4.0e5)
    assert rel(got, ref) < 2e-6
    plain = plan.make_probe(0.02, 120.0).cpu().numpy()
    assert rel(plain, oracle.probe(n, g.pixel_size, g.wavelength, 0.02, 120.0)) < 2e-6


def test_reconstruction_error_matches_the_oracle(dev):
    """The paper's relative reconstruction error after the per-slice complex scale, on a seeded
    estimate against a reference, with and without a coverage mask."""
    from oracle import metrics
    from paper_2205_03902_amd import abi, synth
    ref = synth.complex_field((3, 70, 90), 31)
    est = (ref * np.array([0.8 * np.exp(0.4j), 1.2, -1j])[:, None, None]
           + 0.05 * synth.complex_field((3, 70, 90), 32)).astype(np.complex64)
    mask = np.zeros((70, 90), dtype=np.float32)
    mask[5:60, 10:80] = 1.0
    for mk in (None, mask):
        errs, mean = metrics.reconstruction_error(est, ref, mk)
        got = abi.reconstruction_error(_t(est, dev), _t(ref, dev), None if mk is None else _t(mk, dev)).cpu().numpy()
        assert np.abs(got[:3] - errs).max() < 1e-9 and abs(got[3] - mean) < 1e-9, (got, errs)


def test_translation_aligned_reconstruction_error_matches_the_oracle(dev):
    """With a common translation of the estimate's slices searched over |d| <= max_shift: the same
    translation and errors as the oracle's brute-force search, on a translated, rescaled and
    perturbed copy (with and without a mask) and on an untranslated one."""
    from oracle import metrics
    from paper_2205_03902_amd import abi, synth
    ref = synth.complex_field((3, 70, 90), 33)
    base = (ref * np.array([0.8 * np.exp(0.4j), 1.2, -1j])[:, None, None]
            + 0.05 * synth.complex_field((3, 70, 90), 34))
    mask = np.zeros((70, 90), dtype=np.float32)
    mask[5:60, 10:80] = 1.0
    for s, r in (((3, -5), 6), ((0, 0), 2), ((-2, 1), 3)):
        est = np.roll(base, s, axis=(1, 2)).astype(np.complex64)
        for mk in (None, mask):
            errs, mean, d = metrics.reconstruction_error_aligned(est, ref, mk, max_shift=r)
            sh = torch.zeros(2, dtype=torch.int32, device=dev)
            got = abi.reconstruction_error(_t(est, dev), _t(ref, dev), None if mk is None else _t(mk, dev),
                                           max_shift=r, shift=sh).cpu().numpy()
            assert tuple(sh.cpu().numpy()) == d == (-s[0], -s[1])
            assert np.abs(got[:3] - errs).max() < 1e-9 and abs(got[3] - mean) < 1e-9, (got, errs)
