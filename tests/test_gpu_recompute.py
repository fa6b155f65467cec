"""Exit-wave recomputation: the adjoint with every k-th incident wave stored and the rest recomputed
from the nearest stored wave below it (checkpoint_every = k), against the store-every-wave plan and
against the FP64 oracle, on both execution paths.

Recomputing psi_m repeats the forward chain's own FP32 operations from a stored wave, so every mode
computes the same values; the bar against the store-all plan is 1e-6 (the printed differences show
how close), against the oracle the gradient bar 1e-4."""
import numpy as np
import pytest

from parity_cases import make_case, rel, small_geometry, small_positions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_CASES = {}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def case_for(n, m=5):
    key = (n, m)
    if key not in _CASES:
        g = small_geometry(n, n_slices=m)
        print(f"[case] n={n} obj={g.obj_h} M={g.n_slices} S={g.n_pos}", flush=True)
        _CASES[key] = make_case(g, positions=small_positions(g))
    return _CASES[key]


def _plan(c, dev, k, lines, budget=0):
    from paper_2205_03902_amd import abi
    plan = abi.Plan.from_geometry(c.geo, positions=c.model.positions, budget_bytes=budget, device=dev,
                                  checkpoint_every=k)
    if lines:
        plan.set_path(abi.MS_PATH_LINES)
    return plan


PATHS = [(32, False), (64, False), (128, False), (64, True), (256, True)]


@pytest.mark.parametrize("n, lines", PATHS)
def test_recomputed_waves_give_the_stored_wave_gradients(dev, n, lines):
    c = case_for(n)
    M = c.geo.n_slices
    args = (_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev))
    ref = _plan(c, dev, 1, lines)
    assert ref.checkpoint_every == 1
    l1, g1, p1 = ref.adjoint(*args)
    ref_l, ref_gs, ref_gp, _ = c.model.loss_grad(c.probe, c.start, c.measured)
    for k in (2, 3, M):
        plan = _plan(c, dev, k, lines)
        assert plan.checkpoint_every == k
        assert plan.workspace_bytes < ref.workspace_bytes
        for rep in range(2):                    # the work slot is reused: a second call is the same
            lk, gk, pk = plan.adjoint(*args)
            dl = abs(lk.item() - l1.item()) / l1.item()
            dg, dp = rel(gk.cpu().numpy(), g1.cpu().numpy()), rel(pk.cpu().numpy(), p1.cpu().numpy())
            bitwise = torch.equal(gk, g1) and torch.equal(pk, p1)
            print(f"n={n} lines={lines} k={k}: vs stored waves loss {dl:.1e} slices {dg:.1e} probe {dp:.1e} "
                  f"(bitwise {bitwise}); vs oracle slices {rel(gk.cpu().numpy(), ref_gs):.2e}")
            assert dl < 1e-6 and dg < 1e-6 and dp < 1e-6
            assert abs(lk.item() - ref_l) / ref_l < 1e-5
            assert rel(gk.cpu().numpy(), ref_gs) < 1e-4 and rel(pk.cpu().numpy(), ref_gp) < 1e-4


@pytest.mark.parametrize("n, lines", [(64, False), (64, True)])
def test_recomputation_with_batches_and_without_the_probe_gradient(dev, n, lines):
    """A budget below the no-stored-wave footprint cuts the positions into batches (k = M); the
    slice gradients are then accumulated batch by batch, slice by slice."""
    from paper_2205_03902_amd import abi
    c = case_for(n)
    M = c.geo.n_slices
    args = (_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev))
    l1, g1, _ = _plan(c, dev, 1, lines).adjoint(*args)
    pb, keep = abi.make_problem(c.geo.n, c.geo.obj_h, c.geo.obj_w, M, c.model.positions, c.geo.gaps(),
                                c.geo.pixel_size, c.geo.wavelength, checkpoint_every=M)
    full = abi.workspace_size(pb)
    plan = _plan(c, dev, 0, lines, budget=int(full * 0.8))
    assert plan.checkpoint_every == M and plan.batch < c.geo.n_pos
    lk, gk, pk = plan.adjoint(*args, want_probe=False)
    assert pk is None
    assert abs(lk.item() - l1.item()) <= 1e-6 * l1.item()
    assert rel(gk.cpu().numpy(), g1.cpu().numpy()) < 1e-6


@pytest.mark.parametrize("n, lines", [(64, False), (256, True)])
def test_full_gradient_step_with_recomputed_waves(dev, n, lines):
    """ms_full_step also needs every slice's overlap map sum_s |psi_m^s|^2 for its step sizes: with
    recomputed waves each slice's map is scattered with its gradient."""
    c = case_for(n)
    M = c.geo.n_slices
    p, m = _t(c.probe, dev), _t(c.measured, dev)
    out = []
    for k in (1, M):
        plan = _plan(c, dev, k, lines)
        s = _t(c.start, dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        mu = torch.zeros(M, dtype=torch.float64, device=dev)
        plan.full_step(1, p, s, m, loss=loss, mu=mu, step_scale=1.0 / M)
        out.append((s.cpu().numpy(), loss.item(), mu.cpu().numpy()))
    (s1, l1, mu1), (sk, lk, muk) = out
    assert abs(lk - l1) <= 1e-6 * l1
    assert np.abs(muk / mu1 - 1).max() < 1e-6
    assert rel(sk - c.start, s1 - c.start) < 1e-5
    ref_s, ref_l, ref_mu = c.model.full_step(c.probe, c.start, c.measured, 1, step_scale=1.0 / M)
    assert np.abs(muk / ref_mu - 1).max() < 1e-5
    assert rel(sk - c.start, ref_s - c.start) < 1e-3


def test_config2_block_through_the_autograd_function_with_recomputed_waves(dev):
    """Config 2's chain (256^2 windows, 10 slices at 1.5 A) on a 16-position block, with every exit
    wave recomputed from the probe (checkpoint_every = M), through the torch.autograd.Function: the
    gradients of the loss with respect to every slice and the probe against the FP64 oracle and
    against the oracle's central differences along 24 seeded directions."""
    from paper_2205_03902_amd import abi, configs, synth
    from paper_2205_03902_amd.autograd import amplitude_loss
    geo = configs.CFG2
    block = geo.positions()[[1950, 1951, 1952, 1953, 2014, 2015, 2016, 2017, 2078, 2079, 2080, 2081,
                             2142, 2143, 2144, 2145]]
    print("[case] config 2 block, recomputed waves, autograd", flush=True)
    c = make_case(geo, positions=block)
    plan = abi.Plan.from_geometry(geo, positions=block, device=dev, checkpoint_every=geo.n_slices)
    assert plan.checkpoint_every == geo.n_slices
    p_t = _t(c.probe, dev).requires_grad_(True)
    s_t = _t(c.start, dev).requires_grad_(True)
    loss = amplitude_loss(plan, p_t, s_t, _t(c.measured, dev))
    loss.backward()
    # torch's gradient of a real loss is 2 dL/d conj(z)
    g_s = s_t.grad.cpu().numpy().astype(np.complex128) / 2
    g_p = p_t.grad.cpu().numpy().astype(np.complex128) / 2
    ref_l, ref_gs, ref_gp, _ = c.model.loss_grad(c.probe, c.start, c.measured)
    print(f"config 2 block (recomputed): loss {abs(loss.item() - ref_l) / ref_l:.2e} "
          f"slices {rel(g_s, ref_gs):.2e} probe {rel(g_p, ref_gp):.2e}")
    assert abs(loss.item() - ref_l) / ref_l < 1e-5
    assert rel(g_s, ref_gs) < 1e-4 and rel(g_p, ref_gp) < 1e-4
    start, probe = c.start.astype(np.complex128), c.probe.astype(np.complex128)
    s_dirs = synth.complex_directions(start.shape, 24, seed=geo.seed + 2)
    p_dirs = synth.complex_directions(probe.shape, 24, seed=geo.seed + 7) * 0.01
    eps = 1e-5
    for d, dp in zip(s_dirs, p_dirs):
        fd = (c.model.loss(probe + eps * dp, start + eps * d, c.measured)
              - c.model.loss(probe - eps * dp, start - eps * d, c.measured)) / (2 * eps)
        got = 2 * (np.vdot(g_s, d).real + np.vdot(g_p, dp).real)
        assert abs(got - fd) <= 1e-4 * abs(fd), (got, fd)
