"""GPU checks of the incident waves carried between Algorithm 1's layer steps on the line path
(ms_plan_set_layer_carry): a layer step that follows one for the same layer, or the layer before,
with the same buffers starts its forward chain from the wave the previous step left.  The results
are bit for bit those of the whole chain: whole sweeps with repeated layer steps and probe steps,
steps out of order, other entry points in between (which drop the wave), the fused path."""
import numpy as np
import pytest

from parity_cases import make_case
from paper_2205_03902_amd import configs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
_CASES = {}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def case_for(n):
    if n not in _CASES:
        if n == 64:
            g = configs.small(n=64, obj=128, n_slices=5, scan=(6, 6), step_px=10.0, seed=21, defocus=25.0)
        else:
            g = configs.small(n=256, obj=384, n_slices=4, scan=(4, 4), step_px=24.0, seed=22, defocus=25.0)
        print(f"[case] layer carry n={g.n} M={g.n_slices} S={g.n_pos}", flush=True)
        _CASES[n] = make_case(g)
    return _CASES[n]


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _plan(c, dev, lines=True):
    from paper_2205_03902_amd import abi
    plan = abi.Plan.from_geometry(c.geo, positions=c.model.positions, device=dev, checkpoint_every=1)
    plan.set_path(abi.MS_PATH_LINES if lines else abi.MS_PATH_FUSED)
    return plan


def _sweeps(c, dev, carry, lines=True):
    from paper_2205_03902_amd import layerwise
    plan = _plan(c, dev, lines)
    probe, slices, meas = _t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev)
    h = layerwise.reconstruct(plan, probe, slices, meas, sweeps=2, k_steps=2, probe_steps=1, carry=carry)
    return slices.cpu().numpy(), probe.cpu().numpy(), np.array(h.loss), np.array(h.mu), h.seconds


@pytest.mark.parametrize("n", [64, 256])
def test_sweeps_with_the_carried_wave_are_the_whole_chains(dev, n):
    c = case_for(n)
    s1, p1, l1, m1, t1 = _sweeps(c, dev, True)
    s0, p0, l0, m0, t0 = _sweeps(c, dev, False)
    print(f"layer carry n={n}: {t1 * 1e3:.1f} ms against {t0 * 1e3:.1f} ms for two sweeps")
    assert np.array_equal(s1, s0) and np.array_equal(p1, p0)
    assert np.array_equal(l1, l0) and np.array_equal(m1, m0)


def test_steps_out_of_order_and_other_calls_in_between(dev):
    c = case_for(64)
    order = [2, 3, 3, 0, 1, 2, "adjoint", 3, 4, 2, 1]
    results = []
    for carry in (1, 0):
        plan = _plan(c, dev)
        plan.set_layer_carry(carry)
        probe, slices, meas = _t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev)
        out = torch.zeros(2, dtype=torch.float64, device=dev)
        losses = []
        for step in order:
            if step == "adjoint":
                plan.adjoint(probe, slices, meas)
                continue
            plan.layer_step(step, 1, probe, slices, meas, loss=out[0:1], mu=out[1:2])
            losses.append(out[0].item())
        results.append((slices.cpu().numpy(), losses))
    assert np.array_equal(results[0][0], results[1][0]) and results[0][1] == results[1][1]


def test_the_fused_path_ignores_the_carry(dev):
    c = case_for(64)
    s1, p1, l1, _, _ = _sweeps(c, dev, True, lines=False)
    s0, p0, l0, _, _ = _sweeps(c, dev, False, lines=False)
    assert np.array_equal(s1, s0) and np.array_equal(p1, p0) and np.array_equal(l1, l0)


def test_carried_wave_with_the_poisson_objective_and_tilted_illumination(dev):
    """The carry changes only where a layer step's forward chain starts: with the Poisson deviance
    (its own residual and step) and tilted illumination (the tilt terms of the propagator) the
    sweeps are again bit for bit those of the whole chain."""
    from paper_2205_03902_amd import abi, layerwise
    c = case_for(64)
    g = c.geo
    print("[case] layer carry with the Poisson objective and a tilt, n=64", flush=True)
    runs = []
    for carry in (True, False):
        plan = abi.Plan(g.n, g.obj_h, g.obj_w, g.n_slices, c.model.positions, g.gaps(), g.pixel_size, g.wavelength,
                        tilt_y=0.012, tilt_x=-0.007, device=dev, checkpoint_every=1)
        plan.set_path(abi.MS_PATH_LINES)
        plan.set_objective(abi.MS_OBJECTIVE_POISSON)
        probe, slices, meas = _t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev)
        h = layerwise.reconstruct(plan, probe, slices, meas, sweeps=2, k_steps=2, probe_steps=1, carry=carry)
        runs.append((slices.cpu().numpy(), probe.cpu().numpy(), np.array(h.loss), np.array(h.mu)))
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
    assert np.all(np.isfinite(runs[0][2]))
