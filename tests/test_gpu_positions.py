"""GPU parity of the scan-position gradient, its curvature bound and the position step against
the FP64 oracle, on both execution paths, with sub-pixel, integer and wrapping positions and
with several batches; and a refinement run that brings displaced positions back."""
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


def case_for(n, integer=False):
    key = (n, integer)
    if key not in _CASES:
        g = small_geometry(n, n_slices=3, seed=41)
        pos = small_positions(g)
        if integer:
            pos = np.floor(pos)
            pos[1] += 0.5                         # one sub-pixel class next to the integer ones
        print(f"[case] positions n={n} integer={integer}", flush=True)
        _CASES[key] = make_case(g, positions=pos)
    return _CASES[key]


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _plan(c, dev, path, budget=0):
    from paper_2205_03902_amd import abi
    # every wave stored: a budget then splits the positions into batches
    plan = abi.Plan.from_geometry(c.geo, positions=c.model.positions, budget_bytes=budget, device=dev,
                                  checkpoint_every=1)
    plan.set_path(path)
    return plan


@pytest.mark.parametrize("n,path,integer", [(64, 1, False), (128, 1, False), (64, 2, False), (256, 2, False),
                                            (64, 1, True), (64, 2, True)])
def test_position_gradient_matches_the_oracle(dev, n, path, integer):
    c = case_for(n, integer)
    plan = _plan(c, dev, path)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    g, cv = plan.position_grad(_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev), loss=loss)
    ref_l, ref_g, ref_c = c.model.position_grad(c.probe, c.start, c.measured)
    print(f"grad rel {rel(g.cpu().numpy(), ref_g):.2e} curv rel {rel(cv.cpu().numpy(), ref_c):.2e}")
    assert abs(loss.item() - ref_l) < 1e-5 * ref_l
    assert rel(g.cpu().numpy(), ref_g) < 1e-4
    assert rel(cv.cpu().numpy(), ref_c) < 1e-5


def test_position_step_matches_the_oracle_and_batches_agree(dev):
    from paper_2205_03902_amd import abi
    c = case_for(64)
    one = _plan(c, dev, 1)
    ws = abi.workspace_size(one.pb)
    n2 = 64 * 64
    per_pos = c.geo.n_slices * n2 * 12 + n2 * 16
    small = _plan(c, dev, 1, budget=ws - 6 * per_pos)
    assert 1 < small.batch < c.geo.n_pos
    p, s, m = _t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev)
    pos0 = np.asarray(c.model.positions, dtype=np.float64)
    a = _t(pos0, dev)
    b = _t(pos0, dev)
    one.position_step(a, p, s, m, step_scale=2.0)
    small.position_step(b, p, s, m, step_scale=2.0)
    _, ref_g, ref_c = c.model.position_grad(c.probe, c.start, c.measured)
    ref = pos0 - 2.0 * ref_g / ref_c
    assert rel(a.cpu().numpy() - pos0, ref - pos0) < 1e-4
    assert rel(b.cpu().numpy() - pos0, a.cpu().numpy() - pos0) < 1e-6


@pytest.mark.parametrize("path", [1, 2])
def test_refinement_brings_displaced_positions_back(dev, path):
    import oracle
    from paper_2205_03902_amd import abi, layerwise
    c = case_for(64)
    g = c.geo
    # true positions at half pixels, displaced by up to 0.2 px, so that no position changes its
    # patch origin on the way back (the loss of the patch model jumps slightly where it does);
    # noise-free patterns, the true object and probe; every position is its own sub-pixel class
    true_pos = np.floor(np.asarray(c.model.positions, dtype=np.float64)) + 0.5
    md_true = oracle.Model(g.n, g.obj_h, g.obj_w, g.n_slices, true_pos, g.gaps(), g.pixel_size, g.wavelength)
    meas = md_true.forward(c.probe, c.truth).astype(np.float32)
    off = np.random.default_rng(12).uniform(-0.2, 0.2, true_pos.shape)
    md0 = oracle.Model(g.n, g.obj_h, g.obj_w, g.n_slices, true_pos + off, g.gaps(), g.pixel_size, g.wavelength)
    plan = abi.Plan.from_geometry(g, positions=true_pos + off, device=dev)
    plan.set_path(path)
    assert plan.shift_classes == len(true_pos)
    p, s, m = _t(c.probe, dev), _t(c.truth, dev), _t(meas, dev)
    plan, pos, losses = layerwise.refine_positions(plan, p, s, m, passes=12)
    err0 = np.sqrt(np.mean(off ** 2))
    err = np.sqrt(np.mean((pos.cpu().numpy() - true_pos) ** 2))
    print(f"refinement: rms error {err0:.3f} -> {err:.3f} px, loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert abs(losses[0] - md0.loss(c.probe, c.truth, meas)) < 1e-4 * losses[0]
    assert all(b <= a for a, b in zip(losses, losses[1:])), losses
    # the same run with the oracle reaches rms 0.028 px from 0.122 px in 12 passes
    assert err < 0.4 * err0
