"""GPU parity of the line-kernel path (one launch per slice, 16 lines per workgroup):
forced at N = 32, 64, 128 where the fused kernel also exists, and the only path at N = 256."""
import numpy as np
import pytest

from parity_cases import make_case, rel, small_geometry, small_positions

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_FWD = 1e-5
TOL_GRAD = 1e-4
_CASES = {}


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def case_for(n):
    if n not in _CASES:
        g = small_geometry(n)
        print(f"[case] n={n} obj={g.obj_h} M={g.n_slices} S={g.n_pos}", flush=True)
        _CASES[n] = make_case(g, positions=small_positions(g))
    return _CASES[n]


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _plan(c, dev, budget=0):
    from paper_2205_03902_amd import abi
    # every wave stored: a budget then splits the positions into batches
    plan = abi.Plan.from_geometry(c.geo, positions=c.model.positions, budget_bytes=budget, device=dev,
                                  checkpoint_every=1)
    plan.set_path(abi.MS_PATH_LINES)
    return plan


@pytest.mark.parametrize("n", [32, 64, 128, 256])
def test_lines_forward_and_adjoint(dev, n):
    c = case_for(n)
    plan = _plan(c, dev)
    p, s, m = _t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev)
    inten, ew = plan.forward(p, s, exit_waves=True)
    ref_i, ref_e = c.model.forward(c.probe, c.start, exit_waves=True)
    ei, ee = rel(inten.cpu().numpy(), ref_i), rel(ew.cpu().numpy(), ref_e)
    loss, gs, gp = plan.adjoint(p, s, m)
    ref_l, ref_gs, ref_gp, _ = c.model.loss_grad(c.probe, c.start, c.measured)
    el = abs(loss.item() - ref_l) / ref_l
    egs, egp = rel(gs.cpu().numpy(), ref_gs), rel(gp.cpu().numpy(), ref_gp)
    print(f"lines n={n}: intensity {ei:.2e} exit {ee:.2e} loss {el:.2e} grad slices {egs:.2e} probe {egp:.2e}")
    assert ei < TOL_FWD and ee < TOL_FWD and el < TOL_FWD and egs < TOL_GRAD and egp < TOL_GRAD


@pytest.mark.parametrize("n", [64, 256])
def test_lines_layer_and_probe_steps(dev, n):
    c = case_for(n)
    plan = _plan(c, dev)
    p, m = _t(c.probe, dev), _t(c.measured, dev)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    for layer in range(c.geo.n_slices):            # first, middle and last layer
        s = _t(c.start, dev)
        plan.layer_step(layer, 1, p, s, m, loss=out[0:1], mu=out[1:2])
        ref_s, ref_l, ref_mu = c.model.layer_step(c.probe, c.start, c.measured, layer, 1)
        assert abs(out[0].item() - ref_l) / ref_l < TOL_FWD
        assert abs(out[1].item() - ref_mu) / ref_mu < TOL_FWD
        assert rel(s.cpu().numpy(), ref_s) < TOL_FWD
    p0 = (c.probe * np.exp(0.05j)).astype(np.complex64)
    pt = _t(p0, dev)
    plan.probe_step(1, pt, _t(c.start, dev), m, subset=[0, 4, 8], loss=out[0:1], mu=out[1:2])
    ref_p, ref_l, ref_mu = c.model.probe_step(p0, c.start, c.measured, [0, 4, 8], 1)
    assert abs(out[0].item() - ref_l) / ref_l < TOL_FWD
    assert rel(pt.cpu().numpy(), ref_p) < TOL_FWD
    assert rel(pt.cpu().numpy() - p0, ref_p - p0) < 10 * TOL_GRAD


def test_lines_make_probe_256(dev):
    import oracle
    c = case_for(256)
    plan = _plan(c, dev)
    got = plan.make_probe(c.geo.alpha, c.geo.defocus).cpu().numpy()
    ref = oracle.probe(256, c.geo.pixel_size, c.geo.wavelength, c.geo.alpha, c.geo.defocus)
    assert rel(got, ref) < 2e-6


def test_lines_equal_fused_up_to_rounding(dev):
    """The two execution paths compute the same quantities (N = 128)."""
    from paper_2205_03902_amd import abi
    c = case_for(128)
    fused = abi.Plan.from_geometry(c.geo, positions=c.model.positions, device=dev)
    lines = _plan(c, dev)
    args = (_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev))
    l1, g1, p1 = fused.adjoint(*args)
    l2, g2, p2 = lines.adjoint(*args)
    assert rel(g2.cpu().numpy(), g1.cpu().numpy()) < 1e-5
    assert rel(p2.cpu().numpy(), p1.cpu().numpy()) < 1e-5
    assert abs(l1.item() - l2.item()) < 1e-6 * l1.item()
