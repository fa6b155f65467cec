"""GPU checks of the 256 x 256 workloads (line-kernel path).

config 2 (512^2 object, 10 slices, 4096 positions, noise free) and config 4 (1024^2,
12 slices, 16384 positions) are run at full size on the GPU; the oracle recomputes a
sample of positions one by one.  Gradients at full size are checked through a property
that holds at any size (the loss and gradient of a set of positions are the sums over a
partition of it); the gradient itself is compared with the oracle, and with the oracle's
finite differences along 24 seeded directions, on a 16-position block of config 2."""
import numpy as np
import pytest

from parity_cases import make_case, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _t(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def _sample(geo, k):
    return np.linspace(0, geo.n_pos - 1, k).round().astype(int)


@pytest.fixture(scope="module")
def cfg2():
    from paper_2205_03902_amd import configs
    geo = configs.CFG2
    print("[case] config 2 (256 px, 10 slices, 4096 positions)", flush=True)
    # measured patterns come from the oracle on a 16-position block; the full-size checks
    # below use oracle forwards of sampled positions only
    block = geo.positions()[[1950, 1951, 1952, 1953, 2014, 2015, 2016, 2017, 2078, 2079, 2080, 2081,
                             2142, 2143, 2144, 2145]]
    return geo, make_case(geo, positions=block)


def test_config2_full_size_forward_sampled(dev, cfg2):
    import oracle
    from paper_2205_03902_amd import abi
    geo, c = cfg2
    plan = abi.Plan.from_geometry(geo, device=dev)
    inten = plan.forward(_t(c.probe, dev), _t(c.start, dev))
    pick = _sample(geo, 12)
    sub = oracle.Model.from_geometry(geo, positions=geo.positions()[pick])
    ref = sub.forward(c.probe, c.start)
    assert rel(inten[torch.from_numpy(pick).to(dev)].cpu().numpy(), ref) < 1e-5
    # Parseval: a unit-energy probe through pure-phase slices keeps unit energy, and the
    # detector sum of a unitary-scaled transform is N^2 times it
    sums = inten.double().sum(dim=(1, 2)).cpu().numpy()
    assert np.abs(sums / geo.n ** 2 - 1).max() < 1e-5


def test_config2_full_size_gradient_is_additive_over_a_partition(dev, cfg2):
    from paper_2205_03902_amd import abi
    geo, c = cfg2
    pos = geo.positions()
    full = abi.Plan.from_geometry(geo, device=dev)
    p, s = _t(c.probe, dev), _t(c.start, dev)
    # synthetic measured patterns for all positions: the GPU forward of the truth
    meas = full.forward(p, _t(c.truth, dev))
    loss, gs, gp = full.adjoint(p, s, meas)
    halves = [np.arange(0, geo.n_pos, 2), np.arange(1, geo.n_pos, 2)]
    l_sum, g_sum, p_sum = 0.0, torch.zeros_like(gs), torch.zeros_like(gp)
    for h in halves:
        part = abi.Plan.from_geometry(geo, positions=pos[h], device=dev)
        lh, gh, ph = part.adjoint(p, s, meas[torch.from_numpy(h).to(dev)].contiguous())
        l_sum += lh.item()
        g_sum += gh
        p_sum += ph
    assert abs(l_sum - loss.item()) <= 1e-6 * loss.item()
    assert rel(g_sum.cpu().numpy(), gs.cpu().numpy()) < 1e-5
    assert rel(p_sum.cpu().numpy(), gp.cpu().numpy()) < 1e-5


def test_config2_block_gradient_matches_oracle_and_finite_differences(dev, cfg2):
    from paper_2205_03902_amd import abi, synth
    geo, c = cfg2
    plan = abi.Plan.from_geometry(geo, positions=c.model.positions, device=dev)
    loss, gs, gp = plan.adjoint(_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev))
    ref_l, ref_gs, ref_gp, _ = c.model.loss_grad(c.probe, c.start, c.measured)
    assert abs(loss.item() - ref_l) / ref_l < 1e-5
    assert rel(gs.cpu().numpy(), ref_gs) < 1e-4 and rel(gp.cpu().numpy(), ref_gp) < 1e-4
    # 24 seeded directions over slices (+) probe: FP64 oracle loss, central difference at
    # step 1e-5 (truncation ~ eps^2, rounding ~ 1e-16 |L| / eps, both far below 1e-4)
    g_s = gs.cpu().numpy().astype(np.complex128)
    g_p = gp.cpu().numpy().astype(np.complex128)
    start, probe = c.start.astype(np.complex128), c.probe.astype(np.complex128)
    s_dirs = synth.complex_directions(start.shape, 24, seed=geo.seed + 2)
    p_dirs = synth.complex_directions(probe.shape, 24, seed=geo.seed + 7) * 0.01
    eps = 1e-5
    for d, dp in zip(s_dirs, p_dirs):
        fd = (c.model.loss(probe + eps * dp, start + eps * d, c.measured)
              - c.model.loss(probe - eps * dp, start - eps * d, c.measured)) / (2 * eps)
        got = 2 * (np.vdot(g_s, d).real + np.vdot(g_p, dp).real)
        assert abs(got - fd) <= 1e-4 * abs(fd), (got, fd)


def test_config4_full_size_forward_and_batched_adjoint(dev):
    import oracle
    from paper_2205_03902_amd import abi, configs, synth
    geo = configs.CFG4
    print("[case] config 4 (256 px, 1024^2 object, 12 slices, 16384 positions)", flush=True)
    probe = oracle.probe(geo.n, geo.pixel_size, geo.wavelength, geo.alpha, geo.defocus).astype(np.complex64)
    truth = synth.transmissions(synth.specimen(geo))
    start = synth.unit_phase_field(truth.shape, geo.seed + 3, 0.3)
    # with every wave stored, a 16 GiB budget splits the scan into batches
    plan = abi.Plan.from_geometry(geo, budget_bytes=16 << 30, device=dev, checkpoint_every=1)
    assert plan.batch < geo.n_pos
    p = _t(probe, dev)
    inten = plan.forward(p, _t(start, dev))
    pick = _sample(geo, 8)
    ipick = torch.from_numpy(pick).to(dev)
    sub = oracle.Model.from_geometry(geo, positions=geo.positions()[pick])
    assert rel(inten[ipick].cpu().numpy(), sub.forward(probe, start)) < 1e-5
    del inten
    meas = plan.forward(p, _t(truth, dev))
    s = _t(start, dev)
    loss, gs, gp = plan.adjoint(p, s, meas)
    # batched (2048 positions a batch) and one-shot plans agree on loss and gradients
    whole = abi.Plan.from_geometry(geo, device=dev)
    assert whole.batch == geo.n_pos
    l1, g1, p1 = whole.adjoint(p, s, meas)
    assert abs(l1.item() - loss.item()) <= 1e-6 * l1.item()
    assert rel(gs.cpu().numpy(), g1.cpu().numpy()) < 1e-6
    assert rel(gp.cpu().numpy(), p1.cpu().numpy()) < 1e-6
    del whole, g1, p1
    # the sampled positions' loss against the oracle
    sub_plan = abi.Plan.from_geometry(geo, positions=geo.positions()[pick], device=dev)
    ms = meas[ipick].contiguous()
    ls, _, _ = sub_plan.adjoint(p, s, ms)
    ref = sub.loss(probe, start, ms.cpu().numpy())
    assert abs(ls.item() - ref) / ref < 1e-5


def test_config4_block_gradients_match_the_oracle(dev):
    """Config 4's 12-slice chain on the line kernels against the FP64 oracle: loss, every slice
    gradient and the probe gradient of a 16-position block (a 4 x 4 piece of the raster in the
    object's interior, plus windows moved across the object's edges so that the patches wrap)."""
    from paper_2205_03902_amd import abi, configs
    geo = configs.CFG4
    pos = geo.positions()
    block = pos[[8256, 8257, 8258, 8259, 8384, 8385, 8386, 8387, 8512, 8513, 8514, 8515, 8640, 8641, 8642, 8643]]
    block[3] = (geo.obj_h - 100.0, geo.obj_w - 37.0)      # wraps through the bottom-right corner
    block[12] = (-20.0, 500.0)                             # wraps through the top edge
    print(f"[case] config 4 block: 16 positions, M={geo.n_slices}", flush=True)
    c = make_case(geo, positions=block)
    plan = abi.Plan.from_geometry(geo, positions=block, device=dev)
    loss, gs, gp = plan.adjoint(_t(c.probe, dev), _t(c.start, dev), _t(c.measured, dev))
    ref_l, ref_gs, ref_gp, _ = c.model.loss_grad(c.probe, c.start, c.measured)
    el, egs, egp = abs(loss.item() - ref_l) / ref_l, rel(gs.cpu().numpy(), ref_gs), rel(gp.cpu().numpy(), ref_gp)
    per_slice = [rel(gs[m].cpu().numpy(), ref_gs[m]) for m in range(geo.n_slices)]
    print(f"config 4 block: loss {el:.2e} grad slices {egs:.2e} (worst slice {max(per_slice):.2e}) probe {egp:.2e}")
    assert el < 1e-5 and egs < 1e-4 and egp < 1e-4
    assert max(per_slice) < 1e-4


def test_config4_thirty_sweeps_with_the_probe(dev):
    """Config 4 as specified: 30 sweeps of Algorithm 1 (Sec. 3.3), each followed by a probe step
    (Sec. 3.5) over all 16384 positions, from t = 1 and the probe of 1.1x the defocus, on Poisson
    counts at 1e5 electrons a pattern.  The oracle takes minutes a pass at this size, so the run is
    checked by what holds at any size: the majorised steps of Sec. 3.2 never raise the loss (390
    steps); the first sweep with the incident waves carried between layer steps is the sweep
    without them, bit for bit; and at the end the loss of sampled positions is the oracle's at the
    final slices and probe."""
    import oracle
    from paper_2205_03902_amd import abi, configs, datagen, layerwise, synth
    geo = configs.CFG4
    print(f"[case] config 4, {geo.iterations} sweeps with probe steps from the 1.1x-defocus probe", flush=True)
    plan = abi.Plan.from_geometry(geo, device=dev)
    truth = _t(synth.transmissions(synth.specimen(geo)), dev)
    inten = plan.forward(plan.make_probe(geo.alpha, geo.defocus), truth)
    meas = datagen.poisson(inten, geo.dose, seed=geo.seed + 1, stream_id=0)
    del inten, truth
    p0 = plan.make_probe(geo.alpha, 1.1 * geo.defocus)
    start = torch.ones((geo.n_slices, geo.obj_h, geo.obj_w), dtype=torch.complex64, device=dev)
    s_ref, p_ref = start.clone(), p0.clone()
    h_ref = layerwise.reconstruct(plan, p_ref, s_ref, meas, sweeps=1, probe_steps=1, carry=False)
    s, p = start.clone(), p0.clone()
    h = layerwise.reconstruct(plan, p, s, meas, sweeps=1, probe_steps=1)
    same = (torch.equal(torch.view_as_real(s), torch.view_as_real(s_ref))
            and torch.equal(torch.view_as_real(p), torch.view_as_real(p_ref)))
    del s_ref, p_ref, start
    h2 = layerwise.reconstruct(plan, p, s, meas, sweeps=geo.iterations - 1, probe_steps=1)
    losses = np.array(h.loss + h2.loss)
    l_end = plan.adjoint(p, s, meas)[0].item()
    print(f"config 4, {geo.iterations} sweeps: loss {losses[0]:.4e} -> {l_end:.4e} in "
          f"{h.seconds + h2.seconds:.1f} s; first sweep with and without the carry equal: {same}")
    assert same and h.loss == h_ref.loss
    assert len(losses) == geo.iterations * (geo.n_slices + 1)
    assert (np.diff(losses) <= 1e-6 * losses[0]).all() and l_end <= losses[-1] * (1 + 1e-6)
    assert l_end < 0.5 * losses[0]
    pick = _sample(geo, 8)
    sub = oracle.Model.from_geometry(geo, positions=geo.positions()[pick])
    sub_plan = abi.Plan.from_geometry(geo, positions=geo.positions()[pick], device=dev)
    ms = meas[torch.from_numpy(pick).to(dev)].contiguous()
    ls, _, _ = sub_plan.adjoint(p, s, ms)
    ref = sub.loss(p.cpu().numpy(), s.cpu().numpy(), ms.cpu().numpy())
    print(f"sampled end-state loss: {ls.item():.6e} (oracle {ref:.6e})")
    assert abs(ls.item() - ref) / ref < 1e-5
