"""GPU checks of the learned-initialisation pipeline on the config-3 geometry (config 1's:
320^2 object, 6 slices, 1024 positions).

* The network input is the phase of the coarse slices over the centre crop and the target
  the true potential there (pad channels zero).
* The layer-wise sweeps never raise the loss (the descent guarantee of the step rule).
* The initialisation path is wired right: initialising the crop with the true potential
  (what a perfect network would predict) gives a loss far below the plain method's loss
  after T sweeps, and the control (zero potential) starts from the restart loss.
* time_to_loss reports consistent times and sweep counts.
* A network trained briefly (a few hundred generated specimens, a few epochs) starts held-out
  specimens below the zero-potential control and reaches the plain run's loss sooner.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sim():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_03902_amd import learned_init
    print("[case] learned-init simulator, config-3 geometry", flush=True)
    return learned_init.Simulator(learned_init.Setup(sweeps=6), "cuda")


def test_example_input_and_target(sim):
    from paper_2205_03902_amd import learned_init
    s = sim.s
    x = torch.empty((s.crop, s.crop, 8), dtype=torch.bfloat16, device=sim.device)
    y = torch.empty((s.crop, s.crop, 6), dtype=torch.float32, device=sim.device)
    learned_init.make_example(sim, 39500, x, y)
    xc = x.float().cpu().numpy()
    assert np.all(xc[..., 6:] == 0) and np.all(np.abs(xc) <= np.pi + 1e-2) and np.abs(xc[..., :6]).max() > 0
    pot = sim.pot.cpu().numpy()
    o = s.offset
    assert np.array_equal(y.cpu().numpy(), pot[:, o:o + s.crop, o:o + s.crop].transpose(1, 2, 0))


def test_sweeps_never_raise_the_loss(sim):
    sim.load(39501)
    t = sim.start()
    M = sim.plan.n_slices
    losses = torch.zeros((4, M), dtype=torch.float64, device=sim.device)
    for k in range(4):
        sim.sweep(t, losses, k)
    seq = losses.cpu().numpy().ravel()
    assert np.all(np.diff(seq) <= 1e-9 * seq[0]), seq


def test_true_potential_initialisation_beats_the_plain_run(sim):
    from paper_2205_03902_amd import datagen
    s = sim.s
    M = sim.plan.n_slices
    sim.load(39502)
    t = sim.start()
    lp = torch.zeros((s.sweeps + 1, M), dtype=torch.float64, device=sim.device)
    for k in range(s.sweeps):
        sim.sweep(t, lp, k)
    sim.loss(t, lp[s.sweeps, 0:1])
    t2 = sim.start()
    lc = torch.zeros((s.coarse_sweeps, M), dtype=torch.float64, device=sim.device)
    for k in range(s.coarse_sweeps):
        sim.sweep(t2, lc, k)
    vt = datagen.crop_potential(sim.pot, s.offset, s.offset, s.crop, s.crop)
    datagen.apply_init(vt, t2, s.offset, s.offset, s.kappa)
    li = torch.zeros(1, dtype=torch.float64, device=sim.device)
    sim.loss(t2, li)
    # the truth's loss is the noise floor; the plain run after T sweeps is still above it
    truth = torch.zeros(1, dtype=torch.float64, device=sim.device)
    sim.loss(sim.truth, truth)
    assert li.item() < lp[s.sweeps, 0].item()
    assert abs(li.item() - truth.item()) <= 1e-3 * truth.item()


def test_time_to_loss_report(sim):
    from paper_2205_03902_amd import learned_init
    from paper_2205_03902_amd.unet import UNet
    net = UNet(6, 6, base=8, levels=2, height=sim.s.crop, width=sim.s.crop, max_batch=1, device=sim.device)
    net.init_he(3)
    r = learned_init.time_to_loss(sim, net, 39503)
    assert r["sweeps_plain"] <= sim.s.sweeps and r["t_plain_ms"] > 0
    assert np.all(np.diff(r["plain_curve"]) <= 1e-9 * r["plain_curve"][0])
    assert np.all(np.diff(r["learned_curve"]) <= 1e-9 * r["learned_curve"][0])
    if r["accepted"]:
        k = r["sweeps_learned"]
        assert r["learned_curve"][k - 1] <= r["L_plain"] and (k == 1 or r["learned_curve"][k - 2] > r["L_plain"])
    s = learned_init.summarize([r, r])
    assert s["n"] == 2 and s["ratio_median"] == pytest.approx(r["t_learned_ms"] / r["t_plain_ms"])


def test_a_briefly_trained_network_beats_the_control(sim):
    from paper_2205_03902_amd import learned_init
    from paper_2205_03902_amd.unet import UNet
    s = sim.s
    M = sim.plan.n_slices
    X, Y, _ = learned_init.generate(sim, s.train_first, 256)
    net = UNet(M, M, base=32, levels=4, height=s.crop, width=s.crop, max_batch=16, device=sim.device)
    net.init_he(seed=s.geo.seed)
    tr, _, _ = learned_init.train(net, X, Y, epochs=6, batch=16, lr=1e-3, seed=1)
    del X, Y
    rows = [learned_init.time_to_loss(sim, net, s.test_first + i) for i in range(4)]
    for r in rows:
        print(f"trained net, specimen {r['index']}: loss at init learned {r['loss_at_learned_init']:.4e} control "
              f"{r['loss_at_control_init']:.4e}; t_learned / t_control {r['t_learned_ms'] / r['t_control_ms']:.3f}")
    assert tr[-1] < tr[0]
    assert all(r["loss_at_learned_init"] < r["loss_at_control_init"] for r in rows)
    assert np.median([r["t_learned_ms"] / r["t_control_ms"] for r in rows]) < 1.0


@pytest.fixture(scope="module")
def tiled():
    """The 12-slice workload's arrangement on a small geometry: training on the 2 x 2 tiles of 64^2
    that cover a 128^2 object, the network applied to the whole object."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_03902_amd import configs, learned_init
    geo = configs.small(n=64, obj=128, n_slices=4, scan=(6, 6), step_px=12.0, seed=77, defocus=50.0)
    print("[case] learned-init simulator, 2 x 2 tiles of 64^2, whole 128^2 object", flush=True)
    return learned_init.Simulator(learned_init.Setup(geo=geo, crop=64, grid=2, whole=True, sweeps=4), "cuda")


def test_tiles_cover_the_whole_objects_input_and_target(tiled):
    from paper_2205_03902_amd import datagen, learned_init
    s, M = tiled.s, tiled.plan.n_slices
    offsets = s.train_offsets()
    assert offsets == [(0, 0), (0, 64), (64, 0), (64, 64)] and s.window == (0, 0, 128, 128)
    X, Y, _ = learned_init.generate(tiled, 500, 1)
    assert X.shape == (4, 64, 64, 8) and Y.shape == (4, 64, 64, M)
    # the same coarse reconstruction again, read over the whole object
    tiled.load(500)
    t = tiled.start()
    scratch = torch.zeros((s.coarse_sweeps, M), dtype=torch.float64, device=tiled.device)
    for k in range(s.coarse_sweeps):
        tiled.sweep(t, scratch, k)
    xw = datagen.crop_phase(t, 0, 0, 128, 128, 8).cpu()
    pot = tiled.pot.cpu().numpy()
    for r, (y0, x0) in enumerate(offsets):
        assert torch.equal(X[r].cpu(), xw[y0:y0 + 64, x0:x0 + 64])
        assert np.array_equal(Y[r].cpu().numpy(), pot[:, y0:y0 + 64, x0:x0 + 64].transpose(1, 2, 0))


def test_whole_object_network_takes_the_trained_weights_and_reports(tiled):
    from paper_2205_03902_amd import learned_init
    from paper_2205_03902_amd.unet import UNet
    s, M = tiled.s, tiled.plan.n_slices
    net = UNet(M, M, base=8, levels=2, height=s.crop, width=s.crop, max_batch=4, device=tiled.device)
    net.init_he(5)
    whole = UNet(M, M, base=8, levels=2, height=128, width=128, max_batch=1, device=tiled.device)
    whole.set_params(net.get_params(net.shapes()))
    a, b = net.get_params(net.shapes()), whole.get_params(whole.shapes())
    assert all(np.array_equal(a[k][j], b[k][j]) for k in a for j in range(2))
    r = learned_init.time_to_loss(tiled, whole, 501)
    assert r["sweeps_plain"] <= s.sweeps and r["t_plain_ms"] > 0
    for curve in ("plain_curve", "learned_curve", "control_curve"):
        assert np.all(np.diff(r[curve]) <= 1e-9 * r[curve][0]), curve
    assert r["init_ms"] > 0 and np.isfinite(r["loss_at_learned_init"])
