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
