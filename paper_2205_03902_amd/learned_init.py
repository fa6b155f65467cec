"""Learned initialisation of the layer-wise reconstruction (the 'config 3' workload, and the
same comparison on the 16384-position, 12-slice workload).

The plain method starts Algorithm 1 (Sec. 3.3) from t = 1 and runs T sweeps.  The
learned path runs 2 coarse sweeps from t = 1, feeds the phases of the coarse slices
over a centre crop to a U-Net that predicts the slice potentials there, sets
t = exp(i kappa V_hat) over the crop (coarse slices elsewhere) and refines with
further sweeps.  Its cost is compared by time to reach the plain method's final loss
L_plain on the same data; a prediction is accepted only if the refinement reaches
L_plain within T sweeps, otherwise the plain result stands and the learned attempt
adds to its time.

On the 1024^2, 12-slice workload the network has 12 channels, is trained on the 4 x 4 grid
of 256^2 tiles of each training specimen (simulated at the workload's full geometry, so that
the tiles see its scan overlap), and is applied to the whole object at once: the network is
fully convolutional, so the trained weights serve a 1024^2 instance unchanged.

Everything runs on the device: specimens, simulation and noise (datagen), the
multislice steps (libimsp), the network and Adam (unet).  This module only sequences
the calls and reads back the losses.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Tuple

import numpy as np
import torch

from . import abi, configs, datagen, synth
from .unet import UNet


@dataclasses.dataclass
class Setup:
    geo: configs.Geometry = configs.CFG3
    crop: int = 256
    kappa: float = synth.KAPPA
    coarse_sweeps: int = 2
    sweeps: int = 20                 # T
    dose: float = 1e5
    train_first: int = 30000         # training specimens train_first .. train_first + n_train - 1
    test_first: int = 39000          # held-out specimens
    noise_seed: int = 31
    grid: int = 1                    # training crops per specimen and axis: 1 = the centre crop,
                                     # g = the g x g tiles of crop x crop that cover the object
    whole: bool = False              # the network initialises the whole object, not the centre crop

    @property
    def family(self) -> datagen.SpecimenFamily:
        g = self.geo
        return datagen.SpecimenFamily(g.n_slices, g.obj_h, g.obj_w, pixel_size=g.pixel_size, seed=self.geo.seed)

    @property
    def offset(self) -> int:
        return (self.geo.obj_h - self.crop) // 2

    def train_offsets(self) -> List[Tuple[int, int]]:
        """Top-left corners of the training crops of one specimen."""
        if self.grid == 1:
            return [(self.offset, self.offset)]
        if self.grid * self.crop != self.geo.obj_h or self.grid * self.crop != self.geo.obj_w:
            raise ValueError("the tiles must cover the object exactly")
        return [(i * self.crop, j * self.crop) for i in range(self.grid) for j in range(self.grid)]

    @property
    def window(self) -> Tuple[int, int, int, int]:
        """(y0, x0, h, w): where the network's prediction initialises the slices."""
        if self.whole:
            return 0, 0, self.geo.obj_h, self.geo.obj_w
        return self.offset, self.offset, self.crop, self.crop


def setup_for(config: int, sweeps=None) -> Setup:
    """The learned-initialisation workloads: 3 (config 1's geometry, 6 slices, centre crop, T = 20)
    and 4 (the 1024^2, 12-slice, 16384-position geometry, whole object, T = 30)."""
    if config == 3:
        return Setup(sweeps=20 if sweeps is None else sweeps)
    if config == 4:
        return Setup(geo=configs.CFG4, grid=4, whole=True, sweeps=configs.CFG4.iterations if sweeps is None else sweeps,
                     noise_seed=41)
    raise ValueError("learned initialisation is defined for configs 3 and 4")


class Simulator:
    """One specimen at a time: its potential, true slices and noisy patterns on the device."""

    def __init__(self, setup: Setup, device):
        g = setup.geo
        self.s = setup
        self.plan = abi.Plan.from_geometry(g, device=device)
        self.device = self.plan.device
        self.probe = self.plan.make_probe(g.alpha, g.defocus)
        # each layer step continues from the incident wave the previous one left (the line path;
        # the same results, fewer launches); start() and edited() drop it whenever the slices
        # change other than by a layer step
        self.plan.set_layer_carry(1)
        shape = (g.n_slices, g.obj_h, g.obj_w)
        self.pot = torch.empty(shape, dtype=torch.float32, device=self.device)
        self.truth = torch.empty(shape, dtype=torch.complex64, device=self.device)
        self.meas = torch.empty((self.plan.n_pos, g.n, g.n), dtype=torch.float32, device=self.device)
        self.loss_buf = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.grad_buf = torch.empty(shape, dtype=torch.complex64, device=self.device)

    def load(self, index: int):
        datagen.make_specimen(self.s.family, index, self.s.kappa, potential=self.pot, slices=self.truth)
        self.plan.forward(self.probe, self.truth, out=self.meas)
        datagen.poisson(self.meas, self.s.dose, self.s.noise_seed, index, out=self.meas)

    def start(self):
        t = torch.empty_like(self.truth)
        t.fill_(1.0)
        self.edited()
        return t

    def edited(self):
        """The slices were written other than by a layer step: drop the carried incident wave."""
        self.plan.set_layer_carry(1)

    def sweep(self, slices, losses: torch.Tensor, row: int):
        """One Algorithm 1 sweep in place; losses[row, l] = loss before layer step l."""
        for layer in range(self.plan.n_slices):
            self.plan.layer_step(layer, 1, self.probe, slices, self.meas, loss=losses[row, layer:layer + 1])

    def loss(self, slices, out: torch.Tensor):
        self.plan.adjoint(self.probe, slices, self.meas, want_probe=False, grad_slices=self.grad_buf, loss=out)


def make_example(sim: Simulator, index: int, x_out, y_out):
    """Network inputs (coarse phases, bf16 [crop][crop][in_pad]) and targets (potential,
    [crop][crop][M]) of one specimen: one crop, or with a leading axis one row per training crop."""
    s = sim.s
    offsets = s.train_offsets()
    if x_out.dim() == 3:
        if len(offsets) != 1:
            raise ValueError("this setup takes several crops a specimen: pass one row per crop")
        x_out, y_out = x_out[None], y_out[None]
    sim.load(index)
    t = sim.start()
    scratch = torch.zeros((s.coarse_sweeps, sim.plan.n_slices), dtype=torch.float64, device=sim.device)
    for k in range(s.coarse_sweeps):
        sim.sweep(t, scratch, k)
    for r, (y0, x0) in enumerate(offsets):
        datagen.crop_phase(t, y0, x0, s.crop, s.crop, x_out.shape[-1], out=x_out[r])
        datagen.crop_potential(sim.pot, y0, x0, s.crop, s.crop, out=y_out[r])


def generate(sim: Simulator, first: int, count: int, in_pad: int = 0, log=None):
    """Training examples of specimens first .. first + count - 1: len(train_offsets()) rows each.
    in_pad: the network input's channels (0: the slice count rounded up to a multiple of 8)."""
    s = sim.s
    M = s.geo.n_slices
    in_pad = in_pad or (M + 7) // 8 * 8
    tiles = len(s.train_offsets())
    X = torch.empty((count * tiles, s.crop, s.crop, in_pad), dtype=torch.bfloat16, device=sim.device)
    Y = torch.empty((count * tiles, s.crop, s.crop, M), dtype=torch.float32, device=sim.device)
    t0 = last = time.perf_counter()
    for i in range(count):
        make_example(sim, first + i, X[i * tiles:(i + 1) * tiles], Y[i * tiles:(i + 1) * tiles])
        if log and ((i + 1) % 250 == 0 or time.perf_counter() - last > 20.0):
            torch.cuda.synchronize(sim.device)
            last = time.perf_counter()
            log(f"generated {i + 1}/{count} specimens in {last - t0:.1f} s")
    torch.cuda.synchronize(sim.device)
    return X, Y, time.perf_counter() - t0


def train(net: UNet, X, Y, epochs: int, batch: int, lr: float = 1e-3, seed: int = 0, Xv=None, Yv=None, log=None):
    """Adam on contiguous mini-batches, batch order shuffled every epoch.  Returns per-epoch
    mean training loss and held-out loss."""
    n = X.shape[0] // batch
    rng = np.random.Generator(np.random.PCG64(seed))
    losses = torch.zeros((epochs, n), dtype=torch.float64, device=net.device)
    held = []
    out = torch.empty((batch,) + tuple(Y.shape[1:]), dtype=torch.float32, device=net.device)
    t0 = time.perf_counter()
    for e in range(epochs):
        for j, b in enumerate(rng.permutation(n)):
            sl = slice(int(b) * batch, int(b) * batch + batch)
            net.backward(X[sl], Y[sl], out=out, loss=losses[e, j:j + 1])
            net.adam_step(lr=lr)
        if Xv is not None:
            held.append(evaluate(net, Xv, Yv, batch))
        if log:
            torch.cuda.synchronize(net.device)
            log(f"epoch {e + 1}/{epochs}: train {losses[e].mean().item():.4e}"
                + (f" held-out {held[-1]:.4e}" if held else "") + f" ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize(net.device)
    return losses.mean(dim=1).cpu().tolist(), held, time.perf_counter() - t0


def evaluate(net: UNet, X, Y, batch: int) -> float:
    """Mean centred MSE over a data set (forward passes; the gradient buffer is overwritten)."""
    n = X.shape[0] // batch
    acc = torch.zeros(n, dtype=torch.float64, device=net.device)
    out = torch.empty((batch,) + tuple(Y.shape[1:]), dtype=torch.float32, device=net.device)
    for j in range(n):
        sl = slice(j * batch, j * batch + batch)
        net.backward(X[sl], Y[sl], out=out, loss=acc[j:j + 1])
    return float(acc.mean().item())


def _run_sweeps(sim: Simulator, t, count: int, losses, ends: List):
    for k in range(count):
        sim.sweep(t, losses, k)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record()
        ends.append(ev)


def _init_path(sim: Simulator, net, x, vhat, T: int):
    """Coarse sweeps from t = 1, then t = exp(i kappa V_hat) over the crop with V_hat from the
    network (net given) or zero (net None: the control that keeps only the restart to unit
    modulus), then T refinement sweeps.  Returns (losses after refinement sweeps 1..T,
    their end times in ms from the start, loss at the initialisation, initialisation time)."""
    s = sim.s
    M = sim.plan.n_slices
    y0, x0, h, w = s.window
    ll = torch.zeros((s.coarse_sweeps + T + 1, M), dtype=torch.float64, device=sim.device)
    t = sim.start()
    start = torch.cuda.Event(enable_timing=True)
    start.record()
    _run_sweeps(sim, t, s.coarse_sweeps, ll, [])
    if net is not None:
        datagen.crop_phase(t, y0, x0, h, w, net.in_pad, out=x[0])
        net.forward(x, out=vhat)
    datagen.apply_init(vhat[0], t, y0, x0, s.kappa)
    sim.edited()
    init_done = torch.cuda.Event(enable_timing=True)
    init_done.record()
    ends: List = []
    refine = ll[s.coarse_sweeps:]
    _run_sweeps(sim, t, T, refine, ends)
    sim.loss(t, refine[T, 0:1])
    torch.cuda.synchronize(sim.device)
    return (refine[1:, 0].cpu().numpy(), np.array([start.elapsed_time(e) for e in ends]),
            float(refine[0, 0].item()), float(start.elapsed_time(init_done)))


def _reach(losses, ms, target, fallback_ms):
    hit = np.nonzero(losses <= target)[0]
    if hit.size:
        return True, float(ms[hit[0]]), int(hit[0]) + 1
    return False, float(ms[-1]) + fallback_ms, None


def time_to_loss(sim: Simulator, net: UNet, index: int) -> Dict:
    """Plain, learned and control runs on held-out specimen `index`; times from HIP events (ms).
    net: an instance of the size of the setup's window (batch 1)."""
    s = sim.s
    T, M = s.sweeps, sim.plan.n_slices
    sim.load(index)
    torch.cuda.synchronize(sim.device)
    # plain: T sweeps from t = 1; loss after sweep k = loss before the first layer step of sweep k + 1
    lp = torch.zeros((T + 1, M), dtype=torch.float64, device=sim.device)
    t = sim.start()
    start = torch.cuda.Event(enable_timing=True)
    start.record()
    ends: List = []
    _run_sweeps(sim, t, T, lp, ends)
    sim.loss(t, lp[T, 0:1])
    torch.cuda.synchronize(sim.device)
    plain_loss = lp[1:, 0].cpu().numpy()
    plain_ms = np.array([start.elapsed_time(e) for e in ends])
    L_plain = float(plain_loss[-1])
    k_plain = int(np.argmax(plain_loss <= L_plain))
    t_plain = float(plain_ms[k_plain])

    _, _, h, w = s.window
    x = torch.empty((1, h, w, net.in_pad), dtype=torch.bfloat16, device=sim.device)
    vhat = torch.zeros((1, h, w, M), dtype=torch.float32, device=sim.device)
    c_loss, c_ms, c_init, _ = _init_path(sim, None, x, vhat, T)
    l_loss, l_ms, l_init, init_ms = _init_path(sim, net, x, vhat, T)
    acc, t_learned, k_learned = _reach(l_loss, l_ms, L_plain, float(plain_ms[-1]))
    c_acc, t_control, k_control = _reach(c_loss, c_ms, L_plain, float(plain_ms[-1]))
    return dict(index=index, L_plain=L_plain, t_plain_ms=t_plain, sweeps_plain=k_plain + 1,
                accepted=acc, t_learned_ms=t_learned, sweeps_learned=k_learned, init_ms=init_ms,
                loss_at_learned_init=l_init, learned_final=float(l_loss[-1]),
                control_accepted=c_acc, t_control_ms=t_control, sweeps_control=k_control,
                loss_at_control_init=c_init, control_final=float(c_loss[-1]),
                plain_curve=plain_loss.tolist(), learned_curve=l_loss.tolist(), control_curve=c_loss.tolist())


def summarize(rows: List[Dict]) -> Dict:
    ratio = np.array([r["t_learned_ms"] / r["t_plain_ms"] for r in rows])
    q1, med, q3 = np.percentile(ratio, [25, 50, 75])
    cratio = np.array([r["t_control_ms"] / r["t_plain_ms"] for r in rows])
    lc = np.array([r["t_learned_ms"] / r["t_control_ms"] for r in rows])
    return dict(n=len(rows), acceptance=float(np.mean([r["accepted"] for r in rows])),
                ratio_median=float(med), ratio_q1=float(q1), ratio_q3=float(q3),
                control_acceptance=float(np.mean([r["control_accepted"] for r in rows])),
                control_ratio_median=float(np.median(cratio)),
                learned_over_control_median=float(np.median(lc)),
                learned_over_control_q1=float(np.percentile(lc, 25)),
                learned_over_control_q3=float(np.percentile(lc, 75)),
                final_loss_learned_over_plain_median=float(np.median([r["learned_final"] / r["L_plain"] for r in rows])),
                final_loss_learned_over_control_median=float(np.median([r["learned_final"] / r["control_final"]
                                                                        for r in rows])),
                t_plain_ms_median=float(np.median([r["t_plain_ms"] for r in rows])),
                t_learned_ms_median=float(np.median([r["t_learned_ms"] for r in rows])))


def unet_throughput(net: UNet, X, Y, batch: int, reps: int = 10) -> Dict:
    """Forward and training-step rates of the network (HIP events, warm)."""
    out = torch.empty((batch,) + tuple(Y.shape[1:]), dtype=torch.float32, device=net.device)
    loss = torch.zeros(1, dtype=torch.float64, device=net.device)
    x, y = X[:batch], Y[:batch]
    for _ in range(2):
        net.forward(x, out=out)
        net.backward(x, y, out=out, loss=loss)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record()
    for _ in range(reps):
        net.forward(x, out=out)
    e1.record()
    for _ in range(reps):
        net.backward(x, y, out=out, loss=loss)
    e2.record()
    torch.cuda.synchronize(net.device)
    fwd_ms, bwd_ms = e0.elapsed_time(e1) / reps, e1.elapsed_time(e2) / reps
    f = net.flops_per_sample() * batch
    return dict(batch=batch, forward_ms=fwd_ms, forward_tflops=f / fwd_ms * 1e-9,
                train_step_ms=bwd_ms, train_tflops=3 * f / bwd_ms * 1e-9,
                gflop_per_sample=net.flops_per_sample() * 1e-9, peak_bf16_tflops=2500.0)


def main(argv=None, log=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="learned initialisation: generate, train, time to loss")
    ap.add_argument("--config", type=int, default=3, choices=(3, 4),
                    help="3: config 1's geometry, centre crop; 4: the 1024^2, 12-slice workload, whole object")
    ap.add_argument("--train", type=int, default=None,
                    help="training specimens (default 2000; 125 for config 4, whose specimens give 16 tiles each)")
    ap.add_argument("--test", type=int, default=None, help="held-out specimens (default 100; 3 for config 4)")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--sweeps", type=int, default=None, help="T (default 20; 30 for config 4)")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("a GPU is required")
    if log is None:
        log = lambda m: print(f"[learned-init] {m}", file=sys.stderr, flush=True)
    setup = setup_for(args.config, args.sweeps)
    n_train = args.train if args.train is not None else (2000 if args.config == 3 else 125)
    n_test = args.test if args.test is not None else (100 if args.config == 3 else 3)
    sim = Simulator(setup, "cuda")
    M = setup.geo.n_slices
    tiles = len(setup.train_offsets())
    X, Y, t_gen = generate(sim, setup.train_first, n_train, log=log)
    log(f"training set: {n_train} specimens, {X.shape[0]} crops, in {t_gen:.1f} s "
        f"({1e3 * t_gen / n_train:.2f} ms a specimen)")
    # held-out loss while training: crops of the first held-out specimens, whole batches of them
    if tiles == 1:
        n_val = max(args.batch, (min(n_test, 256) // args.batch) * args.batch)
    else:
        n_val = -(-args.batch // tiles)
    Xv, Yv, _ = generate(sim, setup.test_first, n_val)
    net = UNet(M, M, base=32, levels=4, height=setup.crop, width=setup.crop, max_batch=args.batch, device="cuda")
    net.init_he(seed=setup.geo.seed)
    thr = unet_throughput(net, X, Y, args.batch)
    log(f"unet: forward {thr['forward_tflops']:.1f} TFLOP/s, training step {thr['train_tflops']:.1f} TFLOP/s "
        f"(batch {args.batch})")
    net.init_he(seed=setup.geo.seed)
    tr, held, t_train = train(net, X, Y, args.epochs, args.batch, lr=args.lr, seed=1, Xv=Xv, Yv=Yv, log=log)
    del X, Y, Xv, Yv
    _, _, h, w = setup.window
    if (h, w) != (setup.crop, setup.crop):
        # the same weights in an instance of the window's size, batch 1 (the network is fully
        # convolutional)
        trained = net
        net = UNet(M, M, base=32, levels=4, height=h, width=w, max_batch=1, device="cuda")
        net.set_params(trained.get_params(trained.shapes()))
        del trained
    rows = []
    for i in range(n_test):
        rows.append(time_to_loss(sim, net, setup.test_first + i))
        r = rows[-1]
        log(f"held-out {r['index']}: plain {r['t_plain_ms']:.1f} ms ({r['sweeps_plain']} sweeps), "
            f"learned {r['t_learned_ms']:.1f} ms ({r['sweeps_learned']} sweeps), control {r['t_control_ms']:.1f} ms "
            f"({r['sweeps_control']} sweeps); final loss learned / control {r['learned_final'] / r['control_final']:.4f}")
    summ = summarize(rows)
    where = (f"U-Net trained on the {setup.grid} x {setup.grid} tiles of {setup.crop}^2, applied to the whole "
             f"{h} x {w} object" if setup.whole else f"U-Net on the {setup.crop}^2 centre crop")
    result = dict(workload=f"{setup.geo.name}: {M} slices, {setup.geo.obj_h}^2 object, {sim.plan.n_pos} positions, "
                           + where,
                  train=n_train, train_crops=n_train * tiles, test=n_test, epochs=args.epochs, batch=args.batch,
                  lr=args.lr, sweeps=setup.sweeps, coarse_sweeps=setup.coarse_sweeps, generation_s=t_gen,
                  training_s=t_train, train_loss=tr, heldout_loss=held, unet=thr, time_to_loss=summ, rows=rows)
    log(json.dumps(summ))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(result, f, indent=1)
    return result


if __name__ == "__main__":
    main()
