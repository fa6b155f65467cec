#!/usr/bin/env python3
"""Throughput of the layer-wise multislice hot path on one MI355X.

One step is one fused loss-and-gradient pass (ms_adjoint) over every scan
position of the workload: shifted probes, the forward multislice chain, the
far-field modulus residual, the adjoint chain back to the probe, the
deterministic scatter of the per-position gradients into every slice, the
probe-gradient reduction and the FP64 loss.  The metric counts
S * M position-slice forward+adjoint updates per step.

The headline workload is the largest single-GPU one: 256 x 256 windows, a
1024 x 1024 object of 12 slices and 16384 scan positions (line kernels).  The
128 x 128 workload (fused kernel) is reported beside it.

Prints ONE JSON line.  Also reported (outside the timed region): one
Algorithm 1 sweep (M layer steps and one probe step) and one forward pass.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "position-slice fwd+adjoint updates/s; time-to-loss, learned init vs plain"
UNIT = "position-slice fwd+adjoint updates/s"
HBM_PEAK = 8.0e12            # B/s, MI355X HBM3E
ALU_PEAK = 78.6e12           # FP32 FMA flop/s without packed FP32: 256 CU x 64 lanes x 2 x 2.4 GHz
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2205_03902_amd", "csrc")
# the sources of each per-position kernel family (a traffic record is valid for these only)
KERNEL_SOURCES = {"fused": ["ms_kernels.hpp", "fft_lines.hpp"],
                  "lines": ["line_kernels.hpp", "ms_kernels.hpp", "fft_lines.hpp", "ms_lib.hip"]}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(family: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[family]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def guarded(out: dict, key: str, leg):
    """Runs a leg that follows the headline measurement; if it raises, the error is logged and
    recorded under `key`, and the line with the headline is still printed."""
    try:
        out[key] = leg()
    except Exception as e:  # noqa: BLE001 -- any failure of the leg, recorded in the line
        log(f"bench: {key} failed: {e!r}")
        out[key] = {"error": repr(e)}


def model_per_launch(geo):
    """Algorithmic bytes and flops of the per-position kernels of one adjoint pass over all
    positions (one fused launch, or the 2M + 1 line launches).

    Bytes per position: measured intensities 4 N^2, incident waves stored and
    reloaded 2 (M-1) 8 N^2, slice-gradient patches M 8 N^2, probe-gradient
    patch 8 N^2 (object-patch gathers are cache reuse and not counted; so is the
    half-propagated window the line kernels pass between their launches, which a
    window held on chip would not need).
    Flops per position: (4M - 2) 2D FFTs of 10 N^2 log2 N, plus 30 N^2 M
    pointwise (transmission, propagator, gradient products) and 20 N^2 for the
    modulus residual.
    """
    n2 = geo.n * geo.n
    M = geo.n_slices
    bytes_pos = 4 * n2 + 8 * n2 * (2 * (M - 1) + M + 1)
    flops_pos = (4 * M - 2) * 10 * n2 * math.log2(geo.n) + 30 * n2 * M + 20 * n2
    return bytes_pos * geo.n_pos, flops_pos * geo.n_pos


def pass_bytes(geo):
    """Whole-pass byte model: 32 N^2 M + 4 N^2 per position plus 24 H W M."""
    n2 = geo.n * geo.n
    return (32 * n2 * geo.n_slices + 4 * n2) * geo.n_pos + 24 * geo.obj_h * geo.obj_w * geo.n_slices


def traffic_file(geo, family: str) -> str:
    return os.path.join(PROFILES, f"{family}_adjoint_traffic_{geo.name}.json")


def traffic_record(geo, family: str):
    """The counter record of the per-position kernels (HBM bytes per pass, and where measured the
    VALU instructions per pass), taken with rocprofv3 on this workload and on the current kernel
    sources; None for any other workload, path or source."""
    try:
        with open(traffic_file(geo, family)) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("workload") != geo.name or rec.get("family") != family:
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash(family):
        return None
    return rec


def cpu_baseline(geo, n_sample: int, truth=None):
    """The FP64 oracle on a sample of the same workload (one fwd+adj pass over n_sample evenly
    spaced positions).  The rate is per position-slice update, so it carries over to the whole
    workload linearly (each position's chain is independent; the scatter is a small part)."""
    import numpy as np

    import oracle
    from paper_2205_03902_amd import synth
    pos = geo.positions()
    pick = np.linspace(0, geo.n_pos - 1, n_sample).round().astype(int)
    md = oracle.Model.from_geometry(geo, positions=pos[pick])
    probe = oracle.probe(geo.n, geo.pixel_size, geo.wavelength, geo.alpha, geo.defocus)
    if truth is None:
        truth = synth.transmissions(synth.specimen(geo))
    meas = md.forward(probe, truth)
    if geo.dose > 0:
        meas = synth.poisson_counts(meas, geo.dose, geo.seed + 1)
    start = np.ones_like(truth)
    t0 = time.perf_counter()
    md.loss_grad(probe, start, meas)
    secs = time.perf_counter() - t0
    sample = (f"{n_sample} of {geo.n_pos} positions (evenly spaced), one fwd+adj pass, {secs:.2f} s wall, FP64")
    if n_sample < geo.n_pos:
        sample += (f"; the whole pass extrapolated linearly: {secs * geo.n_pos / n_sample:.0f} s")
    return {"value": n_sample * geo.n_slices / secs, "unit": UNIT, "cores": oracle.max_threads(),
            "kind": "oracle", "cpu": cpu_model(), "sample": sample,
            "extrapolated": n_sample < geo.n_pos}


def cpu_model() -> str:
    """The host CPU's model name, as the kernel reports it."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def coverage_mask(geo, positions):
    """H x W float32: 1 where at least one scan window covers the pixel (periodic object)."""
    import numpy as np
    cover = np.zeros((geo.obj_h, geo.obj_w), dtype=bool)
    rows = np.arange(geo.n)
    for py, px in np.asarray(positions, dtype=np.float64):
        ys = (int(np.floor(py)) + rows) % geo.obj_h
        xs = (int(np.floor(px)) + rows) % geo.obj_w
        cover[np.ix_(ys, xs)] = True
    return cover.astype(np.float32)


def algorithm2_benchmark(n: int, m: int, iterations: int = 3, a_steps: int = 5, cpu_baseline: bool = False):
    """Algorithm 2 (sparse matrix decomposition) on the full-field model: an N x N object, a
    probe moved by integer shifts on an 8 x 8 grid (S = 64), M slices.  Measurements come from
    the multislice forward of the layer-wise path (the two models agree for integer shifts of a
    periodic object).  Reports ms per iteration (A estimate with `a_steps` steps, one
    decomposition pass, the next A; the probe matrix and its norm are set up before the timed
    region), with the iteration's byte model and its GEMM flops.  With cpu_baseline, the CPU
    baseline leg also times one iteration of the FP64 oracle on the same problem."""
    import numpy as np
    import torch

    from paper_2205_03902_amd import abi, smd, synth
    dev = torch.device("cuda:0")
    step = n // 8
    pos = np.array([[y * step, x * step] for y in range(8) for x in range(8)], dtype=np.float64)
    S = pos.shape[0]
    dx, lam = 0.2, 0.0251
    dz = [2.0] * (m - 1)
    ms = abi.Plan(n, n, n, m, pos, dz, dx, lam, device=dev)
    probe = ms.make_probe(0.02, 30.0)
    truth = torch.from_numpy(synth.unit_phase_field((m, n, n), 7, 0.5)).to(dev)
    meas = ms.forward(probe, truth)
    plan = smd.SmdPlan(n, m, pos, dz, dx, lam, device=dev)
    start = torch.ones((m, n, n), dtype=torch.complex64, device=dev)
    plan.set_probe(probe)
    plan.iterate(meas, start.clone(), 1.0, 1, 1)                 # warm-up
    hist = torch.zeros(iterations, dtype=torch.float64, device=dev)
    sl = start.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.iterate(meas, sl, 1.0, iterations, a_steps, hist)
    torch.cuda.synchronize()
    secs = (time.perf_counter() - t0) / iterations
    n2 = n * n
    # The dense formulation would spend 8 (4 a S N^4 + (4(M-1) + 2M) N^6) flops per iteration;
    # here only the two N^4 S products with the probe matrix per estimate step are GEMMs, every
    # G and F product is an FFT propagation of the N^2 images of a matrix.
    gemm_flops = a_steps * 2 * 8 * n2 * n2 * S
    matrix = n2 * n2 * 8
    # bytes: per estimate step A read twice and written once; per decomposition 5 (M - 1)
    # image passes (compose old, suffixes, V, compose new, next A) reading and writing a matrix,
    # the gradient's column sums reading V and S_l per layer, X and the trace sums
    model_bytes = a_steps * 3 * matrix + (5 * (m - 1) * 2 + 2 * m + 2 + 2) * matrix
    res = {"n": n, "slices": m, "positions": S, "iterations": iterations, "a_steps": a_steps,
           "ms_per_iteration": secs * 1e3, "gemm_flops_per_iteration": gemm_flops,
           "model_bytes_per_iteration": model_bytes, "model_gb_per_s": model_bytes / secs / 1e9,
           "dense_equivalent_flops_per_iteration": 8 * (a_steps * 4 * n2 * n2 * S + (4 * (m - 1) + 2 * m) * n2 ** 3),
           "matrix_loss": [float(h) for h in hist.cpu().numpy()]}
    if cpu_baseline:   # the oracle's time, as the cpu_baseline leg reports it for the main step
        from oracle import smd as osmd
        import oracle
        pr = probe.cpu().numpy().astype(np.complex128)
        gs = [osmd.propagator_matrix(oracle.propagator(n, dx, lam, d)) for d in dz]
        mm = meas.cpu().numpy().reshape(S, n2).T.astype(np.float64)
        t1 = time.perf_counter()
        ro, rl, rh = osmd.algorithm2(pr, pos, mm, np.ones((m, n, n), complex), gs, iterations=1, a_steps=a_steps)
        res["oracle_s_per_iteration"] = time.perf_counter() - t1
        res["oracle_threads"] = oracle.max_threads()
    return res


def unet_forward_benchmark(reps: int, batch: int = 16):
    """The learned initialisation's network alone: 4 levels, 32 base channels, 256^2 crops of 6 slices,
    He-initialised, forward passes at `batch` on a seeded input; HIP events over `reps` passes, and the
    flops of every layer (for per-dispatch counters)."""
    import numpy as np
    import torch
    from paper_2205_03902_amd.unet import UNet, to_nhwc_bf16
    dev = torch.device("cuda:0")
    net = UNet(6, 6, base=32, levels=4, height=256, width=256, max_batch=batch, device=dev)
    net.init_he(seed=7)
    rng = np.random.Generator(np.random.PCG64(8))
    x = to_nhwc_bf16(torch.from_numpy(rng.standard_normal((batch, 6, 256, 256)).astype(np.float32)).to(dev), net.in_pad)
    out = torch.empty((batch, 256, 256, 6), dtype=torch.float32, device=dev)
    for _ in range(3):
        net.forward(x, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.forward(x, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    layers = {}
    for name, shp in net.shapes().items():
        level = int(name[3]) if name.startswith(("enc", "dec")) else 0
        px = (256 >> level) ** 2
        k = shp[2] * shp[3]
        layers[name] = {"shape": list(shp), "pixels": px,
                        "gflop": batch * 2.0 * px * shp[0] * shp[1] * (1 if k == 4 and name.endswith("up") else k) / 1e9}
    f = net.flops_per_sample() * batch
    return {"batch": batch, "reps": reps, "forward_ms": ms, "forward_tflops": f / ms * 1e-9,
            "gflop_per_pass": f / 1e9, "layers": layers}


def copy_calibration():
    """A plain device copy of known size, for scaling HBM traffic counters."""
    import torch
    n = 1 << 28                      # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: read {a.numel() * 4 / 1024:.0f} KiB, wrote {b.numel() * 4 / 1024:.0f} KiB")


def device_record():
    """What the device reports about itself, and the HBM rate a plain device copy reaches: the
    measured ceiling beside the published 8 TB/s for the HBM-bound kernels."""
    import torch
    prop = torch.cuda.get_device_properties(0)
    n = 1 << 28                      # 1 GiB of float32 each way
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    rec = {"name": prop.name, "compute_units": prop.multi_processor_count,
           "hbm_gib": round(prop.total_memory / 2 ** 30, 1),
           "copy_GB_s": round(2 * n * 4 / sec / 1e9, 1), "copy_bytes": 2 * n * 4}
    del a, b
    torch.cuda.empty_cache()
    return rec


def time_adjoint(geo, steps: int, warmup: int, dev, batch: int = 0, checkpoint_every: int = 0):
    """Plan, inputs and `steps` timed adjoint passes of one workload.  Inputs are resident in HBM
    before the timed region: the probe and measured patterns are made on the GPU (the probe of
    the 10 %-longer defocus is the start, slices t = 1).  checkpoint_every: which incident waves
    the adjoint stores (1 all, M none; 0 all unless a batch budget is set)."""
    import torch
    from paper_2205_03902_amd import abi, datagen, synth
    log(f"bench: {geo.name} N={geo.n} H=W={geo.obj_h} M={geo.n_slices} S={geo.n_pos}")
    budget = 0
    if batch and batch < geo.n_pos:
        # workspace of a plan whose batches hold `batch` positions
        pb, keep = abi.make_problem(geo.n, geo.obj_h, geo.obj_w, geo.n_slices, geo.positions(), geo.gaps(),
                                    geo.pixel_size, geo.wavelength)
        full = abi.workspace_size(pb)
        # bytes a position adds, as the library counts them: the mean over the problem against
        # a one-position problem (a second position alone also adds shift classes and partials)
        p1, keep1 = abi.make_problem(geo.n, geo.obj_h, geo.obj_w, geo.n_slices, geo.positions()[:1],
                                     geo.gaps(), geo.pixel_size, geo.wavelength)
        per_pos = (full - abi.workspace_size(p1)) // max(geo.n_pos - 1, 1)
        budget = full - (geo.n_pos - batch) * per_pos
    plan = abi.Plan.from_geometry(geo, budget_bytes=budget, device=dev, checkpoint_every=checkpoint_every)
    log(f"bench: {plan.batch} positions per batch, incident waves stored every {plan.checkpoint_every} slices, "
        f"workspace {plan.workspace_bytes / 2 ** 30:.1f} GiB")
    probe_true = plan.make_probe(geo.alpha, geo.defocus)
    truth_np = synth.transmissions(synth.specimen(geo))
    truth = torch.from_numpy(truth_np).to(dev)
    inten = plan.forward(probe_true, truth)
    measured = datagen.poisson(inten, geo.dose, seed=geo.seed + 1, stream_id=0) if geo.dose > 0 else inten
    del inten
    slices = torch.ones((geo.n_slices, geo.obj_h, geo.obj_w), dtype=torch.complex64, device=dev)
    probe = plan.make_probe(geo.alpha, 1.1 * geo.defocus)
    gs = torch.empty_like(slices)
    gp = torch.empty_like(probe)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    for _ in range(warmup):
        plan.adjoint(probe, slices, measured, grad_slices=gs, grad_probe=gp, loss=loss)
    torch.cuda.synchronize()
    # HIP events on the stream every launch is enqueued on
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # one timed region per batch for every wave stored, M + 1 per batch when waves are recomputed
    n_batches = -(-geo.n_pos // plan.batch)
    plan.profile_begin(steps * n_batches * (geo.n_slices + 2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.adjoint(probe, slices, measured, grad_slices=gs, grad_probe=gp, loss=loss)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, launches = plan.profile_end()
    ms = e0.elapsed_time(e1) / steps
    kern = kern_ms / steps
    family = "lines" if geo.n > 128 else "fused"
    log(f"bench: {steps} steps, {ms:.3f} ms/step (events), {wall * 1e3 / steps:.3f} ms/step (wall), "
        f"{family} kernels {kern:.3f} ms per pass ({launches} timed regions), loss {loss.item():.6e}")
    return {"plan": plan, "probe": probe, "probe_true": probe_true, "slices": slices, "measured": measured,
            "truth": truth,
            "truth_np": truth_np, "gs": gs, "gp": gp, "ms": ms, "kernel_ms": kern, "family": family,
            "loss": loss.item(), "batch": plan.batch, "checkpoint_every": plan.checkpoint_every,
            "workspace_bytes": plan.workspace_bytes}


def roofline(geo, family: str, kernel_ms: float):
    """Roofline record of the per-position kernels of one pass (the dominant kernel family)."""
    byt, flo = model_per_launch(geo)
    k_s = kernel_ms * 1e-3
    hbm = {"bound": "hbm", "achieved": byt / k_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s"}
    hbm["frac"] = hbm["achieved"] / hbm["peak"]
    alu = {"bound": "alu", "achieved": flo / k_s / 1e12, "peak": ALU_PEAK / 1e12, "unit": "TFLOP/s"}
    alu["frac"] = alu["achieved"] / alu["peak"]
    roof = dict(alu if alu["frac"] >= hbm["frac"] else hbm)
    other = hbm if roof["bound"] == "alu" else alu
    rec = traffic_record(geo, family)
    roof["traffic"] = rec.get("bytes_per_pass") if rec else None
    if roof["traffic"]:
        # the counted bytes over this run's kernel time: the achieved HBM rate
        roof["traffic_GB_s"] = roof["traffic"] / k_s / 1e9
    if rec and rec.get("valu_issue_ms_per_pass"):
        # the share of the kernel time the counted VALU instructions alone take at one 4-cycle
        # issue per wave64 instruction on 1024 SIMDs at 2.4 GHz (FP32 VALU utilisation)
        roof["valu_issue_frac"] = rec["valu_issue_ms_per_pass"] / kernel_ms
    if family == "fused":
        roof["kernel"] = f"fused_kernel<{geo.n}, adjoint> (one launch per pass)"
    else:
        roof["kernel"] = (f"line_kernel<{geo.n}, frame> (forward and far field) and line_band_kernel<{geo.n}, frame> "
                          f"(adjoint): the {2 * geo.n_slices + 1} launches of one pass, timed together")
    roof["kernel_ms"] = kernel_ms
    roof["other"] = {k: other[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roof["algorithmic_bytes_per_launch"] = byt
    roof["algorithmic_flops_per_launch"] = flo
    return roof


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=4, help="workload geometry (0..4); 4 is the headline")
    ap.add_argument("--cpu-sample", type=int, default=1024, help="positions in the oracle's timing sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the sweep and forward timings")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 128 x 128 workload and the recomputed-wave run of the 10-slice workload")
    ap.add_argument("--checkpoint-every", type=int, default=0,
                    help="incident waves the adjoint stores: 1 all, k every k-th, >= M none (0: all unless --batch)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--batch", type=int, default=0,
                    help="about this many positions per batch (0 = all at once): sets the plan's workspace "
                         "budget; the log reports the batch the plan chose")
    ap.add_argument("--no-time-to-loss", action="store_true",
                    help="skip the learned-initialisation runs (generation, training, time to loss)")
    ap.add_argument("--ttl-train", type=int, default=2000, help="training specimens of the time-to-loss run")
    ap.add_argument("--ttl-test", type=int, default=100, help="held-out specimens of the time-to-loss run")
    ap.add_argument("--ttl-epochs", type=int, default=20, help="training epochs of the time-to-loss run")
    ap.add_argument("--ttl4-train", type=int, default=32,
                    help="training specimens (16 tiles each) of the 1024^2, 12-slice time-to-loss run")
    ap.add_argument("--ttl4-test", type=int, default=2, help="held-out specimens of that run")
    ap.add_argument("--time-to-loss-config4", action="store_true",
                    help="run that comparison with its full protocol: 125 training specimens (2000 tiles) and 8 "
                         "held-out (about 14 minutes)")
    ap.add_argument("--unet-only", type=int, default=0, metavar="REPS",
                    help="time only the network's forward pass (256^2 crops of 6 slices, batch 16) REPS times "
                         "and print its JSON with the flops of every layer")
    ap.add_argument("--algorithm2-only", type=int, default=0, metavar="N",
                    help="time only Algorithm 2 at window N (M = 3) and print its JSON")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}, WORLD_SIZE {world}): the library "
              "implements the single-GPU hot path; sharding positions over GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration()
        return

    if args.unet_only:
        torch.cuda.set_device(0)
        print(json.dumps(unet_forward_benchmark(args.unet_only)), flush=True)
        return

    if args.algorithm2_only:
        torch.cuda.set_device(0)
        print(json.dumps(algorithm2_benchmark(args.algorithm2_only, 3)), flush=True)
        return

    from paper_2205_03902_amd import configs, layerwise
    from paper_2205_03902_amd import abi
    geo = configs.CONFIGS[args.config]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    run = time_adjoint(geo, args.steps, args.warmup, dev, args.batch, args.checkpoint_every)
    plan, probe, slices, measured = run["plan"], run["probe"], run["slices"], run["measured"]
    gs, gp, truth = run["gs"], run["gp"], run["truth"]
    ms = run["ms"]
    batch = run["batch"]
    value = geo.n_pos * geo.n_slices / (ms * 1e-3)
    roof = roofline(geo, run["family"], run["kernel_ms"])

    extras = {}
    if not args.no_extras:
        extras["device"] = device_record()
        # one forward pass
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for _ in range(3):
            plan.forward(probe, slices)
        torch.cuda.synchronize()
        extras["forward_ms"] = (time.perf_counter() - f0) * 1e3 / 3
        probe_start_err = (torch.linalg.vector_norm(probe - run["probe_true"]) /
                           torch.linalg.vector_norm(run["probe_true"])).item()
        # one Algorithm 1 sweep: M layer steps and one probe step over all positions
        sl = slices.clone()
        pr = probe.clone()
        h = layerwise.reconstruct(plan, pr, sl, measured, sweeps=1, k_steps=1, probe_steps=1)
        extras["sweep_ms"] = h.seconds * 1e3
        extras["sweep_losses"] = [h.loss[0], h.loss[-1]]
        # the paper's relative reconstruction error over the pixels some window covers, before and
        # after the sweep (which also steps the probe), after a common translation of the slices
        # (|d| <= 4 px) and a complex scale per slice
        cover = coverage_mask(geo, geo.positions())
        mask_t = torch.from_numpy(cover).to(dev)
        shift = torch.zeros(2, dtype=torch.int32, device=dev)
        r0 = abi.reconstruction_error(slices, truth, mask_t, max_shift=4)
        r1 = abi.reconstruction_error(sl, truth, mask_t, max_shift=4, shift=shift)
        extras["recon_error_start_after_sweep"] = [r0[-1].item(), r1[-1].item()]
        extras["recon_error_shift_after_sweep"] = [int(v) for v in shift.cpu().tolist()]
        del sl, pr
        # the full-gradient (Jacobi) variant from the same start: 4 steps against one sweep,
        # with the layer steps as they are and averaged (step scale 1/M)
        end = torch.zeros(1, dtype=torch.float64, device=dev)
        for tag, scale in (("full_step", 1.0), ("full_step_avg", 1.0 / geo.n_slices)):
            sl = slices.clone()
            fl = torch.zeros(1, dtype=torch.float64, device=dev)
            losses = []
            torch.cuda.synchronize()
            t0f = time.perf_counter()
            for _ in range(4):
                plan.full_step(1, probe, sl, measured, loss=fl, step_scale=scale)
                losses.append(fl.clone())
            torch.cuda.synchronize()
            extras[f"{tag}_ms"] = (time.perf_counter() - t0f) * 1e3 / 4
            plan.adjoint(probe, sl, measured, grad_slices=gs, grad_probe=gp, loss=end)
            extras[f"{tag}_losses"] = [x.item() for x in losses] + [end.item()]
            del sl
        sl2 = slices.clone()
        layerwise.reconstruct(plan, probe.clone(), sl2, measured, sweeps=1)
        plan.adjoint(probe, sl2, measured, grad_slices=gs, grad_probe=gp, loss=end)
        extras["sweep_loss_after"] = end.item()
        del sl2
        # the workload's whole reconstruction: its layer-wise sweeps (30 for the 16384-position
        # workload), each followed by a probe step over all positions (joint probe estimation), from
        # t = 1 and the 1.1x-defocus probe; the final loss and the aligned error against the truth
        sl3, pr3 = slices.clone(), probe.clone()
        hr = layerwise.reconstruct(plan, pr3, sl3, measured, sweeps=geo.iterations, probe_steps=1)
        shift3 = torch.zeros(2, dtype=torch.int32, device=dev)
        r3 = abi.reconstruction_error(sl3, truth, mask_t, max_shift=4, shift=shift3)
        probe_true_err = (torch.linalg.vector_norm(pr3 - run["probe_true"]) /
                          torch.linalg.vector_norm(run["probe_true"])).item()
        extras["reconstruction"] = {"sweeps": geo.iterations, "probe_steps_per_sweep": 1, "seconds": hr.seconds,
                                    "loss_first_last": [hr.loss[0], hr.loss[-1]],
                                    "loss_never_rises": bool(all(b <= a * (1 + 1e-6) for a, b in
                                                                 zip(hr.loss, hr.loss[1:]))),
                                    "recon_error": r3[-1].item(), "recon_shift": [int(v) for v in shift3.cpu().tolist()],
                                    "probe_rel_error_start_end": [probe_start_err, probe_true_err]}
        del sl3, pr3
        extras["pass_model_bytes"] = pass_bytes(geo)
        # scan-position gradient and curvature bound over all positions (a probe-mode pass)
        gpos = torch.empty((geo.n_pos, 2), dtype=torch.float64, device=dev)
        cpos = torch.empty_like(gpos)
        plan.position_grad(probe, slices, measured, gpos, cpos)
        torch.cuda.synchronize()
        t0p = time.perf_counter()
        for _ in range(3):
            plan.position_grad(probe, slices, measured, gpos, cpos)
        torch.cuda.synchronize()
        extras["position_grad_ms"] = (time.perf_counter() - t0p) * 1e3 / 3
        log("bench: Algorithm 2 (sparse matrix decomposition) at N = 32 and 64")
        extras["algorithm2"] = [algorithm2_benchmark(32, 3, cpu_baseline=not args.no_cpu_baseline),
                                algorithm2_benchmark(64, 3)]

    truth_np = run["truth_np"]
    del run, plan, probe, slices, measured, gs, gp, truth
    torch.cuda.empty_cache()
    if not args.no_secondary and args.config != 1:
        # the 128 x 128 workload on the fused kernel, beside the headline
        g1 = configs.CFG1
        r1 = time_adjoint(g1, args.steps, args.warmup, dev)
        extras["cfg1"] = {"workload": f"{g1.name}: {g1.n}x{g1.n} window, {g1.obj_h}x{g1.obj_w} object, "
                                      f"{g1.n_slices} slices, {g1.n_pos} positions",
                          "value": g1.n_pos * g1.n_slices / (r1["ms"] * 1e-3), "unit": UNIT,
                          "ms_per_step": r1["ms"], "roofline": roofline(g1, r1["family"], r1["kernel_ms"])}
        del r1
        torch.cuda.empty_cache()
    if not args.no_secondary and args.config != 2:
        # the 10-slice 256 x 256 workload with every incident wave stored and with none (each
        # recomputed from the probe during the adjoint)
        g2 = configs.CFG2
        legs = {}
        for k in (1, g2.n_slices):
            r2 = time_adjoint(g2, max(3, args.steps // 4), 1, dev, checkpoint_every=k)
            legs[f"checkpoint_every_{k}"] = {"ms_per_step": r2["ms"], "kernel_ms": r2["kernel_ms"],
                                             "value": g2.n_pos * g2.n_slices / (r2["ms"] * 1e-3),
                                             "workspace_gib": r2["workspace_bytes"] / 2 ** 30,
                                             "loss": r2["loss"]}
            del r2
            torch.cuda.empty_cache()
        extras["cfg2_waves_stored_vs_recomputed"] = dict(
            workload=f"{g2.name}: {g2.n}x{g2.n} window, {g2.obj_h}x{g2.obj_w} object, {g2.n_slices} slices, "
                     f"{g2.n_pos} positions", unit=UNIT, **legs)

    out = {"metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{geo.name}: {geo.n}x{geo.n} window, {geo.obj_h}x{geo.obj_w} object, "
                                  f"{geo.n_slices} slices, {geo.n_pos} positions",
                      "n": geo.n, "obj": geo.obj_h, "slices": geo.n_slices, "positions": geo.n_pos,
                      "parallelism": "single GPU, " + ("positions in one batch" if batch == geo.n_pos
                                                       else f"{batch} positions per batch")},
           "roofline": roof}
    out.update(extras)
    if not args.no_time_to_loss:
        from paper_2205_03902_amd import learned_init

        def ttl3():
            log("bench: learned initialisation (generate, train, time to loss)")
            res = learned_init.main(["--train", str(args.ttl_train), "--test", str(args.ttl_test),
                                     "--epochs", str(args.ttl_epochs)], log=log)
            return dict(res["time_to_loss"], workload=res["workload"], train=res["train"], test=args.ttl_test,
                        epochs=res["epochs"], sweeps=res["sweeps"], generation_s=res["generation_s"],
                        training_s=res["training_s"], heldout_loss=res["heldout_loss"][-1:], unet=res["unet"])
        guarded(out, "time_to_loss", ttl3)
    if not args.no_time_to_loss or args.time_to_loss_config4:
        # the same comparison on the headline workload: by default a reduced training set (32
        # specimens, 512 tiles) and 2 held-out specimens; the full protocol with the flag
        from paper_2205_03902_amd import learned_init
        train4, test4 = (125, 8) if args.time_to_loss_config4 else (args.ttl4_train, args.ttl4_test)

        def ttl4():
            log(f"bench: learned initialisation on the 1024^2, 12-slice workload ({train4} training specimens, "
                f"{test4} held-out)")
            torch.cuda.empty_cache()
            res = learned_init.main(["--config", "4", "--train", str(train4), "--test", str(test4)], log=log)
            return dict(res["time_to_loss"], workload=res["workload"], train=res["train"],
                        train_crops=res["train_crops"], test=res["test"], epochs=res["epochs"], sweeps=res["sweeps"],
                        generation_s=res["generation_s"], training_s=res["training_s"],
                        heldout_loss=res["heldout_loss"][-1:])
        guarded(out, "time_to_loss_cfg4", ttl4)
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(geo, min(args.cpu_sample, geo.n_pos), truth=truth_np)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
