"""Algorithm 1 (layer-wise estimation, Sec. 3.3) with the optional probe step of Sec. 3.5.

Each sweep visits the layers l = 1..M in order (Gauss-Seidel: the layers
before l already hold their new values, eq. Layerwise_Prefix_Suffix) and runs
K amplitude-flow steps on layer l through ms_layer_step; a probe step may
follow every sweep.  Losses and step sizes stay on the device until the run
ends, so the loop never waits for the GPU.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import torch

from .abi import Plan, check_finite


@dataclasses.dataclass
class History:
    loss: List[float]          # loss before each layer / probe step
    mu: List[float]            # step size of each step
    kind: List[str]            # "layer<l>" or "probe"
    seconds: float             # wall time of the run (GPU work included)


def reconstruct(plan: Plan, probe: torch.Tensor, slices: torch.Tensor, measured: torch.Tensor, sweeps: int,
                k_steps: int = 1, probe_steps: int = 0, subset: Optional[list] = None,
                carry: bool = True) -> History:
    """Runs `sweeps` sweeps in place on `slices` (and `probe` when probe_steps > 0).  carry: each
    layer step starts its forward chain from the incident wave the previous one left (the same
    results; the buffers change only through these calls meanwhile)."""
    M = plan.n_slices
    plan.set_layer_carry(1 if carry else 0)
    per_sweep = M + (1 if probe_steps > 0 else 0)
    buf = torch.zeros((max(sweeps * per_sweep, 1), 2), dtype=torch.float64, device=plan.device)
    kinds = []
    torch.cuda.synchronize(plan.device)
    t0 = time.perf_counter()
    i = 0
    for _ in range(sweeps):
        for layer in range(M):
            plan.layer_step(layer, k_steps, probe, slices, measured, loss=buf[i, 0:1], mu=buf[i, 1:2])
            kinds.append(f"layer{layer}")
            i += 1
        if probe_steps > 0:
            plan.probe_step(probe_steps, probe, slices, measured, subset=subset, loss=buf[i, 0:1], mu=buf[i, 1:2])
            kinds.append("probe")
            i += 1
    torch.cuda.synchronize(plan.device)
    secs = time.perf_counter() - t0
    plan.set_layer_carry(0)
    h = buf[:i].cpu().numpy()
    check_finite(h[:, 0], "reconstruct")
    return History(loss=h[:, 0].tolist(), mu=h[:, 1].tolist(), kind=kinds, seconds=secs)


def refine_positions(plan: Plan, probe: torch.Tensor, slices: torch.Tensor, measured: torch.Tensor, passes: int,
                     step_scale: float = 1.0, positions=None, adaptive: bool = True):
    """Scan-position refinement at fixed probe and slices, `passes` gradient passes in all.

    Each pass is one ms_position_step: the loss at the plan's positions and the step
    -scale grad / curv from them.  With `adaptive`, a step whose new positions lower the loss
    is accepted and the next scale doubled; one that raises it is undone and the step retaken
    from the accepted positions at half the scale.  The plan's geometry is host data, so new
    positions are read back and a plan of those positions is built (same geometry, path and
    objective).  positions: the plan's positions (default: those it was built from).
    Returns (plan of the accepted positions, those positions (device float64 [S, 2]), the
    accepted losses in order)."""
    import numpy as np
    if positions is None:
        positions = plan.positions()
    dev = plan.device
    pos_a = torch.as_tensor(np.asarray(positions, dtype=np.float64).reshape(-1, 2), device=dev).clone()
    lbuf = torch.zeros(1, dtype=torch.float64, device=dev)
    scale = float(step_scale)
    plan_a = plan
    cand = pos_a.clone()
    plan_a.position_step(cand, probe, slices, measured, scale, loss=lbuf)
    loss_a = lbuf.item()
    check_finite(loss_a, "refine_positions")
    losses = [loss_a]
    for _ in range(int(passes) - 1):
        plan_c = plan_a.with_positions(cand.cpu().numpy())
        nxt = cand.clone()
        next_scale = 2.0 * scale if adaptive else scale
        plan_c.position_step(nxt, probe, slices, measured, next_scale, loss=lbuf)
        loss_c = lbuf.item()
        check_finite(loss_c, "refine_positions")
        if loss_c <= loss_a or not adaptive:
            plan_a, pos_a, loss_a, scale = plan_c, cand, loss_c, next_scale
            losses.append(loss_c)
            cand = nxt
        else:
            scale *= 0.5
            cand = pos_a.clone()
            plan_a.position_step(cand, probe, slices, measured, scale, loss=lbuf)
    return plan_a, pos_a, losses
