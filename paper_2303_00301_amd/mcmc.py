"""Host-side MCMC drivers around the C ABI: step-size warm-up.

The paper calibrates one global delta for the Kalman samplers toward a target
acceptance rate (Sec. 4, experimental setup) without specifying the mechanism.
Here: a Robbins-Monro recursion on log delta,
    log delta_{k+1} = log delta_k + k^{-0.6} (accept_k - target),
run for a fixed number of warm-up steps, after which delta is frozen (so the
timed chain is a fixed-kernel MH chain).
"""
from __future__ import annotations

import math

import torch

from . import sampler as S


def tune_delta(model: "S.DeviceModel", y: torch.Tensor, x: torch.Tensor, delta0: float,
               order: int, n_warmup: int, target: float = 0.3, seed: int = 0,
               block: int = 0) -> dict:
    """Returns dict(delta=frozen delta, x=state after warm-up, history=[...])."""
    dev = x.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    N, d = model.N, model.dx
    log_d = math.log(delta0)
    hist = []
    ws = S.Workspace(dev)
    x = x.clone()
    for k in range(1, n_warmup + 1):
        xi = torch.randn((2, N, d), dtype=torch.float64, device=dev, generator=gen)
        un = torch.rand((1,), dtype=torch.float64, device=dev, generator=gen).clamp_(min=1e-300)
        out = S.mh_step(model, y, x, math.exp(log_d), order, xi, un, x_out=x, block=block, ws=ws)
        acc = float(out["accepted"].item())
        hist.append((math.exp(log_d), acc))
        log_d += k ** -0.6 * (acc - target)
    return dict(delta=math.exp(log_d), x=x, history=hist)
