"""Stillinger-Weber energy as a torch.autograd.Function.

Forward evaluates the per-system energy E_s(x, strain_s, theta) in the HIP
library; backward calls the library's gradient pass with the upstream
gradient as its scale, which returns dL/dx = -F dL/dE, dL/dstrain = Xi
dL/dE (the virial dE/dstrain, 3x3 per system) and dL/dtheta = sum_s dL/dE_s
dE_s/dtheta for theta = (A, B, p, q, a, lambda_sw, gamma, sigma, epsilon).
Strains must be diagonal (orthorhombic boxes); the gradient with respect to
every strain component, off-diagonal ones included, is returned.  The
function is differentiable once.
"""
from __future__ import annotations

import torch

from . import swfe

PARAM_NAMES = swfe.PARAM_NAMES


def theta_of(params: dict) -> torch.Tensor:
    return torch.tensor([params[k] for k in PARAM_NAMES], dtype=torch.float64)


def _params_from_theta(base: dict, theta: torch.Tensor) -> dict:
    vals = theta.detach().cpu().tolist()
    out = dict(base)
    out.update(dict(zip(PARAM_NAMES, vals)))
    return out


class SWEnergy(torch.autograd.Function):
    """E = SWEnergy.apply(x, strain, theta, engine).

    x: (3, n_total) FP64 on the engine's device (packed systems, the layout of
    Engine.x); strain: (n_sys, 3, 3) FP64 (any device); theta: (9,) FP64.
    Returns the (n_sys,) energies."""

    @staticmethod
    def forward(ctx, x, strain, theta, engine):
        engine.x.copy_(x.detach())
        engine.set_params(_params_from_theta(engine.params, theta))
        st = strain.detach().cpu().numpy().reshape(engine.n_sys, 9)
        use_strain = bool((st != 0).any())
        out = engine.compute_forces(strain=st if use_strain else None)
        ctx.engine = engine
        ctx.strain = st if use_strain else None
        ctx.devices = (x.device, strain.device, theta.device)
        ctx.save_for_backward(x, theta)
        return out[:, 0].clone()

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, gE):
        eng = ctx.engine
        x, theta = ctx.saved_tensors
        eng.x.copy_(x.detach())
        eng.set_params(_params_from_theta(eng.params, theta))
        gs = gE.detach().to(device=eng.device, dtype=torch.float64).contiguous()
        gx = torch.empty_like(eng.x)
        out = eng.compute_forces(param_grad=True, strain=ctx.strain, grad_scale=gs, grad_x=gx)
        g_strain = out[:, 2:11].reshape(eng.n_sys, 3, 3)
        g_theta = out[:, 11:20].sum(dim=0)
        dx, ds, dt = ctx.devices
        return gx.to(dx), g_strain.to(ds), g_theta.to(dt), None


def sw_energy(x, strain, theta, engine):
    return SWEnergy.apply(x, strain, theta, engine)
