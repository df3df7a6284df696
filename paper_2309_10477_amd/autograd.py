"""torch.autograd.Function over the library's adjoint kernels.

HestonAdjoint.apply(theta, spec) returns the Monte-Carlo price as a 0-d
float64 tensor; its backward runs the reverse sweep over the checkpoints the
forward stored and returns grad * d price / d theta for
theta = (S0, v0, r, kappa, theta, sigma, rho).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import ADJOINT_PARAMS, FP32, GREEKS_PATHWISE, Context, Options, ckpt_bytes


@dataclass
class AdjointSpec:
    K: float
    T: float
    opt_type: int
    n_paths: int
    n_steps: int
    seed: int
    precision: int = FP32
    every: int = 16
    scheme: int = 0
    fixings: tuple | None = None
    ctx: Context | None = None
    last: dict = field(default_factory=dict)  # standard errors of the last call

    def params(self, theta) -> dict:
        t = [float(v) for v in theta]
        d = dict(zip(ADJOINT_PARAMS, t))
        d.update(K=self.K, T=self.T)
        return d

    def options(self) -> Options:
        return Options(precision=self.precision, scheme=self.scheme, greeks=GREEKS_PATHWISE,
                       fixings=self.fixings)


class HestonAdjoint(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta: torch.Tensor, spec: AdjointSpec):
        if spec.ctx is None:
            spec.ctx = Context(theta.device.index if theta.is_cuda else 0)
        ctx = spec.ctx
        dev = f"cuda:{ctx.device}"
        nbytes = ckpt_bytes(spec.n_paths, spec.n_steps, spec.every, spec.precision)
        ckpt = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        params = spec.params(theta.detach().cpu())
        (price, se), ms = ctx.adjoint_forward(params, spec.opt_type, spec.n_paths, spec.n_steps,
                                              spec.seed, ckpt, spec.every, spec.options())
        spec.last["price"] = (price, se)
        spec.last["forward_ms"] = ms
        fctx.spec = spec
        fctx.params = params
        fctx.save_for_backward(ckpt)
        fctx.theta_device = theta.device
        return torch.tensor(price, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(fctx, grad_out: torch.Tensor):
        (ckpt,) = fctx.saved_tensors
        spec = fctx.spec
        g = float(grad_out.detach().cpu())
        grads, ms = spec.ctx.adjoint_backward(fctx.params, spec.opt_type, spec.n_paths,
                                              spec.n_steps, spec.seed, ckpt, spec.every, g,
                                              spec.options())
        spec.last["grads"] = grads
        spec.last["backward_ms"] = ms
        out = torch.tensor([v for v, _ in grads], dtype=torch.float64, device=fctx.theta_device)
        return out, None
