"""The engine's NLL as a differentiable torch operation.

`NLL(engine, stream)` is a module whose forward runs one device evaluation
(fold, bin stages, Poisson NLL with priors, Eq. 3-6 and 9) and whose backward
returns the adjoint gradient computed in that same pass, scaled by the
incoming gradient. No finite differences and no host round trip: the
parameter vector and the outputs stay in device memory, and the engine's
stream is ordered against torch's current stream with stream waits.
"""
from __future__ import annotations

import torch

from . import nufold as nf


class _NLLFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, module):
        th = theta.detach().to(dtype=torch.float64).contiguous()
        if th.numel() != module.engine.P:
            raise ValueError(f"theta has {th.numel()} entries, the model {module.engine.P}")
        out = torch.empty(1 + module.engine.P, dtype=torch.float64, device=th.device)
        status = torch.zeros(1, dtype=torch.int32, device=th.device)
        cur = torch.cuda.current_stream(th.device)
        module.stream.wait_stream(cur)
        module.engine.eval_device(th.data_ptr(), out.data_ptr(), status.data_ptr(), want_grad=True)
        cur.wait_stream(module.stream)
        for t in (th, out, status):
            t.record_stream(module.stream)
        ctx.save_for_backward(out)
        ctx.theta_dtype = theta.dtype
        module.last_status = status
        return out[0].clone()

    @staticmethod
    def backward(ctx, grad_output):
        (out,) = ctx.saved_tensors
        return (grad_output * out[1:]).to(ctx.theta_dtype), None


class NLL(torch.nn.Module):
    """engine: an nufold.Engine created with stream=stream.cuda_stream, with
    events and data set. forward(theta) -> scalar NLL tensor (float64)."""

    def __init__(self, engine: nf.Engine, stream: torch.cuda.Stream):
        super().__init__()
        self.engine = engine
        self.stream = stream
        self.last_status = None

    def forward(self, theta):
        return _NLLFunction.apply(theta, self)

    @staticmethod
    def create(desc, events, data, mode="m64"):
        """Engine on a new stream, with events and data (lists per dataset) set."""
        stream = torch.cuda.Stream()
        eng = nf.Engine(desc, mode, stream=stream.cuda_stream)
        for d, ev in enumerate(events):
            eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
            eng.set_data(d, data[d])
        return NLL(eng, stream)
