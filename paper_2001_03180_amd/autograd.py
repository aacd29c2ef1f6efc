"""torch.autograd.Function around the integrator and its adjoint.

integrate(x0, v0, ...) runs the integrator (mstar_integrate_record: adaptive
steps, MST coordinates) and returns the end state (x, v, t) as tensors; its
backward pass runs mstar_replay_adjoint on the recorded steps, i.e. the
gradient of the discrete map with the step-size controller frozen
(discretise, then differentiate).  The end time t is an output because the
map advances a fixed number of fictitious steps: for an objective at a fixed
physical time t_end, write it in terms of x + v (t_end - t) and the gradient
flows through t as well.
"""
from __future__ import annotations

import numpy as np
import torch

from .mstar import Context, params as _params


class _Integrate(torch.autograd.Function):
    """Device tensors stay on the device (the library's device-pointer path);
    host tensors go through host arrays.  Both give the same bits."""

    @staticmethod
    def forward(fctx, x0, v0, m, t0, t_end, max_accepted, mctx, p, checkpoint_every):
        dev = x0.device
        on_dev = x0.is_cuda
        if on_dev:
            mm = torch.as_tensor(m, dtype=torch.float64, device=dev)
            xs, vs, rc, st, H = mctx.integrate_record(mm, x0.detach().contiguous(), v0.detach().contiguous(), t0,
                                                      t_end, max_accepted, p)
        else:
            mm = m
            xs, vs, rc, st, H = mctx.integrate_record(m, x0.detach().numpy(), v0.detach().numpy(), t0, t_end,
                                                      max_accepted, p)
        fctx.save_for_backward(x0, v0)
        fctx.info = (mm, t0, H, mctx, p, checkpoint_every, on_dev)
        fctx.stats = st
        x = xs if on_dev else torch.as_tensor(xs)
        v = vs if on_dev else torch.as_tensor(vs)
        t = torch.tensor(st["t_reached"], dtype=torch.float64, device=dev)
        return x, v, t

    @staticmethod
    def backward(fctx, gx, gv, gt):
        x0, v0 = fctx.saved_tensors
        mm, t0, H, mctx, p, ce, on_dev = fctx.info
        gtn = float(gt) if gt is not None else 0.0
        if on_dev:
            z = torch.zeros_like(x0)
            gxd = gx.detach().contiguous() if gx is not None else z
            gvd = gv.detach().contiguous() if gv is not None else z
            gx0, gv0 = mctx.replay_adjoint(mm, x0.detach().contiguous(), v0.detach().contiguous(), t0, H, gxd, gvd,
                                           gtn, ce, p)
        else:
            z = np.zeros((len(mm), 3))
            gxn = gx.detach().numpy() if gx is not None else z
            gvn = gv.detach().numpy() if gv is not None else z
            gx0, gv0 = mctx.replay_adjoint(mm, x0.detach().numpy(), v0.detach().numpy(), t0, H, gxn, gvn, gtn, ce, p)
            gx0, gv0 = torch.as_tensor(gx0), torch.as_tensor(gv0)
        return gx0, gv0, None, None, None, None, None, None, None


def integrate(x0: torch.Tensor, v0: torch.Tensor, m, t0: float, t_end: float, max_accepted: int = 10 ** 9,
              ctx: Context | None = None, checkpoint_every: int = 50, **kw):
    """Differentiable end state (x, v, t) of the integration from (x0, v0) at t0
    to t_end (or max_accepted accepted GBS steps, whichever comes first)."""
    ctx = ctx or Context(0)
    p = _params(**kw)
    return _Integrate.apply(x0, v0, np.ascontiguousarray(m, dtype=np.float64), float(t0), float(t_end),
                            int(max_accepted), ctx, p, int(checkpoint_every))
