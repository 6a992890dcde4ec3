"""torch.autograd binding of the adjoint: the membrane-potential loss of a
simulation window as a differentiable function of the synaptic weights.

    w = torch.tensor(weights_pA, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = window_loss(net, w, window=2000, ckpt_every=200, v_target=-58.0)
    loss.backward()          # w.grad = dL/dw, spike pattern of the window held fixed

The forward sets the network's weights to rint(w * 2^16) / 2^16 pA, simulates
the window and runs the reverse-time adjoint in the same library call
(``mc_adjoint``); backward scales the stored gradient by the incoming one.
The gradient is taken at the quantised weights with the quantisation and the
spike pattern frozen (the loss is then quadratic in the weights).  A float32
``w`` selects float32 gradient accumulation (from float64 adjoint states);
float64 gives float64 gradients.  All arithmetic runs in libmc's kernels;
torch provides the device buffers only.
"""
from __future__ import annotations

import torch

from . import mc

if mc._lib is not None and not mc.loaded_after_torch:
    raise ImportError("libmc was loaded before torch: import torch (or this module) before the first "
                      "paper_2111_04398_amd.mc call so that one HIP runtime serves both")


class _WindowLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, w: torch.Tensor, net: mc.Network, window: int, ckpt_every: int, v_target: float):
        if w.device.type != "cuda" or w.dim() != 1 or w.numel() != net.M:
            raise ValueError(f"w must be a 1-D device tensor of {net.M} weights (pA)")
        if w.dtype not in (torch.float32, torch.float64):
            raise TypeError("w must be float32 or float64")
        w64 = w.detach().to(torch.float64).contiguous()
        grad = torch.empty(net.M, dtype=w.dtype, device=w.device)
        torch.cuda.current_stream(w.device).synchronize()   # w64 is written on torch's stream
        net.set_weights(w64.data_ptr())
        loss = net.adjoint(window, ckpt_every, v_target, fp32=(w.dtype == torch.float32), grad_ptr=grad.data_ptr())
        ctx.save_for_backward(grad)
        return torch.tensor(loss, dtype=torch.float64, device=w.device)

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        (grad,) = ctx.saved_tensors
        return grad * g.to(grad.dtype), None, None, None, None


def window_loss(net: mc.Network, w: torch.Tensor, window: int, ckpt_every: int, v_target: float) -> torch.Tensor:
    """Loss L = 1/(N S) sum (V - v_target)^2 over the next `window` steps of
    `net` (which advances by `window` steps), differentiable in `w`."""
    return _WindowLoss.apply(w, net, int(window), int(ckpt_every), float(v_target))


def fit_weights(net: mc.Network, window: int, ckpt_every: int, v_target: float, iters: int, eta: float,
                fp32: bool = False) -> list:
    """Gradient descent on the explicitly stored weights (the Discussion of
    the paper notes that storing every synapse keeps plasticity and learning
    possible).  Every iteration restarts the window from the network state
    at the call, takes dL/dw with the spike pattern frozen (``mc_adjoint``)
    and moves every weight by -eta * dL/dw, re-quantised on the device
    (``mc_apply_gradient``); the weights live in the library's store.  torch
    only provides the gradient buffer.  The network ends at the state after
    the last window.  Returns the loss of every iteration (before its step)."""
    start = net.save_state()
    grad = torch.empty(net.M, dtype=torch.float32 if fp32 else torch.float64, device="cuda")
    losses = []
    for it in range(iters):
        if it:
            net.load_state(start)
        losses.append(net.adjoint(window, ckpt_every, v_target, fp32, grad.data_ptr()))
        net.apply_gradient(grad.data_ptr(), fp32, eta)
    return losses
