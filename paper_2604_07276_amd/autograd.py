"""torch.autograd.Function over the DPA-1 library's forward/adjoint split.

The forward runs the library's forward half (dp_forward_device) and returns
the atomic energies e_i; the backward runs the library's hand-written adjoint
(dp_backward_device) with the incoming gradient as per-atom weights, so
d(sum_i w_i e_i)/dx comes out of the same kernels that produce the forces
(F = -dE/dx, Eq. (2); E = sum_i e_i, Eq. (5)).  Ghost atoms receive their
gradient too (Eq. (7)).  The embedding-net part of the adjoint always
recomputes its activations from the first layer instead of storing them.

A handle keeps the activations of its latest forward only: a backward whose
forward has been superseded by another forward on the same handle raises.
The backward first waits for the forward and raises on the conditions the
device found there (a neighbour overflow, an out-of-range type), so a
truncated neighbour list never yields a gradient.  The coordinates are saved
with save_for_backward: an in-place change between forward and backward
(the adjoint reads them) raises torch's version-counter error.
"""

from __future__ import annotations

import torch

from .binding import Model


class DPA1AtomicEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coords, model: Model, types, box, nloc: int, nghost: int):
        if not coords.is_cuda or coords.dtype != torch.float64:
            raise TypeError("coords must be a float64 CUDA tensor [nloc + nghost, 3]")
        x = coords.detach().contiguous()
        t = types.to(device=x.device, dtype=torch.int32).contiguous()
        e_tot = torch.empty(1, dtype=torch.float64, device=x.device)
        e = torch.empty(max(nloc, 1), dtype=torch.float64, device=x.device)
        model.forward_device(x, t, box, nloc, nghost, e_tot, e)
        model._fwd_serial = getattr(model, "_fwd_serial", 0) + 1
        ctx.model = model
        ctx.serial = model._fwd_serial
        # the adjoint reads these buffers; x shares coords' version counter
        # when no copy was needed, so in-place edits of coords are caught
        ctx.save_for_backward(x, t)
        ctx.nall = x.shape[0]
        ctx.nloc = nloc
        return e[:nloc]

    @staticmethod
    def backward(ctx, grad_e):
        model = ctx.model
        if getattr(model, "_fwd_serial", None) != ctx.serial:
            raise RuntimeError("the model handle ran another forward since this one; "
                               "its activations are gone")
        x, _ = ctx.saved_tensors
        # device-side status of the forward (neighbour overflow, bad type)
        model.sync()
        grad = torch.empty((ctx.nall, 3), dtype=torch.float64, device=x.device)
        w = grad_e.detach().to(torch.float64).contiguous()
        if ctx.nloc == 0:
            w = None
        model.backward_device(grad, atom_weight=w)
        return grad, None, None, None, None, None


def atomic_energies(model: Model, coords, types, box, nloc: int, nghost: int):
    """e_i for the local atoms, differentiable with respect to coords."""
    return DPA1AtomicEnergy.apply(coords, model, types, box, nloc, nghost)
