"""torch.autograd.Function over the fused AF loss (the differentiable AF
module of the paper's FFT-accelerated evaluation).

Forward runs ``sqngd_af_forward`` and saves only its inputs; backward runs
``sqngd_af_backward``, which recomputes the FFT stages instead of keeping the
delay x Doppler cube. Gradients of complex inputs follow torch's convention
for real losses, dL/dRe + j dL/dIm, which is also the library's.
"""
from __future__ import annotations

import torch

from . import native as nat


class AFLoss(torch.autograd.Function):
    """loss[i] of every problem of ``batch``.

    z: float32 logits (flat, packed), h: complex64 filters (flat, packed),
    s_given: complex64 waveforms for wave_mode GIVEN, else None."""

    @staticmethod
    def forward(ctx, z, h, batch, wave_mode=nat.WAVE_SOFT, s_given=None):
        z_ = z.detach().contiguous() if z is not None else None
        h_ = h.detach().contiguous()
        s_ = s_given.detach().contiguous() if s_given is not None else None
        stats = batch.af_forward(z_, h_, wave_mode, s_given=s_)
        ctx.batch = batch
        ctx.wave_mode = wave_mode
        ctx.save_for_backward(z_, h_, s_)
        return stats.view(torch.float32)[:, 0].clone()

    @staticmethod
    def backward(ctx, grad_out):
        z, h, s = ctx.saved_tensors
        need_z = ctx.needs_input_grad[0] and ctx.wave_mode != nat.WAVE_GIVEN
        need_h = ctx.needs_input_grad[1]
        need_s = len(ctx.needs_input_grad) > 4 and ctx.needs_input_grad[4]
        gl = grad_out.detach().to(torch.float32).contiguous()
        gz, gh, gs = ctx.batch.af_backward(z, h, ctx.wave_mode, s_given=s, grad_loss=gl,
                                           want_z=need_z, want_h=need_h, want_s=need_s)
        return gz, gh, None, None, gs


def af_loss(z, h, batch, wave_mode=nat.WAVE_SOFT, s_given=None):
    """Per-problem loss tensor [nprob] with gradients to z, h (and s_given)."""
    return AFLoss.apply(z, h, batch, wave_mode, s_given)
