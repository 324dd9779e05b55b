"""torch.autograd wrappers around the library's forward and backward calls.

The library returns dL/d conj(s) (the conjugate Wirtinger derivative of
Sec. 4.2); torch's gradient of a real loss with respect to a complex leaf is
twice that, so the wrappers scale by 2.
"""
import torch

from .af import Plan


class AFMagnitude(torch.autograd.Function):
    """s (packed complex64) -> a = sqrt(|chi|^2/E^2 + eps) grids (packed float32).

    Each call gets its own workspace so that spectra stored by the forward
    (store mode) belong to that call's backward.
    """

    @staticmethod
    def forward(ctx, s, plan: Plan):
        ws = plan.new_workspace()
        mag, _, _ = plan.forward(s.detach(), mag=True, ws=ws)
        ctx.plan = plan
        ctx.ws = ws
        ctx.save_for_backward(s)
        return mag

    @staticmethod
    def backward(ctx, grad_mag):
        (s,) = ctx.saved_tensors
        g = ctx.plan.backward(s.detach(), grad_mag.contiguous().to(torch.float32), ws=ctx.ws)
        return 2.0 * g, None


class AFLoss(torch.autograd.Function):
    """s -> per-waveform loss w_isl ISL + w_psl softPSL (float32[B])."""

    @staticmethod
    def forward(ctx, s, plan: Plan, w_isl=1.0, w_psl=0.0, temp=0.05, band_w=None):
        terms, g, _ = plan.loss(s.detach(), w_isl=w_isl, w_psl=w_psl, temp=temp, band_w=band_w,
                                grad=True, ws=plan.new_workspace())
        ctx.g = g
        ctx.owner = plan.owner_index(s.device)
        return terms[:, 0].clone()

    @staticmethod
    def backward(ctx, grad_loss):
        # every sample of waveform b takes that waveform's upstream
        return 2.0 * ctx.g * grad_loss[ctx.owner], None, None, None, None, None


class CrossAFMagnitude(torch.autograd.Function):
    """(s, u) (packed complex64, the same lengths) -> a = sqrt(|chi_su|^2 /
    (E_s E_u) + eps) grids of the cross-ambiguity (packed float32); the
    gradient flows to both inputs.  The backward's workspace lives only for
    the call, so the plan's own serves every call on a stream."""

    @staticmethod
    def forward(ctx, s, u, plan: Plan):
        mag, _, _ = plan.cross_forward(s.detach(), u.detach(), mag=True)
        ctx.plan = plan
        ctx.save_for_backward(s, u)
        return mag

    @staticmethod
    def backward(ctx, grad_mag):
        s, u = ctx.saved_tensors
        gs, gu = ctx.plan.cross_backward(s.detach(), u.detach(), grad_mag.contiguous().to(torch.float32))
        return 2.0 * gs, 2.0 * gu, None


def cross_af_magnitude(s, u, plan):
    return CrossAFMagnitude.apply(s, u, plan)


def af_magnitude(s, plan):
    return AFMagnitude.apply(s, plan)


def af_loss(s, plan, w_isl=1.0, w_psl=0.0, temp=0.05, band_w=None):
    """Loss per waveform with a gradient that flows to s."""
    return AFLoss.apply(s, plan, w_isl, w_psl, temp, band_w)
