"""Differentiable warp + energy step.

WarpEnergy.apply(I_a, u, I_b, lam, levels) returns, per batch item, the energy
sum_l [ SSD(I_a^l(x + u^l(x)), I_b^l) + lam |grad u^l|^2 ] over a pyramid of
``levels`` levels (2x2 block means of the images, half block means of u).
Forward and backward are the library's kernels: the backward recomputes the
pyramid instead of storing it and applies the scatter-add transpose of the
bilinear gather for dE/dI_a.  float32 tensors use the float32 kernels,
float64 tensors the float64 instantiations (for gradcheck).
"""
from __future__ import annotations

import torch

from . import api


class WarpEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Ia, u, Ib, lam=0.1, levels=1):
        Ia, u, Ib = Ia.contiguous(), u.contiguous(), Ib.contiguous()
        ctx.save_for_backward(Ia, u, Ib)
        ctx.lam = float(lam)
        ctx.levels = int(levels)
        return api.pyramid_energy(Ia, u, Ib, lam, levels)

    @staticmethod
    def backward(ctx, gE):
        Ia, u, Ib = ctx.saved_tensors
        need = ctx.needs_input_grad[:3]
        dIa, du, dIb = api.pyramid_energy_backward(
            Ia, u, Ib, ctx.lam, ctx.levels, gE.contiguous().to(torch.float64), need)
        return dIa, du, dIb, None, None


def warp_energy(Ia, u, Ib, lam=0.1, levels=1):
    return WarpEnergy.apply(Ia, u, Ib, lam, levels)
