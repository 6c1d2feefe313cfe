"""torch.autograd.Function over libnnpot.

Forward: (neighbor list kept or rebuilt under the skin rule) -> descriptors
-> per-species MLP -> per-structure energies, with forces from the
hand-written adjoint.  Backward: dL/dpos = -dL/dE_c F_k and dL/dW, dL/db from
nn_energy_forces_grad (Sec. II.A: the loss is minimised over the MLP
parameters with forces as derivatives of the energy).  All compute runs in
the HIP library; this module only passes tensors.
"""
from __future__ import annotations

import torch

from . import nnpot


class NNPotFn(torch.autograd.Function):
    """E_struct [B] (float64) = f(pos [N,3] float64, *weights) for a Potential.

    The weights must be the Potential's own device tensors (pot.dmodel.tensors,
    species-major, W then b per layer): the library reads them by address.
    A Potential holds the forces of its last forward, so run backward before
    the next forward on the same Potential."""

    @staticmethod
    def forward(ctx, pos, pot, flags, *weights):
        pot.pos.copy_(pos.detach())
        nnpot.nn_build_neighbors(pot.sys, pot.rc, pot.skin, pot.nl, pot.ws)
        E, _, _ = pot.energy_forces(flags=flags)
        ctx.pot, ctx.flags = pot, flags
        return E.clone()

    @staticmethod
    def backward(ctx, gE):
        pot = ctx.pot
        need_pos = ctx.needs_input_grad[0]
        need_w = any(ctx.needs_input_grad[3:])
        dpos, wg = pot.grad(gE.detach().to(torch.float64).contiguous(), flags=ctx.flags, positions=need_pos,
                            weights=need_w)
        gw = []
        if need_w:
            for layers in wg:
                for dW, db in layers:
                    gw += [dW, db]
        else:
            gw = [None] * (len(ctx.needs_input_grad) - 3)
        return (dpos.to(torch.float64) if need_pos else None, None, None, *gw)


def energy(pot: "nnpot.Potential", pos: torch.Tensor, flags: int = 0) -> torch.Tensor:
    """Per-structure energies with autograd through positions and weights."""
    return NNPotFn.apply(pos, pot, flags, *pot.dmodel.tensors)
