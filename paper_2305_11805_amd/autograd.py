"""torch.autograd.Function over libnnpot.

Forward: (neighbor list kept or rebuilt under the skin rule) -> descriptors
-> per-species MLP -> per-structure energies, with forces from the
hand-written adjoint.  Backward: dL/dpos = -dL/dE_c F_k and dL/dW, dL/db from
nn_energy_forces_grad (Sec. II.A: the loss is minimised over the MLP
parameters with forces as derivatives of the energy).  energy_forces() also
returns the forces as an output, so a loss on forces (force matching) reaches
the weights; its position gradient (a Hessian product) is not provided.  All
compute runs in the HIP library; this module only passes tensors.
"""
from __future__ import annotations

import torch

from . import nnpot


def _check_current(ctx):
    """The backward pass reads the Potential's list, descriptors and forces:
    refuse it if another evaluation replaced them after this forward."""
    if ctx.pot.evals != ctx.token:
        raise RuntimeError("the Potential was evaluated again after this forward pass; run backward before the "
                           "next evaluation on the same Potential (or use one Potential per graph)")


def _weight_grads(wg, n):
    if wg is None:
        return [None] * n
    gw = []
    for layers in wg:
        for dW, db in layers:
            gw += [dW, db]
    return gw


class NNPotFn(torch.autograd.Function):
    """E_struct [B] (float64) = f(pos [N,3] float64, *weights) for a Potential.

    The weights must be the Potential's own device tensors (pot.dmodel.tensors,
    species-major, W then b per layer): the library reads them by address.
    A Potential holds the forces of its last forward, so backward must run
    before the next evaluation on the same Potential; it raises otherwise."""

    @staticmethod
    def forward(ctx, pos, pot, flags, *weights):
        pot.pos.copy_(pos.detach())
        pot.build_neighbors(check=False)
        E, _, _ = pot.energy_forces(flags=flags)
        ctx.pot, ctx.flags, ctx.token = pot, flags, pot.evals
        return E.clone()

    @staticmethod
    def backward(ctx, gE):
        _check_current(ctx)
        pot = ctx.pot
        need_pos = ctx.needs_input_grad[0]
        need_w = any(ctx.needs_input_grad[3:])
        dpos, wg = pot.grad(gE.detach().to(torch.float64).contiguous(), flags=ctx.flags, positions=need_pos,
                            weights=need_w)
        gw = _weight_grads(wg if need_w else None, len(ctx.needs_input_grad) - 3)
        return (dpos.to(torch.float64) if need_pos else None, None, None, *gw)


class NNPotEFFn(torch.autograd.Function):
    """(E_struct [B] float64, F [N,3] float32) = f(pos, *weights).

    Backward takes dL/dE and dL/dF: the weight gradient includes the force
    term; positions get -dL/dE_c F_k when dL/dF is absent or zero, and a
    request for the position gradient of a nonzero dL/dF raises."""

    @staticmethod
    def forward(ctx, pos, pot, flags, *weights):
        pot.pos.copy_(pos.detach())
        pot.build_neighbors(check=False)
        E, _, F = pot.energy_forces(flags=flags)
        ctx.pot, ctx.flags, ctx.token = pot, flags, pot.evals
        return E.clone(), F.clone()

    @staticmethod
    def backward(ctx, gE, gF):
        _check_current(ctx)
        pot = ctx.pot
        need_pos = ctx.needs_input_grad[0]
        need_w = any(ctx.needs_input_grad[3:])
        if gF is not None and not bool(torch.any(gF != 0)):
            gF = None
        if need_pos and gF is not None:
            raise RuntimeError("the position gradient of a loss on forces is not provided")
        if gE is None:
            gE = torch.zeros(pot.sys.n_structs, dtype=torch.float64, device=pot.dev)
        dL_dE = gE.detach().to(torch.float64).contiguous()
        dL_dF = None if gF is None else gF.detach().to(torch.float32).contiguous()
        dpos, wg = pot.grad(dL_dE, flags=ctx.flags, positions=need_pos, weights=need_w, dL_dF=dL_dF)
        gw = _weight_grads(wg if need_w else None, len(ctx.needs_input_grad) - 3)
        return (dpos.to(torch.float64) if need_pos else None, None, None, *gw)


def energy(pot: "nnpot.Potential", pos: torch.Tensor, flags: int = 0) -> torch.Tensor:
    """Per-structure energies with autograd through positions and weights."""
    return NNPotFn.apply(pos, pot, flags, *pot.dmodel.tensors)


def energy_forces(pot: "nnpot.Potential", pos: torch.Tensor, flags: int = 0):
    """(E_struct, F) with autograd through the weights for losses on both
    (force matching), and through positions for a loss on energies."""
    return NNPotEFFn.apply(pos, pot, flags, *pot.dmodel.tensors)
