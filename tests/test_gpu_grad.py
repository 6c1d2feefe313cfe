"""Gradients through the C ABI: autograd.Function vs forces, central finite
differences of the GPU energy, and the weight gradient of the energy loss
against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

pytestmark = pytest.mark.gpu


def test_autograd_position_gradient_is_minus_forces():
    import torch
    from paper_2305_11805_amd.autograd import energy
    w = synth.config(1, scale=0.25)
    pot = nnpot.Potential(w.system, w.params, w.model)
    pos = pot.pos.clone().requires_grad_(True)
    E = energy(pot, pos)
    E.sum().backward()
    F = pot.F.double()
    assert torch.equal(pos.grad, -F)


def test_forces_match_finite_differences_bulk4096():
    """4th-order central differences, h = 1e-2 A, of the GPU energy (FP32
    atomic energies summed in FP64; only atoms within reach of the moved
    atom change, bitwise, between evaluations) on 32 seeded atoms."""
    import torch
    w = synth.config(1)
    pot = nnpot.Potential(w.system, w.params, w.model)
    pot.build_neighbors()
    _, _, F = pot.energy_forces()
    F = F.double().cpu().numpy()
    base = w.system.pos.copy()
    rng = np.random.Generator(np.random.PCG64(2024))
    atoms = rng.choice(w.system.n_atoms, size=32, replace=False)
    h = 1e-2

    def E_at(k, a, dx):
        p = base.copy()
        p[k, a] += dx
        pot.set_positions(p)
        pot.build_neighbors(check=False)
        E, _, _ = pot.energy_forces(forces=False)
        return float(E.sum().item())

    worst = 0.0
    for k in atoms:
        for a in range(3):
            fd = -(-E_at(k, a, 2 * h) + 8 * E_at(k, a, h) - 8 * E_at(k, a, -h) + E_at(k, a, -2 * h)) / (12 * h)
            worst = max(worst, abs(fd - F[k, a]))
    pot.set_positions(base)
    print(f"max |F_fd - F| = {worst:.2e} eV/A", flush=True)
    assert worst <= 1e-3


@pytest.mark.parametrize("cfg,scale,flags", [(0, 1.0, 0), (2, 0.03, 0), (2, 0.03, nnpot.NN_BF16X3_MLP),
                                             (3, 0.05, 0)])
def test_weight_gradient_matches_oracle(cfg, scale, flags):
    w = synth.config(cfg, scale=scale)
    s, p = w.system, w.params
    T = synth.energy_targets(w.seed, s.n_structs)
    nl = oracle.neighbors_cells(s, p.rc)
    L_ref, Es_ref, flat = oracle.energy_loss_grad(p, w.model, s, nl, T)
    ref = oracle.unflatten_grads(w.model, flat)
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    pot.energy_forces(flags=flags)
    dL_dE = 2.0 * (Es_ref - T) / s.n_structs
    _, got = pot.grad(dL_dE, flags=flags, positions=False)
    nnpot.nn_check(pot.nl)
    worst = 0.0
    for sp in range(len(ref)):
        for (dW_r, db_r), (dW_g, db_g) in zip(ref[sp], got[sp]):
            for r_, g_ in ((dW_r, dW_g), (db_r, db_g)):
                g_ = g_.double().cpu().numpy().reshape(r_.shape)
                scale_ = max(np.abs(r_).max(), 1e-12)
                worst = max(worst, np.abs(g_ - r_).max() / scale_)
    print(f"cfg{cfg} flags={flags}: max |d dW| / max |dW| = {worst:.2e}", flush=True)
    assert worst <= 1e-4


def test_weight_gradient_deterministic():
    w = synth.config(2, scale=0.03)
    pot = nnpot.Potential(w.system, w.params, w.model)
    pot.build_neighbors()
    pot.energy_forces()
    g = np.linspace(-1, 1, w.system.n_structs)
    outs = []
    for _ in range(2):
        _, got = pot.grad(g, positions=False)
        outs.append([t.cpu().numpy().copy() for layers in got for pair in layers for t in pair])
    for a, b in zip(*outs):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
