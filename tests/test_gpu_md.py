"""Repeated evaluation with a skinned neighbor list (random-walk MD shape of
the 262144-atom workload, cut to 16384 atoms) and HIP graph capture."""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import F_TOL, oracle_sampled_forces

pytestmark = pytest.mark.gpu


def md_workload(scale=1 / 16):
    w = synth.config(4, scale=scale)
    return w, w.extra["skin"], w.extra["step_sigma"]


def test_skin_rebuild_rule_and_fresh_list_equivalence():
    import torch
    w, skin, sigma = md_workload()
    s, p = w.system, w.params
    skinned = nnpot.Potential(s, p, w.model, skin=skin, capacity_margin=1.6)
    fresh = nnpot.Potential(s, p, w.model, skin=0.0, capacity_margin=1.6)
    pos = s.pos.copy()
    ref = None
    n_rebuild = 0
    steps = 30
    for k, xi in enumerate(synth.md_displacements(w.seed, s.n_atoms, steps, sigma)):
        if k:
            pos = pos + xi
        skinned.set_positions(pos)
        fresh.set_positions(pos)
        skinned.build_neighbors()
        fresh.build_neighbors()
        rebuilt = int(skinned.meta[3].item())
        # host rule: rebuild when some atom moved more than skin/2 since the last build
        if ref is None:
            expect = 1
        else:
            d = pos - ref
            d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            expect = int(np.any(~(d2 <= (0.5 * skin) ** 2)))
        assert rebuilt == expect, (k, rebuilt, expect)
        if rebuilt:
            ref = pos.copy()
            n_rebuild += 1
        Es, Ea, Fs = [t.cpu().numpy().copy() for t in skinned.energy_forces()]
        Ef, Eaf, Ff = [t.cpu().numpy().copy() for t in fresh.energy_forces()]
        # same staged neighbor sequence: identical energies; forces equal up to
        # the order of the per-row gather (the skinned rows hold extra zeros)
        assert np.array_equal(Ea, Eaf) and np.array_equal(Es, Ef)
        assert np.abs(Fs - Ff).max() <= 1e-5 * np.abs(Ff).max()
        if k in (0, steps - 1):
            t = np.random.Generator(np.random.PCG64(k)).choice(s.n_atoms, 16, replace=False)
            wk = synth.Workload(w.name, synth.System(pos, s.species, s.atom_ptr, s.cell, s.pbc), p, w.model, w.seed)
            _, _, F_ref = oracle_sampled_forces(wk, t)
            assert np.abs(Fs[t] - F_ref).max() <= F_TOL
    nnpot.nn_check(skinned.nl)
    print(f"rebuilds: {n_rebuild} in {steps} steps", flush=True)
    assert 1 < n_rebuild < steps


@pytest.mark.parametrize("flags", [0, nnpot.NN_BF16X3_MLP])
def test_graph_replay_matches_eager(flags):
    """One MD step (skinned list build + energies + forces) captured in a HIP
    graph; replays with fresh positions, with eager work and synchronizations
    between them, must equal an eager Potential bitwise."""
    import torch
    w, skin, sigma = md_workload(scale=1 / 32)
    s, p = w.system, w.params
    g_pot = nnpot.Potential(s, p, w.model, skin=skin, capacity_margin=1.6, flags=flags)
    e_pot = nnpot.Potential(s, p, w.model, skin=skin, capacity_margin=1.6, flags=flags)
    # warm up (first build) outside the graph
    g_pot.build_neighbors()
    g_pot.energy_forces()
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        nnpot.nn_build_neighbors(g_pot.sys, g_pot.rc, g_pot.skin, g_pot.nl, g_pot.ws)
        nnpot.nn_energy_forces(g_pot.sys, g_pot.nl, g_pot.params, g_pot.dmodel.struct, flags, 0, g_pot.E_struct,
                               g_pot.E_atom, g_pot.F, g_pot.ws)
    torch.cuda.synchronize()
    pos = s.pos.copy()
    e_pot.build_neighbors()
    for k, xi in enumerate(synth.md_displacements(w.seed, s.n_atoms, 12, sigma)):
        pos = pos + xi
        g_pot.set_positions(pos)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        e_pot.set_positions(pos)
        e_pot.build_neighbors(check=False)
        e_pot.energy_forces()
        torch.cuda.synchronize()
        for a, b in ((g_pot.E_struct, e_pot.E_struct), (g_pot.F, e_pot.F), (g_pot.meta[:4], e_pot.meta[:4])):
            assert torch.equal(a, b), k
    nnpot.nn_check(g_pot.nl)
