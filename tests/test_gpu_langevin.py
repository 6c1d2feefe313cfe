"""Langevin dynamics through nn_md_langevin against the FP64 oracle's BAOAB
integrator on the same seeded velocities and noise.

Trajectory bar: an error of at most F_TOL (the per-evaluation force bar) in
every force of every step moves a velocity by at most dt a F_TOL per step
(a = ACCEL / m) and a position by the sum of those; over n steps
    |dv| <= n dt a F_TOL,   |dx| <= n^2 dt^2 a F_TOL / 2
as long as the trajectories have not separated (a few fs here, far below the
time on which nearby trajectories diverge)."""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import F_TOL

pytestmark = pytest.mark.gpu


def mixed_batch():
    rng = np.random.Generator(np.random.PCG64(33))
    p = synth.mbp_params(2, 4.0, 16, 8, 4)
    systems = []
    for L, n in [(3.5, 6), (5.5, 20)]:
        cell = np.array([[L, 0, 0], [0.3, L * 0.97, 0], [-0.2, 0.4, L * 1.03]])
        systems.append(synth.single(rng.uniform(0, 1, (n, 3)) @ cell, rng.integers(0, 2, n), cell=cell,
                                    pbc=(1, 1, 1)))
    cl = synth.clusters_system(rng, [9, 13], lambda n: 5.0, 0.9, 2)
    model = synth.random_model(2, p.dim, [64, 32], 9, in_scale=3.0)
    return synth.Workload("small periodic cells + clusters", synth.concat(systems + [cl]), p, model, 33)


def run_both(w, masses, steps, dt, friction, kT, skin=0.0, v_sigma=0.005, seed=1):
    import torch
    s, p = w.system, w.params
    inv_m = 1.0 / np.asarray(masses, np.float64)
    v0, noise = synth.md_inputs(seed, s.n_atoms, steps, v_sigma)
    x_r, v_r, F_r, E_r = oracle.md_langevin(p, w.model, s, v0, inv_m, dt, friction, kT, noise, steps)
    pot = nnpot.Potential(s, p, w.model, skin=skin)
    pot.build_neighbors()
    pot.energy_forces()
    dev = pot.dev
    vel = torch.tensor(v0, dtype=torch.float64, device=dev)
    im = torch.tensor(inv_m, dtype=torch.float64, device=dev)
    xi = torch.tensor(noise, device=dev)
    E = pot.md_langevin(steps, vel, im, dt, friction, kT, noise=xi)
    nnpot.nn_check(pot.nl)
    got = (pot.pos.cpu().numpy(), vel.cpu().numpy(), pot.F.double().cpu().numpy(), E.cpu().numpy())
    return got, (x_r, v_r, F_r, E_r), inv_m, pot


def check_trajectory(got, ref, inv_m, steps, dt, n_atoms_struct):
    (x, v, F, E), (x_r, v_r, F_r, E_r) = got, ref
    a = oracle.ACCEL * inv_m.max()
    dv_bar = steps * dt * a * F_TOL
    dx_bar = 0.5 * steps * steps * dt * dt * a * F_TOL
    dx, dv = np.abs(x - x_r).max(), np.abs(v - v_r).max()
    dF = np.abs(F - F_r).max()
    dE = np.max(np.abs(E - E_r) / np.maximum(n_atoms_struct, 1))
    print(f"  |dx| {dx:.2e} (bar {dx_bar:.1e})  |dv| {dv:.2e} (bar {dv_bar:.1e})  "
          f"|dF| {dF:.2e}  |dE|/atom {dE:.2e}", flush=True)
    assert dx <= dx_bar and dv <= dv_bar
    assert dF <= F_TOL and dE <= 1e-4


def test_langevin_small_cells_and_clusters_match_oracle():
    w = mixed_batch()
    masses = np.asarray([12.011, 1.008])[w.system.species]
    steps, dt = 20, 0.5
    print(f"[langevin] {w.name}: {w.system.n_atoms} atoms, {steps} steps", flush=True)
    got, ref, inv_m, _ = run_both(w, masses, steps, dt, 0.02, 0.02585)
    check_trajectory(got, ref, inv_m, steps, dt, np.diff(w.system.atom_ptr))


def test_langevin_bulk_with_skin_rebuilds_matches_oracle():
    """1024-atom periodic bulk, skin 0.5 A and fast atoms, so the list is
    rebuilt on the device during the run; the oracle builds a fresh list at
    rc every step."""
    w = synth.config(1, scale=0.25)
    n = w.system.n_atoms
    steps, dt = 6, 1.0
    print(f"[langevin] {w.name}, skin 0.5, {steps} steps", flush=True)
    got, ref, inv_m, pot = run_both(w, np.full(n, synth.CARBON_MASS), steps, dt, 0.01, 0.02585, skin=0.5,
                                    v_sigma=0.05)
    builds = int(pot.meta[2].item())
    print(f"  list builds: {builds}", flush=True)
    assert builds >= 2
    check_trajectory(got, ref, inv_m, steps, dt, np.array([n]))


def test_langevin_graph_replay_equals_eager_bitwise():
    import torch
    w = synth.md_cells(4)
    s = w.system
    steps = 10
    v0, noise = synth.md_inputs(2, s.n_atoms, steps, 0.005)
    pot = nnpot.Potential(s, w.params, w.model, skin=1.0)
    pot.build_neighbors()
    pot.energy_forces()
    x0, F0 = pot.pos.clone(), pot.F.clone()
    vel = torch.tensor(v0, dtype=torch.float64, device=pot.dev)
    im = torch.full((s.n_atoms,), 1.0 / synth.CARBON_MASS, dtype=torch.float64, device=pot.dev)
    xi = torch.tensor(noise, device=pot.dev)
    E = torch.empty((steps, s.n_structs), dtype=torch.float64, device=pot.dev)
    pot.md_langevin(steps, vel, im, 0.5, 0.01, 0.02585, noise=xi, E_pot=E)
    torch.cuda.synchronize()
    eager = [t.clone() for t in (pot.pos, vel, pot.F, E)]

    def reset():
        pot.pos.copy_(x0)
        vel.copy_(torch.tensor(v0, dtype=torch.float64, device=pot.dev))
        pot.F.copy_(F0)
        pot.build_neighbors()  # the list of the start positions
        torch.cuda.synchronize()
    reset()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        pot.md_langevin(steps, vel, im, 0.5, 0.01, 0.02585, noise=xi, E_pot=E)
    for rep in range(3):
        reset()
        g.replay()
        torch.cuda.synchronize()
        nnpot.nn_check(pot.nl)
        for a, b in zip(eager, (pot.pos, vel, pot.F, E)):
            assert torch.equal(a, b), f"replay {rep} differs"


def test_constant_energy_16_atom_cell():
    """Without friction (velocity Verlet) over 200 steps of 0.5 fs on the
    16-atom cell: the GPU's E_pot + E_kin stays within twice the oracle's own
    largest deviation (the O(dt^2) oscillation of the integrator) plus 1e-4 eV."""
    import torch
    w = synth.md_cells(1)
    s = w.system
    steps, dt = 200, 0.5
    inv_m = np.full(s.n_atoms, 1.0 / synth.CARBON_MASS)
    v0, _ = synth.md_inputs(3, s.n_atoms, 1, 0.005)

    def ke(v):
        return 0.5 * np.sum(np.sum(v * v, axis=1) / inv_m) / oracle.ACCEL

    # oracle path, one step at a time for the kinetic energy along the way
    E0, _, _ = oracle.energy_forces(w.params, w.model, s, oracle.neighbors_cells(s, w.params.rc))
    Et0 = E0.sum() + ke(v0)
    cur, v, dev_ref = s, v0, 0.0
    for _ in range(steps):
        x, v, _, E = oracle.md_langevin(w.params, w.model, cur, v, inv_m, dt, 0.0, 0.0, None, 1)
        cur = synth.System(x, s.species, s.atom_ptr, s.cell, s.pbc)
        dev_ref = max(dev_ref, abs(E.sum() + ke(v) - Et0))
    pot = nnpot.Potential(s, w.params, w.model, skin=1.0)
    pot.build_neighbors()
    pot.energy_forces()
    vel = torch.tensor(v0, dtype=torch.float64, device=pot.dev)
    im = torch.tensor(inv_m, dtype=torch.float64, device=pot.dev)
    dev_gpu = 0.0
    Eg0 = float(pot.E_struct.sum().item()) + ke(v0)
    E = torch.empty((1, s.n_structs), dtype=torch.float64, device=pot.dev)
    for _ in range(steps):
        pot.md_langevin(1, vel, im, dt, 0.0, 0.0, E_pot=E)
        dev_gpu = max(dev_gpu, abs(float(E.sum().item()) + ke(vel.cpu().numpy()) - Eg0))
    nnpot.nn_check(pot.nl)
    print(f"  max |dE_tot|: gpu {dev_gpu:.2e} eV, oracle {dev_ref:.2e} eV", flush=True)
    assert dev_gpu <= 2 * dev_ref + 1e-4


@pytest.mark.parametrize("network", ["small", "middle", "big"])
def test_langevin_table2_networks_match_oracle(network):
    """The like-for-like Table II shape: 16-atom periodic carbon cells (four of
    them batched) with the Carbon descriptor of Sec. III.B (D = 152) and each
    Table II network, 300 K, 0.5 fs, skin 1 A (the bench's setting)."""
    w = synth.md_cells(4, network=network)
    masses = np.full(w.system.n_atoms, synth.CARBON_MASS)
    steps, dt = 20, 0.5
    print(f"[langevin] {w.name}: {w.system.n_atoms} atoms, {steps} steps", flush=True)
    got, ref, inv_m, _ = run_both(w, masses, steps, dt, 0.01, 0.025852, skin=1.0)
    check_trajectory(got, ref, inv_m, steps, dt, np.diff(w.system.atom_ptr))
