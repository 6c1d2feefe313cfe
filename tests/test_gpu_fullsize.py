"""Parity at the full workload sizes, in the launch configuration bench.py
times: whole-system checks where the oracle can afford them (2048 clusters),
seeded samples of rows, descriptors and forces otherwise (32768 and 262144
atoms), and properties that hold at any size."""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL, descriptor_errors, list_rows_equal, oracle_sampled_forces

pytestmark = pytest.mark.gpu

_w = {}


def workload(i):
    if i not in _w:
        _w[i] = synth.config(i)
    return _w[i]


def test_batched_clusters_full():
    """2048 clusters of 5-60 atoms in one launch per stage: lists, energies,
    forces (FP32 and split BF16) and the energy-loss weight gradient against
    the oracle on the whole batch."""
    w = workload(2)
    s, p = w.system, w.params
    print(f"[full] {w.name}: {s.n_atoms} atoms", flush=True)
    ref_nl = oracle.neighbors_brute(s, p.rc)
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    got = pot.neighbor_list_host()
    ok, msg = list_rows_equal(got, ref_nl)
    assert ok, msg
    Es_ref, Ea_ref, F_ref = oracle.energy_forces(p, w.model, s, ref_nl)
    n_c = np.diff(s.atom_ptr)
    for flags in (0, nnpot.NN_BF16X3_MLP):
        Es, Ea, F = [t.cpu().numpy().copy() for t in pot.energy_forces(flags=flags)]
        e_err = np.max(np.abs(Es - Es_ref) / n_c)
        f_err = np.abs(F - F_ref).max()
        print(f"  flags={flags}: E/atom {e_err:.2e}  F {f_err:.2e}", flush=True)
        assert e_err <= E_TOL and f_err <= F_TOL
    T = synth.energy_targets(w.seed, s.n_structs)
    _, Es_o, flat = oracle.energy_loss_grad(p, w.model, s, ref_nl, T)
    ref = oracle.unflatten_grads(w.model, flat)
    pot.energy_forces(flags=0)
    _, g = pot.grad(2.0 * (Es_o - T) / s.n_structs, positions=False)
    nnpot.nn_check(pot.nl)
    worst = max(np.abs(gg.double().cpu().numpy().reshape(rr.shape) - rr).max() / max(np.abs(rr).max(), 1e-12)
                for sp in range(len(ref)) for pr, pg in zip(ref[sp], g[sp]) for rr, gg in zip(pr, pg))
    print(f"  weight gradient max rel {worst:.2e}", flush=True)
    assert worst <= 1e-4


@pytest.mark.parametrize("cfg", [3, 4])
def test_bulk_full_size_sampled(cfg):
    w = workload(cfg)
    s, p = w.system, w.params
    skin = float(w.extra.get("skin", 0.0))
    print(f"[full] {w.name}: {s.n_atoms} atoms, skin {skin}", flush=True)
    pot = nnpot.Potential(s, p, w.model, skin=skin)
    pot.build_neighbors()
    rng = np.random.Generator(np.random.PCG64(100 + cfg))
    rows = np.sort(rng.choice(s.n_atoms, size=256, replace=False))
    # list rows at the build radius (rc + skin) are identical
    got = pot.neighbor_list_host()
    ref_rows = oracle.neighbors_cells(s, p.rc + skin, rows=rows)
    ok, msg = list_rows_equal(got, ref_rows, rows=rows)
    assert ok, msg
    # descriptors of the sampled atoms
    G = pot.descriptors().cpu().numpy()
    G_ref = oracle.descriptors(p, s, oracle.neighbors_cells(s, p.rc, rows=rows))
    err = descriptor_errors(G[rows], G_ref)
    print(f"  descriptors: max |dG|/tol {err:.3f}", flush=True)
    assert err <= 1.0
    # forces of 32 sampled atoms, FP32 and split BF16; energies of their rows
    t = rows[:32]
    row_ids, E_rows, F_ref = oracle_sampled_forces(w, t)
    for flags in (0, nnpot.NN_BF16X3_MLP):
        _, Ea, F = [x.cpu().numpy().copy() for x in pot.energy_forces(flags=flags)]
        f_err = np.abs(F[t] - F_ref).max()
        e_err = np.abs(Ea[row_ids] - E_rows).max()
        print(f"  flags={flags}: F {f_err:.2e}  E_atom {e_err:.2e}", flush=True)
        assert f_err <= F_TOL and e_err <= E_TOL
        Fd = F.astype(np.float64)
        assert np.abs(Fd.sum(0)).max() <= 1e-6 * np.abs(Fd).max() * s.n_atoms
    nnpot.nn_check(pot.nl)
