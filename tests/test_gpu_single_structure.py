"""Neighbor lists of a single structure.  Up to 4096 atoms, one structure
takes the single-block binning launch (geometry, bin counts, bin starts and
the bin-ordered copy in one block); larger ones and batches take the
per-structure passes.  Both sides of that limit, a dilute triclinic cell
whose bins are merged, an open molecule, a small periodic cell with lattice
images and unwrapped positions must give the oracle's list entry for entry,
with a consistent reverse index.  Bad inputs of a single structure (a
non-finite position, an atom pointer array that does not end at N) are
reported by nn_check.  Structures of no, one and two atoms give the oracle's
(empty or one-pair) list, energy and forces."""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL, list_rows_equal

pytestmark = pytest.mark.gpu

ONE_BLOCK_ATOMS = 4096
RC = 4.6


def uniform_cell(n, rho, seed, tric=False, unwrap=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    L = (n / rho) ** (1.0 / 3.0)
    cell = np.array([[L, 0, 0], [0.31 * L, 0.95 * L, 0], [-0.2 * L, 0.17 * L, 1.05 * L]]) if tric else np.eye(3) * L
    pos = rng.uniform(0, 1, (n, 3)) @ cell
    if unwrap:
        pos = pos + rng.integers(-1, 2, (n, 3)) @ cell  # some atoms one whole cell away
    return synth.single(pos, rng.integers(0, 2, n), cell=cell, pbc=(1, 1, 1))


def open_molecule(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.standard_normal((n, 3))
    pos = d / np.linalg.norm(d, axis=1, keepdims=True) * (rng.uniform(0, 1, (n, 1)) ** (1 / 3) * 12.0)
    return synth.single(pos + 3.0, rng.integers(0, 2, n))


CASES = {
    "bulk_at_limit": lambda: uniform_cell(ONE_BLOCK_ATOMS, 0.08, 1201),
    "bulk_over_limit": lambda: uniform_cell(ONE_BLOCK_ATOMS + 1, 0.08, 1202),
    "dilute_triclinic": lambda: uniform_cell(300, 0.0003, 1203, tric=True),
    "open_molecule": lambda: open_molecule(1000, 1204),
    "small_cell_images": lambda: uniform_cell(40, 0.09, 1205, tric=True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_single_structure_list_matches_oracle(name):
    s = CASES[name]()
    p = synth.mbp_params(2, RC, 8, 4, 4)
    ref = oracle.neighbors_cells(s, p.rc)
    rows = np.diff(ref["offsets"])
    print(f"[single structure] {name}: {s.n_atoms} atoms, {int(ref['offsets'][-1])} entries, "
          f"rows max {rows.max()}", flush=True)
    pot = nnpot.Potential(s, p, None)
    pot.build_neighbors()
    got = pot.neighbor_list_host()
    assert np.array_equal(got["offsets"], ref["offsets"])
    ok, msg = list_rows_equal(got, ref)
    assert ok, msg
    off = got["offsets"]
    row_of = np.repeat(np.arange(len(off) - 1), np.diff(off))
    assert np.array_equal(got["nbr"][got["rev"]], row_of)
    assert np.array_equal(got["shift"][got["rev"]], -got["shift"])
    # a second build on the same buffers gives the same list
    pot.build_neighbors()
    again = pot.neighbor_list_host()
    for k in ("offsets", "nbr", "shift", "rev"):
        assert np.array_equal(again[k], got[k]), k


@pytest.mark.parametrize("n", [ONE_BLOCK_ATOMS, ONE_BLOCK_ATOMS + 1])
def test_single_structure_non_finite_position_is_reported(n):
    s = uniform_cell(n, 0.08, 1206)
    p = synth.mbp_params(2, RC, 8, 4, 4)
    pot = nnpot.Potential(s, p, None)
    pot.build_neighbors()
    pos = s.pos.copy()
    pos[7, 1] = np.nan
    pot.set_positions(pos)
    print(f"[single structure] non-finite position, {n} atoms", flush=True)
    pot.build_neighbors(check=False)
    with pytest.raises(nnpot.NNError, match="non-finite"):
        nnpot.nn_check(pot.nl)
    with pytest.raises(nnpot.NNError, match="neighbor count failed"):  # the counting pass too
        nnpot.nn_count_neighbors(pot.sys, pot.rc, pot.ws)


@pytest.mark.parametrize("skin", [0.0, 0.3])
def test_single_structure_bad_atom_ptr_is_reported(skin):
    import torch
    s = uniform_cell(500, 0.08, 1207)
    p = synth.mbp_params(2, RC, 8, 4, 4)
    pot = nnpot.Potential(s, p, None, skin=skin)
    pot.build_neighbors()
    good = pot.neighbor_list_host()
    ptr = pot.atom_ptr.clone()
    pot.atom_ptr[1] = s.n_atoms - 1  # does not end at N
    pot.set_positions(s.pos + 0.2)  # a skin list must rebuild too
    print(f"[single structure] atom_ptr ending at N - 1, skin {skin}", flush=True)
    pot.build_neighbors(check=False)
    torch.cuda.synchronize()
    with pytest.raises(nnpot.NNError, match="atom_ptr"):
        nnpot.nn_check(pot.nl)
    pot.atom_ptr.copy_(ptr)
    pot.set_positions(s.pos)
    pot.build_neighbors()
    again = pot.neighbor_list_host()
    for k in ("offsets", "nbr", "shift", "rev"):
        assert np.array_equal(again[k], good[k]), k


@pytest.mark.parametrize("n", [0, 1, 2])
def test_tiny_single_structure_energy_forces_match_oracle(n):
    """No atoms, one isolated atom (energy of a zero descriptor) and a pair:
    the single-block binning launch, an empty list and the energy sums."""
    rng = np.random.Generator(np.random.PCG64(40 + n))
    s = synth.single(rng.uniform(0, 3, (n, 3)), rng.integers(0, 2, n))
    p = synth.mbp_params(2, RC, 8, 4, 4)
    model = synth.random_model(2, p.dim, [64, 32], 7, in_scale=2.0)
    ref = oracle.neighbors_cells(s, p.rc)
    Es_ref, _, F_ref = oracle.energy_forces(p, model, s, ref)
    print(f"[single structure] {n} atoms", flush=True)
    pot = nnpot.Potential(s, p, model)
    pot.build_neighbors()
    got = pot.neighbor_list_host()
    assert np.array_equal(got["offsets"], ref["offsets"])
    ok, msg = list_rows_equal(got, ref)
    assert ok, msg
    Es, _, F = pot.energy_forces()
    nnpot.nn_check(pot.nl)
    assert abs(float(Es.cpu().numpy()[0]) - Es_ref[0]) <= E_TOL * max(n, 1)
    if n:
        assert float(np.abs(F.cpu().numpy() - F_ref).max()) <= F_TOL
