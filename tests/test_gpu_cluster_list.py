"""The cluster list passes (batches whose structures all have at most 64
atoms and no periodic direction) against the FP64 oracle's lists, entry for
entry, with the reverse index; batches that need the generic passes (a
65-atom structure, a periodic cell) fall back to them for the whole list.
Also: the counting call, non-finite positions, the skin rule, and
repeatability.
"""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import list_rows_equal

pytestmark = pytest.mark.gpu


def check_list(pot, s, radius):
    ref = oracle.neighbors_cells(s, radius)
    got = pot.neighbor_list_host()
    assert np.array_equal(got["offsets"], ref["offsets"])
    ok, why = list_rows_equal(got, ref)
    assert ok, why
    off = got["offsets"]
    row_of = np.repeat(np.arange(len(off) - 1), np.diff(off))
    assert np.array_equal(got["nbr"][got["rev"]], row_of)
    assert np.array_equal(got["shift"][got["rev"]], -got["shift"])
    assert np.array_equal(got["rev"][got["rev"]], np.arange(off[-1]))
    return got


def clusters(seed, sizes, n_species=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.clusters_system(rng, sizes, lambda n: (max(n, 1) / 0.05) ** (1 / 3), 0.9, n_species)


CASES = {
    "batch": lambda: clusters(71, list(np.random.Generator(np.random.PCG64(1)).integers(1, 65, 300))),
    "sizes_63_64": lambda: clusters(72, [63, 64, 64, 1, 2, 64]),
    "with_65": lambda: clusters(73, [10, 65, 30, 64]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_cluster_batch_list_matches_oracle(name):
    s = CASES[name]()
    p = synth.mbp_params(3, 4.6, 8, 4, 4)
    print(f"[cluster list] {name}: {s.n_structs} structures, {s.n_atoms} atoms, "
          f"largest {int(np.diff(s.atom_ptr).max())}", flush=True)
    pot = nnpot.Potential(s, p, None)
    pot.build_neighbors()
    got = check_list(pot, s, p.rc)
    assert nnpot.nn_count_neighbors(pot.sys, p.rc, pot.ws) == int(got["offsets"][-1])
    pot.build_neighbors()  # rebuilt: the same list bit for bit
    again = pot.neighbor_list_host()
    for k in ("offsets", "nbr", "shift", "rev"):
        assert np.array_equal(again[k], got[k]), k


def test_batch_with_a_periodic_cell_takes_the_generic_passes():
    rng = np.random.Generator(np.random.PCG64(74))
    cl = clusters(75, [12, 30, 50])
    cell = synth.single(rng.uniform(0, 7.0, (16, 3)), rng.integers(0, 3, 16), cell=np.eye(3) * 7.0, pbc=(1, 1, 1))
    s = synth.concat([cl, cell])
    p = synth.mbp_params(3, 4.6, 8, 4, 4)
    pot = nnpot.Potential(s, p, None)
    pot.build_neighbors()
    check_list(pot, s, p.rc)


def test_cluster_batch_non_finite_position_is_reported():
    s = clusters(76, [20, 30, 40])
    p = synth.mbp_params(3, 4.6, 8, 4, 4)
    pot = nnpot.Potential(s, p, None)
    pot.build_neighbors()
    pos = s.pos.copy()
    pos[25, 2] = np.inf
    pot.set_positions(pos)
    pot.build_neighbors(check=False)
    with pytest.raises(nnpot.NNError, match="non-finite"):
        nnpot.nn_check(pot.nl)


def test_cluster_batch_skin_rule():
    """With a skin the list holds the pairs within rc + skin; small moves keep
    it, a move past skin/2 rebuilds it, and the rebuilt list is the oracle's
    at the new positions."""
    s = clusters(77, [25, 40, 60, 8])
    p = synth.mbp_params(3, 4.6, 8, 4, 4)
    skin = 0.6
    pot = nnpot.Potential(s, p, None, skin=skin)
    pot.build_neighbors()
    check_list(pot, s, p.rc + skin)
    builds = int(pot.meta[2].item())
    pos = s.pos.copy()
    pos[3] += 0.1  # below skin / 2
    pot.set_positions(pos)
    pot.build_neighbors()
    assert int(pot.meta[2].item()) == builds
    pos[3] += 0.3  # now 0.4 > skin / 2
    pot.set_positions(pos)
    pot.build_neighbors()
    assert int(pot.meta[2].item()) == builds + 1
    s2 = synth.System(pos, s.species, s.atom_ptr, s.cell, s.pbc)
    check_list(pot, s2, p.rc + skin)
