"""Device-side error paths of the C ABI (forced from the inputs; every
kernel still runs to completion and bounds its own accesses):

- list capacity below the entries needed: NN_E_CAPACITY with the needed
  size from nn_check, zero forces, and a list of that size equal to the
  oracle's;
- a periodic cell narrower than three bins for a structure over 256 atoms:
  NN_E_CELL (synchronously from nn_count_neighbors, from nn_check after a
  build);
- a species index out of range: NN_E_DEVICE, and a correct result once the
  input is fixed;
- more than 192 neighbors inside rc: NN_E_DEVICE;
- NN_REUSE_DESCRIPTORS after a list rebuild: NN_E_DEVICE and zero forces.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL, list_rows_equal

pytestmark = pytest.mark.gpu


def check_status(pot):
    """(status, info) of nn_check without raising."""
    import torch
    info = C.c_int64(0)
    st = nnpot.lib().nn_check(C.byref(pot.nl), C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(info))
    return st, int(info.value), nnpot.nn_last_error()


def test_capacity_overflow_reports_size_then_exact_rebuild():
    w = synth.config(1, scale=0.25)
    s, p = w.system, w.params
    ref = oracle.neighbors_cells(s, p.rc)
    nnz = int(ref["offsets"][-1])
    pot = nnpot.Potential(s, p, w.model, capacity=nnz // 3)
    pot.build_neighbors(check=False)
    _, _, F = pot.energy_forces()
    st, info, msg = check_status(pot)
    print(f"[capacity] status {st} info {info} (oracle nnz {nnz}): {msg}", flush=True)
    assert st == nnpot.STATUS_CODE["NN_E_CAPACITY"] and info == nnz
    assert not F.any().item()  # no valid list: zero forces
    assert check_status(pot)[0] == 0  # nn_check cleared the error word
    pot2 = nnpot.Potential(s, p, w.model, capacity=info)
    pot2.build_neighbors()
    got = pot2.neighbor_list_host()
    assert np.array_equal(got["offsets"], ref["offsets"])
    ok, why = list_rows_equal(got, ref)
    assert ok, why
    Es, _, F = [t.cpu().numpy() for t in pot2.energy_forces()]
    Es_ref, _, F_ref = oracle.energy_forces(p, w.model, s, ref)
    assert np.abs(F - F_ref).max() <= F_TOL and np.max(np.abs(Es - Es_ref) / s.n_atoms) <= E_TOL


def narrow_cell_system():
    rng = np.random.Generator(np.random.PCG64(8))
    L = 12.0  # 2.4 rc: fewer than three bins of width rc per direction
    return synth.single(rng.uniform(0, L, (300, 3)), np.zeros(300, np.int32), cell=np.eye(3) * L, pbc=(1, 1, 1))


def test_narrow_cell_large_structure():
    s = narrow_cell_system()
    p = synth.mbp_params(1, 5.0, 8, 4, 4)
    with pytest.raises(nnpot.NNError) as e:
        nnpot.Potential(s, p, None)  # sizing the list counts the neighbors synchronously
    assert e.value.status == nnpot.STATUS_CODE["NN_E_CELL"]
    pot = nnpot.Potential(s, p, None, capacity=200000)
    pot.build_neighbors(check=False)
    st, _, msg = check_status(pot)
    print(f"[cell] status {st}: {msg}", flush=True)
    assert st == nnpot.STATUS_CODE["NN_E_CELL"]


@pytest.mark.parametrize("cfg,scale", [(0, 1.0), (1, 0.05)])
def test_species_out_of_range_then_fixed(cfg, scale):
    import torch
    w = synth.config(cfg, scale=scale)
    s, p = w.system, w.params
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    bad = pot.species.clone()
    bad[3] = p.n_species  # one past the last species
    pot.species.copy_(bad)
    pot.energy_forces()
    st, _, msg = check_status(pot)
    print(f"[species] cfg{cfg}: status {st}: {msg}", flush=True)
    assert st == nnpot.STATUS_CODE["NN_E_DEVICE"] and "species" in msg
    pot.species.copy_(torch.tensor(s.species, dtype=torch.int32, device=pot.dev))
    Es, _, F = [t.cpu().numpy() for t in pot.energy_forces()]
    nnpot.nn_check(pot.nl)
    nl = oracle.neighbors_cells(s, p.rc)
    Es_ref, _, F_ref = oracle.energy_forces(p, w.model, s, nl)
    assert np.abs(F - F_ref).max() <= F_TOL
    assert np.max(np.abs(Es - Es_ref) / np.maximum(np.diff(s.atom_ptr), 1)) <= E_TOL


def test_too_many_neighbors():
    rng = np.random.Generator(np.random.PCG64(9))
    pos = rng.uniform(0, 2.5, (250, 3))  # every pair within rc: 249 neighbors each (> 192)
    s = synth.single(pos, np.zeros(250, np.int32), cell=np.eye(3) * 3.0)
    p = synth.mbp_params(1, 4.6, 8, 4, 4)
    model = synth.random_model(1, p.dim, [64, 32], 3)
    pot = nnpot.Potential(s, p, model)
    pot.build_neighbors()  # the list itself is fine (rows of 249 <= 1024)
    _, _, F = pot.energy_forces()
    st, _, msg = check_status(pot)
    print(f"[too many] status {st}: {msg}", flush=True)
    assert st == nnpot.STATUS_CODE["NN_E_DEVICE"] and "too many" in msg
    assert not F.any().item()  # every row is over the limit: zero pair gradients


def test_reuse_after_rebuild_is_refused():
    w = synth.config(1, scale=0.1)
    s, p = w.system, w.params
    big = 1 << 40
    pot = nnpot.Potential(s, p, w.model, mem_budget=big, flags=nnpot.NN_STORE_JACOBIAN)
    pot.build_neighbors()
    _, _, F0 = [t.cpu().numpy().copy() for t in pot.energy_forces(flags=nnpot.NN_STORE_JACOBIAN)]
    _, _, F1 = [t.cpu().numpy().copy() for t in pot.energy_forces(flags=nnpot.NN_REUSE_DESCRIPTORS)]
    nnpot.nn_check(pot.nl)
    assert np.array_equal(F0, F1)
    pot.build_neighbors()  # a rebuild (no skin): the stored rows refer to the old list
    _, _, F2 = pot.energy_forces(flags=nnpot.NN_REUSE_DESCRIPTORS)
    st, _, msg = check_status(pot)
    print(f"[stale] status {st}: {msg}", flush=True)
    assert st == nnpot.STATUS_CODE["NN_E_DEVICE"] and "stale" in msg
    assert not F2.any().item()
    # storing again makes reuse valid
    pot.energy_forces(flags=nnpot.NN_STORE_JACOBIAN)
    _, _, F3 = [t.cpu().numpy().copy() for t in pot.energy_forces(flags=nnpot.NN_REUSE_DESCRIPTORS)]
    nnpot.nn_check(pot.nl)
    assert np.array_equal(F0, F3)
