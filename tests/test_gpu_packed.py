"""The packed descriptor passes (four short-row atoms per wave) against the
FP64 oracle, forced with NNPOT_PLAN="0,0,m".

Cases: the 4-species cluster batch of the small-molecule workload; the
12-atom clusters; one-species clusters (the one-species adjoint and the
identity grouping); clusters of 1-4 atoms (atoms with no or one neighbor,
empty species-pair segments); the cluster geometry at rc 6 (rows on both
sides of the 32-entry packing limit, so the packed and the one-atom
long-row kernels share a launch); a list with a skin (entries beyond rc);
every angular shape the ABI accepts; a run-time mBP exponent.  Each checks
descriptors, energies and forces at the bars of the other parity tests, for
the FP32 and split-BF16 MLPs, then the weight gradient of an energy loss
against the one-atom plan.  Also: bitwise repeatability, and the device
error paths (capacity overflow, a species out of range) under the packed
plan.
"""
import ctypes as C
import os

import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL, descriptor_errors

pytestmark = pytest.mark.gpu

PACKED = "0,0,4"
_cache = {}


def first_layer_scale(p, s):
    G = oracle.descriptors(p, s, oracle.neighbors_cells(s, p.rc))
    return float(np.sqrt(p.dim) / np.sqrt(np.mean(np.sum(G * G, axis=1))))


def workload(name):
    if name in _cache:
        return _cache[name]
    skin = 0.0
    if name == "clusters4":
        w = synth.config(2, scale=0.03)
        s, p, model = w.system, w.params, w.model
    elif name == "cfg0":
        w = synth.config(0)
        s, p, model = w.system, w.params, w.model
    else:
        rng = np.random.Generator(np.random.PCG64(5100 + len(name)))
        nt, nra, zeta = 8, 4, 50.0
        if name == "one_species":
            s = synth.clusters_system(rng, rng.integers(5, 41, size=40), lambda n: (n / 0.05) ** (1 / 3), 0.9, 1)
            S, rc = 1, 4.6
        elif name == "tiny":
            s = synth.clusters_system(rng, [1, 2, 3, 4, 1, 2, 3, 4, 2, 2], lambda n: 3.0, 0.9, 3)
            S, rc = 3, 4.6
        elif name == "mixed_rows":
            s = synth.clusters_system(rng, rng.integers(20, 61, size=24), lambda n: (n / 0.05) ** (1 / 3), 0.9, 4)
            S, rc = 4, 6.0
        elif name == "skin":
            s = synth.clusters_system(rng, rng.integers(5, 41, size=40), lambda n: (n / 0.05) ** (1 / 3), 0.9, 4)
            S, rc, skin = 4, 4.6, 0.8
        elif name == "zeta8":
            s = synth.clusters_system(rng, rng.integers(5, 41, size=40), lambda n: (n / 0.05) ** (1 / 3), 0.9, 2)
            S, rc, zeta = 2, 4.6, 8.0
        elif name.startswith("shape"):
            nt, nra = (int(x) for x in name[5:].split("x"))
            s = synth.clusters_system(rng, rng.integers(5, 41, size=40), lambda n: (n / 0.05) ** (1 / 3), 0.9, 3)
            S, rc = 3, 4.6
        else:
            raise KeyError(name)
        p = synth.mbp_params(S, rc, 16, nt, nra, zeta=zeta)
        model = synth.random_model(S, p.dim, [64, 32], 91 + len(name), in_scale=first_layer_scale(p, s))
    nl = oracle.neighbors_cells(s, p.rc)
    G_ref = oracle.descriptors(p, s, nl)
    Es_ref, _, F_ref = oracle.energy_forces(p, model, s, nl)
    _cache[name] = (s, p, model, skin, nl, G_ref, Es_ref, F_ref)
    return _cache[name]


class plan:
    def __init__(self, value):
        self.value = value

    def __enter__(self):
        os.environ["NNPOT_PLAN"] = self.value

    def __exit__(self, *a):
        os.environ.pop("NNPOT_PLAN", None)


CASES = ["clusters4", "cfg0", "one_species", "tiny", "mixed_rows", "skin", "zeta8",
         "shape8x8", "shape16x8", "shape16x4", "shape4x8", "shape4x4"]


@pytest.mark.parametrize("name", CASES)
def test_packed_matches_oracle(name):
    s, p, model, skin, nl, G_ref, Es_ref, F_ref = workload(name)
    rows = np.diff(nl["offsets"])
    print(f"[packed] {name}: {s.n_atoms} atoms, D = {p.dim}, rows <= 32: {int((rows <= 32).sum())}, "
          f"longer: {int((rows > 32).sum())}", flush=True)
    pot = nnpot.Potential(s, p, model, skin=skin)
    pot.build_neighbors()
    n_c = np.maximum(np.diff(s.atom_ptr), 1)
    with plan(PACKED):
        G = pot.descriptors().cpu().numpy()
        assert descriptor_errors(G, G_ref) <= 1.0, descriptor_errors(G, G_ref)
        for flags in (0, nnpot.NN_BF16X3_MLP):
            Es, _, F = [t.cpu().numpy() for t in pot.energy_forces(flags=flags)]
            e = float(np.max(np.abs(Es - Es_ref) / n_c))
            f = float(np.abs(F - F_ref).max()) if F.size else 0.0
            print(f"[packed] {name} flags {flags}: E/atom {e:.2e} F {f:.2e}", flush=True)
            assert e <= E_TOL and f <= F_TOL, (flags, e, f)
        nnpot.nn_check(pot.nl)
        _, g_pk = pot.grad(np.ones(s.n_structs), positions=False)
    with plan("1,1,4"):
        _, g_one = pot.grad(np.ones(s.n_structs), positions=False)
    for la, lb in zip(g_pk, g_one):
        for (dw_a, db_a), (dw_b, db_b) in zip(la, lb):
            for a, b in ((dw_a, dw_b), (db_a, db_b)):
                a, b = a.cpu().numpy(), b.cpu().numpy()
                scale = max(float(np.abs(b).max()), 1e-30)
                assert float(np.abs(a - b).max()) <= 1e-4 * scale


def test_packed_is_bitwise_repeatable():
    """The full 2048-cluster batch, the list rebuilt before each run: the
    atoms a wave packs (and so the order of its sums) must not depend on the
    list's bin order, whose order within a bin is that of the binning
    atomics."""
    w = synth.config(2)
    pot = nnpot.Potential(w.system, w.params, w.model)
    runs = []
    with plan(PACKED):
        for _ in range(4):
            pot.build_neighbors()
            G = pot.descriptors().cpu().numpy().copy()
            runs.append([G] + [t.cpu().numpy().copy() for t in pot.energy_forces()])
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert np.array_equal(a, b)


def check_status(pot):
    import torch
    info = C.c_int64(0)
    st = nnpot.lib().nn_check(C.byref(pot.nl), C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(info))
    return st, int(info.value), nnpot.nn_last_error()


def test_packed_capacity_overflow_gives_zeros():
    s, p, model, skin, nl, *_ = workload("clusters4")
    nnz = int(nl["offsets"][-1])
    pot = nnpot.Potential(s, p, model, capacity=nnz // 3)
    pot.build_neighbors(check=False)
    import torch
    pot.G = torch.ones((pot.N, pot.D), dtype=torch.float32, device=pot.dev)
    with plan(PACKED):
        G = pot.descriptors()
        _, _, F = pot.energy_forces()
    st, info, msg = check_status(pot)
    print(f"[packed capacity] status {st} info {info}: {msg}", flush=True)
    assert st == nnpot.STATUS_CODE["NN_E_CAPACITY"] and info == nnz
    assert not G.any().item() and not F.any().item()


def test_packed_species_out_of_range_then_fixed():
    import torch
    s, p, model, skin, nl, G_ref, Es_ref, F_ref = workload("clusters4")
    pot = nnpot.Potential(s, p, model)
    pot.build_neighbors()
    bad = pot.species.clone()
    bad[3] = p.n_species
    pot.species.copy_(bad)
    with plan(PACKED):
        pot.energy_forces()
        st, _, msg = check_status(pot)
        print(f"[packed species] status {st}: {msg}", flush=True)
        assert st == nnpot.STATUS_CODE["NN_E_DEVICE"] and "species" in msg
        pot.species.copy_(torch.tensor(s.species, dtype=torch.int32, device=pot.dev))
        Es, _, F = [t.cpu().numpy() for t in pot.energy_forces()]
    nnpot.nn_check(pot.nl)
    assert np.abs(F - F_ref).max() <= F_TOL
    assert np.max(np.abs(Es - Es_ref) / np.maximum(np.diff(s.atom_ptr), 1)) <= E_TOL
