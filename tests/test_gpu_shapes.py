"""Every angular shape the ABI accepts, against the FP64 oracle.

(n_theta, n_rs_ang) in {4, 16} x {4, 8} (the 8 x 8 and 8 x 4 shapes of the
workloads are covered elsewhere); 16 x 8 with 24 radial bins on one species
is the Carbon descriptor of Sec. III.B (D = 152).  Each shape runs on a
one-species periodic bulk cell and on a batch of small 4-species clusters
(the several-species pair-block path), through descriptors, energies and
forces, the stored Jacobian and the descriptor tangent, at the bars of the
other parity tests.
"""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL, descriptor_errors, tangent_error, tangent_error_with_floor, tangent_noise_floor
from test_gpu_stored import expand_jacobian

pytestmark = pytest.mark.gpu

SHAPES = [(16, 8), (16, 4), (4, 8), (4, 4)]
_cache = {}


def first_layer_scale(p, s):
    """sqrt(D) over the RMS descriptor row norm (oracle descriptors): keeps
    first-layer pre-activations O(1) so the forces are not ~0."""
    G = oracle.descriptors(p, s, oracle.neighbors_cells(s, p.rc))
    return float(np.sqrt(p.dim) / np.sqrt(np.mean(np.sum(G * G, axis=1))))


def workload(kind, nt, nra):
    key = (kind, nt, nra)
    if key in _cache:
        return _cache[key]
    if kind == "bulk":
        # Sec. III.B shape: one species, Rc 5, 24 radial bins
        rng = np.random.Generator(np.random.PCG64(4000 + 10 * nt + nra))
        s = synth.bulk_system(rng, 432, 0.1, 1.2, [432])  # side 16.3 A: three bins of rc
        p = synth.mbp_params(1, 5.0, 24, nt, nra)
        hidden = [64, 32]
    else:
        w0 = synth.config(2, scale=0.02)
        s = w0.system
        p = synth.mbp_params(4, 4.6, 16, nt, nra)
        hidden = [64, 32]
    model = synth.random_model(p.n_species, p.dim, hidden, 77 + nt + nra, in_scale=first_layer_scale(p, s))
    w = synth.Workload(f"{kind} {nt}x{nra}", s, p, model, 0)
    nl = oracle.neighbors_cells(s, p.rc)
    _cache[key] = (w, nl)
    return w, nl


CASES = [(k, nt, nra) for nt, nra in SHAPES for k in ("bulk", "clusters")]


def ids(c):
    return f"{c[0]}-{c[1]}x{c[2]}"


def test_paper_carbon_descriptor_size():
    w, _ = workload("bulk", 16, 8)
    pot = nnpot.Potential(w.system, w.params, w.model)
    assert pot.D == 152


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_descriptors_and_energy_forces(case):
    w, nl = workload(*case)
    s, p = w.system, w.params
    print(f"[shape] {w.name}: D = {p.dim}, {s.n_atoms} atoms", flush=True)
    G_ref = oracle.descriptors(p, s, nl)
    Es_ref, _, F_ref = oracle.energy_forces(p, w.model, s, nl)
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    G = pot.descriptors().cpu().numpy()
    for flags in (0, nnpot.NN_BF16X3_MLP):
        Es, _, F = [t.cpu().numpy() for t in pot.energy_forces(flags=flags)]
        nnpot.nn_check(pot.nl)
        e = np.max(np.abs(Es - Es_ref) / np.maximum(np.diff(s.atom_ptr), 1))
        f = np.abs(F - F_ref).max()
        print(f"  flags {flags}: E/atom {e:.2e}  F {f:.2e} (|F|max {np.abs(F_ref).max():.2f})", flush=True)
        assert e <= E_TOL and f <= F_TOL
    err = descriptor_errors(G, G_ref)
    print(f"  max |dG| / tol = {err:.3f}", flush=True)
    assert err <= 1.0
    assert np.abs(F_ref).max() > 0.05  # the forces are not trivially small


@pytest.mark.parametrize("case", [c for c in CASES if c[0] == "bulk"] + [("clusters", 16, 8)], ids=ids)
def test_stored_jacobian_and_stored_forces(case):
    w, nl_ref = workload(*case)
    s, p = w.system, w.params
    if case[0] == "clusters":  # fewer structures: the dense expansion is [nnz][D][3]
        n = int(np.searchsorted(s.atom_ptr, 400))
        s = synth.System(s.pos[:s.atom_ptr[n]], s.species[:s.atom_ptr[n]], s.atom_ptr[:n + 1], s.cell[:n], s.pbc[:n])
        nl_ref = oracle.neighbors_cells(s, p.rc)
    big = 1 << 40
    pot = nnpot.Potential(s, p, w.model, mem_budget=big, flags=nnpot.NN_STORE_JACOBIAN)
    pot.build_neighbors()
    _, J = pot.jacobian()
    nnpot.nn_check(pot.nl)
    nl = pot.neighbor_list_host()
    _, dG = oracle.descriptors(p, s, nl_ref, jacobian=True)
    got = expand_jacobian(J.cpu().numpy().astype(np.float64)[:len(nl["nbr"])], nl, s.species, p)
    scale_e = np.maximum(np.abs(dG).max(axis=(1, 2)), 1e-12)
    err = (np.abs(got - dG).max(axis=(1, 2)) / scale_e).max()
    print(f"[jacobian] {w.name}: max per-entry |dJ| / max |J| = {err:.2e}", flush=True)
    assert err <= 1e-4
    Es_ref, _, F_ref = oracle.energy_forces(p, w.model, s, nl_ref)
    _, _, F0 = [t.cpu().numpy().copy() for t in pot.energy_forces(flags=0)]
    Es1, _, F1 = [t.cpu().numpy().copy() for t in pot.energy_forces(flags=nnpot.NN_STORE_JACOBIAN)]
    nnpot.nn_check(pot.nl)
    assert np.abs(F1 - F_ref).max() <= F_TOL
    assert np.max(np.abs(Es1 - Es_ref) / np.maximum(np.diff(s.atom_ptr), 1)) <= E_TOL
    assert np.abs(F1 - F0).max() <= 1e-5 * np.abs(F0).max()


@pytest.mark.parametrize("case", CASES, ids=ids)
def test_descriptor_tangent(case):
    w, nl = workload(*case)
    s, p = w.system, w.params
    v = np.random.Generator(np.random.PCG64(55)).standard_normal((s.n_atoms, 3)).astype(np.float32)
    U_ref = oracle.descriptor_tangent(p, s, nl, v.astype(np.float64))
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    U = pot.descriptor_tangent(v).double().cpu().numpy()
    nnpot.nn_check(pot.nl)
    # bar: 1e-4 of the block's largest entry in the row, plus four times the
    # spread of the FP64 tangent under FP32-sized displacement noise (elements
    # whose terms cancel are not better conditioned than that)
    floor = tangent_noise_floor(p, s, nl, v.astype(np.float64))
    err = tangent_error_with_floor(U, U_ref, p, floor)
    print(f"[tangent] {w.name}: max |dU| / block scale = {tangent_error(U, U_ref, p):.2e}, "
          f"against the bar with the noise floor {err:.2f}", flush=True)
    assert err <= 1.0
