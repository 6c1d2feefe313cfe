"""The layer-by-layer MLP path: networks of one to three hidden layers, any
widths, and a different architecture per species (Sec. II.A), including the
three networks of Table II (64-32, 256-128, 1024-512-256) on the Carbon
descriptor of Sec. III.B (D = 152).  Energies and forces, the weight
gradient of an energy loss and of a loss on energies and forces, against
the FP64 oracle at the bars of the other parity tests."""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL

pytestmark = pytest.mark.gpu

WG_REL = 1e-4


def first_layer_scale(p, s):
    G = oracle.descriptors(p, s, oracle.neighbors_cells(s, p.rc))
    return float(np.sqrt(p.dim) / np.sqrt(np.mean(np.sum(G * G, axis=1))))


def carbon_bulk(n=432, seed=4242):
    rng = np.random.Generator(np.random.PCG64(seed))
    return synth.bulk_system(rng, n, 0.1, 1.2, [n])


def carbon_params():
    return synth.mbp_params(1, 5.0, 24, 16, 8)  # Sec. III.B: 24 radial + 8 x 16 angular, D = 152


_cache = {}


def workload(name):
    if name in _cache:
        return _cache[name]
    if name.startswith("table2"):
        hidden = {"table2-small": [64, 32], "table2-middle": [256, 128], "table2-big": [1024, 512, 256]}[name]
        s = carbon_bulk()
        p = carbon_params()
        model = synth.random_model(1, p.dim, hidden, 31, in_scale=first_layer_scale(p, s))
        w = synth.Workload(name, s, p, model, 31)
    elif name == "per-species":
        w0 = synth.config(0)
        hid = [[64, 32], [48], [32, 24, 16], [96, 40]]
        model = synth.random_model_per_species(w0.params.dim, hid, 33, in_scale=synth.IN_SCALE[0])
        w = synth.Workload(name, w0.system, w0.params, model, w0.seed)
    elif name == "per-species-tanh-batch":
        w0 = synth.config(2, scale=0.03)
        hid = [[40, 24], [64, 48, 32], [16], [128, 64]]
        model = synth.random_model_per_species(w0.params.dim, hid, 35, act="tanh", in_scale=synth.IN_SCALE[2])
        w = synth.Workload(name, w0.system, w0.params, model, w0.seed)
    elif name == "three-hidden-bulk-2sp":
        w0 = synth.config(4, scale=1 / 128)
        model = synth.random_model(2, w0.params.dim, [96, 64, 32], 37, in_scale=synth.IN_SCALE[4])
        w = synth.Workload(name, w0.system, w0.params, model, w0.seed)
    else:
        raise KeyError(name)
    nl = oracle.neighbors_cells(w.system, w.params.rc)
    _cache[name] = (w, nl)
    return _cache[name]


NAMES = ["table2-small", "table2-middle", "table2-big", "per-species", "per-species-tanh-batch",
         "three-hidden-bulk-2sp"]


def grad_error(got, ref):
    worst = 0.0
    for sp in range(len(ref)):
        for (dW_r, db_r), (dW_g, db_g) in zip(ref[sp], got[sp]):
            for r_, g_ in ((dW_r, dW_g), (db_r, db_g)):
                g_ = g_.double().cpu().numpy().reshape(r_.shape)
                worst = max(worst, float(np.abs(g_ - r_).max() / max(np.abs(r_).max(), 1e-30)))
    return worst


@pytest.mark.parametrize("name", NAMES)
def test_energy_forces(name):
    w, nl = workload(name)
    s, p = w.system, w.params
    Es_ref, Ea_ref, F_ref = oracle.energy_forces(p, w.model, s, nl)
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    Es, Ea, F = [t.cpu().numpy() for t in pot.energy_forces()]
    nnpot.nn_check(pot.nl)
    e = np.max(np.abs(Es - Es_ref) / np.maximum(np.diff(s.atom_ptr), 1))
    f = np.abs(F - F_ref).max()
    print(f"[layers] {name}: E/atom {e:.2e}  F {f:.2e} (|F|max {np.abs(F_ref).max():.2f}, "
          f"|E_atom| max {np.abs(Ea_ref).max():.2f})", flush=True)
    assert e <= E_TOL and f <= F_TOL
    assert np.abs(Ea - Ea_ref).max() <= E_TOL
    assert np.abs(F_ref).max() > 0.05


@pytest.mark.parametrize("name", NAMES)
def test_energy_loss_weight_gradient(name):
    w, nl = workload(name)
    s, p = w.system, w.params
    T = synth.energy_targets(w.seed, s.n_structs)
    _, Es_ref, flat = oracle.energy_loss_grad(p, w.model, s, nl, T)
    ref = oracle.unflatten_grads(w.model, flat)
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    pot.energy_forces()
    _, got = pot.grad(2.0 * (Es_ref - T) / s.n_structs, positions=False)
    nnpot.nn_check(pot.nl)
    err = grad_error(got, ref)
    print(f"[layers] {name}: energy-loss max |d dW| / max |dW| = {err:.2e}", flush=True)
    assert err <= WG_REL


@pytest.mark.parametrize("name", NAMES)
def test_force_loss_weight_gradient(name):
    w, nl = workload(name)
    s, p = w.system, w.params
    rng = np.random.Generator(np.random.PCG64(w.seed + 9))
    gE = rng.standard_normal(s.n_structs)
    gF = rng.standard_normal((s.n_atoms, 3)).astype(np.float32)
    ref = oracle.unflatten_grads(w.model, oracle.force_loss_grad(p, w.model, s, nl, gE, gF.astype(np.float64)))
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    pot.energy_forces()
    _, got = pot.grad(gE, positions=False, dL_dF=gF)
    nnpot.nn_check(pot.nl)
    err = grad_error(got, ref)
    print(f"[layers] {name}: force-loss max |d dW| / max |dW| = {err:.2e}", flush=True)
    assert err <= WG_REL


def test_layered_path_deterministic_and_bf16_refused():
    w, _ = workload("per-species")
    pot = nnpot.Potential(w.system, w.params, w.model)
    pot.build_neighbors()
    outs = []
    for _ in range(2):
        Es, _, F = pot.energy_forces()
        _, g = pot.grad(np.linspace(-1, 1, w.system.n_structs), positions=False)
        outs.append([Es.cpu().numpy().copy(), F.cpu().numpy().copy()] +
                    [t.cpu().numpy().copy() for layers in g for pair in layers for t in pair])
    for a, b in zip(*outs):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    with pytest.raises(nnpot.NNError) as e:
        pot.energy_forces(flags=nnpot.NN_BF16X3_MLP)
    assert e.value.status == nnpot.STATUS_CODE["NN_E_UNSUPPORTED"]
