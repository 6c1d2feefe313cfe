"""The row-block MLP (plan value 1: 64 atoms per block, the weights staged in
LDS) against the FP64 oracle, forced with NNPOT_PLAN="f,a,1": energies,
forces and the weight gradient of an energy loss for both fused shapes
(64-32 on the 4-species clusters, 128-128 on the one- and two-species bulk
cells), the Gaussian, ReLU and tanh activations, species tiles with a ragged
last block, and bitwise repeatability; then its BF16 modes, split (hi + lo)
operands to the stated tolerances and plain BF16 to its rounding model."""
import os

import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL

pytestmark = pytest.mark.gpu


class plan:
    def __init__(self, value):
        self.value = value

    def __enter__(self):
        os.environ["NNPOT_PLAN"] = self.value

    def __exit__(self, *a):
        os.environ.pop("NNPOT_PLAN", None)


def workload(name):
    if name == "cfg2s":
        return synth.config(2, scale=0.05)
    if name == "cfg1s":
        return synth.config(1, scale=0.25)
    if name == "cfg4s":
        return synth.config(4, scale=1 / 128)
    w = synth.config(2, scale=0.03)  # activation variants on the cluster shape
    act = name.split("_")[1]
    model = [(widths, [act, act, "linear"], Ws, bs) for (widths, acts, Ws, bs) in w.model]
    return synth.Workload(f"{w.name} {act}", w.system, w.params, model, w.seed)


@pytest.mark.parametrize("name", ["cfg2s", "cfg1s", "cfg4s", "act_relu", "act_tanh"])
def test_row_block_mlp_matches_oracle(name):
    w = workload(name)
    s, p = w.system, w.params
    nl = oracle.neighbors_cells(s, p.rc)
    Es_ref, _, F_ref = oracle.energy_forces(p, w.model, s, nl)
    T = synth.energy_targets(w.seed, s.n_structs)
    _, Es_l, flat = oracle.energy_loss_grad(p, w.model, s, nl, T)
    ref = oracle.unflatten_grads(w.model, flat)
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    n_c = np.maximum(np.diff(s.atom_ptr), 1)
    fw = "0" if name.startswith(("cfg2", "act")) else "1"
    with plan(f"{fw},{fw},1"):
        assert pot.launch_plan() == (int(fw), int(fw), 1)
        Es, _, F = [t.cpu().numpy() for t in pot.energy_forces()]
        e = float(np.max(np.abs(Es - Es_ref) / n_c))
        f = float(np.abs(F - F_ref).max())
        print(f"[mlp rows] {name}: E/atom {e:.2e} F {f:.2e}", flush=True)
        assert e <= E_TOL and f <= F_TOL
        again = [t.cpu().numpy() for t in pot.energy_forces()]
        assert np.array_equal(again[0], Es) and np.array_equal(again[2], F)
        dL_dE = 2.0 * (Es_l - T) / s.n_structs
        _, got = pot.grad(dL_dE, positions=False)
        nnpot.nn_check(pot.nl)
    worst = 0.0
    for sp in range(len(ref)):
        for (dW_r, db_r), (dW_g, db_g) in zip(ref[sp], got[sp]):
            for r_, g_ in ((dW_r, dW_g), (db_r, db_g)):
                g_ = g_.double().cpu().numpy().reshape(r_.shape)
                worst = max(worst, np.abs(g_ - r_).max() / max(np.abs(r_).max(), 1e-12))
    print(f"[mlp rows] {name}: weight gradient {worst:.2e} of its scale", flush=True)
    assert worst <= 1e-4


@pytest.mark.parametrize("name", ["cfg2s", "cfg1s", "cfg4s", "act_tanh"])
def test_row_block_bf16_modes(name):
    w = workload(name)
    s, p = w.system, w.params
    nl = oracle.neighbors_cells(s, p.rc)
    Es_ref, Ea_ref, F_ref = oracle.energy_forces(p, w.model, s, nl)
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    n_c = np.maximum(np.diff(s.atom_ptr), 1)
    fw = "0" if name.startswith(("cfg2", "act")) else "1"
    with plan(f"{fw},{fw},1"):
        # split operands: about 16 significant bits each, the stated tolerances
        Es, _, F = [t.cpu().numpy() for t in pot.energy_forces(flags=nnpot.NN_BF16X3_MLP)]
        e = float(np.max(np.abs(Es - Es_ref) / n_c))
        f = float(np.abs(F - F_ref).max())
        print(f"[mlp rows] {name} bf16x3: E/atom {e:.2e} F {f:.2e}", flush=True)
        assert e <= E_TOL and f <= F_TOL
        again = [t.cpu().numpy() for t in pot.energy_forces(flags=nnpot.NN_BF16X3_MLP)]
        assert np.array_equal(again[0], Es) and np.array_equal(again[2], F)
        # plain BF16 (unit roundoff u = 2^-9 on every operand): 16 u of the
        # largest atomic energy / force component, as for the tile kernel
        _, Ea, F = [t.cpu().numpy() for t in pot.energy_forces(flags=nnpot.NN_BF16_MLP)]
        u = 2.0 ** -9
        e = float(np.abs(Ea - Ea_ref).max())
        f = float(np.abs(F - F_ref).max())
        print(f"[mlp rows] {name} bf16: E/atom {e:.2e} F {f:.2e}", flush=True)
        assert e <= 16 * u * max(1.0, np.abs(Ea_ref).max())
        assert f <= 16 * u * max(1.0, np.abs(F_ref).max())
    nnpot.nn_check(pot.nl)


# Descriptor lengths the row-block kernels do not take: D = 76 (a multiple of 4,
# not of 8: the FP32 row-block kernel, the split-BF16 mode falls back to the
# tile kernel) and D = 77 (both fall back), with plan value 1 forced.
@pytest.mark.parametrize("n_rad,hidden", [(12, [64, 32]), (13, [64, 32]), (12, [128, 128]), (13, [128, 128])])
def test_row_plan_on_descriptor_lengths_it_does_not_take(n_rad, hidden):
    rng = np.random.Generator(np.random.PCG64(5100 + n_rad))
    s = synth.bulk_system(rng, 432, 0.1, 1.2, [432])
    p = synth.mbp_params(1, 5.0, n_rad, 8, 8)
    G = oracle.descriptors(p, s, oracle.neighbors_cells(s, p.rc))
    scale = float(np.sqrt(p.dim) / np.sqrt(np.mean(np.sum(G * G, axis=1))))
    model = synth.random_model(1, p.dim, hidden, 91 + n_rad, in_scale=scale)
    nl = oracle.neighbors_cells(s, p.rc)
    Es_ref, _, F_ref = oracle.energy_forces(p, model, s, nl)
    pot = nnpot.Potential(s, p, model)
    pot.build_neighbors()
    with plan("1,1,1"):
        for flags in (0, nnpot.NN_BF16X3_MLP):
            Es, _, F = [t.cpu().numpy() for t in pot.energy_forces(flags=flags)]
            e = float(np.max(np.abs(Es - Es_ref)) / s.n_atoms)
            f = float(np.abs(F - F_ref).max())
            print(f"[mlp rows] D {p.dim} {hidden} flags {flags}: E/atom {e:.2e} F {f:.2e}", flush=True)
            assert e <= E_TOL and f <= F_TOL
    nnpot.nn_check(pot.nl)
