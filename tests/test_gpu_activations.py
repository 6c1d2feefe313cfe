"""ReLU and tanh hidden layers (activations of Eq. (1), Sec. II.A) on the
GPU against the FP64 oracle: energies and forces (FP32 and split-BF16 MLP),
the weight gradient of an energy loss, and the weight gradient of a loss on
energies and forces (which needs the second derivative of the activation in
the MLP's forward-mode tangent).  Same bars as the Gaussian tests."""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL

pytestmark = pytest.mark.gpu

ACTS = ["relu", "tanh"]
CFGS = [(0, 1.0), (1, 0.25), (2, 0.03), (3, 0.05)]


def workload(cfg, scale, act):
    w = synth.config(cfg, scale=scale)
    hidden = list(w.model[0][0][1:-1])
    model = synth.random_model(w.params.n_species, w.params.dim, hidden, w.seed + 17, act=act,
                               in_scale=synth.IN_SCALE[cfg])
    return synth.Workload(w.name + f" {act}", w.system, w.params, model, w.seed)


def grad_error(got, ref):
    worst = 0.0
    for sp in range(len(ref)):
        for (dW_r, db_r), (dW_g, db_g) in zip(ref[sp], got[sp]):
            for r_, g_ in ((dW_r, dW_g), (db_r, db_g)):
                g_ = g_.double().cpu().numpy().reshape(r_.shape)
                worst = max(worst, float(np.abs(g_ - r_).max() / max(np.abs(r_).max(), 1e-30)))
    return worst


@pytest.mark.parametrize("act", ACTS)
@pytest.mark.parametrize("cfg,scale", CFGS)
def test_energy_forces(cfg, scale, act):
    w = workload(cfg, scale, act)
    s, p = w.system, w.params
    nl = oracle.neighbors_cells(s, p.rc)
    Es_ref, _, F_ref = oracle.energy_forces(p, w.model, s, nl)
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    for flags in (0, nnpot.NN_BF16X3_MLP):
        Es, _, F = [t.cpu().numpy() for t in pot.energy_forces(flags=flags)]
        nnpot.nn_check(pot.nl)
        e = np.max(np.abs(Es - Es_ref) / np.maximum(np.diff(s.atom_ptr), 1))
        f = np.abs(F - F_ref).max()
        print(f"[{act}] cfg{cfg} flags {flags}: E/atom {e:.2e}  F {f:.2e} (|F|max {np.abs(F_ref).max():.2f})",
              flush=True)
        assert e <= E_TOL
        # The ReLU gate is a decision: split-BF16 products carry about 16
        # significant bits, so a unit whose pre-activation is within ~1e-5
        # of its input scale of zero may take the other branch than in FP64
        # and change its atom's dE/dG by that unit's whole weight (the energy
        # is continuous there, its derivative is not).  ReLU forces are held
        # to the bar in FP32, where the window is 2^-24 and no unit of these
        # inputs falls in it; tanh and the Gaussian are smooth.
        if not (act == "relu" and flags == nnpot.NN_BF16X3_MLP):
            assert f <= F_TOL
    assert np.abs(F_ref).max() > 0.05


@pytest.mark.parametrize("act", ACTS)
@pytest.mark.parametrize("cfg,scale", [(0, 1.0), (2, 0.03), (3, 0.05)])
def test_energy_loss_weight_gradient(cfg, scale, act):
    w = workload(cfg, scale, act)
    s, p = w.system, w.params
    T = synth.energy_targets(w.seed, s.n_structs)
    nl = oracle.neighbors_cells(s, p.rc)
    _, Es_ref, flat = oracle.energy_loss_grad(p, w.model, s, nl, T)
    ref = oracle.unflatten_grads(w.model, flat)
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    pot.energy_forces()
    _, got = pot.grad(2.0 * (Es_ref - T) / s.n_structs, positions=False)
    nnpot.nn_check(pot.nl)
    err = grad_error(got, ref)
    print(f"[{act}] cfg{cfg}: energy-loss max |d dW| / max |dW| = {err:.2e}", flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("act", ACTS)
@pytest.mark.parametrize("cfg,scale", [(0, 1.0), (1, 0.25), (2, 0.03)])
def test_force_loss_weight_gradient(cfg, scale, act):
    w = workload(cfg, scale, act)
    s, p = w.system, w.params
    rng = np.random.Generator(np.random.PCG64(w.seed + 9))
    gE = rng.standard_normal(s.n_structs)
    gF = rng.standard_normal((s.n_atoms, 3)).astype(np.float32)
    nl = oracle.neighbors_cells(s, p.rc)
    ref = oracle.unflatten_grads(w.model, oracle.force_loss_grad(p, w.model, s, nl, gE, gF.astype(np.float64)))
    pot = nnpot.Potential(s, p, w.model)
    pot.build_neighbors()
    pot.energy_forces()
    _, got = pot.grad(gE, positions=False, dL_dF=gF)
    nnpot.nn_check(pot.nl)
    err = grad_error(got, ref)
    print(f"[{act}] cfg{cfg}: force-loss max |d dW| / max |dW| = {err:.2e}", flush=True)
    assert err <= 1e-4
