"""Every launch plan against the FP64 oracle.

A plan (waves per atom of the descriptor forward and adjoint passes, 0 for
the packed passes, waves per MLP tile) changes only the order of some sums, so each one must meet the
same bars; NNPOT_PLAN forces one on every call.  One-species bulk, a
2-species bulk and the 4-species cluster batch cover the one-species,
several-species and pair-block forward paths."""
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL

pytestmark = pytest.mark.gpu

PLANS = list(itertools.product((0, 1, 2, 4), (0, 1, 2, 4), (1, 4, 8)))
_cache = {}


def case(name):
    if name not in _cache:
        w = {"cfg1s": lambda: synth.config(1, scale=0.25), "cfg4s": lambda: synth.config(4, scale=1 / 128),
             "cfg2s": lambda: synth.config(2, scale=0.03)}[name]()
        nl = oracle.neighbors_cells(w.system, w.params.rc)
        Es, _, F = oracle.energy_forces(w.params, w.model, w.system, nl)
        _cache[name] = (w, Es, F)
    return _cache[name]


@pytest.mark.parametrize("name", ["cfg1s", "cfg4s", "cfg2s"])
def test_every_plan_matches_oracle(name):
    w, Es_ref, F_ref = case(name)
    s = w.system
    pot = nnpot.Potential(s, w.params, w.model)
    pot.build_neighbors()
    n_c = np.maximum(np.diff(s.atom_ptr), 1)
    worst_e = worst_f = 0.0
    try:
        for plan in PLANS:
            os.environ["NNPOT_PLAN"] = ",".join(map(str, plan))
            for flags in (0, nnpot.NN_BF16X3_MLP):
                Es, _, F = [t.cpu().numpy() for t in pot.energy_forces(flags=flags)]
                e = float(np.max(np.abs(Es - Es_ref) / n_c))
                f = float(np.abs(F - F_ref).max())
                assert e <= E_TOL and f <= F_TOL, (plan, flags, e, f)
                worst_e, worst_f = max(worst_e, e), max(worst_f, f)
            # the gradient kernels follow the plan too
            _, g = pot.grad(np.ones(s.n_structs), positions=False)
            assert all(np.isfinite(t.cpu().numpy()).all() for layers in g for pair in layers for t in pair)
        nnpot.nn_check(pot.nl)
    finally:
        os.environ.pop("NNPOT_PLAN", None)
    print(f"[plans] {name}: {len(PLANS)} plans, worst E/atom {worst_e:.2e}, F {worst_f:.2e}", flush=True)
