"""Launch tuning: nn_autotune picks waves per atom / per MLP tile by timing;
the tuned plan must keep every result within the oracle tolerances, be
bitwise reproducible, and nn_autotune_reset must bring back the default
plan's results bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,flags", [("cfg1", 0), ("cfg3s", 0), ("cfg3s", nnpot.NN_BF16X3_MLP),
                                        ("cfg2s", 0)])
def test_autotuned_plan_matches_oracle(name, flags):
    import torch
    w = {"cfg1": lambda: synth.config(1), "cfg3s": lambda: synth.config(3, scale=0.1),
         "cfg2s": lambda: synth.config(2, scale=0.05)}[name]()
    s, p = w.system, w.params
    print(f"[tune] {name} flags {flags}: {w.name}", flush=True)
    nnpot.nn_autotune_reset()
    pot = nnpot.Potential(s, p, w.model, flags=flags)
    pot.build_neighbors()
    Es0, _, F0 = (t.clone() for t in pot.energy_forces())
    plan = pot.autotune()
    print(f"  plan {plan}", flush=True)
    assert plan[0] in (0, 1, 2, 4) and plan[1] in (0, 1, 2, 4) and plan[2] in (1, 4, 8)
    Es, _, F = (t.clone() for t in pot.energy_forces())
    Es2, _, F2 = pot.energy_forces()
    assert torch.equal(Es, Es2) and torch.equal(F, F2)
    nl = oracle.neighbors_cells(s, p.rc)
    Es_ref, _, F_ref = oracle.energy_forces(p, w.model, s, nl)
    n_c = np.diff(s.atom_ptr)
    e_err = float(np.max(np.abs(Es.cpu().numpy() - Es_ref) / np.maximum(n_c, 1)))
    f_err = float(np.max(np.abs(F.cpu().numpy() - F_ref)))
    print(f"  E/atom {e_err:.2e}  F {f_err:.2e}", flush=True)
    assert e_err <= E_TOL and f_err <= F_TOL
    nnpot.nn_autotune_reset()
    Es3, _, F3 = pot.energy_forces()
    assert torch.equal(Es3, Es0) and torch.equal(F3, F0)


def test_autotune_writes_the_cache_file(tmp_path, monkeypatch):
    """nn_autotune with NN_AUTOTUNE_CACHE set writes its plan under the
    workload's key; a fresh process (host only) then reads it back through
    nn_launch_plan."""
    import json
    import os
    import subprocess
    import sys
    path = str(tmp_path / "plans.json")
    monkeypatch.setenv("NN_AUTOTUNE_CACHE", path)
    w = synth.config(0)
    s, p = w.system, w.params
    nnpot.nn_autotune_reset()
    pot = nnpot.Potential(s, p, w.model, capacity=4000)
    pot.build_neighbors()
    plan = list(pot.autotune())
    assert pot.launch_plan() == tuple(plan)
    entries = json.load(open(path))
    n = int(s.n_atoms)
    key = [n.bit_length(), ((4000 + n - 1) // n + 2) // 4, p.n_species, p.n_theta,
           p.n_rs_ang, p.n_rad, 64, 32, 0]
    assert {"key": key, "plan": plan} in entries, (entries, key, plan)
    nnpot.nn_autotune_reset()
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, here)
    from test_autotune_cache import QUERY
    env = dict(os.environ, PYTHONPATH=os.path.dirname(here) + os.pathsep + os.environ.get("PYTHONPATH", ""))
    env.pop("NNPOT_PLAN", None)
    r = subprocess.run([sys.executable, "-c", QUERY], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert json.loads(r.stdout.strip().splitlines()[-1])["plan"] == plan
