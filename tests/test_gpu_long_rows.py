"""The one-wave descriptor forward and adjoint over rows of more than 128
list entries (the one-pass staging takes up to 128; longer rows are staged
in two passes).  A dense two-species bulk cell at rc 6.5 A with a 0.5 A skin
has rows of 123 to 168 entries (about 115 neighbors inside rc), so both
staging paths run in one call.  Descriptors, energies and forces against
the FP64 oracle at the bars of the other parity tests, for one and for two
waves per atom.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL, descriptor_errors

pytestmark = pytest.mark.gpu


def test_rows_on_both_sides_of_the_short_block():
    rng = np.random.Generator(np.random.PCG64(6200))
    s = synth.bulk_system(rng, 1000, 0.1, 1.2, [500, 500])
    p = synth.mbp_params(2, 6.5, 16, 8, 8)
    nl = oracle.neighbors_cells(s, p.rc)
    G_ref = oracle.descriptors(p, s, nl)
    scale = float(np.sqrt(p.dim) / np.sqrt(np.mean(np.sum(G_ref * G_ref, axis=1))))
    model = synth.random_model(2, p.dim, [128, 128], 62, in_scale=scale)
    Es_ref, _, F_ref = oracle.energy_forces(p, model, s, nl)
    pot = nnpot.Potential(s, p, model, skin=0.5)
    pot.build_neighbors()
    rows = np.diff(pot.offsets.cpu().numpy())
    print(f"[long rows] entries per row {rows.min()}..{rows.max()}, {(rows > 128).sum()} over 128", flush=True)
    assert (rows > 128).sum() > 0 and (rows <= 128).sum() > 0
    try:
        for plan in ("1,1,1", "2,2,1"):
            os.environ["NNPOT_PLAN"] = plan
            G = pot.descriptors().cpu().numpy()
            rel = descriptor_errors(G, G_ref)
            Es, _, F = [t.cpu().numpy() for t in pot.energy_forces()]
            e = float(np.max(np.abs(Es - Es_ref)) / s.n_atoms)
            f = float(np.abs(F - F_ref).max())
            print(f"[long rows] plan {plan}: G {rel:.2e} E/atom {e:.2e} F {f:.2e}", flush=True)
            assert rel <= 1.0 and e <= E_TOL and f <= F_TOL
        nnpot.nn_check(pot.nl)
    finally:
        os.environ.pop("NNPOT_PLAN", None)
