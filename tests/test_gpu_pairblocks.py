"""Small molecules with several species: the forward and tangent passes give
each species-pair block its own 4-lane MFMA block when an atom has at most
256 triplets, there are at most 16 pair blocks (S <= 5) and one wave works
on an atom (the default plan for several species and short rows).  Dense
seeded clusters put atoms on both sides of the 256-triplet limit; species
drawn with unequal weights leave some pair blocks without triplets.  Cases:
5 species with the mBP term (compile-time exponent 50) and with the
standard BP term, 3 species with a run-time mBP exponent, and 6 species
(21 pair blocks: every atom takes the chunked path).  Bars: descriptors
1e-5 relative, energies 1e-4 eV/atom, forces 1e-3 eV/A, tangents 1e-4 of
their block's scale, all against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2305_11805_amd import nnpot, synth

from helpers import E_TOL, F_TOL, descriptor_errors, tangent_error

pytestmark = pytest.mark.gpu

FUSE_TRIPLETS = 256


def dense_clusters(S, params, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    weights = np.linspace(1.0, 0.3, S)
    sys_ = synth.clusters_system(rng, [1, 2, 3, 9, 20, 34, 48, 64], lambda n: (n / 0.1) ** (1.0 / 3.0) + 1.0, 0.9,
                                 S, species_p=weights / weights.sum())
    model = synth.random_model(S, params.dim, [64, 32], seed, in_scale=2.0)
    return synth.Workload(f"{S}-species dense clusters", sys_, params, model, seed)


CASES = {
    "s5_mbp": lambda: dense_clusters(5, synth.mbp_params(5, 4.6, 8, 8, 4), 501),
    "s5_bp": lambda: dense_clusters(5, synth.bp_params(5, 4.6, 8, zetas=(1, 2, 4, 9), etas=(0.02, 0.1, 0.3, 0.7)),
                                    502),
    "s3_zeta7": lambda: dense_clusters(3, synth.mbp_params(3, 4.6, 8, 8, 8, zeta=7.0), 503),
    "s6_mbp": lambda: dense_clusters(6, synth.mbp_params(6, 4.6, 8, 8, 4), 504),
}
_cache = {}


def case(name):
    if name not in _cache:
        w = CASES[name]()
        nl = oracle.neighbors_cells(w.system, w.params.rc)
        _cache[name] = (w, nl)
    return _cache[name]


def potential(w, nl):
    nnpot.nn_autotune_reset()  # the default plan, not one tuned earlier in this process
    nnz = int(nl["offsets"][-1])
    cap = nnz + 16
    assert cap <= 24 * w.system.n_atoms  # short rows: one wave per atom for the forward and tangent
    pot = nnpot.Potential(w.system, w.params, w.model, capacity=cap)
    pot.build_neighbors()
    return pot


def test_cases_straddle_the_triplet_limit():
    for name in ("s5_mbp", "s5_bp", "s3_zeta7"):
        w, nl = case(name)
        n = np.diff(nl["offsets"])
        t = n * (n - 1) // 2
        assert (t <= FUSE_TRIPLETS).sum() > 0 and (t > FUSE_TRIPLETS).sum() > 0, name
        assert (n == 0).any() and ((n > 0) & (n < 3)).any(), name


@pytest.mark.parametrize("name", list(CASES))
def test_descriptors_match_oracle(name):
    w, nl = case(name)
    print(f"[pair blocks] descriptors {name}: {w.system.n_atoms} atoms, D = {w.params.dim}", flush=True)
    G_ref = oracle.descriptors(w.params, w.system, nl)
    pot = potential(w, nl)
    G = pot.descriptors().cpu().numpy()
    nnpot.nn_check(pot.nl)
    err = descriptor_errors(G, G_ref)
    print(f"  max |dG| / tol = {err:.3f}", flush=True)
    assert err <= 1.0


@pytest.mark.parametrize("name", list(CASES))
def test_energy_forces_match_oracle(name):
    w, nl = case(name)
    print(f"[pair blocks] E/F {name}", flush=True)
    Es_ref, _, F_ref = oracle.energy_forces(w.params, w.model, w.system, nl)
    pot = potential(w, nl)
    Es, _, F = pot.energy_forces()
    nnpot.nn_check(pot.nl)
    n_c = np.diff(w.system.atom_ptr).astype(np.float64)
    e_err = float(np.max(np.abs(Es.cpu().numpy() - Es_ref) / n_c))
    f_err = float(np.abs(F.cpu().numpy() - F_ref).max())
    print(f"  E/atom {e_err:.2e} eV, F {f_err:.2e} eV/A", flush=True)
    assert e_err <= E_TOL and f_err <= F_TOL


@pytest.mark.parametrize("name", list(CASES))
def test_descriptor_tangent_matches_oracle(name):
    w, nl = case(name)
    print(f"[pair blocks] tangent {name}", flush=True)
    v = np.random.Generator(np.random.PCG64(w.seed + 7)).standard_normal((w.system.n_atoms, 3))
    v32 = v.astype(np.float32)
    U_ref = oracle.descriptor_tangent(w.params, w.system, nl, v32.astype(np.float64))
    pot = potential(w, nl)
    U = pot.descriptor_tangent(v32).double().cpu().numpy()
    nnpot.nn_check(pot.nl)
    err = tangent_error(U, U_ref, w.params)
    print(f"  max |dU| / block scale = {err:.2e}", flush=True)
    assert err <= 1e-4
