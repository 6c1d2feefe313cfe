"""Seeded synthetic inputs: atomic configurations, descriptor hyperparameters
and random MLP weights.

This module only draws inputs.  It holds none of the method's arithmetic (no
descriptor, network or force code) and is the one module shared by the GPU
path's callers and by the tests that feed the same arrays to the oracle.

Workloads stand in for the paper's data sets, which are not available here:
  * configs 0 and 2: small organic molecules with {H, C, N, O} (the rMD17
    benchmark of Sec. III.A) -- non-periodic clusters;
  * configs 1, 3, 4: bulk periodic cells (the Carbon data of Sec. III.B and
    the repeated MD evaluation of Table II).
Placement is random sequential addition (RSA): uniform candidates, rejected
when closer than d_min to an accepted atom (minimum image in periodic boxes).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

SEED_BASE = 1000


@dataclass
class System:
    """A batch of structures.  Atoms of structure c are [atom_ptr[c], atom_ptr[c+1])."""
    pos: np.ndarray        # [N, 3] float64 (Angstrom)
    species: np.ndarray    # [N] int32
    atom_ptr: np.ndarray   # [B+1] int64
    cell: np.ndarray       # [B, 3, 3] float64, rows = lattice vectors a, b, c
    pbc: np.ndarray        # [B, 3] uint8

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_structs(self) -> int:
        return int(self.atom_ptr.shape[0] - 1)


@dataclass
class MBPParams:
    """Descriptor hyperparameters (grids as explicit arrays)."""
    n_species: int
    rc: float
    eta_rad: float
    rs_rad: np.ndarray
    theta_s: np.ndarray
    eta_ang: float
    rs_ang: np.ndarray
    zeta: float = 50.0
    eps: float = 1e-3
    # kind 1: the standard BP angular term instead of mBP, with per angle
    # term p an integer exponent bp_zeta[p] and sign bp_lambda[p], and per
    # radius term q a width bp_eta[q] (theta_s, rs_ang, eta_ang, zeta, eps
    # are then unused)
    kind: int = 0
    bp_zeta: np.ndarray = None
    bp_lambda: np.ndarray = None
    bp_eta: np.ndarray = None

    @property
    def n_rad(self) -> int:
        return int(len(self.rs_rad))

    @property
    def n_theta(self) -> int:
        return int(len(self.bp_zeta) if self.kind == 1 else len(self.theta_s))

    @property
    def n_rs_ang(self) -> int:
        return int(len(self.bp_eta) if self.kind == 1 else len(self.rs_ang))

    @property
    def dim(self) -> int:
        S = self.n_species
        return self.n_rad * S + self.n_theta * self.n_rs_ang * S * (S + 1) // 2


# A model is a list over species of (widths, activations, [W_l], [b_l]) with
# W_l of shape [widths[l], widths[l-1]] in float64.
Model = List[Tuple[List[int], List[str], List[np.ndarray], List[np.ndarray]]]


@dataclass
class Workload:
    name: str
    system: System
    params: MBPParams
    model: Model
    seed: int
    extra: dict = field(default_factory=dict)


def mbp_params(n_species, rc, n_rad, n_theta, n_rs_ang, eta_rad=16.0, eta_ang=12.0, zeta=50.0,
               eps=1e-3, r_min=0.5) -> MBPParams:
    """Evenly spaced grids: radial centres r_min..rc (inclusive), angular
    radial centres r_min..rc (inclusive), angle centres (p + 1/2) pi / n_theta."""
    return MBPParams(
        n_species=n_species, rc=float(rc), eta_rad=float(eta_rad),
        rs_rad=np.linspace(r_min, rc, n_rad), theta_s=(np.arange(n_theta) + 0.5) * np.pi / n_theta,
        eta_ang=float(eta_ang), rs_ang=np.linspace(r_min, rc, n_rs_ang), zeta=float(zeta), eps=float(eps))


def bp_params(n_species, rc, n_rad, zetas=(1, 2, 4, 16), etas=(0.005, 0.02, 0.06, 0.15), eta_rad=16.0,
              r_min=0.5) -> MBPParams:
    """Standard BP descriptor: the mBP radial part (same grid rule) and angular
    terms for every zeta in `zetas` with lambda = +1 and -1 (p = 2 z + l) and
    every radius width in `etas` (1/A^2)."""
    zl = [(float(z), lam) for z in zetas for lam in (1.0, -1.0)]
    return MBPParams(
        n_species=n_species, rc=float(rc), eta_rad=float(eta_rad), rs_rad=np.linspace(r_min, rc, n_rad),
        theta_s=np.zeros(0), eta_ang=0.0, rs_ang=np.zeros(0), zeta=0.0, eps=0.0, kind=1,
        bp_zeta=np.array([z for z, _ in zl]), bp_lambda=np.array([l for _, l in zl]),
        bp_eta=np.asarray(etas, np.float64))


def random_model(n_species, D, hidden: Sequence[int], seed, act="gaussian", in_scale=1.0, n_out=1) -> Model:
    """Per-species MLP D -> hidden... -> n_out with W, b ~ N(0, 1/fan_in),
    seeded per species and layer.  The first layer's draws are multiplied by
    in_scale (the inverse of a typical descriptor magnitude) so that the
    Gaussian units are neither saturated nor flat."""
    model = []
    widths = [D] + list(hidden) + [n_out]
    acts = [act] * len(hidden) + ["linear"]
    for s in range(n_species):
        Ws, bs = [], []
        for l in range(1, len(widths)):
            rng = np.random.Generator(np.random.PCG64([seed, s, l]))
            std = 1.0 / np.sqrt(widths[l - 1])
            W = rng.normal(0.0, std, size=(widths[l], widths[l - 1]))
            b = rng.normal(0.0, std, size=(widths[l],))
            if l == 1:
                W *= in_scale
            Ws.append(W)
            bs.append(b)
        model.append((list(widths), list(acts), Ws, bs))
    return model


def random_model_per_species(D, hidden_per_species: Sequence[Sequence[int]], seed, act="gaussian",
                             in_scale=1.0) -> Model:
    """Per-species networks of different depths and widths (Sec. II.A lets
    each species have its own architecture): species s gets
    D -> hidden_per_species[s]... -> 1, drawn as in random_model."""
    model = []
    for s, hidden in enumerate(hidden_per_species):
        one = random_model(len(hidden_per_species), D, list(hidden), seed, act=act, in_scale=in_scale)
        model.append(one[s])
    return model


# ----------------------------------------------------------------------------
# placement
# ----------------------------------------------------------------------------

def rsa_cluster(rng, n, box, d_min, max_tries=100000) -> np.ndarray:
    """n points uniform in [0, box)^3, none closer than d_min (no periodicity)."""
    pts = np.empty((n, 3))
    k, tries = 0, 0
    while k < n:
        c = rng.uniform(0.0, box, size=3)
        tries += 1
        if tries > max_tries:
            raise RuntimeError("RSA did not converge")
        if k and np.min(np.sum((pts[:k] - c) ** 2, axis=1)) < d_min * d_min:
            continue
        pts[k] = c
        k += 1
    return pts


def rsa_periodic(rng, n, L, d_min) -> np.ndarray:
    """n points uniform in a periodic cube of side L with minimum-image
    distance >= d_min, placed in batches (candidates are accepted in draw
    order, so the result is the sequential RSA of the drawn stream)."""
    from scipy.spatial import cKDTree

    acc = np.empty((0, 3))
    while acc.shape[0] < n:
        need = n - acc.shape[0]
        cand = rng.uniform(0.0, L, size=(max(64, int(need * 1.15) + 16), 3))
        cand = np.minimum(cand, np.nextafter(L, 0.0))
        if acc.shape[0]:
            tree = cKDTree(acc, boxsize=L)
            dist, _ = tree.query(cand, k=1, distance_upper_bound=d_min)
            cand = cand[~(dist < d_min)]
        if cand.shape[0] == 0:
            continue
        ctree = cKDTree(cand, boxsize=L)
        pairs = ctree.query_pairs(d_min, output_type="ndarray")
        keep = np.ones(cand.shape[0], bool)
        if pairs.size:
            conflicts = [[] for _ in range(cand.shape[0])]
            for a, b in pairs:
                lo, hi = (a, b) if a < b else (b, a)
                conflicts[hi].append(lo)
            for idx in range(cand.shape[0]):
                if conflicts[idx] and any(keep[j] for j in conflicts[idx]):
                    keep[idx] = False
        acc = np.concatenate([acc, cand[keep][:need]])
    return acc


def _cube(L):
    return np.diag([L, L, L]).astype(np.float64)


def clusters_system(rng, sizes, box_of, d_min, n_species, species_p=None) -> System:
    pos, sp, ptr, cell = [], [], [0], []
    for n in sizes:
        L = box_of(n)
        pos.append(rsa_cluster(rng, n, L, d_min))
        sp.append(rng.choice(n_species, size=n, p=species_p).astype(np.int32))
        ptr.append(ptr[-1] + n)
        cell.append(_cube(L))
    B = len(sizes)
    return System(np.concatenate(pos), np.concatenate(sp), np.asarray(ptr, np.int64), np.stack(cell),
                  np.zeros((B, 3), np.uint8))


def bulk_system(rng, n, density, d_min, species_counts) -> System:
    L = (n / density) ** (1.0 / 3.0)
    pos = rsa_periodic(rng, n, L, d_min)
    sp = np.concatenate([np.full(c, s, np.int32) for s, c in enumerate(species_counts)])
    rng.shuffle(sp)
    return System(pos, sp, np.asarray([0, n], np.int64), _cube(L)[None], np.ones((1, 3), np.uint8))


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

# Scale applied to the first-layer weights: sqrt(D) over the typical RMS norm
# of a descriptor row of that workload (rounded), so that first-layer
# pre-activations are O(1) and the Gaussian units are in their sensitive
# range.  A fixed constant per workload, not computed from the data.
IN_SCALE = {0: 14.0, 1: 0.45, 2: 12.0, 3: 3.3, 4: 0.6}


# The standard BP descriptor on the geometries of configs 0-2 (desc="bp"):
# radial grid as for mBP, angular terms zeta in {1, 2, 4, 8} (molecules) or
# {1, 2, 4, 16} (bulk) with lambda = +-1, and 4 or 8 radius widths; the
# first-layer scale follows the same rule as IN_SCALE.
BP_ANGULAR = {0: ((1, 2, 4, 8), (0.01, 0.05, 0.15, 0.4)),
              1: ((1, 2, 4, 16), (0.001, 0.01, 0.03, 0.06, 0.1, 0.2, 0.4, 0.8)),
              2: ((1, 2, 4, 8), (0.01, 0.05, 0.15, 0.4))}
BP_IN_SCALE = {0: 7.0, 1: 0.14, 2: 6.0}


def config(idx: int, scale: float = 1.0, desc: str = "mbp") -> Workload:
    """Workload `idx` (0..4).  `scale` < 1 shrinks bulk systems (same density
    and hyperparameters) for fast tests; it does not apply to clusters.
    desc="bp" (configs 0-2) keeps the system and swaps the mBP angular term
    for the standard BP one (same radial grid and MLP widths)."""
    w = _config_mbp(idx, scale)
    if desc == "mbp":
        return w
    if desc != "bp" or idx not in BP_ANGULAR:
        raise ValueError(f"descriptor {desc!r} for config {idx}")
    zetas, etas = BP_ANGULAR[idx]
    p0 = w.params
    p = bp_params(p0.n_species, p0.rc, p0.n_rad, zetas=zetas, etas=etas, eta_rad=p0.eta_rad)
    hidden = list(w.model[0][0][1:-1])
    model = random_model(p.n_species, p.dim, hidden, w.seed, in_scale=BP_IN_SCALE[idx])
    name = w.name.replace(f"{p0.n_theta}x{p0.n_rs_ang} bins", f"BP {p.n_theta}x{p.n_rs_ang} terms")
    name = name.replace(f" + {p0.n_theta}x{p0.n_rs_ang} ", f" + BP {p.n_theta}x{p.n_rs_ang} ")
    return Workload(name, w.system, p, model, w.seed, w.extra)


def _config_mbp(idx: int, scale: float = 1.0) -> Workload:
    seed = SEED_BASE + idx
    rng = np.random.Generator(np.random.PCG64(seed))
    if idx == 0:
        sys = clusters_system(rng, [12] * 16, lambda n: 6.0, 0.9, 4)
        p = mbp_params(4, 4.6, 16, 8, 4)
        model = random_model(4, p.dim, [64, 32], seed, in_scale=IN_SCALE[0])
        name = "16 clusters x 12 atoms, 4 species, Rc 4.6, 16 + 8x4 bins, MLP D-64-32-1"
    elif idx == 1:
        n = max(16, int(round(4096 * scale)))
        sys = bulk_system(rng, n, 0.1, 1.2, [n])
        p = mbp_params(1, 5.0, 32, 8, 8)
        model = random_model(1, p.dim, [128, 128], seed, in_scale=IN_SCALE[1])
        name = f"periodic bulk {n} atoms, 1 species, rho 0.1, Rc 5.0, 32 + 8x8 bins, MLP D-128-128-1"
    elif idx == 2:
        nb = max(1, int(round(2048 * scale)))
        sizes = rng.integers(5, 61, size=nb)
        sys = clusters_system(rng, sizes, lambda n: (n / 0.05) ** (1.0 / 3.0), 0.9, 4)
        p = mbp_params(4, 4.6, 16, 8, 4)
        model = random_model(4, p.dim, [64, 32], seed, in_scale=IN_SCALE[2])
        name = f"{nb} clusters of 5-60 atoms, 4 species, rho 0.05, Rc 4.6, 16 + 8x4 bins, MLP D-64-32-1"
    elif idx == 3:
        n = max(64, int(round(32768 * scale)) // 4 * 4)
        sys = bulk_system(rng, n, 0.09, 1.2, [n // 4] * 4)
        p = mbp_params(4, 5.0, 32, 8, 8)
        model = random_model(4, p.dim, [128, 128], seed, in_scale=IN_SCALE[3])
        name = f"periodic bulk {n} atoms, 4 species, rho 0.09, Rc 5.0, 32 + 8x8 bins, MLP D-128-128-1"
    elif idx == 4:
        n = max(64, int(round(262144 * scale)) // 2 * 2)
        sys = bulk_system(rng, n, 0.09, 1.2, [n // 2] * 2)
        p = mbp_params(2, 6.0, 48, 8, 8)
        model = random_model(2, p.dim, [128, 128], seed, in_scale=IN_SCALE[4])
        name = f"periodic bulk {n} atoms, 2 species, rho 0.09, Rc 6.0, 48 + 8x8 bins, MLP D-128-128-1"
    else:
        raise ValueError(idx)
    extra = {}
    if idx == 4:
        extra = {"skin": 0.5, "steps": 100, "step_sigma": 0.02}
    return Workload(name, sys, p, model, seed, extra)


# Charge equilibration (Sec. II.B) on charged two-species clusters shaped like
# the paper's Na9Cl8+ / Na8Cl8+ test (17 and 16 atoms, total charge +1).
# The paper's descriptor length 45 has no (n_theta, n_rs_ang) among the
# compiled angular shapes, so the stand-in uses 16 radial + 4 x 4 angular
# bins (D = 80) with the paper's network: two hidden layers of 15 units and
# an output layer of 3 (local energy, electronegativity, hardness).  The
# output biases start from per-species references (eV, eV/e, eV/e^2: the
# Mulliken electronegativity and hardness of Na and Cl); Gaussian charge
# widths 1.0 and 1.2 A.  Atoms are placed by RSA in a 9 A cube with a 2.2 A
# minimum distance.
QEQ_SIGMA = (1.0, 1.2)
QEQ_REF = ((0.0, 2.85, 4.6), (0.0, 8.3, 9.4))


def qeq_model(D, seed, hidden=(15, 15), in_scale=1.0) -> Model:
    model = random_model(2, D, list(hidden), seed, in_scale=in_scale, n_out=3)
    for s, (widths, acts, Ws, bs) in enumerate(model):
        bs[-1] = bs[-1] + np.asarray(QEQ_REF[s])
    return model


def qeq_clusters(n_clusters: int, seed: int = SEED_BASE + 7):
    """(Workload, total charges [B]): n_clusters charged NaCl-like clusters,
    alternately 9 Na + 8 Cl and 8 Na + 8 Cl, each of total charge +1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, sp, ptr, cell = [], [], [0], []
    for c in range(n_clusters):
        n_na = 9 if c % 2 == 0 else 8
        n = n_na + 8
        pos.append(rsa_cluster(rng, n, 9.0, 2.2))
        s = np.array([0] * n_na + [1] * 8, np.int32)
        rng.shuffle(s)
        sp.append(s)
        ptr.append(ptr[-1] + n)
        cell.append(_cube(9.0))
    system = System(np.concatenate(pos), np.concatenate(sp), np.asarray(ptr, np.int64), np.stack(cell),
                    np.zeros((n_clusters, 3), np.uint8))
    p = mbp_params(2, 6.0, 16, 4, 4, eta_rad=4.0, eta_ang=3.0, zeta=8.0)
    model = qeq_model(p.dim, seed, in_scale=QEQ_IN_SCALE)
    name = f"{n_clusters} charged clusters Na9Cl8+ / Na8Cl8+ (Q = +1), Rc 6.0, 16 + 4x4 bins, MLP D-15-15-3"
    return Workload(name, system, p, model, seed, {"sigma": QEQ_SIGMA}), np.ones(n_clusters)


# Atomic masses (amu) of the four species the molecular workloads draw
# ({H, C, N, O}); the bulk workloads are carbon.
SPECIES_MASS = (1.008, 12.011, 14.007, 15.999)
CARBON_MASS = 12.011


# The three networks of Table II (hidden widths), on the Carbon descriptor
# of Sec. III.B: one species, Rc 5 A, 24 radial bins and 8 radius x 16 angle
# bins (D = 152).  First-layer scale 0.45: sqrt(D) over the RMS descriptor
# row norm of these 16-atom cells (27.2), a fixed constant like IN_SCALE.
TABLE2_HIDDEN = {"small": [64, 32], "middle": [256, 128], "big": [1024, 512, 256]}
TABLE2_IN_SCALE = 0.45
QEQ_IN_SCALE = 5.4  # sqrt(D) over the RMS descriptor row norm of these clusters


def md_cells(n_cells: int = 1, network: str = None) -> Workload:
    """The repeated-evaluation shape of Table II: 16-atom periodic carbon
    cells at the config-1 density and minimum distance (cube side 5.43 A,
    narrower than 2 Rc, so several images of each atom are neighbors);
    n_cells independent cells are batched as structures.  network=None: the
    config-1 descriptor and MLP; "small" / "middle" / "big": the Carbon
    descriptor of Sec. III.B (D = 152) with that Table II network."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 5))
    cells = [bulk_system(rng, 16, 0.1, 1.2, [16]) for _ in range(n_cells)]
    if network is None:
        p = mbp_params(1, 5.0, 32, 8, 8)
        model = random_model(1, p.dim, [128, 128], SEED_BASE + 1, in_scale=IN_SCALE[1])
        name = f"{n_cells} periodic carbon cell(s) of 16 atoms, rho 0.1, Rc 5.0, 32 + 8x8 bins, MLP D-128-128-1"
    else:
        hidden = TABLE2_HIDDEN[network]
        p = mbp_params(1, 5.0, 24, 16, 8)
        model = random_model(1, p.dim, hidden, SEED_BASE + 6, in_scale=TABLE2_IN_SCALE)
        name = (f"{n_cells} periodic carbon cell(s) of 16 atoms, rho 0.1, Rc 5.0, 24 + 8x16 bins (D = 152), "
                f"Table II {network} MLP D-{'-'.join(map(str, hidden))}-1")
    return Workload(name, concat(cells), p, model, SEED_BASE + 5, {"mass": CARBON_MASS})


def md_inputs(seed: int, n_atoms: int, n_steps: int, v_sigma: float):
    """Initial velocities N(0, v_sigma) (Angstrom/fs, FP64 [N, 3]) and the
    Langevin noise: standard normal FP32 [n_steps, N, 3]."""
    rng = np.random.Generator(np.random.PCG64([seed, 13]))
    v0 = rng.normal(0.0, v_sigma, size=(n_atoms, 3))
    noise = rng.standard_normal(size=(n_steps, n_atoms, 3), dtype=np.float32)
    return v0, noise


def md_displacements(seed: int, n_atoms: int, steps: int, sigma: float):
    """Generator of per-step Gaussian displacements (cumulative random walk)."""
    rng = np.random.Generator(np.random.PCG64([seed, 7]))
    for _ in range(steps):
        yield rng.normal(0.0, sigma, size=(n_atoms, 3))


def energy_targets(seed: int, n_structs: int) -> np.ndarray:
    """Seeded targets T_c ~ N(0, 1) for the energy loss."""
    return np.random.Generator(np.random.PCG64([seed, 11])).normal(size=n_structs)


def force_targets(seed: int, n_atoms: int) -> np.ndarray:
    """Seeded force targets F*_k ~ N(0, 1) eV/A per component for a force-matching loss."""
    return np.random.Generator(np.random.PCG64([seed, 12])).normal(size=(n_atoms, 3))


def single(pos, species, cell=None, pbc=(0, 0, 0)) -> System:
    """One structure from explicit arrays (tests and small examples)."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    if cell is None:
        span = np.ptp(pos, axis=0) if pos.shape[0] else np.zeros(3)
        cell = np.diag(np.maximum(span, 1.0) + 1.0)
    return System(pos, np.asarray(species, np.int32), np.asarray([0, pos.shape[0]], np.int64),
                  np.asarray(cell, np.float64).reshape(1, 3, 3), np.asarray(pbc, np.uint8).reshape(1, 3))


def concat(systems: Sequence[System]) -> System:
    ptr = [0]
    for s in systems:
        ptr += list(ptr[-1] + np.cumsum(np.diff(s.atom_ptr)))
    return System(np.concatenate([s.pos for s in systems]), np.concatenate([s.species for s in systems]),
                  np.asarray(ptr, np.int64), np.concatenate([s.cell for s in systems]),
                  np.concatenate([s.pbc for s in systems]))
