"""Plain FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``nnref.c`` (plain C, double precision, no
fast-math, no FP contraction) through ctypes and shares no code with the GPU
library.  Inputs are plain arrays (any object with the attributes named
below); nothing here imports the product package.

What each function computes, and the passage of the PANNA 2.0 paper it
follows, is stated in ``nnref.c``; the Langevin integrator written here in
numpy (``md_langevin``) states it in its docstring.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nnref.c")
_LIB_PATH = os.path.join(_HERE, "libnnref.so")
_MAX_LAYERS = 8  # REF_MAX_LAYERS in nnref.c

ACT = {"linear": 0, "gaussian": 1, "relu": 2, "tanh": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -ffp-contract=off, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math", "-ffp-contract=off",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _System(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("n_structs", C.c_int32), ("pos", C.c_void_p),
                ("species", C.c_void_p), ("atom_ptr", C.c_void_p), ("cell", C.c_void_p),
                ("pbc", C.c_void_p)]


class _NList(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("rows", C.c_void_p), ("offsets", C.c_void_p),
                ("nbr", C.c_void_p), ("shift", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("rc", C.c_double), ("n_rad", C.c_int32),
                ("eta_rad", C.c_double), ("rs_rad", C.c_void_p), ("n_theta", C.c_int32),
                ("theta_s", C.c_void_p), ("n_rs_ang", C.c_int32), ("eta_ang", C.c_double),
                ("rs_ang", C.c_void_p), ("zeta", C.c_double), ("eps", C.c_double),
                ("kind", C.c_int32), ("bp_zeta", C.c_void_p), ("bp_lambda", C.c_void_p), ("bp_eta", C.c_void_p)]


class _Model(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_layers", C.c_void_p), ("arch", C.c_void_p),
                ("act", C.c_void_p), ("params", C.c_void_p), ("poff", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.nnref_neighbors_brute.restype = C.c_int64
        L.nnref_neighbors_brute.argtypes = [P, C.c_double, C.c_int, P, C.c_int64, C.c_int64, P, P, P]
        L.nnref_neighbors_cells.restype = C.c_int64
        L.nnref_neighbors_cells.argtypes = [P, C.c_double, P, C.c_int64, C.c_int64, P, P, P]
        L.nnref_descriptor_dim.restype = C.c_int64
        L.nnref_descriptor_dim.argtypes = [C.c_int32] * 4
        L.nnref_descriptors.restype = None
        L.nnref_descriptors.argtypes = [P, P, P, P, P]
        L.nnref_mlp.restype = None
        L.nnref_mlp.argtypes = [P, C.c_int64, P, P, C.c_int64, P, P]
        L.nnref_atom_energies.restype = None
        L.nnref_atom_energies.argtypes = [P, P, P, P, P, P]
        L.nnref_forces.restype = None
        L.nnref_forces.argtypes = [P, P, P, P, P, C.c_int64, P, P]
        L.nnref_energy_forces.restype = None
        L.nnref_energy_forces.argtypes = [P, P, P, P, P, P, P]
        L.nnref_energy_loss_grad.restype = C.c_double
        L.nnref_energy_loss_grad.argtypes = [P, P, P, P, P, P, P, C.c_int64]
        L.nnref_descriptor_tangent.restype = None
        L.nnref_descriptor_tangent.argtypes = [P, P, P, P, P]
        L.nnref_force_loss_grad.restype = None
        L.nnref_force_loss_grad.argtypes = [P, P, P, P, P, P, P, C.c_int64]
        L.nnref_num_threads.restype = C.c_int
        L.nnref_num_threads.argtypes = []
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Keep:
    """Holds numpy arrays alive while a ctypes struct points at them."""

    def __init__(self):
        self.items = []

    def __call__(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.items.append(a)
        return a


def _c_system(sys, keep):
    pos = keep(sys.pos, np.float64)
    sp = keep(sys.species, np.int32)
    ptr = keep(sys.atom_ptr, np.int64)
    cell = keep(sys.cell, np.float64)
    pbc = keep(sys.pbc, np.uint8)
    return _System(pos.shape[0], ptr.shape[0] - 1, _ptr(pos), _ptr(sp), _ptr(ptr), _ptr(cell), _ptr(pbc))


def _c_params(p, keep):
    """Descriptor parameters; p.kind = 1 selects the standard BP angular term
    with per-term p.bp_zeta, p.bp_lambda (n_theta of them) and p.bp_eta
    (n_rs_ang of them)."""
    rs_rad = keep(p.rs_rad, np.float64)
    kind = int(getattr(p, "kind", 0))
    if kind == 1:
        bz, bl, be = keep(p.bp_zeta, np.float64), keep(p.bp_lambda, np.float64), keep(p.bp_eta, np.float64)
        return _Params(p.n_species, p.rc, rs_rad.size, p.eta_rad, _ptr(rs_rad), bz.size, None, be.size, 0.0, None,
                       0.0, 0.0, 1, _ptr(bz), _ptr(bl), _ptr(be))
    th = keep(p.theta_s, np.float64)
    rs_ang = keep(p.rs_ang, np.float64)
    return _Params(p.n_species, p.rc, rs_rad.size, p.eta_rad, _ptr(rs_rad), th.size, _ptr(th),
                   rs_ang.size, p.eta_ang, _ptr(rs_ang), p.zeta, p.eps, 0, None, None, None)


def _c_model(model, keep):
    """model: sequence over species of (widths, acts, Ws, bs) in FP64."""
    S = len(model)
    n_layers = np.zeros(S, np.int32)
    arch = np.zeros((S, _MAX_LAYERS + 1), np.int32)
    act = np.zeros((S, _MAX_LAYERS), np.int32)
    chunks, poff, off = [], np.zeros(S, np.int64), 0
    for s, (widths, acts, Ws, bs) in enumerate(model):
        L = len(Ws)
        n_layers[s] = L
        arch[s, :L + 1] = widths
        act[s, :L] = [ACT[a] if isinstance(a, str) else a for a in acts]
        poff[s] = off
        for W, b in zip(Ws, bs):
            chunks += [np.asarray(W, np.float64).ravel(), np.asarray(b, np.float64).ravel()]
            off += W.size + b.size
    params = np.concatenate(chunks)
    return _Model(S, _ptr(keep(n_layers, np.int32)), _ptr(keep(arch, np.int32)), _ptr(keep(act, np.int32)),
                  _ptr(keep(params, np.float64)), _ptr(keep(poff, np.int64))), params.size


def _c_nlist(nl, keep):
    offsets = keep(nl["offsets"], np.int64)
    nbr = keep(nl["nbr"], np.int32)
    shift = keep(nl["shift"], np.int32)
    rows = nl.get("rows")
    rows = None if rows is None else keep(rows, np.int64)
    return _NList(offsets.size - 1, _ptr(rows), _ptr(offsets), _ptr(nbr), _ptr(shift))


def descriptor_dim(n_species, n_rad, n_theta, n_rs_ang) -> int:
    return int(lib().nnref_descriptor_dim(n_species, n_rad, n_theta, n_rs_ang))


def _neighbors(fn, sys, cutoff, rows, extra):
    keep = _Keep()
    csys = _c_system(sys, keep)
    n_rows = sys.pos.shape[0] if rows is None else len(rows)
    rows_a = None if rows is None else keep(rows, np.int64)
    offsets = np.zeros(n_rows + 1, np.int64)
    args = (C.byref(csys), cutoff) + ((extra,) if extra is not None else ())
    nnz = fn(*args, _ptr(rows_a), n_rows, 0, _ptr(offsets), None, None)
    nbr = np.zeros(max(nnz, 1), np.int32)
    shift = np.zeros((max(nnz, 1), 3), np.int32)
    nnz2 = fn(*args, _ptr(rows_a), n_rows, nnz, _ptr(offsets), _ptr(nbr), _ptr(shift))
    assert nnz2 == nnz
    out = {"offsets": offsets, "nbr": nbr[:nnz], "shift": shift[:nnz]}
    if rows is not None:
        out["rows"] = np.asarray(rows, np.int64)
    return out


def neighbors_brute(sys, cutoff, rows=None, extra_images=0):
    """Brute-force neighbor list (all atoms x all images in range)."""
    return _neighbors(lib().nnref_neighbors_brute, sys, cutoff, rows, int(extra_images))


def neighbors_cells(sys, cutoff, rows=None):
    """Cell-binned neighbor list: same set and row order as the brute force."""
    return _neighbors(lib().nnref_neighbors_cells, sys, cutoff, rows, None)


def descriptors(params, sys, nl, jacobian=False):
    """G[n_rows][D] (and dG[nnz][D][3] = dG_row/d(d_e) if jacobian)."""
    keep = _Keep()
    cp, cs, cn = _c_params(params, keep), _c_system(sys, keep), _c_nlist(nl, keep)
    D = descriptor_dim(params.n_species, params.n_rad, params.n_theta, params.n_rs_ang)
    n_rows = len(nl["offsets"]) - 1
    G = np.zeros((n_rows, D))
    dG = np.zeros((len(nl["nbr"]), D, 3)) if jacobian else None
    lib().nnref_descriptors(C.byref(cp), C.byref(cs), C.byref(cn), _ptr(G), _ptr(dG))
    return (G, dG) if jacobian else G


def mlp(model, species, G, backward=True):
    """Per-atom energies E[n] and (optionally) lambda = dE/dG [n][D]."""
    keep = _Keep()
    cm, _ = _c_model(model, keep)
    G = keep(G, np.float64)
    sp = keep(species, np.int32)
    E = np.zeros(G.shape[0])
    lam = np.zeros_like(G) if backward else None
    lib().nnref_mlp(C.byref(cm), G.shape[0], _ptr(sp), _ptr(G), G.shape[1], _ptr(E), _ptr(lam))
    return (E, lam) if backward else E


def atom_energies(params, model, sys, nl, pair_grads=False):
    """E for each row atom, and (optionally) dE_i/dd_e for every entry e."""
    keep = _Keep()
    cp, cm, cs, cn = _c_params(params, keep), _c_model(model, keep)[0], _c_system(sys, keep), _c_nlist(nl, keep)
    E = np.zeros(len(nl["offsets"]) - 1)
    pg = np.zeros((len(nl["nbr"]), 3)) if pair_grads else None
    lib().nnref_atom_energies(C.byref(cp), C.byref(cm), C.byref(cs), C.byref(cn), _ptr(E), _ptr(pg))
    return (E, pg) if pair_grads else E


def forces(params, model, sys, nl, targets):
    """Forces on target atoms; nl must hold the rows of targets and their neighbors."""
    keep = _Keep()
    cp, cm, cs, cn = _c_params(params, keep), _c_model(model, keep)[0], _c_system(sys, keep), _c_nlist(nl, keep)
    t = keep(targets, np.int64)
    E = np.zeros(len(nl["offsets"]) - 1)
    F = np.zeros((t.size, 3))
    lib().nnref_forces(C.byref(cp), C.byref(cm), C.byref(cs), C.byref(cn), _ptr(t), t.size, _ptr(E), _ptr(F))
    return E, F


def energy_forces(params, model, sys, nl):
    """Full evaluation: (E_struct[B], E_atom[N], F[N][3]); nl must cover all atoms."""
    keep = _Keep()
    cp, cm, cs, cn = _c_params(params, keep), _c_model(model, keep)[0], _c_system(sys, keep), _c_nlist(nl, keep)
    N, B = sys.pos.shape[0], len(sys.atom_ptr) - 1
    Es, Ea, F = np.zeros(B), np.zeros(N), np.zeros((N, 3))
    lib().nnref_energy_forces(C.byref(cp), C.byref(cm), C.byref(cs), C.byref(cn), _ptr(Es), _ptr(Ea), _ptr(F))
    return Es, Ea, F


def energy_loss_grad(params, model, sys, nl, targets):
    """(L, E_struct, flat dL/dparams) for L = mean_c (E_c - T_c)^2."""
    keep = _Keep()
    cp, cs, cn = _c_params(params, keep), _c_system(sys, keep), _c_nlist(nl, keep)
    cm, n_params = _c_model(model, keep)
    T = keep(targets, np.float64)
    Es = np.zeros(len(sys.atom_ptr) - 1)
    dp = np.zeros(n_params)
    L = lib().nnref_energy_loss_grad(C.byref(cp), C.byref(cm), C.byref(cs), C.byref(cn), _ptr(T), _ptr(Es),
                                     _ptr(dp), n_params)
    return L, Es, dp


def descriptor_tangent(params, sys, nl, v):
    """u[rows][D]: derivative of each row atom's descriptor along the
    displacement field v [N][3] (sum over atoms k of dG_i/dx_k . v_k)."""
    keep = _Keep()
    cp, cs, cn = _c_params(params, keep), _c_system(sys, keep), _c_nlist(nl, keep)
    V = keep(np.asarray(v, np.float64).reshape(-1, 3), np.float64)
    D = descriptor_dim(params.n_species, params.n_rad, params.n_theta, params.n_rs_ang)
    u = np.zeros((cn.n_rows, D))
    lib().nnref_descriptor_tangent(C.byref(cp), C.byref(cs), C.byref(cn), _ptr(V), _ptr(u))
    return u


def force_loss_grad(params, model, sys, nl, gE=None, gF=None):
    """Flat dL/dparams for upstream gradients gE [B] = dL/dE_c and gF [N][3] =
    dL/dF_k (either may be None)."""
    keep = _Keep()
    cp, cs, cn = _c_params(params, keep), _c_system(sys, keep), _c_nlist(nl, keep)
    cm, n_params = _c_model(model, keep)
    E = None if gE is None else keep(np.asarray(gE, np.float64), np.float64)
    Fv = None if gF is None else keep(np.asarray(gF, np.float64).reshape(-1, 3), np.float64)
    dp = np.zeros(n_params)
    lib().nnref_force_loss_grad(C.byref(cp), C.byref(cm), C.byref(cs), C.byref(cn), _ptr(E), _ptr(Fv), _ptr(dp),
                                n_params)
    return dp


def unflatten_grads(model, flat):
    """Split a flat parameter-gradient vector into per-species [(dW_l, db_l), ...]."""
    out, off = [], 0
    for widths, acts, Ws, bs in model:
        layers = []
        for W, b in zip(Ws, bs):
            dW = flat[off:off + W.size].reshape(W.shape)
            off += W.size
            db = flat[off:off + b.size].copy()
            off += b.size
            layers.append((dW, db))
        out.append(layers)
    return out


def loss(atom_ptr, E, E_ref, F=None, F_ref=None, energy_kind="quad", force_kind="quad", per_atom=False,
         energy_weight=1.0, force_weight=1.0):
    """Loss of Sec. II.A (energy and force errors with a relative weight, each
    a quadratic or exponential function of the difference, energies per
    configuration or per atom), with its derivatives:
        L = w_E mean_c l_E(dE_c) + w_F mean_(k,a) l_F(F_ka - F*_ka),
        dE_c = E_c - T_c  or  (E_c - T_c) / N_c,  l(x) = x^2 or exp(x^2) - 1.
    Returns (L, dL/dE [B], dL/dF [N][3] or None)."""
    def term(kind, x):
        if kind == "exp":
            return np.exp(x * x) - 1.0, 2.0 * x * np.exp(x * x)
        return x * x, 2.0 * x
    E = np.asarray(E, np.float64)
    n = np.diff(np.asarray(atom_ptr, np.int64)).astype(np.float64)
    scale = 1.0 / np.maximum(n, 1.0) if per_atom else np.ones_like(E)
    B = E.size
    lE, dE = term(energy_kind, (E - np.asarray(E_ref, np.float64)) * scale)
    L = energy_weight / B * lE.sum()
    dL_dE = energy_weight / B * dE * scale
    dL_dF = None
    if F is not None:
        d = np.asarray(F, np.float64) - np.asarray(F_ref, np.float64)
        lF, dF = term(force_kind, d)
        L += force_weight / d.size * lF.sum()
        dL_dF = force_weight / d.size * dF
    return L, dL_dE, dL_dF


# (eV / Angstrom) / amu in Angstrom / fs^2: eV = 1.602176634e-19 J,
# amu = 1.66053906660e-27 kg, Angstrom^2 / fs^2 = 1e10 m^2 / s^2
ACCEL = 1.602176634e-19 / 1.66053906660e-27 / 1e10


class _Sys:
    def __init__(self, pos, species, atom_ptr, cell, pbc):
        self.pos, self.species, self.atom_ptr, self.cell, self.pbc = pos, species, atom_ptr, cell, pbc


def md_langevin(params, model, sys, vel, inv_mass, dt, friction, kT, noise, n_steps, cutoff=None):
    """Langevin dynamics on the potential, as in the repeated evaluation of
    Table II (Sec. III.B), by the BAOAB splitting (Leimkuhler and Matthews,
    2013): per step
        v += dt/2 F/m;  x += dt/2 v;  v = c1 v + c2 sqrt(kT/m) xi;  x += dt/2 v;
        F = F(x) (fresh cell list at `cutoff`, default rc);  v += dt/2 F/m,
    with c1 = exp(-friction dt), c2 = sqrt(1 - c1^2), xi = noise[step].
    Units: Angstrom, fs, eV, amu.  Returns (x, v, F, E_pot [n_steps][B])."""
    x = np.array(sys.pos, np.float64, copy=True).reshape(-1, 3)
    v = np.array(vel, np.float64, copy=True).reshape(-1, 3)
    a = (np.asarray(inv_mass, np.float64) * ACCEL)[:, None]
    rc = params.rc if cutoff is None else cutoff

    def eval_at(xx):
        s = _Sys(xx, sys.species, sys.atom_ptr, sys.cell, sys.pbc)
        E, _, F = energy_forces(params, model, s, neighbors_cells(s, rc))
        return E, F

    _, F = eval_at(x)
    c1 = np.exp(-friction * dt)
    c2 = np.sqrt(max(0.0, 1.0 - c1 * c1))
    sigma = np.sqrt(kT * a)
    E_pot = []
    for n in range(n_steps):
        v = v + 0.5 * dt * a * F
        x = x + 0.5 * dt * v
        xi = np.asarray(noise[n], np.float64).reshape(-1, 3) if friction > 0 else 0.0
        v = c1 * v + c2 * sigma * xi
        x = x + 0.5 * dt * v
        E, F = eval_at(x)
        v = v + 0.5 * dt * a * F
        E_pot.append(E)
    return x, v, F, np.array(E_pot).reshape(n_steps, -1)


def num_threads() -> int:
    return int(lib().nnref_num_threads())
