"""ctypes binding of libnnpot (include/nnpot.h).

The functions nn_* below have the names and arguments of the C ABI; they only
marshal arguments.  Device memory comes from torch tensors on the current HIP
device and work is enqueued on torch's current stream.  `Potential` bundles
the buffers one evaluation needs.  There is no fallback: if libnnpot.so is
missing, or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnnpot.so")

NN_MAX_SPECIES = 8
NN_MAX_LAYERS = 4
NN_BF16_MLP = 1
NN_STORE_JACOBIAN = 2
NN_BF16X3_MLP = 4
NN_REUSE_DESCRIPTORS = 8
NN_DESC_MBP = 0
NN_DESC_BP = 1
NN_LOSS_QUAD = 0
NN_LOSS_EXP = 1
ACT = {"linear": 0, "gaussian": 1, "relu": 2, "tanh": 3}
STATUS = {0: "NN_OK", 1: "NN_E_INVALID", 2: "NN_E_CAPACITY", 3: "NN_E_CELL", 4: "NN_E_WORKSPACE",
          5: "NN_E_UNSUPPORTED", 6: "NN_E_HIP", 7: "NN_E_DEVICE"}
STATUS_CODE = {v: k for k, v in STATUS.items()}


class NNError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class nn_system(C.Structure):
    _fields_ = [("n_atoms", C.c_int64), ("n_structs", C.c_int32), ("pos", C.c_void_p), ("species", C.c_void_p),
                ("atom_ptr", C.c_void_p), ("cell", C.c_void_p), ("pbc", C.c_void_p)]


class nn_nlist(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("offsets", C.c_void_p), ("nbr", C.c_void_p), ("shift", C.c_void_p),
                ("rev", C.c_void_p), ("ref_pos", C.c_void_p), ("meta", C.c_void_p), ("order", C.c_void_p),
                ("radius", C.c_double)]


class nn_mbp_params(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("rc", C.c_double), ("n_rad", C.c_int32), ("eta_rad", C.c_double),
                ("rs_rad", C.c_void_p), ("n_theta", C.c_int32), ("theta_s", C.c_void_p), ("n_rs_ang", C.c_int32),
                ("eta_ang", C.c_double), ("rs_ang", C.c_void_p), ("zeta", C.c_double), ("eps", C.c_double),
                ("kind", C.c_int32), ("bp_zeta", C.c_void_p), ("bp_lambda", C.c_void_p), ("bp_eta", C.c_void_p)]


class nn_mlp(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("width", C.c_int32 * (NN_MAX_LAYERS + 1)),
                ("act", C.c_int32 * NN_MAX_LAYERS), ("W", C.c_void_p * NN_MAX_LAYERS),
                ("b", C.c_void_p * NN_MAX_LAYERS)]


class nn_model(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("mlp", nn_mlp * NN_MAX_SPECIES)]


class nn_loss_params(C.Structure):
    _fields_ = [("energy_kind", C.c_int32), ("force_kind", C.c_int32), ("per_atom", C.c_int32),
                ("energy_weight", C.c_double), ("force_weight", C.c_double)]


class nn_qeq_params(C.Structure):
    _fields_ = [("sigma", C.c_void_p), ("coulomb", C.c_double)]


class nn_langevin(C.Structure):
    _fields_ = [("dt", C.c_double), ("friction", C.c_double), ("kT", C.c_double)]


_lib = None
EXPORTS = ("nn_descriptor_dim", "nn_workspace_size", "nn_count_neighbors", "nn_build_neighbors", "nn_descriptors",
           "nn_energy_forces", "nn_energy_forces_noalloc", "nn_energy_forces_grad", "nn_energy_forces_qeq",
           "nn_energy_forces_qeq_grad", "nn_descriptor_tangent", "nn_md_langevin", "nn_loss", "nn_autotune", "nn_autotune_reset",
           "nn_launch_plan", "nn_check",
           "nn_last_error", "nn_timing", "nn_timing_read",
           "nn_jacobian_stride")
STAGES = ("neighbors", "species", "weights", "desc_fwd", "mlp", "energy", "desc_adj", "force_gather", "desc_jac",
          "jac_contract")


def lib():
    """Open libnnpot.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_11805_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, SZ, D = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
        L.nn_descriptor_dim.restype = I64
        L.nn_descriptor_dim.argtypes = [P]
        L.nn_workspace_size.restype = I32
        L.nn_workspace_size.argtypes = [I64, I32, I64, P, P, I32, SZ, C.POINTER(SZ)]
        L.nn_count_neighbors.restype = I32
        L.nn_count_neighbors.argtypes = [P, D, C.POINTER(I64), P, SZ, P]
        L.nn_build_neighbors.restype = I32
        L.nn_build_neighbors.argtypes = [P, D, D, P, P, SZ, P]
        L.nn_descriptors.restype = I32
        L.nn_descriptors.argtypes = [P, P, P, P, P, P, SZ, P]
        L.nn_energy_forces.restype = I32
        L.nn_energy_forces.argtypes = [P, P, P, P, I32, SZ, P, P, P, P, SZ, P]
        L.nn_energy_forces_noalloc.restype = I32
        L.nn_energy_forces_noalloc.argtypes = [P, P, P, P, I32, P, P, P, P]
        L.nn_energy_forces_qeq.restype = I32
        L.nn_energy_forces_qeq.argtypes = [P, P, P, P, P, P, P, P, P, P, SZ, P]
        L.nn_energy_forces_qeq_grad.restype = I32
        L.nn_energy_forces_qeq_grad.argtypes = [P, P, P, P, P, P, P, P, SZ, P]
        L.nn_descriptor_tangent.restype = I32
        L.nn_descriptor_tangent.argtypes = [P, P, P, P, P, P]
        L.nn_md_langevin.restype = I32
        L.nn_md_langevin.argtypes = [P, P, P, P, P, C.c_double, C.c_double, P, P, I32, P, P, I32, P, P, P, SZ, P]
        L.nn_loss.restype = I32
        L.nn_loss.argtypes = [P, P, P, P, P, P, P, P, P, P, SZ, P]
        L.nn_energy_forces_grad.restype = I32
        L.nn_energy_forces_grad.argtypes = [P, P, P, P, I32, P, P, P, P, P, P, P, SZ, P]
        L.nn_autotune.restype = I32
        L.nn_autotune.argtypes = [P, P, P, P, I32, P, SZ, P, P]
        L.nn_autotune_reset.restype = None
        L.nn_autotune_reset.argtypes = []
        L.nn_launch_plan.restype = I32
        L.nn_launch_plan.argtypes = [P, P, P, P, I32, P]
        L.nn_check.restype = I32
        L.nn_check.argtypes = [P, P, C.POINTER(I64)]
        L.nn_last_error.restype = C.c_char_p
        L.nn_last_error.argtypes = []
        L.nn_jacobian_stride.restype = I64
        L.nn_jacobian_stride.argtypes = [P]
        L.nn_timing.restype = I32
        L.nn_timing.argtypes = [I32]
        L.nn_timing_read.restype = I32
        L.nn_timing_read.argtypes = [P, P]
        _lib = L
    return _lib


def _ok(status: int):
    if status != 0:
        raise NNError(status, lib().nn_last_error().decode())


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# the C entry points, same names
# ---------------------------------------------------------------------------

def nn_descriptor_dim(params: nn_mbp_params) -> int:
    return int(lib().nn_descriptor_dim(C.byref(params)))


def nn_workspace_size(n_atoms, n_structs, capacity, params=None, model=None, flags=0, mem_budget=0) -> int:
    out = C.c_size_t(0)
    _ok(lib().nn_workspace_size(n_atoms, n_structs, capacity, C.byref(params) if params else None,
                                C.byref(model) if model else None, flags, mem_budget, C.byref(out)))
    return int(out.value)


def nn_count_neighbors(sys: nn_system, radius: float, ws, stream=None) -> int:
    n = C.c_int64(0)
    _ok(lib().nn_count_neighbors(C.byref(sys), radius, C.byref(n), _p(ws), ws.numel(), _stream(stream)))
    return int(n.value)


def nn_build_neighbors(sys: nn_system, rc: float, skin: float, nl: nn_nlist, ws, stream=None):
    _ok(lib().nn_build_neighbors(C.byref(sys), rc, skin, C.byref(nl), _p(ws), ws.numel(), _stream(stream)))


def nn_descriptors(sys, nl, params, G, jac, ws, stream=None):
    _ok(lib().nn_descriptors(C.byref(sys), C.byref(nl), C.byref(params), _p(G), _p(jac), _p(ws),
                             0 if ws is None else ws.numel(), _stream(stream)))


def nn_descriptor_tangent(sys, nl, params, v, U, stream=None):
    _ok(lib().nn_descriptor_tangent(C.byref(sys), C.byref(nl), C.byref(params), _p(v), _p(U), _stream(stream)))


def nn_energy_forces(sys, nl, params, model, flags, mem_budget, E_struct, E_atom, F, ws, stream=None):
    _ok(lib().nn_energy_forces(C.byref(sys), C.byref(nl), C.byref(params), C.byref(model), flags, mem_budget,
                               _p(E_struct), _p(E_atom), _p(F), _p(ws), ws.numel(), _stream(stream)))


def nn_energy_forces_noalloc(sys, nl, params, model, flags, E_struct, E_atom, F, stream=None):
    _ok(lib().nn_energy_forces_noalloc(C.byref(sys), C.byref(nl), C.byref(params), C.byref(model), flags,
                                       _p(E_struct), _p(E_atom), _p(F), _stream(stream)))


def nn_energy_forces_qeq(sys, nl, params, model, qp, total_charge, E_struct, charges, F, ws, stream=None):
    _ok(lib().nn_energy_forces_qeq(C.byref(sys), C.byref(nl), C.byref(params), C.byref(model), C.byref(qp),
                                   _p(total_charge), _p(E_struct), _p(charges), _p(F), _p(ws), ws.numel(),
                                   _stream(stream)))


def nn_energy_forces_qeq_grad(sys, nl, params, model, dL_dE, dW, db, ws, stream=None):
    _ok(lib().nn_energy_forces_qeq_grad(C.byref(sys), C.byref(nl), C.byref(params), C.byref(model), _p(dL_dE),
                                        _ptr_table(dW), _ptr_table(db), _p(ws), ws.numel(), _stream(stream)))


def _ptr_table(tensors):
    """[species][layer] tensors (or None) -> C array of NN_MAX_SPECIES*NN_MAX_LAYERS device pointers."""
    if tensors is None:
        return None
    arr = (C.c_void_p * (NN_MAX_SPECIES * NN_MAX_LAYERS))()
    for s, layers in enumerate(tensors):
        for l, t in enumerate(layers):
            arr[s * NN_MAX_LAYERS + l] = None if t is None else t.data_ptr()
    return arr


def nn_energy_forces_grad(sys, nl, params, model, flags, dL_dE, dL_dF, F, dL_dpos, dW, db, ws, stream=None):
    """dW, db: [species][layer] lists of FP32 device tensors (or None);
    dL_dE [B] FP64, dL_dF [N, 3] FP32 (either may be None)."""
    _ok(lib().nn_energy_forces_grad(C.byref(sys), C.byref(nl), C.byref(params), C.byref(model), flags, _p(dL_dE),
                                    _p(dL_dF), _p(F), _p(dL_dpos), _ptr_table(dW), _ptr_table(db), _p(ws),
                                    ws.numel(), _stream(stream)))


def nn_md_langevin(sys, pos, vel, inv_mass, nl, rc, skin, params, model, flags, lp, noise, n_steps, E_pot, F, ws,
                   stream=None):
    _ok(lib().nn_md_langevin(C.byref(sys), _p(pos), _p(vel), _p(inv_mass), C.byref(nl), float(rc), float(skin),
                             C.byref(params), C.byref(model), flags, C.byref(lp), _p(noise), int(n_steps), _p(E_pot),
                             _p(F), _p(ws), ws.numel(), _stream(stream)))


def nn_loss(sys, lp, E, E_ref, F, F_ref, L, dL_dE, dL_dF, ws, stream=None):
    _ok(lib().nn_loss(C.byref(sys), C.byref(lp), _p(E), _p(E_ref), _p(F), _p(F_ref), _p(L), _p(dL_dE), _p(dL_dF),
                      _p(ws), ws.numel(), _stream(stream)))


def nn_autotune(sys, nl, params, model, flags, ws, stream=None) -> tuple:
    """Times the launch variants and stores the fastest plan for this shape
    class; returns (waves/atom forward, waves/atom adjoint, waves/MLP tile)."""
    plan = (C.c_int32 * 3)()
    _ok(lib().nn_autotune(C.byref(sys), C.byref(nl), C.byref(params), C.byref(model), flags, _p(ws), ws.numel(),
                          _stream(stream), plan))
    return tuple(int(v) for v in plan)


def nn_autotune_reset():
    lib().nn_autotune_reset()


def nn_launch_plan(sys, nl, params, model, flags) -> tuple:
    """The plan nn_energy_forces would use (forced, tuned or cached, else
    the fixed rules): (waves/atom forward, waves/atom adjoint, waves/MLP tile)."""
    plan = (C.c_int32 * 3)()
    _ok(lib().nn_launch_plan(C.byref(sys), C.byref(nl), C.byref(params), C.byref(model), flags, plan))
    return tuple(int(v) for v in plan)


def nn_check(nl: nn_nlist, stream=None) -> int:
    info = C.c_int64(0)
    st = lib().nn_check(C.byref(nl), _stream(stream), C.byref(info))
    if st != 0:
        raise NNError(st, lib().nn_last_error().decode())
    return int(info.value)


def nn_last_error() -> str:
    return lib().nn_last_error().decode()


def nn_jacobian_stride(params: nn_mbp_params) -> int:
    return int(lib().nn_jacobian_stride(C.byref(params)))


def nn_timing(enable: bool):
    _ok(lib().nn_timing(1 if enable else 0))


def nn_timing_read() -> dict:
    """{stage: (total ms, launches)} since the last nn_timing(True)."""
    ms = (C.c_double * len(STAGES))()
    n = (C.c_int64 * len(STAGES))()
    _ok(lib().nn_timing_read(ms, n))
    return {name: (ms[k], n[k]) for k, name in enumerate(STAGES)}


# ---------------------------------------------------------------------------
# device buffers for one system
# ---------------------------------------------------------------------------

@dataclass
class DeviceModel:
    struct: nn_model
    tensors: list  # keeps the FP32 weight tensors alive
    grads: Optional[list] = None


def make_params(p) -> tuple:
    """nn_mbp_params from an object with the descriptor hyperparameters
    (host arrays are kept alive in the returned tuple); p.kind = 1 selects
    the standard BP angular term with p.bp_zeta, p.bp_lambda, p.bp_eta."""
    rs_rad = np.ascontiguousarray(p.rs_rad, np.float64)
    if int(getattr(p, "kind", 0)) == NN_DESC_BP:
        bz = np.ascontiguousarray(p.bp_zeta, np.float64)
        bl = np.ascontiguousarray(p.bp_lambda, np.float64)
        be = np.ascontiguousarray(p.bp_eta, np.float64)
        s = nn_mbp_params(p.n_species, p.rc, rs_rad.size, p.eta_rad, rs_rad.ctypes.data, bz.size, None, be.size,
                          0.0, None, 0.0, 0.0, NN_DESC_BP, bz.ctypes.data, bl.ctypes.data, be.ctypes.data)
        return s, (rs_rad, bz, bl, be)
    th = np.ascontiguousarray(p.theta_s, np.float64)
    rs_ang = np.ascontiguousarray(p.rs_ang, np.float64)
    s = nn_mbp_params(p.n_species, p.rc, rs_rad.size, p.eta_rad, rs_rad.ctypes.data, th.size, th.ctypes.data,
                      rs_ang.size, p.eta_ang, rs_ang.ctypes.data, p.zeta, p.eps, NN_DESC_MBP, None, None, None)
    return s, (rs_rad, th, rs_ang)


def make_model(model, device="cuda") -> DeviceModel:
    """Upload per-species (widths, acts, [W], [b]) FP64 host weights as FP32."""
    import torch
    m = nn_model()
    m.n_species = len(model)
    keep = []
    for s, (widths, acts, Ws, bs) in enumerate(model):
        q = m.mlp[s]
        q.n_layers = len(Ws)
        for l, w in enumerate(widths):
            q.width[l] = int(w)
        for l, a in enumerate(acts):
            q.act[l] = ACT[a] if isinstance(a, str) else int(a)
        for l, (W, b) in enumerate(zip(Ws, bs)):
            tw = torch.tensor(np.asarray(W, np.float32), device=device).contiguous()
            tb = torch.tensor(np.asarray(b, np.float32), device=device).contiguous()
            keep += [tw, tb]
            q.W[l] = tw.data_ptr()
            q.b[l] = tb.data_ptr()
    return DeviceModel(m, keep)


class Potential:
    """Device-side buffers for evaluating one system: positions, list,
    workspace and outputs.  All compute runs in libnnpot."""

    def __init__(self, system, params, model=None, capacity: Optional[int] = None, skin: float = 0.0,
                 capacity_margin: float = 1.25, flags: int = 0, mem_budget: int = 0, device="cuda"):
        import torch
        lib()
        self.torch = torch
        self.dev = torch.device(device)
        self.N, self.B = system.n_atoms, system.n_structs
        self.params_host = params
        self.params, self._keep_params = make_params(params)
        self.D = nn_descriptor_dim(self.params)
        if self.D < 0:
            raise NNError(1, nn_last_error())
        self.rc, self.skin, self.flags, self.mem_budget = float(params.rc), float(skin), flags, int(mem_budget)
        t = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=self.dev)
        self.pos = t(system.pos, torch.float64)
        self.species = t(system.species, torch.int32)
        self.atom_ptr = t(system.atom_ptr, torch.int64)
        self.cell = t(np.asarray(system.cell, np.float64).reshape(-1, 9), torch.float64)
        self.pbc = t(np.asarray(system.pbc, np.uint8).reshape(-1, 3), torch.uint8)
        self.sys = nn_system(self.N, self.B, self.pos.data_ptr(), self.species.data_ptr(), self.atom_ptr.data_ptr(),
                             self.cell.data_ptr(), self.pbc.data_ptr())
        self.dmodel = make_model(model, device) if model is not None else None
        ws0 = nn_workspace_size(self.N, self.B, 0)
        self.ws = torch.empty(ws0, dtype=torch.uint8, device=self.dev)
        if capacity is None:
            n = nn_count_neighbors(self.sys, self.rc + self.skin, self.ws)
            capacity = int(n * capacity_margin) + 64
        self.capacity = int(capacity)
        z = lambda n, dt: torch.zeros(n, dtype=dt, device=self.dev)
        self.offsets = z(self.N + 1, torch.int64)
        self.nbr = z(self.capacity, torch.int32)
        self.shift = z((self.capacity, 4), torch.int8)
        self.rev = z(self.capacity, torch.int32)
        self.ref_pos = z((self.N, 3), torch.float64)
        self.meta = z(8, torch.int64)
        self.order = z(max(self.N, 1), torch.int32)
        self.nl = nn_nlist(self.capacity, self.offsets.data_ptr(), self.nbr.data_ptr(), self.shift.data_ptr(),
                           self.rev.data_ptr(), self.ref_pos.data_ptr(), self.meta.data_ptr(),
                           self.order.data_ptr(), 0.0)
        ws = nn_workspace_size(self.N, self.B, self.capacity, self.params,
                               self.dmodel.struct if self.dmodel else None, flags, self.mem_budget)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=self.dev)
        self.E_struct = z(self.B, torch.float64)
        self.E_atom = z(self.N, torch.float32)
        self.F = z((self.N, 3), torch.float32)
        self.G = None
        # calls through this object that replace the state a backward pass
        # reads (list, workspace descriptors, forces); autograd checks it
        self.evals = 0

    def set_positions(self, pos):
        self.pos.copy_(self.torch.as_tensor(pos, dtype=self.torch.float64))

    def build_neighbors(self, check: bool = True):
        self.evals += 1
        nn_build_neighbors(self.sys, self.rc, self.skin, self.nl, self.ws)
        if check:
            nn_check(self.nl)

    def descriptors(self):
        if self.G is None:
            self.G = self.torch.zeros((self.N, self.D), dtype=self.torch.float32, device=self.dev)
        nn_descriptors(self.sys, self.nl, self.params, self.G, None, self.ws)
        return self.G

    def descriptor_tangent(self, v):
        """U [N, D]: derivative of the descriptors along the displacement field v [N, 3]."""
        torch = self.torch
        v = torch.as_tensor(v, dtype=torch.float32, device=self.dev).reshape(self.N, 3).contiguous()
        U = torch.zeros((self.N, self.D), dtype=torch.float32, device=self.dev)
        nn_descriptor_tangent(self.sys, self.nl, self.params, v, U)
        return U

    def md_langevin(self, n_steps, vel, inv_mass, dt, friction, kT, noise=None, E_pot=None,
                    flags: Optional[int] = None):
        """n_steps of BAOAB Langevin dynamics in place on self.pos / vel
        (FP64 [N, 3], Angstrom/fs), with inv_mass FP64 [N] (1/amu), dt in fs,
        friction in 1/fs, kT in eV and noise FP32 [n_steps, N, 3] standard
        normal draws.  self.F must hold the forces at the current positions
        (energy_forces() or the previous call) and holds those at the new
        ones on return.  Returns E_pot [n_steps, B] (FP64)."""
        torch = self.torch
        f = self.flags if flags is None else flags
        if E_pot is None:
            E_pot = torch.empty((max(int(n_steps), 1), self.B), dtype=torch.float64, device=self.dev)
        lp = nn_langevin(float(dt), float(friction), float(kT))
        self.evals += 1
        nn_md_langevin(self.sys, self.pos, vel, inv_mass, self.nl, self.rc, self.skin, self.params,
                       self.dmodel.struct, f, lp, noise, n_steps, E_pot, self.F, self.ws)
        return E_pot

    def loss(self, E_ref, F_ref=None, energy_kind=NN_LOSS_QUAD, force_kind=NN_LOSS_QUAD, per_atom=False,
             energy_weight=1.0, force_weight=1.0, E=None, F=None):
        """(L [1], dL/dE [B], dL/dF [N, 3] or None) of the loss of Sec. II.A on
        E (default self.E_struct) and F (default self.F) against the targets."""
        torch = self.torch
        E = self.E_struct if E is None else E
        E_ref = torch.as_tensor(E_ref, dtype=torch.float64, device=self.dev).contiguous()
        if F_ref is not None:
            F = self.F if F is None else F
            F_ref = torch.as_tensor(F_ref, dtype=torch.float32, device=self.dev).reshape(self.N, 3).contiguous()
        else:
            F = None
        L = torch.empty(1, dtype=torch.float64, device=self.dev)
        dE = torch.empty(self.B, dtype=torch.float64, device=self.dev)
        dF = torch.empty((self.N, 3), dtype=torch.float32, device=self.dev) if F_ref is not None else None
        lp = nn_loss_params(int(energy_kind), int(force_kind), int(bool(per_atom)), float(energy_weight),
                            float(force_weight))
        nn_loss(self.sys, lp, E, E_ref, F, F_ref, L, dE, dF, self.ws)
        return L, dE, dF

    def autotune(self, flags: Optional[int] = None):
        """nn_autotune on the current list (build it first)."""
        f = self.flags if flags is None else flags
        self.evals += 1
        return nn_autotune(self.sys, self.nl, self.params, self.dmodel.struct, f, self.ws)

    def launch_plan(self, flags: Optional[int] = None):
        """The plan energy_forces would use now (nn_launch_plan)."""
        f = self.flags if flags is None else flags
        return nn_launch_plan(self.sys, self.nl, self.params, self.dmodel.struct, f)

    def energy_forces(self, flags: Optional[int] = None, forces: bool = True, mem_budget: Optional[int] = None):
        f = self.flags if flags is None else flags
        b = self.mem_budget if mem_budget is None else int(mem_budget)
        self.evals += 1
        nn_energy_forces(self.sys, self.nl, self.params, self.dmodel.struct, f, b, self.E_struct,
                         self.E_atom, self.F if forces else None, self.ws)
        return self.E_struct, self.E_atom, self.F

    def energy_forces_qeq(self, total_charge, sigma, coulomb=14.399645, forces: bool = True):
        """(E_struct [B] FP64, charges [N] FP64, F [N, 3] FP32) with charge
        equilibration (Sec. II.B): the model's networks have three outputs per
        atom; sigma [S] are the species' Gaussian charge widths."""
        torch = self.torch
        Qt = torch.as_tensor(total_charge, dtype=torch.float64, device=self.dev).contiguous()
        sig = np.ascontiguousarray(sigma, np.float64)
        qp = nn_qeq_params(sig.ctypes.data, float(coulomb))
        q = torch.empty(self.N, dtype=torch.float64, device=self.dev)
        self.evals += 1
        nn_energy_forces_qeq(self.sys, self.nl, self.params, self.dmodel.struct, qp, Qt, self.E_struct, q,
                             self.F if forces else None, self.ws)
        return self.E_struct, q, self.F

    def grad_qeq(self, dL_dE):
        """[species][layer] (dW, db) of a loss on the energies of the last
        energy_forces_qeq() call."""
        torch = self.torch
        dL_dE = torch.as_tensor(dL_dE, dtype=torch.float64, device=self.dev).contiguous()
        dW, db = [], []
        it = iter(self.dmodel.tensors)
        for s in range(self.dmodel.struct.n_species):
            L = self.dmodel.struct.mlp[s].n_layers
            ws_, bs_ = [], []
            for _ in range(L):
                W, b = next(it), next(it)
                ws_.append(torch.empty_like(W))
                bs_.append(torch.empty_like(b))
            dW.append(ws_)
            db.append(bs_)
        nn_energy_forces_qeq_grad(self.sys, self.nl, self.params, self.dmodel.struct, dL_dE, dW, db, self.ws)
        return [list(zip(w_s, b_s)) for w_s, b_s in zip(dW, db)]

    def jacobian(self):
        """(G [N, D], J [capacity, stride]) via nn_descriptors with a Jacobian buffer."""
        js = nn_jacobian_stride(self.params)
        J = self.torch.zeros((self.capacity, js), dtype=self.torch.float32, device=self.dev)
        G = self.torch.zeros((self.N, self.D), dtype=self.torch.float32, device=self.dev)
        nn_descriptors(self.sys, self.nl, self.params, G, J, self.ws)
        return G, J

    def grad(self, dL_dE=None, flags: Optional[int] = None, positions: bool = True, weights: bool = True,
             dL_dF=None):
        """Backward of E_struct (dL_dE [B]) and F (dL_dF [N, 3]) after
        energy_forces(): (dL/dpos [N,3] or None, [species][layer] (dW, db) or
        None).  The position gradient is only available without dL_dF."""
        torch = self.torch
        f = self.flags if flags is None else flags
        if dL_dE is not None:
            dL_dE = torch.as_tensor(dL_dE, dtype=torch.float64, device=self.dev).contiguous()
        if dL_dF is not None:
            dL_dF = torch.as_tensor(dL_dF, dtype=torch.float32, device=self.dev).reshape(self.N, 3).contiguous()
        dpos = torch.zeros((self.N, 3), dtype=torch.float32, device=self.dev) if positions else None
        dW = db = None
        if weights:
            dW, db = [], []
            it = iter(self.dmodel.tensors)
            for s in range(self.dmodel.struct.n_species):
                L = self.dmodel.struct.mlp[s].n_layers
                ws_, bs_ = [], []
                for _ in range(L):
                    W, b = next(it), next(it)
                    ws_.append(torch.empty_like(W))  # every element is written
                    bs_.append(torch.empty_like(b))
                dW.append(ws_)
                db.append(bs_)
        nn_energy_forces_grad(self.sys, self.nl, self.params, self.dmodel.struct, f, dL_dE, dL_dF, self.F, dpos, dW,
                              db, self.ws)
        return dpos, ([list(zip(w_s, b_s)) for w_s, b_s in zip(dW, db)] if weights else None)

    def neighbor_list_host(self):
        """(offsets, nbr, shift[:, :3]) copied to the host (after a sync)."""
        self.torch.cuda.synchronize()
        off = self.offsets.cpu().numpy()
        nnz = int(off[-1])
        return {"offsets": off, "nbr": self.nbr[:nnz].cpu().numpy(),
                "shift": self.shift[:nnz, :3].cpu().numpy().astype(np.int32), "rev": self.rev[:nnz].cpu().numpy()}
