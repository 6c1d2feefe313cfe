#!/usr/bin/env python3
"""Energy + force throughput of the mBP / per-species MLP path on one MI355X.

One step = one pass of the whole path over the resident input.  The default
workload is the repeated evaluation at scale: a 262144-atom periodic cell
with 2 species (rho = 0.09 A^-3, Rc = 6 A, 48 radial + 8x8 angular bins, MLP
288-128-128-1) whose atoms take a random walk of N(0, 0.02 A) per component
and step.  Each step moves the atoms, tests the 0.5 A skin on the device and
rebuilds the list (cell binning, FP64 inclusion test, row sort, reverse
index) only when an atom moved farther than skin/2, then computes species
grouping, radial + angular descriptors, per-species MLP forward + backward,
FP64 per-structure energies, the descriptor adjoint and the force gather.
Inputs are synthetic and seeded and sit in HBM before the timed region;
--config k selects another workload (those without a walk rebuild the list
every step).

Prints one JSON line: atoms/s, the roofline position of the dominant kernel
(timed live with HIP events on the stream it runs on) and the FP64 oracle's
own throughput on the host cores over a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 256 CU x 4 SIMD x 32 lanes x 2 flop (FMA) x 2.4 GHz: an unpacked v_fma_f32
# retires a wave64 in 2 clocks on gfx950 (paper_2305_11805_amd/probe/issue_rates)
PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
METRIC = "energy+force atoms/sec at stated force error vs FP64 oracle; HBM GB/s"
MODE_FLAGS = {"fp32": 0, "bf16": 1, "bf16x3": 4}  # NN_BF16_MLP, NN_BF16X3_MLP


def ipow_mults(e: int) -> int:
    """Multiplications of binary exponentiation x^e (squarings + extra products)."""
    return (e.bit_length() - 1) + (bin(e).count("1") - 1) if e > 0 else 0


def flop_model(p, n_valid):
    """Algorithmic FP32 work of the two descriptor kernels (FMA = 2 flops,
    each exp2 / sqrt / reciprocal = 1): per (pair, radial bin), per triplet
    (separable angular form) and per pair."""
    NT, NR = p.n_theta, p.n_rs_ang
    P = float(np.sum(n_valid))
    T = float(np.sum(n_valid * (n_valid - 1) / 2))
    if int(getattr(p, "kind", 0)) == 1:
        # standard BP: 1 +- cos, the third side (FP64), its cutoff (sin as 15),
        # s2 and fc fc fc; per angle term (1 + lambda cos)^zeta and the
        # prefactor, per radius term exp(-eta s2) fc fc fc, two flops per bin
        zs = [int(z) for z in p.bp_zeta]
        fwd_trip = 50 + sum(ipow_mults(z) + 1 for z in zs) + 3 * NR + 2 * NT * NR
        adj_trip = 45 + sum(ipow_mults(z - 1) + 4 for z in zs) + 3 * NR + 4 * NT * NR + 4 * NR + 4 * NT + 60
        fwd = T * fwd_trip + P * p.n_rad * 8
        adj = T * adj_trip + P * (p.n_rad * 12 + 6)
        return {"pairs": P, "triplets": T, "desc_fwd": fwd, "desc_adj": adj, "desc_tan": 0.0,
                "per_triplet": {"desc_fwd": fwd_trip, "desc_adj": adj_trip, "desc_tan": 0}}
    z = int(p.zeta)
    geom = 33
    fwd_trip = geom + 4 * NT + NT * ipow_mults(z) + 7 * NR + 2 * NT * NR
    adj_trip = geom + 4 * NT + NT * ipow_mults(z - 1) + NT + 6 * NR + 4 * NT * NR + 5 * NR + 5 * NT + 35
    # tangent along a displacement field: the forward terms, their derivatives
    # (A_dot 5 per angle bin, R_dot 5 per radius bin, cos/ssm/F2/rbar dots 26)
    # and two FMAs per bin
    tan_trip = geom + 4 * NT + NT * ipow_mults(z - 1) + NT + 5 * NT + 26 + 12 * NR + 4 * NT * NR
    fwd = T * fwd_trip + P * p.n_rad * 8
    adj = T * adj_trip + P * (p.n_rad * 12 + 6)
    tan = T * tan_trip + P * (p.n_rad * 12 + 11)
    return {"pairs": P, "triplets": T, "desc_fwd": fwd, "desc_adj": adj, "desc_tan": tan,
            "per_triplet": {"desc_fwd": fwd_trip, "desc_adj": adj_trip, "desc_tan": tan_trip}}


def mlp_flops(w, n_atoms):
    """Algorithmic flops of one MLP launch (forward and backward to dE/dG):
    per atom 2 (D h1 + h1 h2 + h2) forward and 2 (h2 h1 + h1 D) backward."""
    D, h1, h2 = w.model[0][0][:3]
    return float(n_atoms) * (2 * (D * h1 + h1 * h2 + h2) + 2 * (h2 * h1 + h1 * D))


def valid_neighbor_counts(pot, rc):
    nl = pot.neighbor_list_host()
    pos = pot.pos.cpu().numpy()
    cell = pot.cell.cpu().numpy().reshape(-1, 3, 3)
    ptr = pot.atom_ptr.cpu().numpy()
    off = nl["offsets"]
    rows = np.repeat(np.arange(len(off) - 1), np.diff(off))
    struct = np.searchsorted(ptr, rows, side="right") - 1
    d = pos[nl["nbr"]] - pos[rows] + np.einsum("ek,ekl->el", nl["shift"].astype(np.float64), cell[struct])
    valid = np.sum(d * d, axis=1) < rc * rc
    return np.bincount(rows[valid], minlength=len(off) - 1)


SOURCES = {"k_desc": "descriptors.hip", "k_jac": "descriptors.hip", "k_mlp_rows_bf": "mlp_rows.hip", "k_mlp_rows": "mlp_rows.hip", "k_mlp": "mlp.hip", "k_force_gather": "descriptors.hip",
           "k_nb": "neighbors.hip"}


def mlp_rows_plan(plan, mode, w):
    """The row-block MLP kernel the timed steps run (plan value 1 on the
    widths and descriptor sizes it takes: k_mlp_rows in FP32, k_mlp_rows_bf
    in the BF16 modes), else None (the tile kernel k_mlp)."""
    if plan is None or plan[2] != 1:
        return None
    widths = w.model[0][0]
    if len(widths) != 4 or tuple(widths[1:3]) not in ((64, 32), (128, 128)):
        return None
    if mode == "fp32":
        return "k_mlp_rows" if w.params.dim % 4 == 0 else None
    return "k_mlp_rows_bf" if w.params.dim % 8 == 0 else None


def source_hash(kernel="k_desc_adj"):
    """Hash of the source file a kernel is built from and of the compiler
    flags (counter figures are used only while it matches)."""
    from paper_2305_11805_amd import build as nnbuild
    src = next(v for k, v in SOURCES.items() if kernel.startswith(k))
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2305_11805_amd", "csrc", src), "rb") as f:
        h.update(f.read())
    h.update(" ".join(a for a in nnbuild.CFLAGS if not a.startswith("/")).encode())
    return h.hexdigest()[:16]


def oracle_leg(w, target_s=15.0):
    """The FP64 oracle as it stands, on the host cores: per-atom energies and
    per-pair gradients (all of the E + F work) for the first rows of the
    workload at its input positions; if the whole workload takes less than
    target_s, it is evaluated repeatedly until about target_s."""
    import oracle
    oracle.build(force=False)
    s, p = w.system, w.params
    n = min(64, s.n_atoms)
    t0 = time.perf_counter()
    nl = oracle.neighbors_cells(s, p.rc, rows=np.arange(n))
    oracle.atom_energies(p, w.model, s, nl, pair_grads=True)
    dt = time.perf_counter() - t0
    n2 = int(min(s.n_atoms, max(n, n * target_s / max(dt, 1e-3))))
    reps = 1
    if n2 == s.n_atoms:
        reps = max(1, int(round(target_s / max(dt * s.n_atoms / n, 1e-3))))
    rows = np.arange(n2)
    t0 = time.perf_counter()
    for _ in range(reps):
        nl = oracle.neighbors_cells(s, p.rc, rows=rows)
        oracle.atom_energies(p, w.model, s, nl, pair_grads=True)
    dt = time.perf_counter() - t0
    what = f"the first {n2} of {s.n_atoms} atoms" if n2 < s.n_atoms else f"all {s.n_atoms} atoms x {reps} passes"
    return {"value": n2 * reps / dt, "unit": "atoms/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"neighbor rows + E + per-pair dE/dd of {what} (FP64, OpenMP over atoms), {dt:.1f} s"}


def sampled_force_error(w, F, n=16, seed=0, pos=None):
    """Max |F - F_oracle| over n seeded atoms, at positions pos (default:
    the workload's input positions)."""
    import oracle
    from paper_2305_11805_amd import synth
    s = w.system if pos is None else synth.System(np.asarray(pos, np.float64), w.system.species,
                                                  w.system.atom_ptr, w.system.cell, w.system.pbc)
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.sort(rng.choice(s.n_atoms, size=min(n, s.n_atoms), replace=False))
    own = oracle.neighbors_cells(s, w.params.rc, rows=t)
    rows = np.array(sorted(set(t.tolist()) | set(own["nbr"].tolist())), np.int64)
    nl = oracle.neighbors_cells(s, w.params.rc, rows=rows)
    _, F_ref = oracle.forces(w.params, w.model, s, nl, t)
    return float(np.max(np.abs(F[t] - F_ref)))


def read_pmc_csv(path, counter):
    """Per-dispatch values of one counter from a rocprofv3 counter_collection
    CSV: list of (kernel name, value)."""
    import csv
    out = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") == counter:
                out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def ingest_counters(fetch_csv, write_csv, calib_mib, workload, kernels=("k_desc_adj", "k_desc_fwd", "k_mlp_rows")):
    for k in kernels:
        ingest_kernel(fetch_csv, write_csv, calib_mib, workload, k)


def ingest_kernel(fetch_csv, write_csv, calib_mib, workload, kernel):
    """HBM bytes per launch of `kernel` from two rocprofv3 --pmc runs
    (FETCH_SIZE, WRITE_SIZE, KiB per dispatch), each scaled by the ratio of
    the known size of a plain device copy to what the counter read for it."""
    res = {}
    runs = {name: read_pmc_csv(path, name) for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv))}
    # one instantiation for both counters: of those both runs dispatched, the
    # most frequent (the timed steps run one; the launch tuner also runs the
    # others a few times each)
    names = {name: [k for k, _ in rows if f"nnp::{kernel}<" in k or f"nnp::{kernel}(" in k]
             for name, rows in runs.items()}
    both = set(names["FETCH_SIZE"]) & set(names["WRITE_SIZE"])
    if not both:
        raise SystemExit(f"no {kernel} instantiation in both counter runs")
    full = max(sorted(both), key=lambda k: names["FETCH_SIZE"].count(k) + names["WRITE_SIZE"].count(k))
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = runs[name]
        mine = [v for k, v in rows if k == full]
        copies = [v for k, v in rows if "copyBuffer" in k]
        if not copies:
            raise SystemExit(f"{path}: no copy dispatch with {name}")
        known_kib = calib_mib * 1024.0
        calib = max(copies)
        res[name] = {"kernel": full, "kib_per_launch_raw": sum(mine) / len(mine), "launches": len(mine),
                     "copy_kib_raw": calib, "copy_kib_known": known_kib, "scale": known_kib / calib}
    hbm = sum(1024.0 * r["kib_per_launch_raw"] * r["scale"] for r in res.values())
    prof = os.path.join(ROOT, "profiles", "counters.json")
    cnt = {}
    if os.path.exists(prof):
        with open(prof) as f:
            cnt = json.load(f)
    cnt[f"{kernel}:{workload}"] = {"source_hash": source_hash(kernel), "hbm_bytes_per_launch": round(hbm),
                                  "counters": res}
    with open(prof, "w") as f:
        json.dump(cnt, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(cnt[f"{kernel}:{workload}"]))


def _timed(torch, stream, fn, k):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(k):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def suite_config(idx, modes, steps, out):
    """Every workload at full size: throughput (eager step, graph replay,
    standing list) per MLP mode, errors against the FP64 oracle, the oracle's
    own throughput, and the workload-specific extras (batched vs per-structure
    launches and the loss gradient for the cluster batch, the 100-step random
    walk with skin rebuilds for the large bulk cell)."""
    import torch
    import oracle
    from paper_2305_11805_amd import nnpot, synth
    oracle.build(force=False)
    w = synth.config(idx)
    s, p = w.system, w.params
    stream = torch.cuda.current_stream()
    skin = float(w.extra.get("skin", 0.0))
    res = {"config": idx, "workload": w.name, "n_atoms": s.n_atoms, "n_structs": s.n_structs, "modes": {}}
    md = idx == 4
    if md:
        nsteps = int(w.extra["steps"])
        xi = torch.tensor(np.stack(list(synth.md_displacements(w.seed, s.n_atoms, nsteps, w.extra["step_sigma"]))),
                          dtype=torch.float64, device="cuda")
    # oracle reference (full for small workloads, seeded samples for the MD cell)
    t0 = time.perf_counter()
    if not md:
        nl_ref = oracle.neighbors_cells(s, p.rc)
        Es_ref, _, F_ref = oracle.energy_forces(p, w.model, s, nl_ref)
        t_or = time.perf_counter() - t0
        G_ref = oracle.descriptors(p, s, nl_ref)
        res["oracle"] = {"atoms_per_s": s.n_atoms / t_or, "cores": oracle.num_threads(), "seconds": round(t_or, 2),
                         "what": "full neighbor list + E + F"}
    else:
        rng = np.random.Generator(np.random.PCG64(5))
        tgt = np.sort(rng.choice(s.n_atoms, 64, replace=False))
        own = oracle.neighbors_cells(s, p.rc, rows=tgt)
        rows = np.array(sorted(set(tgt.tolist()) | set(own["nbr"].tolist())), np.int64)
        nl_s = oracle.neighbors_cells(s, p.rc, rows=rows)
        _, F0_ref = oracle.forces(p, w.model, s, nl_s, tgt)
        t_or = time.perf_counter() - t0
        res["oracle"] = {"atoms_per_s": len(tgt) / t_or, "cores": oracle.num_threads(), "seconds": round(t_or, 2),
                         "what": f"forces on 64 seeded atoms (rows of {len(rows)} atoms)"}
    n_c = np.diff(s.atom_ptr)
    for mode in modes:
        flags = {"fp32": 0, "bf16": nnpot.NN_BF16_MLP, "bf16x3": nnpot.NN_BF16X3_MLP}[mode]
        pot = nnpot.Potential(s, p, w.model, skin=skin, flags=flags, capacity_margin=1.3 if md else 1.25)
        r = {}

        def build():
            nnpot.nn_build_neighbors(pot.sys, pot.rc, pot.skin, pot.nl, pot.ws)

        def ef():
            nnpot.nn_energy_forces(pot.sys, pot.nl, pot.params, pot.dmodel.struct, flags, 0, pot.E_struct,
                                   pot.E_atom, pot.F, pot.ws)

        if not md:
            def step():
                build()
                ef()
            for _ in range(3):
                step()
            torch.cuda.synchronize()
            nnpot.nn_check(pot.nl)
            r["launch_plan"] = pot.autotune()
            ms = _timed(torch, stream, step, steps) / steps
            r["eager_step"] = {"ms": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1)}
            ms = _timed(torch, stream, ef, steps) / steps
            r["standing_list"] = {"ms": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1)}
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                step()
            torch.cuda.synchronize()
            ms = _timed(torch, stream, g.replay, steps) / steps
            r["graph_replay"] = {"ms": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1)}
            torch.cuda.synchronize()
            nnpot.nn_check(pot.nl)
            Es = pot.E_struct.cpu().numpy()
            F = pot.F.cpu().numpy()
            dE = np.abs(Es - Es_ref) / np.maximum(n_c, 1)
            dF = np.abs(F - F_ref)
            r["errors"] = {"E_per_atom_max": float(dE.max()), "E_per_atom_rms": float(np.sqrt(np.mean(dE ** 2))),
                           "F_max": float(dF.max()), "F_rms": float(np.sqrt(np.mean(dF ** 2)))}
            if mode == modes[0]:
                G = pot.descriptors().cpu().numpy().astype(np.float64)
                floor = 1e-6 * np.max(np.abs(G_ref), axis=1, keepdims=True)
                den = np.maximum(np.abs(G_ref), floor)
                err = np.abs(G - G_ref)
                # rows with no neighbors are all zero on both sides
                r["errors"]["G_max_rel"] = float(np.max(np.where(den > 0, err / np.where(den > 0, den, 1.0), err)))
        else:
            pos0 = pot.pos.clone()
            build()
            ef()
            torch.cuda.synchronize()
            nnpot.nn_check(pot.nl)
            r["launch_plan"] = pot.autotune()
            pot.meta[1] = 0  # the walk starts from a fresh list
            build()
            ef()
            torch.cuda.synchronize()
            F0 = pot.F.cpu().numpy()
            b0 = int(pot.meta[2].item())
            k = [0]

            def md_step():
                pot.pos.add_(xi[k[0]])
                k[0] += 1
                build()
                ef()
            ms = _timed(torch, stream, md_step, nsteps) / nsteps
            nnpot.nn_check(pot.nl)
            r["md_walk"] = {"steps": nsteps, "ms_per_step": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1),
                            "rebuilds": int(pot.meta[2].item()) - b0,
                            "what": "x += N(0, 0.02 A) per component, skin 0.5 A, rebuild when an atom moved > skin/2"}
            F_eager = pot.F.clone()
            # the same walk with each step replayed from a captured graph
            # (skin test, predicated rebuild, E, F); the displacement of the
            # step is copied into the graph's input buffer before each replay
            pot.pos.copy_(pos0)
            pot.meta[1] = 0
            build()
            ef()
            xi_buf = torch.zeros_like(pot.pos)
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                pot.pos.add_(xi_buf)
                build()
                ef()
            torch.cuda.synchronize()
            kg = [0]

            def md_graph_step():
                xi_buf.copy_(xi[kg[0]])
                kg[0] += 1
                g.replay()
            ms = _timed(torch, stream, md_graph_step, nsteps) / nsteps
            nnpot.nn_check(pot.nl)
            r["md_walk_graph"] = {"steps": nsteps, "ms_per_step": round(ms, 4),
                                  "atoms_per_s": round(s.n_atoms / ms * 1e3, 1),
                                  "forces_equal_eager_bitwise": bool(torch.equal(pot.F, F_eager))}
            del g
            ms = _timed(torch, stream, ef, 20) / 20
            r["standing_list"] = {"ms": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1)}
            F_end = pot.F.cpu().numpy()
            pos_end = pot.pos.cpu().numpy()
            s_end = synth.System(pos_end, s.species, s.atom_ptr, s.cell, s.pbc)
            own = oracle.neighbors_cells(s_end, p.rc, rows=tgt)
            rows = np.array(sorted(set(tgt.tolist()) | set(own["nbr"].tolist())), np.int64)
            _, F1_ref = oracle.forces(p, w.model, s_end, oracle.neighbors_cells(s_end, p.rc, rows=rows), tgt)
            r["errors"] = {"F_max_step0_sampled": float(np.max(np.abs(F0[tgt] - F0_ref))),
                           "F_max_last_step_sampled": float(np.max(np.abs(F_end[tgt] - F1_ref)))}
            pot.pos.copy_(pos0)
        res["modes"][mode] = r
        if idx == 2 and mode == modes[0]:
            # loss gradient step: E, F and dL/dW of L = mean_c (E_c - T_c)^2
            T = torch.tensor(synth.energy_targets(w.seed, s.n_structs), dtype=torch.float64, device="cuda")

            def grad_step():
                build()
                ef()
                dL = (2.0 / s.n_structs) * (pot.E_struct - T)
                pot.grad(dL, positions=False, weights=True)
            grad_step()
            ms = _timed(torch, stream, grad_step, steps) / steps
            res["loss_gradient_step"] = {"ms": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1)}
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                grad_step()
            torch.cuda.synchronize()
            g.replay()
            ms = _timed(torch, stream, g.replay, steps) / steps
            res["loss_gradient_step_graph"] = {"ms": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1)}
            del g
            # force-matching step: E, F and dL/dW of
            # L = mean_c (E_c - T_c)^2 + sum_k |F_k - F*_k|^2 / (3N)
            Ft = torch.tensor(synth.force_targets(w.seed, s.n_atoms), dtype=torch.float32, device="cuda")

            def fm_step():
                build()
                ef()
                _, dL, dF = pot.loss(T, Ft)
                pot.grad(dL, positions=False, weights=True, dL_dF=dF)
            fm_step()
            ms = _timed(torch, stream, fm_step, steps) / steps
            res["force_matching_step"] = {"ms": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1)}
            side = torch.cuda.Stream()
            side.wait_stream(stream)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                fm_step()
            torch.cuda.synchronize()
            g.replay()
            ms = _timed(torch, stream, g.replay, steps) / steps
            res["force_matching_step_graph"] = {"ms": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1)}
            del g
            # the same structures, one Potential and one launch sequence each
            sub = 64
            pots = [nnpot.Potential(synth.single(s.pos[s.atom_ptr[c]:s.atom_ptr[c + 1]],
                                                 s.species[s.atom_ptr[c]:s.atom_ptr[c + 1]],
                                                 cell=s.cell[c], pbc=s.pbc[c]), p, w.model)
                    for c in range(sub)]
            n_sub = int(s.atom_ptr[sub])

            def per_structure():
                for q in pots:
                    q.build_neighbors(check=False)
                    q.energy_forces()
            per_structure()
            ms = _timed(torch, stream, per_structure, 5) / 5
            aps = n_sub / ms * 1e3
            res["per_structure_launches"] = {"structures": sub, "atoms": n_sub, "ms": round(ms, 4),
                                             "atoms_per_s": round(aps, 1),
                                             "batched_over_per_structure": round(r["eager_step"]["atoms_per_s"] / aps, 2)}
        del pot
        torch.cuda.empty_cache()
    if len(modes) > 1:
        key = "eager_step" if not md else "md_walk"
        base = res["modes"]["fp32"][key]["atoms_per_s"]
        res["bf16_over_fp32"] = {m: round(res["modes"][m][key]["atoms_per_s"] / base, 3) for m in modes if m != "fp32"}
    out.write(json.dumps(res) + "\n")
    out.flush()
    print(json.dumps(res), flush=True)


def force_matching(args):
    """One force-matching training step per iteration on --config: list
    (re)build, E and F, the loss L = mean_c (E_c - T_c)^2 + sum_k |F_k - F*_k|^2
    / (3N) with its derivatives (nn_loss), then dL/dW (the force term through
    the descriptor tangent and the MLP's forward-mode tangent).  Every step
    runs in the library's kernels.  Prints one JSON line."""
    import torch
    from paper_2305_11805_amd import nnpot, synth
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    w = synth.config(args.config)
    s = w.system
    pot = nnpot.Potential(s, w.params, w.model, skin=float(w.extra.get("skin", 0.0)))
    T = torch.tensor(synth.energy_targets(w.seed, s.n_structs), dtype=torch.float64, device="cuda")
    Ft = torch.tensor(synth.force_targets(w.seed, s.n_atoms), dtype=torch.float32, device="cuda")

    def step():
        pot.build_neighbors(check=False)
        pot.energy_forces()
        _, dL, dF = pot.loss(T, Ft)  # nn_loss: L, dL/dE, dL/dF on the device
        pot.grad(dL, positions=False, weights=True, dL_dF=dF)
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    nnpot.nn_check(pot.nl)
    stream = torch.cuda.current_stream()
    ms = _timed(torch, stream, step, args.steps) / args.steps
    nnpot.nn_check(pot.nl)
    n_valid = valid_neighbor_counts(pot, w.params.rc)
    fm = flop_model(w.params, n_valid)
    res = {"workload": w.name, "step": "force_matching", "n_atoms": s.n_atoms, "steps": args.steps,
           "ms_per_step": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1),
           "desc_tan_flops_per_launch": fm["desc_tan"], "desc_tan_flops_per_triplet": fm["per_triplet"]["desc_tan"]}
    print(json.dumps(res), flush=True)


def md_table2(args):
    """The repeated-evaluation shape of Table II: Langevin dynamics (300 K,
    0.5 fs, friction 0.01 / fs) of 16-atom periodic carbon cells through
    nn_md_langevin, one cell and a batch of independent cells, eager and
    replayed from a HIP graph: the config-1 model, then the Carbon descriptor
    of Sec. III.B (D = 152) with each of the three Table II networks (64-32,
    256-128, 1024-512-256).  Prints one JSON line; the paper's figures
    (0.78-0.79 ms per step per atom, A100 through ASE) are context only."""
    import torch
    from paper_2305_11805_amd import nnpot, synth
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    dt, gamma, kT = 0.5, 0.01, 0.025852
    out = {"step": "langevin_md", "dt_fs": dt, "friction_per_fs": gamma, "kT_eV": kT,
           "paper_context": {"ms_per_step_per_atom": {"small": 0.78, "middle": 0.79, "big": 0.79},
                             "hardware": "A100, ASE driver"}, "runs": []}
    runs = [(None, 1, 1000), (None, args.md_cells, 200)]
    for net in ("small", "middle", "big"):  # the networks of Table II on the Sec. III.B descriptor
        runs += [(net, 1, 1000), (net, args.md_cells, 200)]
    for net, n_cells, steps in runs:
        w = synth.md_cells(n_cells, network=net)
        s = w.system
        pot = nnpot.Potential(s, w.params, w.model, skin=1.0)
        pot.build_neighbors()
        plan = pot.autotune()  # launch plan for this shape class (untimed)
        pot.energy_forces()
        v0, _ = synth.md_inputs(w.seed, s.n_atoms, 1, 0.005)
        vel = torch.tensor(v0, dtype=torch.float64, device="cuda")
        im = torch.full((s.n_atoms,), 1.0 / synth.CARBON_MASS, dtype=torch.float64, device="cuda")
        chunk = 100
        xi = torch.randn((chunk, s.n_atoms, 3), dtype=torch.float32, device="cuda")
        E = torch.empty((chunk, s.n_structs), dtype=torch.float64, device="cuda")

        def run_chunk():
            pot.md_langevin(chunk, vel, im, dt, gamma, kT, noise=xi, E_pot=E)
        run_chunk()
        torch.cuda.synchronize()
        ms = _timed(torch, stream, run_chunk, steps // chunk) / (steps // chunk * chunk)
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            run_chunk()
        torch.cuda.synchronize()
        g.replay()
        ms_g = _timed(torch, stream, g.replay, steps // chunk) / (steps // chunk * chunk)
        nnpot.nn_check(pot.nl)
        del g
        out["runs"].append({"model": w.name.split(", ", 4)[-1], "cells": n_cells, "atoms": s.n_atoms, "steps": steps,
                            "ms_per_step": round(ms, 5), "ms_per_step_graph": round(ms_g, 5),
                            "us_per_step_per_atom_graph": round(ms_g * 1e3 / s.n_atoms, 4),
                            "list_builds": int(pot.meta[2].item()), "launch_plan": list(plan)})
    print(json.dumps(out), flush=True)


def qeq_bench(args):
    """Charge equilibration (Sec. II.B) on a batch of charged NaCl-like
    clusters (--qeq-clusters of 16/17 atoms, total charge +1): per step the
    list build, descriptors, the 3-output networks, the per-structure FP64
    solve, the seeded backward pass, the adjoint, the gather and the Coulomb
    forces.  Reports atoms/s, the stage times, the errors against the FP64
    oracle on the first 64 clusters and the oracle's own throughput there.
    Prints one JSON line."""
    import torch
    from oracle import qeq as oqeq
    import oracle
    from paper_2305_11805_amd import nnpot, synth
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    oracle.build(force=False)
    w, Qc = synth.qeq_clusters(args.qeq_clusters)
    s = w.system
    pot = nnpot.Potential(s, w.params, w.model)
    Qt = torch.tensor(Qc, dtype=torch.float64, device="cuda")
    sig = w.extra["sigma"]

    def step():
        pot.build_neighbors(check=False)
        pot.energy_forces_qeq(Qt, sig)
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    nnpot.nn_check(pot.nl)
    stream = torch.cuda.current_stream()
    ms = _timed(torch, stream, step, args.steps) / args.steps
    nnpot.nn_timing(True)
    step()
    st = nnpot.nn_timing_read()
    nnpot.nn_timing(False)
    nnpot.nn_check(pot.nl)
    E = pot.E_struct.cpu().numpy()
    _, q, F = pot.energy_forces_qeq(Qt, sig)
    q, F = q.cpu().numpy(), F.cpu().numpy()
    # the oracle on the first 64 clusters (timed: its own throughput)
    m = min(64, s.n_structs)
    a1 = int(s.atom_ptr[m])
    sub = synth.System(s.pos[:a1], s.species[:a1], s.atom_ptr[:m + 1], s.cell[:m], s.pbc[:m])
    t0 = time.perf_counter()
    Es_r, q_r, F_r, _ = oqeq.energy_forces_qeq(w.params, w.model, sub, Qc[:m], sig)
    t_or = time.perf_counter() - t0
    out = {"step": "charge_equilibration", "workload": w.name, "n_atoms": s.n_atoms, "steps": args.steps,
           "ms_per_step": round(ms, 4), "atoms_per_s": round(s.n_atoms / ms * 1e3, 1),
           "stages_ms": {k: round(v[0], 5) for k, v in st.items() if v[1]},
           "errors_first_64_clusters": {
               "E_per_atom_max": float(np.max(np.abs(E[:m] - Es_r) / np.diff(sub.atom_ptr))),
               "q_max": float(np.abs(q[:a1] - q_r).max()), "F_max": float(np.abs(F[:a1] - F_r).max())},
           "oracle": {"atoms_per_s": round(a1 / t_or, 1), "what": "numpy FP64 oracle, first 64 clusters",
                      "seconds": round(t_or, 2)}}
    print(json.dumps(out), flush=True)


def stored_mode(args):
    """The stored-Jacobian (precomputed-derivative) mode of Sec. II.A on
    --config: a store step (list, descriptors with the Jacobian, MLP,
    contraction, gather) and a reuse step (MLP, contraction and gather on the
    stored descriptors and Jacobian: training over a fixed set), with the
    achieved HBM GB/s of the two Jacobian kernels against 8 TB/s.  Prints one
    JSON line."""
    import torch
    from paper_2305_11805_amd import nnpot, synth
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    w = synth.config(args.config, desc=args.desc)
    s, p = w.system, w.params
    big = 1 << 42
    pot = nnpot.Potential(s, p, w.model, flags=nnpot.NN_STORE_JACOBIAN, mem_budget=big)
    store_flags = nnpot.NN_STORE_JACOBIAN
    reuse_flags = nnpot.NN_STORE_JACOBIAN | nnpot.NN_REUSE_DESCRIPTORS

    def store():
        nnpot.nn_build_neighbors(pot.sys, pot.rc, pot.skin, pot.nl, pot.ws)
        nnpot.nn_energy_forces(pot.sys, pot.nl, pot.params, pot.dmodel.struct, store_flags, big, pot.E_struct,
                               pot.E_atom, pot.F, pot.ws)

    def reuse():
        nnpot.nn_energy_forces(pot.sys, pot.nl, pot.params, pot.dmodel.struct, reuse_flags, big, pot.E_struct,
                               pot.E_atom, pot.F, pot.ws)
    for _ in range(max(args.warmup, 1)):
        store()
        reuse()
    torch.cuda.synchronize()
    nnpot.nn_check(pot.nl)
    stream = torch.cuda.current_stream()
    ms_store = _timed(torch, stream, store, args.steps) / args.steps
    ms_reuse = _timed(torch, stream, reuse, args.steps) / args.steps
    nnpot.nn_timing(True)
    store()
    reuse()
    st = nnpot.nn_timing_read()
    nnpot.nn_timing(False)
    nnpot.nn_check(pot.nl)
    entries = int(pot.offsets[-1].item())
    js = nnpot.nn_jacobian_stride(pot.params)
    # algorithmic bytes: the Jacobian rows written once and read once; the
    # contraction also reads lambda and writes a 16-B pair gradient per entry
    jac_bytes = 4.0 * js * entries
    con_bytes = jac_bytes + 4.0 * s.n_atoms * p.dim + 16.0 * entries + 4.0 * entries
    cnt = {}
    prof = os.path.join(ROOT, "profiles", "counters.json")
    if os.path.exists(prof):
        with open(prof) as f:
            cnt = json.load(f)

    def kern(stage, name, alg):
        ms_k = st[stage][0] / max(st[stage][1], 1)
        e = {"avg_launch_ms": round(ms_k, 5), "algorithmic_bytes_per_launch": alg,
             "gbs": round(alg / (ms_k / 1e3) / 1e9, 1), "frac_hbm": round(alg / (ms_k / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
        c = cnt.get(f"{name}:{w.name}")
        if c and c.get("source_hash") == source_hash(name):
            e["hbm_bytes_per_launch"] = c["hbm_bytes_per_launch"]
            e["traffic_gbs"] = round(c["hbm_bytes_per_launch"] / (ms_k / 1e3) / 1e9, 1)
        return e
    res = {"workload": w.name, "step": "stored_jacobian", "n_atoms": s.n_atoms, "list_entries": entries,
           "jacobian_floats_per_entry": js, "jacobian_gb": round(jac_bytes / 1e9, 3),
           "store_step": {"ms": round(ms_store, 4), "atoms_per_s": round(s.n_atoms / ms_store * 1e3, 1)},
           "reuse_step": {"ms": round(ms_reuse, 4), "atoms_per_s": round(s.n_atoms / ms_reuse * 1e3, 1)},
           "kernels": {"k_desc_jac": kern("desc_jac", "k_desc_jac", jac_bytes),
                       "k_jac_contract": kern("jac_contract", "k_jac_contract", con_bytes)},
           "peak_hbm_gbs": PEAK_HBM_GBS}
    if args.calib_copy_mib > 0:
        a = torch.empty(args.calib_copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
    print(json.dumps(res), flush=True)


def suite(args):
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    path = args.suite_out
    with open(path, "w") as out:
        for idx in args.suite_configs:
            modes = ["fp32", "bf16x3", "bf16"] if idx in (3, 4) else ["fp32"]
            print(f"[suite] config {idx}", file=sys.stderr, flush=True)
            suite_config(idx, modes, args.steps, out)


def valid_neighbor_counts_gpu(pot, rc):
    """Entries of each row inside rc (the skin list holds rc + skin), from
    the list and positions on the device."""
    import torch
    nnz = int(pot.offsets[-1].item())
    off = pot.offsets
    rows = torch.repeat_interleave(torch.arange(pot.N, device=pot.dev), off[1:] - off[:-1])
    ptr = pot.atom_ptr
    struct = torch.searchsorted(ptr, rows, right=True) - 1
    cell = pot.cell.view(-1, 3, 3)
    sh = pot.shift[:nnz, :3].to(torch.float64)
    img = sh @ cell[0] if pot.B == 1 else torch.einsum("ek,ekl->el", sh, cell[struct])
    d = pot.pos[pot.nbr[:nnz].long()] - pot.pos[rows] + img
    valid = (d * d).sum(1) < rc * rc
    return torch.bincount(rows[valid], minlength=pot.N).cpu().numpy()


def headline(args):
    """The bench line.  Workloads with a random walk (the 262144-atom cell)
    time K steps of the walk from the input positions: per step x += xi_k,
    the device skin test with a predicated list rebuild, then energies and
    forces.  Other workloads rebuild the list every step."""
    import torch
    from paper_2305_11805_amd import nnpot, synth
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    w = synth.config(args.config, desc=args.desc)
    s, p = w.system, w.params
    flags = MODE_FLAGS[args.mode]
    skin = float(w.extra.get("skin", 0.0))
    walk = "steps" in w.extra
    pot = nnpot.Potential(s, p, w.model, skin=skin, flags=flags, capacity_margin=1.3 if walk else 1.25)
    stream = torch.cuda.current_stream()
    pos0 = pot.pos.clone()
    n_disp = max(args.steps, args.warmup, 1)
    xi = None
    if walk:
        xi = torch.tensor(np.stack(list(synth.md_displacements(w.seed, s.n_atoms, n_disp, w.extra["step_sigma"]))),
                          dtype=torch.float64, device="cuda")
    k = [0]

    def build():
        nnpot.nn_build_neighbors(pot.sys, pot.rc, pot.skin, pot.nl, pot.ws)

    def energy_forces(f=flags):
        nnpot.nn_energy_forces(pot.sys, pot.nl, pot.params, pot.dmodel.struct, f, 0, pot.E_struct,
                               pot.E_atom, pot.F, pot.ws)

    def step(f=flags):
        if walk:
            pot.pos.add_(xi[k[0]])
            k[0] += 1
        build()
        energy_forces(f)

    def restart():
        # the walk starts again from the input positions with a fresh list
        torch.cuda.synchronize()
        if walk:
            pot.pos.copy_(pos0)
            pot.meta[1] = 0
            k[0] = 0

    def timed(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    def builds():
        return int(pot.meta[2].item())

    restart()
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    nnpot.nn_check(pot.nl)
    plan = pot.launch_plan() if args.no_autotune else pot.autotune()  # launch plan for this shape class (untimed)
    restart()
    for _ in range(max(args.warmup, 1)):
        step()
    restart()

    # the timed region: K whole steps
    b0 = builds()
    total_ms = timed(step, args.steps)
    n_builds = builds() - b0
    nnpot.nn_check(pot.nl)
    F = pot.F.cpu().numpy()
    pos_end = pot.pos.cpu().numpy()
    # K more steps with the library's per-stage HIP events (on its launch
    # stream): per-kernel launch times for the roofline; the events add a
    # little time to these steps, so they are reported apart
    restart()
    nnpot.nn_timing(True)
    staged_ms = timed(step, args.steps)
    stages = nnpot.nn_timing_read()
    nnpot.nn_timing(False)
    nnpot.nn_check(pot.nl)
    assert np.array_equal(pot.F.cpu().numpy(), F), "the staged pass differs from the timed one"
    n_valid = valid_neighbor_counts_gpu(pot, p.rc)

    variants = {}
    if not args.no_variants:
        # E + F on the list already built (no rebuild)
        ms = timed(energy_forces, args.steps) / args.steps
        variants["steady_state_no_rebuild"] = {"ms_per_step": round(ms, 4), "value": round(s.n_atoms / ms * 1e3, 1)}
        # the whole step replayed from a HIP graph; the walk's displacement is
        # copied into the graph's input buffer before each replay
        restart()
        xi_buf = torch.zeros_like(pot.pos)
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            if walk:
                pot.pos.add_(xi_buf)
            build()
            energy_forces()
        restart()
        kg = [0]

        def replay():
            if walk:
                xi_buf.copy_(xi[kg[0]])
                kg[0] += 1
            graph.replay()
        ms = timed(replay, args.steps) / args.steps
        nnpot.nn_check(pot.nl)
        same = bool(np.array_equal(pot.F.cpu().numpy(), F))
        assert same, "graph replay differs from the eager steps"
        variants["graph_replay"] = {"ms_per_step": round(ms, 4), "value": round(s.n_atoms / ms * 1e3, 1),
                                    "forces_equal_eager_bitwise": same}
        del graph
        # the other MLP precision modes on the same walk, with their sampled
        # force error against the oracle at the final positions
        for mode in ("fp32", "bf16x3", "bf16"):
            if mode == args.mode:
                continue
            restart()
            for _ in range(max(args.warmup, 1)):
                step(MODE_FLAGS[mode])
            restart()
            ms = timed(lambda: step(MODE_FLAGS[mode]), args.steps) / args.steps
            nnpot.nn_check(pot.nl)
            variants[f"mlp_{mode}"] = {
                "ms_per_step": round(ms, 4), "value": round(s.n_atoms / ms * 1e3, 1),
                "force_err_max_sampled_eV_per_A": sampled_force_error(w, pot.F.cpu().numpy(),
                                                                      pos=pot.pos.cpu().numpy())}
        # the same step through torch.autograd.Function: E forward, dE/dpos
        # (= -F, from the adjoint) by backward, at the walk's end positions
        from paper_2305_11805_amd import autograd
        pos_t = pot.pos.clone().requires_grad_(True)

        def ag_step():
            E = autograd.energy(pot, pos_t, flags)
            torch.autograd.grad(E.sum(), pos_t)
        for _ in range(2):
            ag_step()
        ms = timed(ag_step, args.steps) / args.steps
        variants["autograd_function"] = {"ms_per_step": round(ms, 4), "value": round(s.n_atoms / ms * 1e3, 1)}
        if args.config != 1:
            variants["bulk4096_rebuild_every_step"] = small_bulk_line(args, flags)

    if args.calib_copy_mib > 0:
        a = torch.empty(args.calib_copy_mib * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()

    ms_per_step = total_ms / args.steps
    value = s.n_atoms * args.steps / (total_ms / 1e3)
    fm = flop_model(p, n_valid)
    single_kernel = ["desc_adj", "desc_fwd", "mlp", "force_gather", "energy"]
    dom = max(single_kernel, key=lambda kk: stages[kk][0])
    dom_ms = stages[dom][0] / max(stages[dom][1], 1)
    if dom in ("desc_adj", "desc_fwd"):
        achieved = fm[dom] / (dom_ms / 1e3) / 1e12
        roof = {"kernel": {"desc_adj": "k_desc_adj", "desc_fwd": "k_desc_fwd"}[dom], "bound": "alu",
                "achieved": round(achieved, 3), "peak": PEAK_FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_VALU_TFLOPS, 4), "traffic": None,
                "avg_launch_ms": round(dom_ms, 5), "algorithmic_flops_per_launch": fm[dom],
                "flops_per_triplet": fm["per_triplet"][dom]}
    else:
        roof = {"kernel": dom, "bound": "mfma", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "avg_launch_ms": round(dom_ms, 5)}
    cnt = {}
    prof = os.path.join(ROOT, "profiles", "counters.json")
    if os.path.exists(prof):
        with open(prof) as f:
            cnt = json.load(f)

    def hbm_bytes(kernel):
        e = cnt.get(f"{kernel}:{w.name}")
        return e["hbm_bytes_per_launch"] if e and e.get("source_hash") == source_hash(kernel) else None

    t = hbm_bytes(roof["kernel"])
    if t is not None:
        roof["traffic"] = t
        roof["traffic_gbs"] = round(t / (dom_ms / 1e3) / 1e9, 1)
    # every hot kernel against its own roof: the descriptor passes against
    # FP32 VALU and HBM, the MLP against the MFMA peak of its operand type
    kern = {}
    for stage, name in (("desc_fwd", "k_desc_fwd"), ("desc_adj", "k_desc_adj")):
        if stages[stage][1]:
            ms_k = stages[stage][0] / stages[stage][1]
            e = {"avg_launch_ms": round(ms_k, 5), "tflops": round(fm[stage] / (ms_k / 1e3) / 1e12, 3),
                 "frac_fp32_valu": round(fm[stage] / (ms_k / 1e3) / 1e12 / PEAK_FP32_VALU_TFLOPS, 4)}
            b = hbm_bytes(name)
            if b is not None:
                e["hbm_bytes_per_launch"] = b
                e["hbm_gbs"] = round(b / (ms_k / 1e3) / 1e9, 1)
                e["frac_hbm"] = round(b / (ms_k / 1e3) / 1e9 / PEAK_HBM_GBS, 4)
            kern[name] = e
    if stages["mlp"][1]:
        ms_k = stages["mlp"][0] / stages["mlp"][1]
        fl = mlp_flops(w, s.n_atoms)
        peak = {"fp32": PEAK_FP32_MFMA_TFLOPS, "bf16": PEAK_BF16_MFMA_TFLOPS, "bf16x3": PEAK_BF16_MFMA_TFLOPS}[args.mode]
        e = {"avg_launch_ms": round(ms_k, 5), "algorithmic_flops_per_launch": fl,
             "tflops": round(fl / (ms_k / 1e3) / 1e12, 3), "peak_mfma_tflops": peak,
             "frac_mfma": round(fl / (ms_k / 1e3) / 1e12 / peak, 4)}
        mlp_name = mlp_rows_plan(plan, args.mode, w) or "k_mlp"
        b = hbm_bytes(mlp_name)
        if b is not None:
            e["hbm_bytes_per_launch"] = b
            e["hbm_gbs"] = round(b / (ms_k / 1e3) / 1e9, 1)
        kern[mlp_name] = e
    cfg = {"workload": w.name, "n_atoms": s.n_atoms, "n_structs": s.n_structs, "mlp_mode": args.mode,
           "neighbor_build_each_step": skin == 0.0, "skin": skin, "seed": w.seed,
           "launch_plan": None if plan is None else {
               "plan": list(plan), "waves_per_atom_fwd": plan[0], "waves_per_atom_adj": plan[1],
               "mlp": "row blocks of 64 atoms" if mlp_rows_plan(plan, args.mode, w) else f"tiles of 16 atoms, plan {plan[2]}"}}
    if walk:
        cfg["walk"] = {"steps_timed": args.steps, "sigma_A": w.extra["step_sigma"], "list_builds_timed": n_builds,
                       "rule": "rebuild on the device when an atom moved farther than skin/2 since the last build"}
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "atoms/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {"fp32": "f32", "bf16": "bf16-mlp/f32",
                                                        "bf16x3": "bf16x3-mlp/f32"}[args.mode],
        "data": ("synthetic (seeded RSA positions; seeded W, b ~ N(0, 1/fan_in) with the first layer scaled by a "
                 "fixed per-workload constant)"),
        "config": cfg,
        "roofline": roof,
        "stages_ms_per_step": {kk: round(v[0] / args.steps, 5) for kk, v in stages.items()},
        "stage_launches": {kk: int(v[1]) for kk, v in stages.items()},
        "ms_per_step_with_stage_events": round(staged_ms / args.steps, 4),
        "pairs_last_step": fm["pairs"], "triplets_last_step": fm["triplets"], "kernels": kern,
        "variants": variants,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = oracle_leg(w)
        out["force_err_max_sampled_eV_per_A"] = sampled_force_error(w, F, pos=pos_end)
    print(json.dumps(out), flush=True)


def small_bulk_line(args, flags):
    """The 4096-atom bulk cell with the list rebuilt every step (K steps)."""
    import torch
    from paper_2305_11805_amd import nnpot, synth
    w = synth.config(1)
    pot = nnpot.Potential(w.system, w.params, w.model, flags=flags)

    def step():
        nnpot.nn_build_neighbors(pot.sys, pot.rc, pot.skin, pot.nl, pot.ws)
        nnpot.nn_energy_forces(pot.sys, pot.nl, pot.params, pot.dmodel.struct, flags, 0, pot.E_struct,
                               pot.E_atom, pot.F, pot.ws)
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    nnpot.nn_check(pot.nl)
    plan = pot.autotune()
    ms = _timed(torch, torch.cuda.current_stream(), step, args.steps) / args.steps
    nnpot.nn_check(pot.nl)
    return {"workload": w.name, "ms_per_step": round(ms, 4), "value": round(w.system.n_atoms / ms * 1e3, 1),
            "launch_plan": list(plan)}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=4,
                    help="workload index 0-4 (default: 4, the 262144-atom cell's 100-step walk)")
    ap.add_argument("--mode", choices=["fp32", "bf16", "bf16x3"], default="fp32")
    ap.add_argument("--desc", choices=["mbp", "bp"], default="mbp",
                    help="angular descriptor term: mBP (the headline) or standard BP (configs 0-2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the steady-state and graph-replay timings")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch plan")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: turn two rocprofv3 --pmc CSVs of this workload into profiles/counters.json")
    ap.add_argument("--suite", action="store_true",
                    help="measure every workload (one JSON line each) instead of the single bench line")
    ap.add_argument("--suite-configs", type=int, nargs="*", default=[0, 1, 2, 3, 4])
    ap.add_argument("--suite-out", default="suite.jsonl")
    ap.add_argument("--stored", action="store_true",
                    help="time the stored-Jacobian mode (store and reuse steps) on --config instead of the bench line")
    ap.add_argument("--ingest-kernels", nargs="*", default=["k_desc_adj", "k_desc_fwd", "k_mlp_rows"],
                    help="kernels whose counters --ingest-counters keeps")
    ap.add_argument("--md", action="store_true",
                    help="Langevin dynamics of 16-atom cells (the Table II shape) instead of the bench line")
    ap.add_argument("--md-cells", type=int, default=1024, help="cells in the batched --md run")
    ap.add_argument("--qeq", action="store_true",
                    help="time charge equilibration (Sec. II.B) on charged clusters instead of the bench line")
    ap.add_argument("--qeq-clusters", type=int, default=4096, help="clusters in the --qeq run")
    ap.add_argument("--force-matching", action="store_true",
                    help="time the force-matching training step on --config instead of the bench line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    from paper_2305_11805_amd import synth
    if args.suite:
        suite(args)
        return
    if args.force_matching:
        force_matching(args)
        return
    if args.md:
        md_table2(args)
        return
    if args.qeq:
        qeq_bench(args)
        return
    if args.stored:
        stored_mode(args)
        return
    if args.ingest_counters:
        if args.calib_copy_mib <= 0:
            raise SystemExit("--ingest-counters needs --calib-copy-mib of the profiled run")
        ingest_counters(*args.ingest_counters, args.calib_copy_mib, synth.config(args.config, desc=args.desc).name,
                        kernels=tuple(args.ingest_kernels))
        return

    headline(args)


if __name__ == "__main__":
    main()
