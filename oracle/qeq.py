"""Charge equilibration of Sec. II.B in plain FP64 numpy (test infrastructure
only: the tests, the smoke check and the benchmark's CPU leg may use it).

The paper gives the structure of the method -- one network per species with
three outputs per atom, the coefficients of a second-order Taylor expansion
of the atom's energy in its charge (local energy, electronegativity,
hardness), followed by a charge-equilibration layer that returns the charges
and the total energy from a linear system -- and defers the theory to another
work.  The reading implemented here (Goedecker-type Gaussian charges, as in
the equilibration schemes the paper cites):

  E(q) = sum_i [E0_i + chi_i q_i + J_i q_i^2 / 2]
         + k_e [ sum_i q_i^2 / (2 sigma_i sqrt(pi))
                 + sum_{i<j} q_i q_j erf(r_ij / (sqrt(2) gamma_ij)) / r_ij ],
  gamma_ij = sqrt(sigma_i^2 + sigma_j^2),

minimised over the charges of each structure c subject to sum_{i in c} q_i = Q_c
(non-periodic structures).  (E0_i, chi_i, J_i) are the three network outputs of
atom i (Eq. (1) with an output layer of width 3), sigma_i the Gaussian width of
its species and k_e = e^2 / (4 pi eps0).  With A_ij = k_e erf(...)/r_ij (i != j),
A_ii = J_i + k_e / (sigma_i sqrt(pi)), the minimum solves
  A q - mu 1 = -chi,   1^T q = Q,
so every atom ends at the same chemical potential dE/dq_i = mu, and
  E = sum_i E0_i + chi . q / 2 + mu Q / 2.
Since q minimises E at fixed positions and weights, dE/dx and dE/dtheta are the
partial derivatives at fixed q (no derivative of the solve is needed): the
network part backpropagates the output seeds (1, q_i, q_i^2 / 2), and the
Coulomb part adds its pair forces.
"""
from __future__ import annotations

import math

import numpy as np

from . import descriptors, neighbors_brute

KE = 14.399645  # e^2 / (4 pi eps0) in eV * Angstrom / e^2


def _act(code, z):
    if code == "gaussian":
        a = np.exp(-z * z)
        return a, -2.0 * z * a
    if code == "tanh":
        t = np.tanh(z)
        return t, 1.0 - t * t
    if code == "relu":
        return np.maximum(z, 0.0), (z > 0.0).astype(np.float64)
    return z, np.ones_like(z)


def mlp_outputs(model, species, G):
    """Per-atom outputs of each atom's species network (Eq. (1)): out[n][n_out],
    and the per-species intermediate values the backward pass needs."""
    n = G.shape[0]
    n_out = model[0][0][-1]
    out = np.zeros((n, n_out))
    cache = {}
    for s, (widths, acts, Ws, bs) in enumerate(model):
        idx = np.nonzero(species == s)[0]
        if idx.size == 0:
            continue
        a = [G[idx]]
        d = []
        for W, b, act in zip(Ws, bs, acts):
            z = a[-1] @ W.T + b
            y, dy = _act(act, z)
            a.append(y)
            d.append(dy)
        out[idx] = a[-1]
        cache[s] = (idx, a, d)
    return out, cache


def mlp_backward(model, cache, seed, D, n):
    """For per-atom output seeds seed[n][n_out]: lambda = sum_o seed_o d out_o / dG
    [n][D], and the parameter gradient sum_i sum_o seed_io d out_io / dtheta as
    per-species [(dW_l, db_l), ...]."""
    lam = np.zeros((n, D))
    grads = []
    for s, (widths, acts, Ws, bs) in enumerate(model):
        layers = [(np.zeros_like(W), np.zeros_like(b)) for W, b in zip(Ws, bs)]
        if s in cache:
            idx, a, d = cache[s]
            delta = seed[idx] * d[-1]
            for l in range(len(Ws) - 1, -1, -1):
                layers[l] = (delta.T @ a[l], delta.sum(axis=0))
                back = delta @ Ws[l]
                delta = back * d[l - 1] if l > 0 else back
            lam[idx] = delta
        grads.append(layers)
    return lam, grads


def coulomb_matrix(pos, sigma, ke=KE):
    """A0: k_e erf(r / (sqrt(2) gamma)) / r off the diagonal, the Gaussian
    self-interaction k_e / (sigma_i sqrt(pi)) on it."""
    n = pos.shape[0]
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] = ke / (sigma[i] * math.sqrt(math.pi))
        for j in range(i + 1, n):
            r = float(np.linalg.norm(pos[j] - pos[i]))
            g = math.sqrt(sigma[i] ** 2 + sigma[j] ** 2)
            A[i, j] = A[j, i] = ke * math.erf(r / (math.sqrt(2.0) * g)) / r
    return A


def solve(chi, J, A0, Q):
    """Charges q and chemical potential mu minimising chi.q + q^T (A0 + diag J) q / 2
    subject to sum q = Q (the constrained minimum as one linear solve)."""
    n = chi.size
    K = np.zeros((n + 1, n + 1))
    K[:n, :n] = A0 + np.diag(J)
    K[:n, n] = -1.0
    K[n, :n] = 1.0
    rhs = np.concatenate([-chi, [Q]])
    x = np.linalg.solve(K, rhs)
    return x[:n], x[n]


def coulomb_forces(pos, q, sigma, ke=KE):
    """-d/dx of k_e sum_{i<j} q_i q_j erf(r / (sqrt(2) gamma)) / r at fixed q."""
    n = pos.shape[0]
    F = np.zeros((n, 3))
    for i in range(n):
        for j in range(i + 1, n):
            d = pos[i] - pos[j]
            r = float(np.linalg.norm(d))
            a = math.sqrt(2.0 * (sigma[i] ** 2 + sigma[j] ** 2))
            fp = 2.0 / (a * math.sqrt(math.pi)) * math.exp(-(r / a) ** 2) / r - math.erf(r / a) / (r * r)
            g = ke * q[i] * q[j] * fp * d / r  # dE/dx_i
            F[i] -= g
            F[j] += g
    return F


def energy_forces_qeq(params, model, sys, Q, sigma_species, nl=None, ke=KE, weights=None):
    """Total energies E_struct [B], charges q [N], forces F [N][3] and the network
    outputs out [N][3] of non-periodic structures with total charges Q [B].
    With weights [B] (dL/dE_c), also the parameter gradient of sum_c w_c E_c
    (per-species [(dW, db), ...])."""
    assert not np.any(np.asarray(sys.pbc)), "charge equilibration is for non-periodic structures"
    if nl is None:
        nl = neighbors_brute(sys, params.rc)
    G, dG = descriptors(params, sys, nl, jacobian=True)
    N = sys.pos.shape[0]
    out, cache = mlp_outputs(model, sys.species, G)
    E0, chi, J = out[:, 0], out[:, 1], out[:, 2]
    sigma = np.asarray(sigma_species, np.float64)[sys.species]
    B = len(sys.atom_ptr) - 1
    Es, q, F = np.zeros(B), np.zeros(N), np.zeros((N, 3))
    for c in range(B):
        a0, a1 = int(sys.atom_ptr[c]), int(sys.atom_ptr[c + 1])
        if a1 == a0:
            continue
        A0 = coulomb_matrix(sys.pos[a0:a1], sigma[a0:a1], ke)
        qc, mu = solve(chi[a0:a1], J[a0:a1], A0, float(Q[c]))
        q[a0:a1] = qc
        Es[c] = E0[a0:a1].sum() + 0.5 * chi[a0:a1] @ qc + 0.5 * mu * float(Q[c])
        F[a0:a1] += coulomb_forces(sys.pos[a0:a1], qc, sigma[a0:a1], ke)
    seed = np.stack([np.ones(N), q, 0.5 * q * q], axis=1)
    lam, _ = mlp_backward(model, cache, seed, G.shape[1], N)
    # F_k = -sum_i lambda_i . dG_i/dx_k, with dG_i/dx_j = dG[e] for e = (i -> j)
    # and dG_i/dx_i = -sum_e dG[e]
    rows = np.repeat(np.arange(N), np.diff(nl["offsets"]))
    g = np.einsum("ed,edk->ek", lam[rows], dG)
    np.add.at(F, nl["nbr"], -g)
    np.add.at(F, rows, g)
    res = (Es, q, F, out)
    if weights is not None:
        struct = np.repeat(np.arange(B), np.diff(sys.atom_ptr))
        w = np.asarray(weights, np.float64)[struct]
        _, grads = mlp_backward(model, cache, seed * w[:, None], G.shape[1], N)
        res = res + (grads,)
    return res


def energy_only(params, model, sys, Q, sigma_species, ke=KE):
    """E_struct of energy_forces_qeq (for finite differences)."""
    return energy_forces_qeq(params, model, sys, Q, sigma_species, ke=ke)[0]
