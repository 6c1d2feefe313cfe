"""Pins of the charge-equilibration oracle (Sec. II.B; oracle/qeq.py) to
facts that do not come from the oracle itself: closed forms for one and two
atoms, the constraint and the equal chemical potential of the constrained
minimum, minimality, the 3-output network against torch float64, and
central differences of the total energy (which re-solves the charges at
every displaced geometry) for the forces and the weight gradient."""
import math

import numpy as np
import pytest

from paper_2305_11805_amd import synth

KE = 14.399645


@pytest.fixture(scope="module")
def Q(oracle_lib):
    from oracle import qeq
    return qeq


def test_two_atom_solve_closed_form(Q):
    """Two charges q1 + q2 = Q0: equal chemical potential
    chi1 + A11 q1 + A12 q2 = chi2 + A21 q1 + A22 q2 gives
    q1 = (chi2 - chi1 + (A22 - A12) Q0) / (A11 + A22 - 2 A12)."""
    r, s1, s2 = 2.7, 1.0, 1.3
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    A0 = Q.coulomb_matrix(pos, np.array([s1, s2]))
    a = KE * math.erf(r / (math.sqrt(2.0) * math.hypot(s1, s2))) / r  # written out, not A0[0, 1]
    self1, self2 = KE / (s1 * math.sqrt(math.pi)), KE / (s2 * math.sqrt(math.pi))
    assert abs(A0[0, 1] - a) < 1e-13 and abs(A0[0, 0] - self1) < 1e-13 and abs(A0[1, 1] - self2) < 1e-13
    chi, J, Q0 = np.array([3.1, 7.9]), np.array([5.0, 9.0]), 0.4
    q, mu = Q.solve(chi, J, A0, Q0)
    A11, A22 = J[0] + self1, J[1] + self2
    q1 = (chi[1] - chi[0] + (A22 - a) * Q0) / (A11 + A22 - 2 * a)
    assert abs(q[0] - q1) < 1e-13 and abs(q[1] - (Q0 - q1)) < 1e-13
    assert abs(mu - (chi[0] + A11 * q[0] + a * q[1])) < 1e-12


def test_single_atom_energy_closed_form(Q, oracle_lib):
    """One atom of charge Q0: q = Q0 and E = E0 + chi Q0 + (J + k_e / (sigma sqrt(pi))) Q0^2 / 2."""
    p = synth.mbp_params(2, 6.0, 8, 4, 4)
    model = synth.qeq_model(p.dim, 3, hidden=(6, 5))
    s = synth.single(np.zeros((1, 3)), [1], cell=np.eye(3) * 5.0)
    Q0 = -0.7
    Es, q, F, out = Q.energy_forces_qeq(p, model, s, np.array([Q0]), (1.0, 1.2))
    E0, chi, J = out[0]
    assert abs(q[0] - Q0) < 1e-15
    ref = E0 + chi * Q0 + 0.5 * (J + KE / (1.2 * math.sqrt(math.pi))) * Q0 * Q0
    assert abs(Es[0] - ref) < 1e-12
    assert np.all(F == 0.0)


@pytest.fixture(scope="module")
def batch():
    w, Qc = synth.qeq_clusters(4)
    return w, Qc


def test_constraint_chemical_potential_and_minimum(Q, batch):
    w, Qc = batch
    s = w.system
    Es, q, F, out = Q.energy_forces_qeq(w.params, w.model, s, Qc, w.extra["sigma"])
    sigma = np.asarray(w.extra["sigma"])[s.species]
    rng = np.random.Generator(np.random.PCG64(1))
    for c in range(s.n_structs):
        a0, a1 = s.atom_ptr[c], s.atom_ptr[c + 1]
        qc = q[a0:a1]
        assert abs(qc.sum() - Qc[c]) < 1e-12
        A = Q.coulomb_matrix(s.pos[a0:a1], sigma[a0:a1]) + np.diag(out[a0:a1, 2])
        mu = out[a0:a1, 1] + A @ qc  # dE/dq_i
        assert np.ptp(mu) < 1e-10 * max(1.0, np.abs(mu).max())

        def E_of(qq):
            return out[a0:a1, 0].sum() + out[a0:a1, 1] @ qq + 0.5 * qq @ A @ qq
        assert abs(E_of(qc) - Es[c]) < 1e-10 * max(1.0, abs(Es[c]))
        for _ in range(5):  # any change that keeps the total charge raises E
            dq = rng.normal(size=qc.size) * 0.05
            dq -= dq.mean()
            assert E_of(qc + dq) > E_of(qc)


def test_three_output_network_vs_torch(Q):
    torch = pytest.importorskip("torch")
    rng = np.random.Generator(np.random.PCG64(5))
    D, n = 12, 30
    model = synth.random_model(2, D, [7, 5], 9, act="tanh", n_out=3)
    G = rng.uniform(0, 2, (n, D))
    sp = rng.integers(0, 2, n).astype(np.int32)
    seed = rng.normal(size=(n, 3))
    out, cache = Q.mlp_outputs(model, sp, G)
    lam, grads = Q.mlp_backward(model, cache, seed, D, n)
    for s in range(2):
        idx = np.nonzero(sp == s)[0]
        g = torch.tensor(G[idx], requires_grad=True)
        params = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True))
                  for W, b in zip(model[s][2], model[s][3])]
        a = g
        for l, (W, b) in enumerate(params):
            z = a @ W.T + b
            a = torch.tanh(z) if l < len(params) - 1 else z
        np.testing.assert_allclose(out[idx], a.detach().numpy(), rtol=1e-13, atol=1e-14)
        (a * torch.tensor(seed[idx])).sum().backward()
        np.testing.assert_allclose(lam[idx], g.grad.numpy(), rtol=1e-12, atol=1e-14)
        for (dW, db), (W, b) in zip(grads[s], params):
            np.testing.assert_allclose(dW, W.grad.numpy(), rtol=1e-12, atol=1e-14)
            np.testing.assert_allclose(db, b.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_forces_central_differences(Q):
    """F = -dE/dx with the charges re-equilibrated at every displaced
    geometry: checks the envelope argument (no derivative of the solve),
    the Coulomb pair forces and the descriptor chain rule together."""
    w, Qc = synth.qeq_clusters(2)
    s = w.system
    sig = w.extra["sigma"]
    _, _, F, _ = Q.energy_forces_qeq(w.params, w.model, s, Qc, sig)
    h = 1e-5
    rng = np.random.Generator(np.random.PCG64(2))
    for k in rng.choice(s.n_atoms, 6, replace=False):
        for a in range(3):
            pp, pm = s.pos.copy(), s.pos.copy()
            pp[k, a] += h
            pm[k, a] -= h
            Ep = Q.energy_only(w.params, w.model, synth.System(pp, s.species, s.atom_ptr, s.cell, s.pbc), Qc, sig)
            Em = Q.energy_only(w.params, w.model, synth.System(pm, s.species, s.atom_ptr, s.cell, s.pbc), Qc, sig)
            fd = -(Ep.sum() - Em.sum()) / (2 * h)
            assert abs(fd - F[k, a]) < 1e-6 * max(1.0, abs(F[k, a])), (k, a, fd, F[k, a])


def test_weight_gradient_central_differences(Q):
    w, Qc = synth.qeq_clusters(2)
    s = w.system
    sig = w.extra["sigma"]
    wts = np.array([0.7, -1.3])
    grads = Q.energy_forces_qeq(w.params, w.model, s, Qc, sig, weights=wts)[4]
    h = 1e-6
    rng = np.random.Generator(np.random.PCG64(3))
    for sp in range(2):
        for l in range(len(w.model[sp][2])):
            W = w.model[sp][2][l]
            for _ in range(3):
                i, j = rng.integers(0, W.shape[0]), rng.integers(0, W.shape[1])
                vals = []
                for d in (h, -h):
                    W[i, j] += d
                    vals.append(wts @ Q.energy_only(w.params, w.model, s, Qc, sig))
                    W[i, j] -= d
                fd = (vals[0] - vals[1]) / (2 * h)
                got = grads[sp][l][0][i, j]
                assert abs(fd - got) < 1e-6 * max(1.0, abs(got)), (sp, l, i, j, fd, got)
