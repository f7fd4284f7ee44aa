"""Exact density matrix and the stochastic trajectory ensemble (complex128).

``density_matrix``  rho <- |0><0|; each gate rho <- U rho U^dagger; after each
                    gate, each of its channels rho <- sum_j K_j rho K_j^dagger
                    (Eq.(1), Sec. III-F).  This is the exact noisy state the
                    ensemble estimates (the role Qiskit's density-matrix
                    simulator plays in Sec. III-G).
``trajectory``      one member of the ensemble (Sec. III-G): the ideal circuit is
                    rebuilt gate by gate; after gate i, for every channel of gate
                    i in list order, a uniform draw picks Kraus operator j and
                    K_j / sqrt(q_j) is applied (for a Pauli channel this is the
                    Pauli itself).  The draw is Philox(seed; k, s), s = the
                    channel's site number.
``ensemble``        rho_hat = (1/K) sum_k psi_k psi_k^dagger, its diagonal
                    sigma_approx = (1/K) sum_k |psi_k|^2 (Sec. III-G), and the
                    MaxCut energy <C>_k = <psi_k|C|psi_k>, C = sum_e w_e (1 - Z_u Z_v)/2.
"""
import math

import numpy as np

from . import channels as chn
from .gates import gate_matrix
from .philox import site_draws
from .statevector import (apply_kraus_sum, apply_superoperator, apply_to_rho, apply_to_state,
                          rho_matrix, superoperator, zero_state)


def _channels_by_gate(problem):
    by = {}
    for s, ch in enumerate(problem.channels):
        by.setdefault(ch.after_gate, []).append((s, ch))
    return by


def density_matrix(problem, literal=False):
    """Exact rho (2^n x 2^n complex128).  literal=True applies each channel as
    the explicit Kraus sum; otherwise as the equivalent superoperator."""
    n = problem.n_qubits
    rho = np.zeros((2,) * (2 * n), dtype=np.complex128)
    rho[(0,) * (2 * n)] = 1.0
    by = _channels_by_gate(problem)
    for i, g in enumerate(problem.gates):
        rho = apply_to_rho(rho, gate_matrix(g), g.qubits)
        for _, ch in by.get(i, []):
            ops = chn.kraus_ops(ch)
            if literal:
                rho = apply_kraus_sum(rho, ops, ch.qubits)
            else:
                rho = apply_superoperator(rho, superoperator(ops), ch.qubits)
    return rho_matrix(rho).copy()


def noiseless_state(problem):
    n = problem.n_qubits
    psi = zero_state(n)
    for g in problem.gates:
        psi = apply_to_state(psi, gate_matrix(g), g.qubits)
    return psi.reshape(-1).copy()


def site_tables(problem):
    """Per site: selection probabilities, thresholds and inserted operators."""
    tabs = []
    for ch in problem.channels:
        q = chn.selection_probs(ch)
        T = chn.thresholds(q)
        ops = [K / math.sqrt(qj) if qj > 0 else None for K, qj in zip(chn.kraus_ops(ch), q)]
        tabs.append((q, T, ops))
    return tabs


def kraus_indices(problem, seed, k0, K):
    """uint8 [K, S]: index of the Kraus operator picked at every site."""
    S = len(problem.channels)
    idx = np.zeros((K, S), dtype=np.uint8)
    if S == 0 or K == 0:
        return idx
    r = site_draws(seed, k0, K, S)
    for s, (q, T, _) in enumerate(site_tables(problem)):
        Ta = np.array(T, dtype=np.uint64)
        # j = min{j : r < T_j}  ==  number of thresholds <= r
        idx[:, s] = (r[:, s][:, None] >= Ta[None, :]).sum(axis=1).astype(np.uint8)
    return idx


def trajectory(problem, idx_row, tabs=None, max_gates=None):
    """Statevector of one trajectory given its Kraus indices (one per site).

    An inserted operator that is exactly the identity matrix (the no-error
    outcome of a Pauli channel: sqrt(q)/sqrt(q) = 1 exactly) is skipped, which
    changes no bit of the result.  max_gates truncates the circuit (timing
    samples only)."""
    if tabs is None:
        tabs = site_tables(problem)
    n = problem.n_qubits
    by = _channels_by_gate(problem)
    psi = zero_state(n)
    for i, g in enumerate(problem.gates):
        if max_gates is not None and i >= max_gates:
            break
        psi = apply_to_state(psi, gate_matrix(g), g.qubits)
        for s, ch in by.get(i, []):
            op = tabs[s][2][int(idx_row[s])]
            if np.array_equal(op, np.eye(op.shape[0])):
                continue
            psi = apply_to_state(psi, op, ch.qubits)
    return psi.reshape(-1).copy()


def cut_values(n, edges, weights):
    """C(z) = sum_e w_e [z_u != z_v] for every basis index z."""
    z = np.arange(1 << n, dtype=np.int64)
    c = np.zeros(1 << n, dtype=np.float64)
    for (u, v), w in zip(edges, weights):
        c += w * (((z >> u) ^ (z >> v)) & 1)
    return c


def zz_values(n, u, v):
    z = np.arange(1 << n, dtype=np.int64)
    return 1.0 - 2.0 * (((z >> u) ^ (z >> v)) & 1)


def energy(psi, n, edges, weights):
    """<psi|C|psi> (not normalised: unnormalised trajectories keep their weight)."""
    p = np.abs(psi) ** 2
    return float(np.dot(p, cut_values(n, edges, weights)))


def edge_zz(psi, n, edges):
    p = np.abs(psi) ** 2
    return np.array([float(np.dot(p, zz_values(n, u, v))) for u, v in edges])


def ensemble(problem, seed, k0, K, want_states=True):
    """Runs trajectories k0..k0+K-1.  Returns a dict with
    idx [K,S] uint8, energies [K], edge_zz [K,m], and if want_states
    psi [K, 2^n], rho_hat, sigma_approx."""
    n = problem.n_qubits
    idx = kraus_indices(problem, seed, k0, K)
    tabs = site_tables(problem)
    cz = cut_values(n, problem.edges, problem.weights) if problem.edges else None
    psis, en, ezz = [], [], []
    for k in range(K):
        psi = trajectory(problem, idx[k], tabs)
        p = np.abs(psi) ** 2
        en.append(float(np.dot(p, cz)) if cz is not None else 0.0)
        ezz.append([float(np.dot(p, zz_values(n, u, v))) for u, v in problem.edges])
        if want_states:
            psis.append(psi)
    out = dict(idx=idx, energies=np.array(en), edge_zz=np.array(ezz).reshape(K, len(problem.edges)))
    if want_states:
        Psi = np.array(psis)  # [K, 2^n]
        out["psi"] = Psi
        out["rho_hat"] = (Psi.T @ Psi.conj()) / K
        out["sigma_approx"] = (np.abs(Psi) ** 2).sum(axis=0) / K
    return out


def energy_exact(rho, n, edges, weights):
    """Tr(rho C)."""
    return float(np.real(np.dot(np.diag(rho), cut_values(n, edges, weights))))
