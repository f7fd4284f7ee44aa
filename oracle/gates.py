"""Gate matrices (complex128).

Conventions: qubit q is bit q of the basis index; a k-qubit gate acting on
qubits (q_0, ..., q_{k-1}) has local basis index sum_t bit(q_t) << t.
Rotations are exp(-i theta P / 2); the QAOA cost gate on an edge is
zz(gamma) = diag(1, e^{-i gamma}, e^{-i gamma}, 1) = exp(-i gamma (1 - Z Z) / 2),
so a layer of them on every edge is exp(-i gamma C) with C the cut-size
operator of MaxCut (Sec. III-E).
"""
import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
PAULIS = (I2, X, Y, Z)


def rx(theta):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def ry(theta):
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(theta):
    return np.diag([np.exp(-0.5j * theta), np.exp(0.5j * theta)]).astype(np.complex128)


def zz(theta):
    e = np.exp(-1j * theta)
    return np.diag([1.0, e, e, 1.0]).astype(np.complex128)


def cx():
    # control = local bit 0, target = local bit 1: |c t> -> |c, t xor c>
    m = np.zeros((4, 4), dtype=np.complex128)
    for c in (0, 1):
        for t in (0, 1):
            m[c | ((t ^ c) << 1), c | (t << 1)] = 1.0
    return m


def gate_matrix(gate):
    """Matrix of a workloads.Gate in its local little-endian basis."""
    k = gate.kind
    if k == "h":
        return H
    if k == "x":
        return X
    if k == "y":
        return Y
    if k == "z":
        return Z
    if k == "rx":
        return rx(gate.theta)
    if k == "ry":
        return ry(gate.theta)
    if k == "rz":
        return rz(gate.theta)
    if k == "zz":
        return zz(gate.theta)
    if k == "cx":
        return cx()
    if k in ("u1", "u2"):
        d = 2 if k == "u1" else 4
        return np.array(gate.matrix, dtype=np.complex128).reshape(d, d)
    raise ValueError(f"unknown gate kind {k!r}")


def pauli_string(labels):
    """Matrix of P_{labels[0]} (x) ... on local qubits 0, 1, ... (little-endian:
    labels[0] acts on local bit 0)."""
    m = np.array([[1.0 + 0j]])
    for a in labels:
        m = np.kron(PAULIS[a], m)
    return m
