"""Pins of the oracle's gate matrices and tensor application (CPU only).

Gate matrices are checked against scipy's matrix exponential of their
generators; the tensor application against operators built independently by
brute force over basis states."""
import itertools
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import gates as G
from oracle.statevector import apply_to_rho, apply_to_state
from workloads import Gate

X, Y, Z, I2 = G.X, G.Y, G.Z, G.I2


@pytest.mark.parametrize("theta", [0.0, 0.3, -1.7, math.pi, 5.9])
def test_rotations_are_exponentials(theta):
    np.testing.assert_allclose(G.rx(theta), expm(-0.5j * theta * X), atol=1e-14)
    np.testing.assert_allclose(G.ry(theta), expm(-0.5j * theta * Y), atol=1e-14)
    np.testing.assert_allclose(G.rz(theta), expm(-0.5j * theta * Z), atol=1e-14)
    # zz(gamma) = exp(-i gamma (1 - Z(x)Z)/2): the MaxCut cost term, no global phase
    np.testing.assert_allclose(G.zz(theta), expm(-0.5j * theta * (np.eye(4) - np.kron(Z, Z))), atol=1e-14)


def test_hadamard_and_cx():
    np.testing.assert_allclose(G.H @ G.H, I2, atol=1e-15)
    np.testing.assert_allclose(G.H @ Z @ G.H, X, atol=1e-15)
    # cx: control local bit 0, target local bit 1
    for c, t in itertools.product((0, 1), repeat=2):
        e = np.zeros(4)
        e[c | (t << 1)] = 1
        out = G.cx() @ e
        assert out[c | ((t ^ c) << 1)] == 1


def full_operator(n, M, qubits):
    """2^n x 2^n operator of M on `qubits`, by brute force over basis states."""
    d = len(qubits)
    U = np.zeros((1 << n, 1 << n), dtype=complex)
    for col in range(1 << n):
        loc_in = sum(((col >> q) & 1) << t for t, q in enumerate(qubits))
        rest = col
        for q in qubits:
            rest &= ~(1 << q)
        for loc_out in range(1 << d):
            row = rest | sum(((loc_out >> t) & 1) << q for t, q in enumerate(qubits))
            U[row, col] += M[loc_out, loc_in]
    return U


@pytest.mark.parametrize("qubits", [(0,), (2,), (0, 2), (2, 0), (1, 3), (3, 1, 0)])
def test_apply_matches_brute_force(qubits):
    n = 4
    rng = np.random.default_rng(7)
    d = 1 << len(qubits)
    M = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    U = full_operator(n, M, qubits)
    out = apply_to_state(psi.reshape((2,) * n), M, qubits).reshape(-1)
    np.testing.assert_allclose(out, U @ psi, atol=1e-12)
    rho = np.outer(psi, psi.conj())
    out_r = apply_to_rho(rho.reshape((2,) * (2 * n)), M, qubits).reshape(1 << n, 1 << n)
    np.testing.assert_allclose(out_r, U @ rho @ U.conj().T, atol=1e-10)


def test_pauli_string_little_endian():
    # labels[0] acts on local bit 0
    P = G.pauli_string([1, 3])  # X on local bit 0, Z on local bit 1
    np.testing.assert_allclose(P, np.kron(Z, X))


def test_gate_matrix_dispatch():
    assert np.allclose(G.gate_matrix(Gate("rx", (0,), 0.4)), G.rx(0.4))
    u = tuple(np.arange(16) * (1 + 1j))
    assert np.allclose(G.gate_matrix(Gate("u2", (0, 1), 0.0, u)), np.array(u).reshape(4, 4))
