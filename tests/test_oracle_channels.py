"""Pins of the oracle's channels, selection rule and thresholds (CPU only).

Each pin is fixed by something other than the oracle's own formula: closed
forms of the channels derived from their Kraus sets (Sec. III-F), exact
rational arithmetic for the thresholds, and the outcome probabilities of the
two-qubit bit-flip example (Fig. 2) stored under tests/golden/.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import channels as chn
from oracle.statevector import apply_kraus_sum
from workloads import Channel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_rho(d, rng):
    A = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    r = A @ A.conj().T
    return r / np.trace(r)


def as_tensor(r, n):
    return r.reshape((2,) * (2 * n))


def kraus_apply(ch, r, n):
    out = apply_kraus_sum(as_tensor(r, n), chn.kraus_ops(ch), list(range(n)))
    return out.reshape(1 << n, 1 << n)


X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.diag([1.0, -1.0]).astype(complex)


@pytest.mark.parametrize("lam", [0.0, 1e-3, 0.3, 1.0])
def test_depol1_closed_form(lam):
    # Sec. III-F one-qubit depolarizing set: E(rho) = (1-lam) rho + lam I/2
    rng = np.random.default_rng(1)
    r = rand_rho(2, rng)
    out = kraus_apply(Channel(0, "depol1", (0,), lam), r, 1)
    np.testing.assert_allclose(out, (1 - lam) * r + lam * np.eye(2) / 2, atol=1e-15)


def test_depol1_bloch_shrink():
    # Bloch vector shrinks by (1-lam)^m after m applications
    lam, m = 0.07, 9
    rng = np.random.default_rng(2)
    r = rand_rho(2, rng)
    bloch = lambda rr: np.real([np.trace(rr @ P) for P in (X, Y, Z)])
    b0 = bloch(r)
    rr = r
    for _ in range(m):
        rr = kraus_apply(Channel(0, "depol1", (0,), lam), rr, 1)
    np.testing.assert_allclose(bloch(rr), (1 - lam) ** m * b0, atol=1e-14)


@pytest.mark.parametrize("lam", [0.0, 1e-2, 0.5])
def test_depol2_closed_form(lam):
    # 16-Pauli two-qubit depolarizing: E(rho) = (1-lam) rho + lam I/4
    rng = np.random.default_rng(3)
    r = rand_rho(4, rng)
    out = kraus_apply(Channel(0, "depol2", (0, 1), lam), r, 2)
    np.testing.assert_allclose(out, (1 - lam) * r + lam * np.eye(4) / 4, atol=1e-15)


@pytest.mark.parametrize("g", [0.0, 5e-3, 0.4])
def test_ampdamp_closed_form(g):
    rng = np.random.default_rng(4)
    r = rand_rho(2, rng)
    out = kraus_apply(Channel(0, "ampdamp", (0,), g), r, 1)
    exp = np.array([[r[0, 0] + g * r[1, 1], math.sqrt(1 - g) * r[0, 1]],
                    [math.sqrt(1 - g) * r[1, 0], (1 - g) * r[1, 1]]])
    np.testing.assert_allclose(out, exp, atol=1e-15)


def test_bitflip_closed_form():
    p = 0.2
    rng = np.random.default_rng(5)
    r = rand_rho(2, rng)
    out = kraus_apply(Channel(0, "bitflip", (0,), p), r, 1)
    np.testing.assert_allclose(out, (1 - p) * r + p * X @ r @ X, atol=1e-15)


CHANNELS = [Channel(0, "bitflip", (0,), 0.1), Channel(0, "depol1", (0,), 0.01),
            Channel(0, "depol2", (0, 1), 0.02), Channel(0, "ampdamp", (0,), 0.3)]


@pytest.mark.parametrize("ch", CHANNELS, ids=lambda c: c.kind)
def test_trace_preserving(ch):
    ops = chn.kraus_ops(ch)
    d = ops[0].shape[0]
    np.testing.assert_allclose(sum(K.conj().T @ K for K in ops), np.eye(d), atol=1e-15)


@pytest.mark.parametrize("ch", CHANNELS, ids=lambda c: c.kind)
def test_selection_unbiased(ch):
    # sum_j q_j (K_j/sqrt q_j) rho (K_j/sqrt q_j)^dag equals the channel
    ops = chn.kraus_ops(ch)
    q = chn.selection_probs(ch)
    assert abs(sum(q) - 1.0) < 1e-15
    n = len(ch.qubits)
    rng = np.random.default_rng(6)
    r = rand_rho(1 << n, rng)
    est = sum(qj * (K / math.sqrt(qj)) @ r @ (K / math.sqrt(qj)).conj().T for K, qj in zip(ops, q))
    np.testing.assert_allclose(est, kraus_apply(ch, r, n), atol=1e-15)
    # q_j = Tr(K_j^dag K_j)/d (the reading of the selection probabilities)
    np.testing.assert_allclose(q, [np.trace(K.conj().T @ K).real / (1 << n) for K in ops], atol=1e-16)


def test_pauli_channels_insert_paulis():
    # Sec. III-G: the inserted operator of a Pauli channel is the Pauli itself
    for ch in CHANNELS[:3]:
        for K, qj in zip(chn.kraus_ops(ch), chn.selection_probs(ch)):
            P = K / math.sqrt(qj)
            np.testing.assert_allclose(P @ P.conj().T, np.eye(P.shape[0]), atol=1e-15)
            assert np.all(np.isclose(np.abs(P), 0) | np.isclose(np.abs(P), 1))


@pytest.mark.parametrize("q", [[0.99925, 0.00025, 0.00025, 0.00025], [0.5, 0.5],
                               [1 - 15 * 0.01 / 16] + [0.01 / 16] * 15, [0.0, 1.0], [1.0, 0.0]])
def test_thresholds_exact(q):
    T = chn.thresholds(q)
    assert T[-1] == 1 << 32
    c = 0.0
    for j in range(len(q) - 1):
        c = c + q[j]
        # exact rational floor of the binary64 cumulative sum times 2^32
        assert T[j] == min(1 << 32, math.floor(Fraction(c) * (1 << 32)))
    assert all(a <= b for a, b in zip(T, T[1:]))


def test_select_ties_go_up():
    T = [10, 20, 1 << 32]
    assert chn.select(9, T) == 0
    assert chn.select(10, T) == 1        # r == T_0 goes to j+1
    assert chn.select(20, T) == 2
    assert chn.select((1 << 32) - 1, T) == 2
    assert chn.select(0, [0, 1 << 32]) == 1  # zero-probability outcome never picked


def test_fig2_two_bitflips_on_cx():
    """Fig. 2: independent bit-flips on both qubits of a cX give the outcome
    probabilities (1-p)^2, p(1-p), p(1-p), p^2."""
    with open(os.path.join(GOLDEN, "fig2_bitflip_cx.json")) as f:
        g = json.load(f)
    p = g["p"]
    q = chn.selection_probs(Channel(0, "bitflip", (0,), p))  # [X, I]
    probs = {"none": q[1] * q[1], "control_only": q[0] * q[1], "target_only": q[1] * q[0],
             "both": q[0] * q[0]}
    for k, v in g["probabilities"].items():
        assert abs(probs[k] - v) < 1e-15, k
    # the sampled frequencies through the oracle's draws follow them
    from workloads import Gate, Problem
    from oracle.simulate import kraus_indices
    prob = Problem(2, [Gate("cx", (0, 1))],
                   [Channel(0, "bitflip", (0,), p), Channel(0, "bitflip", (1,), p)])
    idx = kraus_indices(prob, 77, 0, 200000)
    both = np.mean((idx[:, 0] == 0) & (idx[:, 1] == 0))
    none = np.mean((idx[:, 0] == 1) & (idx[:, 1] == 1))
    assert abs(both - p * p) < 5 * math.sqrt(p * p / 200000)
    assert abs(none - (1 - p) ** 2) < 5 * math.sqrt((1 - p) ** 2 * (1 - (1 - p) ** 2) / 200000)
