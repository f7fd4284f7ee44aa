"""Pins of the oracle's explicit-Kraus channel branch (CPU only).

A channel of kind "kraus" carries its operators as row-major flattened
complex matrices; the oracle reads the dimension from their length, reshapes
them, and takes q_j = Tr(K_j^dagger K_j)/d (Sec. III-G selection reading).
Nothing here reuses the oracle's own channel formulas as the reference:

* explicit listings of the paper's channels (Sec. III-F), typed here, must
  act as the closed forms (1-lam) rho + lam I/2, (1-lam) rho + lam I/4 and
  the amplitude-damping map, and must give the paper's squared coefficients
  as selection probabilities;
* a non-symmetric two-qubit set (amplitude damping on the first qubit of the
  pair, the identity on the second) pins the row-major reshape and the
  little-endian local index: a transposed or qubit-swapped reading damps the
  wrong way or the wrong qubit;
* random CPTP sets from a Stinespring isometry, whose exact action is
  computed here from the isometry with full-space matrices built by kron,
  pin unbiasedness by exhaustive enumeration of the oracle's trajectories,
  and sum_j q_j = 1 (a wrong dimension breaks it).
"""
import itertools
import math

import numpy as np
import pytest

from oracle import channels as chn
from oracle import simulate as sim
from workloads import Channel, Gate, Problem

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
PAULI = [I2, PX, PY, PZ]


def flat(m):
    return tuple(complex(v) for v in np.asarray(m).reshape(-1))


def rand_rho(d, rng):
    A = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    r = A @ A.conj().T
    return r / np.trace(r)


def embed(M, qubits, n):
    """Full 2^n x 2^n matrix of the local operator M (local index = bit(q0) +
    2 bit(q1)) by explicit index arithmetic, independent of the oracle."""
    N = 1 << n
    out = np.zeros((N, N), dtype=complex)
    k = len(qubits)
    rest_mask = ~sum(1 << q for q in qubits) & (N - 1)
    for col in range(N):
        lc = sum(((col >> q) & 1) << t for t, q in enumerate(qubits))
        for lr in range(1 << k):
            row = col & rest_mask
            for t, q in enumerate(qubits):
                row |= ((lr >> t) & 1) << q
            out[row, col] += M[lr, lc]
    return out


def dm_reference(n, gates, chans, ops_by_site):
    """Exact rho with full-space matrices: gates via the oracle's pinned local
    matrices embedded here, channels via the test's own Kraus matrices."""
    from oracle.gates import gate_matrix
    rho = np.zeros((1 << n, 1 << n), dtype=complex)
    rho[0, 0] = 1.0
    for i, g in enumerate(gates):
        U = embed(gate_matrix(g), g.qubits, n)
        rho = U @ rho @ U.conj().T
        for s, ch in enumerate(chans):
            if ch.after_gate != i:
                continue
            acc = np.zeros_like(rho)
            for K in ops_by_site[s]:
                E = embed(K, ch.qubits, n)
                acc += E @ rho @ E.conj().T
            rho = acc
    return rho


def kraus_channel(after, qubits, mats):
    return Channel(after, "kraus", tuple(qubits), 0.0, tuple(flat(m) for m in mats))


def prep_gates(n):
    # a generic entangled start so that every channel acts on a non-trivial state
    g = []
    for q in range(n):
        g.append(Gate("ry", (q,), 0.3 + 0.4 * q))
        g.append(Gate("rz", (q,), 0.9 - 0.2 * q))
    for q in range(n - 1):
        g.append(Gate("cx", (q, q + 1)))
    return g


def channel_on_rho(ch, r):
    """The oracle's Kraus operators of ch applied to the matrix r by the
    operator sum (its tensor application is pinned against brute-force
    operators elsewhere)."""
    from oracle.statevector import apply_kraus_sum
    n = max(ch.qubits) + 1
    out = apply_kraus_sum(r.reshape((2,) * (2 * n)), chn.kraus_ops(ch), list(ch.qubits))
    return out.reshape(1 << n, 1 << n), len(ch.qubits)


@pytest.mark.parametrize("lam", [1e-3, 0.3, 1.0])
def test_explicit_depol1_listing(lam):
    mats = [math.sqrt(1 - 3 * lam / 4) * I2] + [math.sqrt(lam / 4) * P for P in PAULI[1:]]
    ch = kraus_channel(0, (0,), mats)
    q = chn.selection_probs(ch)
    np.testing.assert_allclose(q, [1 - 3 * lam / 4, lam / 4, lam / 4, lam / 4], rtol=1e-15, atol=1e-17)
    rng = np.random.default_rng(11)
    r = rand_rho(2, rng)
    out, _ = channel_on_rho(ch, r)
    np.testing.assert_allclose(out, (1 - lam) * r + lam * np.eye(2) / 2, atol=1e-15)
    # the inserted operators K_j/sqrt(q_j) are the Paulis themselves
    for K, qj, P in zip(chn.kraus_ops(ch), q, PAULI):
        np.testing.assert_allclose(K / math.sqrt(qj), P, atol=1e-15)


@pytest.mark.parametrize("lam", [1e-2, 0.5])
def test_explicit_depol2_listing(lam):
    mats = []
    for a in range(4):
        for b in range(4):
            w = 1 - 15 * lam / 16 if (a, b) == (0, 0) else lam / 16
            # P_a on local bit 0 (the high index of kron is local bit 1)
            mats.append(math.sqrt(w) * np.kron(PAULI[b], PAULI[a]))
    ch = kraus_channel(0, (0, 1), mats)
    q = chn.selection_probs(ch)
    assert len(q) == 16
    np.testing.assert_allclose(q, [1 - 15 * lam / 16] + [lam / 16] * 15, rtol=1e-15, atol=1e-17)
    rng = np.random.default_rng(12)
    r = rand_rho(4, rng)
    out, _ = channel_on_rho(ch, r)
    np.testing.assert_allclose(out, (1 - lam) * r + lam * np.eye(4) / 4, atol=1e-15)


@pytest.mark.parametrize("g", [5e-3, 0.4])
def test_explicit_ampdamp_listing(g):
    K0 = np.array([[1, 0], [0, math.sqrt(1 - g)]], dtype=complex)
    K1 = np.array([[0, math.sqrt(g)], [0, 0]], dtype=complex)
    ch = kraus_channel(0, (0,), [K0, K1])
    np.testing.assert_allclose(chn.selection_probs(ch), [1 - g / 2, g / 2], rtol=1e-15)
    rng = np.random.default_rng(13)
    r = rand_rho(2, rng)
    out, _ = channel_on_rho(ch, r)
    exp = np.array([[r[0, 0] + g * r[1, 1], math.sqrt(1 - g) * r[0, 1]],
                    [math.sqrt(1 - g) * r[1, 0], (1 - g) * r[1, 1]]])
    np.testing.assert_allclose(out, exp, atol=1e-15)


@pytest.mark.parametrize("pair", [(0, 1), (1, 0), (2, 0)])
def test_explicit_two_qubit_set_orientation(pair):
    """Amplitude damping on the pair's first qubit, identity on the second, as
    a 4x4 explicit set: only qubit pair[0] decays toward |0>."""
    g = 0.3
    K0 = np.array([[1, 0], [0, math.sqrt(1 - g)]], dtype=complex)
    K1 = np.array([[0, math.sqrt(g)], [0, 0]], dtype=complex)
    # local index = bit(pair[0]) + 2 bit(pair[1]); kron(A, B) puts A on local bit 1
    mats = [np.kron(I2, K0), np.kron(I2, K1)]
    n = 3
    gates = prep_gates(n)
    last = len(gates) - 1
    ch = kraus_channel(last, pair, mats)
    np.testing.assert_allclose(chn.selection_probs(ch), [1 - g / 2, g / 2], rtol=1e-15)
    got = sim.density_matrix(Problem(n, gates, [ch]))
    before = sim.density_matrix(Problem(n, gates, []))
    # closed form on qubit a = pair[0], written with basis-index arithmetic
    a = pair[0]
    exp = np.zeros_like(before)
    N = 1 << n
    for i in range(N):
        for j in range(N):
            bi, bj = (i >> a) & 1, (j >> a) & 1
            if bi == 0 and bj == 0:
                exp[i, j] = before[i, j] + g * before[i | (1 << a), j | (1 << a)]
            elif bi == 1 and bj == 1:
                exp[i, j] = (1 - g) * before[i, j]
            else:
                exp[i, j] = math.sqrt(1 - g) * before[i, j]
    np.testing.assert_allclose(got, exp, atol=1e-14)
    # and it equals the named channel on that qubit
    named = sim.density_matrix(Problem(n, gates, [Channel(last, "ampdamp", (a,), g)]))
    np.testing.assert_allclose(got, named, atol=1e-14)


def stinespring_kraus(d, J, rng):
    """J Kraus matrices of a random CPTP map on C^d: blocks of an isometry
    V (J d x d), K_j = V[j d:(j+1) d, :], so sum_j K_j^dag K_j = V^dag V = I."""
    A = rng.normal(size=(J * d, d)) + 1j * rng.normal(size=(J * d, d))
    Q, R = np.linalg.qr(A)
    Q = Q * (np.diag(R) / np.abs(np.diag(R)))  # fix column phases (any isometry will do)
    return [Q[j * d:(j + 1) * d, :] for j in range(J)]


def random_kraus_problem(seed):
    rng = np.random.default_rng(seed)
    n = 3
    gates = prep_gates(n) + [Gate("h", (2,)), Gate("zz", (0, 2), 0.8)]
    ops = [stinespring_kraus(2, 3, rng), stinespring_kraus(4, 4, rng), stinespring_kraus(2, 2, rng)]
    chans = [kraus_channel(1, (1,), ops[0]),
             kraus_channel(len(gates) - 2, (2, 0), ops[1]),
             kraus_channel(len(gates) - 1, (1,), ops[2])]
    return Problem(n, gates, chans), ops


@pytest.mark.parametrize("seed", [21, 22])
def test_random_cptp_selection_sums_to_one(seed):
    pr, ops = random_kraus_problem(seed)
    for ch, mats in zip(pr.channels, ops):
        q = chn.selection_probs(ch)
        assert len(q) == len(mats)
        assert abs(sum(q) - 1.0) < 1e-14
        assert all(v > 0 for v in q)
        T = chn.thresholds(q)
        assert T[-1] == 1 << 32 and all(a <= b for a, b in zip(T, T[1:]))
        # the oracle's operators are the test's matrices, not their transposes
        for K, M in zip(chn.kraus_ops(ch), mats):
            np.testing.assert_allclose(K, M, atol=1e-15)


@pytest.mark.parametrize("seed", [21, 22])
def test_random_cptp_exhaustive_enumeration(seed):
    """Sum over all outcome tuples of prod(q) psi psi^dag (the oracle's
    trajectories with K_j/sqrt(q_j) inserted) equals the exact map computed
    from the isometries: unbiased with no stochastic error."""
    pr, ops = random_kraus_problem(seed)
    ref = dm_reference(pr.n_qubits, pr.gates, pr.channels, ops)
    assert abs(np.trace(ref) - 1) < 1e-13
    np.testing.assert_allclose(sim.density_matrix(pr), ref, atol=1e-13)
    np.testing.assert_allclose(sim.density_matrix(pr, literal=True), ref, atol=1e-13)
    tabs = sim.site_tables(pr)
    acc = 0
    for tup in itertools.product(*[range(len(t[0])) for t in tabs]):
        w = math.prod(tabs[s][0][j] for s, j in enumerate(tup))
        psi = sim.trajectory(pr, np.array(tup), tabs)
        acc = acc + w * np.outer(psi, psi.conj())
    np.testing.assert_allclose(acc, ref, atol=1e-13)


def test_random_cptp_draw_frequencies():
    """The Philox draws pick outcome j of an explicit set with frequency q_j."""
    pr, _ = random_kraus_problem(23)
    K = 100000
    idx = sim.kraus_indices(pr, 4242, 0, K)
    for s, ch in enumerate(pr.channels):
        q = chn.selection_probs(ch)
        for j, qj in enumerate(q):
            f = float(np.mean(idx[:, s] == j))
            assert abs(f - qj) < 5 * math.sqrt(qj * (1 - qj) / K) + 1e-12, (s, j, f, qj)
