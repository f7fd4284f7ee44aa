"""Seeded random circuits and noise models for the tests (every gate kind,
explicit 2x2 / 4x4 unitaries, every channel kind including explicit Kraus
channels with 1..4 operators, several channels after one gate, gates without
noise, a random weighted observable)."""
import numpy as np


def random_unitary(rng, d):
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def random_kraus(rng, d, J):
    """J operators with sum K^dagger K = I: blocks of an isometry (dJ x d)."""
    z = rng.normal(size=(d * J, d)) + 1j * rng.normal(size=(d * J, d))
    q, _ = np.linalg.qr(z)
    return [q[j * d:(j + 1) * d, :] for j in range(J)]


def random_problem(seed, n_range=(1, 8)):
    """n uniform in n_range (inclusive); gates of every kind with random
    angles and explicit unitaries, 0..2 channels of every kind after each."""
    from workloads import Channel, Gate, Problem
    rng = np.random.default_rng(seed)
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    kinds1 = ["h", "x", "y", "z", "rx", "ry", "rz", "u1"]
    kinds2 = ["zz", "cx", "u2"]
    gates, chans = [], []
    for g in range(int(rng.integers(n, 4 * n + 2))):
        two = n >= 2 and rng.random() < 0.4
        if two:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            k = kinds2[int(rng.integers(len(kinds2)))]
            mat = tuple(random_unitary(rng, 4).reshape(-1)) if k == "u2" else None
            gates.append(Gate(k, (a, b), float(rng.uniform(-np.pi, np.pi)), mat))
        else:
            a = int(rng.integers(n))
            k = kinds1[int(rng.integers(len(kinds1)))]
            mat = tuple(random_unitary(rng, 2).reshape(-1)) if k == "u1" else None
            gates.append(Gate(k, (a,), float(rng.uniform(-np.pi, np.pi)), mat))
        for _ in range(int(rng.choice([0, 1, 1, 2]))):
            qs = gates[-1].qubits
            if len(qs) == 2 and rng.random() < 0.5:
                ck = ["depol2", "kraus"][int(rng.integers(2))]
                cq = qs
            else:
                ck = ["bitflip", "depol1", "ampdamp", "kraus"][int(rng.integers(4))]
                cq = (qs[int(rng.integers(len(qs)))],)
            if ck == "kraus":
                d = 2 ** len(cq)
                ops = random_kraus(rng, d, int(rng.integers(1, 5)))
                chans.append(Channel(g, "kraus", cq, 0.0, tuple(tuple(o.reshape(-1)) for o in ops)))
            else:
                chans.append(Channel(g, ck, cq, float(rng.uniform(0.0, 0.3))))
    edges = []
    if n >= 2:
        for _ in range(int(rng.integers(1, 2 * n))):
            a, b = sorted(int(x) for x in rng.choice(n, size=2, replace=False))
            if (a, b) not in edges:
                edges.append((a, b))
    weights = [float(w) for w in rng.uniform(0.1, 2.0, size=len(edges))]
    return Problem(n, gates, chans, edges, weights, [], [], 24, int(rng.integers(1 << 40)), f"random-{seed}")
