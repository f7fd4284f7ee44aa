"""Seeded synthetic inputs for the noisy-QAOA trajectory ensemble.

This module is the only code shared by the CPU oracle (``oracle/``) and the GPU
product path (``paper_2210_15874_amd/``).  It holds input *data* only: graphs,
angles, gate lists, channel lists and the workload table.  It holds none of the
method's arithmetic (no gate matrices, no Kraus operators, no sampling, no
contraction): each side interprets the gate and channel names itself.

Workload shapes follow the paper's experiment (QAOA MaxCut on regular graphs
with depolarizing noise after every gate, Sec. IV Results); the fixed-angle
table the paper uses is not available, so angles are seeded uniform draws in
[0, pi) and graphs are seeded random regular / Erdos-Renyi graphs.

Conventions carried as data:
  * qubit q is bit q of a basis index (little-endian);
  * a gate is (kind, qubits, theta[, matrix]) with kinds
      h, x, y, z                     fixed one-qubit gates
      rx, ry, rz   theta             exp(-i theta P / 2)
      zz           theta             diag(1, e^{-i theta}, e^{-i theta}, 1)
      cx                             control = qubits[0], target = qubits[1]
      u1, u2       matrix            explicit 2x2 / 4x4 complex matrix, row-major,
                                     local index = sum_t bit(qubits[t]) << t
  * a channel is (after_gate, kind, qubits, param[, kraus]) with kinds
      bitflip(p), depol1(lambda), depol2(lambda), ampdamp(gamma), kraus(list)
    Channels attached to the same gate act in list order; a channel's site
    number is its position in the list.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Gate", "Channel", "Problem", "random_regular_graph", "erdos_renyi_graph",
    "uniform_angles", "qaoa_circuit", "depolarizing_noise", "amplitude_damping_after_layers",
    "make_problem", "CONFIGS", "config_problem", "uneven_batch", "poisson_stream",
    "PAPER_EXPERIMENT", "paper_experiment_problem",
]


@dataclass(frozen=True)
class Gate:
    kind: str
    qubits: Tuple[int, ...]
    theta: float = 0.0
    matrix: Optional[Tuple[complex, ...]] = None  # u1 / u2 only, row-major


@dataclass(frozen=True)
class Channel:
    after_gate: int
    kind: str
    qubits: Tuple[int, ...]
    param: float = 0.0
    kraus: Optional[Tuple[Tuple[complex, ...], ...]] = None  # kind == "kraus" only


@dataclass
class Problem:
    """One noisy-circuit job: circuit + noise model + MaxCut observable + K."""
    n_qubits: int
    gates: List[Gate]
    channels: List[Channel]
    edges: List[Tuple[int, int]] = field(default_factory=list)
    weights: List[float] = field(default_factory=list)
    gammas: List[float] = field(default_factory=list)
    betas: List[float] = field(default_factory=list)
    K: int = 0
    seed: int = 0           # Philox key of the job
    name: str = ""

    @property
    def p(self) -> int:
        return len(self.gammas)


# ----------------------------------------------------------------------------- graphs

def random_regular_graph(n: int, d: int, seed: int) -> List[Tuple[int, int]]:
    """Seeded random d-regular simple graph by the pairing (configuration) model
    with rejection.  Edges are returned sorted, each as (u, v) with u < v."""
    if (n * d) % 2 or d >= n:
        raise ValueError("no d-regular graph on n vertices")
    rng = np.random.Generator(np.random.PCG64(seed))
    for _ in range(100000):
        pts = np.repeat(np.arange(n), d)
        rng.shuffle(pts)
        pairs = pts.reshape(-1, 2)
        ok = True
        seen = set()
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            e = (min(a, b), max(a, b))
            if e in seen:
                ok = False
                break
            seen.add(e)
        if ok:
            return sorted(seen)
    raise RuntimeError("pairing model did not converge")


def erdos_renyi_graph(n: int, p_edge: float, seed: int) -> List[Tuple[int, int]]:
    """Seeded G(n, p) graph; may have isolated vertices or no edges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((n, n))
    return [(i, j) for i in range(n) for j in range(i + 1, n) if u[i, j] < p_edge]


def uniform_angles(p: int, seed: int) -> Tuple[List[float], List[float]]:
    """gamma_l, beta_l uniform in [0, pi), l = 1..p."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.random(p) * math.pi
    b = rng.random(p) * math.pi
    return [float(x) for x in g], [float(x) for x in b]


# ----------------------------------------------------------------------------- circuits

def qaoa_circuit(n: int, edges: Sequence[Tuple[int, int]], gammas: Sequence[float],
                 betas: Sequence[float]) -> List[Gate]:
    """QAOA MaxCut ansatz as a gate list: H on every qubit, then for each layer
    a zz(gamma_l) on every edge in sorted order and rx(2 beta_l) on qubits
    0..n-1 (the cost-then-mixer layering of Sec. III-E)."""
    gates = [Gate("h", (q,)) for q in range(n)]
    es = sorted((min(u, v), max(u, v)) for u, v in edges)
    for g, b in zip(gammas, betas):
        gates += [Gate("zz", (u, v), float(g)) for u, v in es]
        gates += [Gate("rx", (q,), 2.0 * float(b)) for q in range(n)]
    return gates


def depolarizing_noise(gates: Sequence[Gate], lam1: float, lam2: float) -> List[Channel]:
    """One depolarizing channel after every gate: depol1(lam1) after one-qubit
    gates, depol2(lam2) after two-qubit gates (Sec. IV: depolarizing noise on
    all of the gates)."""
    ch = []
    for i, g in enumerate(gates):
        if len(g.qubits) == 1:
            if lam1 > 0:
                ch.append(Channel(i, "depol1", g.qubits, float(lam1)))
        else:
            if lam2 > 0:
                ch.append(Channel(i, "depol2", g.qubits, float(lam2)))
    return ch


def amplitude_damping_after_layers(n: int, gates: Sequence[Gate], channels: Sequence[Channel],
                                   gamma: float, p: int) -> List[Channel]:
    """Adds one amplitude-damping channel per qubit after each layer's mixer:
    attached to the rx gate of that qubit in that layer, after its
    depolarizing channel.  Returns the merged list ordered by gate."""
    m = (len(gates) - n) // p - n  # edges per layer
    extra = []
    for layer in range(p):
        first_rx = n + layer * (m + n) + m
        for q in range(n):
            gi = first_rx + q
            assert gates[gi].kind == "rx" and gates[gi].qubits == (q,)
            extra.append(Channel(gi, "ampdamp", (q,), float(gamma)))
    merged = list(channels) + extra
    # stable sort by gate keeps each gate's depolarizing channel first
    order = sorted(range(len(merged)), key=lambda i: (merged[i].after_gate, i >= len(channels), i))
    return [merged[i] for i in order]


def make_problem(n: int, edges, gammas, betas, lam1: float, lam2: float, K: int, seed: int,
                 gamma_ad: float = 0.0, name: str = "") -> Problem:
    gates = qaoa_circuit(n, edges, gammas, betas)
    ch = depolarizing_noise(gates, lam1, lam2)
    if gamma_ad > 0:
        ch = amplitude_damping_after_layers(n, gates, ch, gamma_ad, len(gammas))
    es = sorted((min(u, v), max(u, v)) for u, v in edges)
    return Problem(n, gates, ch, es, [1.0] * len(es), list(gammas), list(betas), K, seed, name)


# ----------------------------------------------------------------------------- workload table

# Seeds: graph 1000+i, angles 2000+i, Philox key 3000+i for workload i.
CONFIGS = {
    0: dict(name="qaoa-n6-p1-3reg-K100", n=6, d=3, p=1, lam1=1e-3, lam2=1e-2, gamma_ad=0.0, K=100),
    1: dict(name="qaoa-n12-p2-3reg-ad-K1024", n=12, d=3, p=2, lam1=1e-3, lam2=1e-2, gamma_ad=5e-3, K=1024),
    2: dict(name="qaoa-n26-p4-3reg-K4096", n=26, d=3, p=4, lam1=1e-3, lam2=1e-2, gamma_ad=0.0, K=4096),
}


def config_problem(i: int, K: Optional[int] = None) -> Problem:
    c = CONFIGS[i]
    edges = random_regular_graph(c["n"], c["d"], 1000 + i)
    g, b = uniform_angles(c["p"], 2000 + i)
    return make_problem(c["n"], edges, g, b, c["lam1"], c["lam2"], K if K is not None else c["K"],
                        3000 + i, gamma_ad=c["gamma_ad"], name=c["name"])


def uneven_batch(n_jobs: int = 64, seed: int = 1003, n_range=(10, 30), p_range=(1, 6),
                 K_range=(256, 8192), lam1: float = 1e-3, lam2: float = 1e-2) -> List[Problem]:
    """Uneven batch of QAOA jobs: n, p, K uniform integers in the given ranges,
    Erdos-Renyi graphs with edge probability 3/(n-1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for j in range(n_jobs):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        gseed, aseed = int(rng.integers(1 << 31)), int(rng.integers(1 << 31))
        edges = erdos_renyi_graph(n, 3.0 / (n - 1), gseed)
        g, b = uniform_angles(p, aseed)
        jobs.append(make_problem(n, edges, g, b, lam1, lam2, K, int(rng.integers(1 << 62)),
                                 name=f"er-n{n}-p{p}-K{K}-j{j}"))
    return jobs


def poisson_stream(n_jobs: int, rate_per_s: float = 200.0, seed: int = 1004, n_range=(10, 30),
                   p_range=(1, 6), K_range=(256, 8192), lam_range=(1e-4, 1e-2)):
    """Arrival times (s) and jobs of a Poisson stream of noisy-QAOA energy jobs;
    depolarizing rates are drawn log-uniformly and independently for 1q / 2q."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, jobs = [], []
    now = 0.0
    lo, hi = math.log(lam_range[0]), math.log(lam_range[1])
    for j in range(n_jobs):   # one job at a time: the first m arrivals do not depend on n_jobs
        now += float(rng.exponential(1.0 / rate_per_s))
        t.append(now)
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        K = int(rng.integers(K_range[0], K_range[1] + 1))
        l1, l2 = math.exp(rng.uniform(lo, hi)), math.exp(rng.uniform(lo, hi))
        edges = erdos_renyi_graph(n, 3.0 / (n - 1), int(rng.integers(1 << 31)))
        g, b = uniform_angles(p, int(rng.integers(1 << 31)))
        jobs.append(make_problem(n, edges, g, b, l1, l2, K, int(rng.integers(1 << 62)),
                                 name=f"stream-n{n}-p{p}-K{K}-j{j}"))
    return t, jobs


# ----------------------------------------------------------------------------- the paper's own experiment

# Sec. IV: QAOA p=2 on 4-regular graphs, depolarizing noise on every gate
# (lambda_1 = 0.001 after one-qubit gates, lambda_2 = 0.004 after two-qubit
# gates), ensembles of 10 .. 1,780 circuits, fixed angles.  The paper's
# fixed-angle table is not available: one seeded angle pair is used for every
# size, namely the first seed from 2100 on whose noiseless output distribution
# has fidelity between 0.85 and 0.95 with the uniform one at n = 6, 8 and 10
# (the paper fixed its angles so that the output is neither close to uniform
# nor to the noiseless state).  Sizes n = 5 .. 12 (a 4-regular graph needs
# n >= 5), three seeded graphs per size, independent Philox keys per repetition.
PAPER_EXPERIMENT = dict(p=2, d=4, lam1=1e-3, lam2=4e-3, n_range=(5, 12), graphs=3,
                        K_values=(10, 20, 50, 100, 200, 500, 1000, 1780), angle_seed=2104)


def paper_experiment_problem(n: int, graph: int = 0, rep: int = 0, K: int = 1780) -> Problem:
    c = PAPER_EXPERIMENT
    edges = random_regular_graph(n, c["d"], 5000 + 100 * graph + n)
    g, b = uniform_angles(c["p"], c["angle_seed"])
    seed = 9_000_000 + (graph * 1024 + rep) * 64 + n
    return make_problem(n, edges, g, b, c["lam1"], c["lam2"], K, seed,
                        name=f"paper-exp-n{n}-g{graph}-r{rep}")
