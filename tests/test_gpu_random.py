"""Seeded random circuits on 1..8 qubits (every gate kind, explicit 2x2 /
4x4 unitaries, every channel kind including explicit Kraus channels with
1..4 operators, several channels after one gate, gates without noise)
through the whole-state-in-LDS lowering, against the oracle's literal
Kraus insertion on the same draws: rho_hat, sigma and per-trajectory
energies."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_15874_amd as stn
    stn.load()
    torch.cuda.set_device(0)


def random_unitary(rng, d):
    z = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def random_kraus(rng, d, J):
    """J operators with sum K^dagger K = I: blocks of an isometry (dJ x d)."""
    z = rng.normal(size=(d * J, d)) + 1j * rng.normal(size=(d * J, d))
    q, _ = np.linalg.qr(z)
    return [q[j * d:(j + 1) * d, :] for j in range(J)]


def random_problem(seed):
    from workloads import Channel, Gate, Problem
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
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


@pytest.mark.parametrize("precision,tol", [(128, 1e-12), (64, 1e-5)])
@pytest.mark.parametrize("seed", list(range(16)))
def test_random_circuit_against_oracle(seed, precision, tol):
    from oracle import simulate as sim
    import paper_2210_15874_amd as stn
    pr = random_problem(seed)
    outputs = stn.OUT_RHO | stn.OUT_DIAG | (stn.OUT_ENERGY if pr.edges else 0)
    res = stn.simulate_batch_ensemble(pr, outputs=outputs, precision=precision)
    ens = sim.ensemble(pr, pr.seed, 0, pr.K)
    scale = max(1.0, float(np.abs(ens["rho_hat"]).max()))
    assert np.abs(res["rho"] - ens["rho_hat"]).max() / scale < tol
    assert np.abs(res["diag"] - ens["sigma_approx"]).max() / scale < tol
    if pr.edges:
        m = sum(pr.weights)
        assert abs(res["energy_mean"] - ens["energies"].mean()) / m < tol
        np.testing.assert_allclose(res["energies"] / m, ens["energies"] / m, atol=tol)


@pytest.mark.parametrize("precision,tol", [(128, 1e-12), (64, 1e-5)])
def test_one_qubit_and_one_trajectory(precision, tol):
    """Degenerate sizes: one qubit (no observable), a single trajectory,
    a channel with a single (unitary) Kraus operator."""
    from oracle import simulate as sim
    from workloads import Channel, Gate, Problem
    import paper_2210_15874_amd as stn
    rng = np.random.default_rng(5)
    u = tuple(random_unitary(rng, 2).reshape(-1))
    one = tuple(tuple(o.reshape(-1)) for o in random_kraus(rng, 2, 1))
    pr = Problem(1, [Gate("h", (0,)), Gate("u1", (0,), 0.0, u), Gate("ry", (0,), 0.7)],
                 [Channel(0, "ampdamp", (0,), 0.3), Channel(1, "kraus", (0,), 0.0, one),
                  Channel(1, "bitflip", (0,), 0.4)], [], [], [], [], 1, 99, "one-qubit")
    for K in (1, 7):
        res = stn.simulate_batch_ensemble(pr, K=K, outputs=stn.OUT_RHO | stn.OUT_DIAG, precision=precision)
        ens = sim.ensemble(pr, pr.seed, 0, K)
        assert res["k_done"] == K
        assert np.abs(res["rho"] - ens["rho_hat"]).max() < tol
