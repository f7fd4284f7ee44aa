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


from random_circuits import random_kraus, random_problem, random_unitary  # noqa: E402


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
