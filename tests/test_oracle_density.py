"""Pins of the exact density-matrix oracle and the trajectory estimator on the
same draws (CPU only): invariants, the noiseless limit against the p=1 QAOA
closed form, exhaustive enumeration of Kraus outcomes, the superoperator form
against the literal operator sum (Eq.(1))."""
import itertools
import math

import numpy as np
import pytest

from oracle import channels as chn
from oracle import simulate as sim
from oracle.statevector import apply_kraus_sum
from workloads import Channel, Gate, Problem, config_problem, make_problem, random_regular_graph


def qaoa_p1_edge(gamma, beta, du, dv, t):
    """Wang, Hadfield, Jiang, Rieffel, PRA 97, 022304 (2018): <C_uv> at p=1,
    du/dv = degree-1 of the endpoints, t = triangles through the edge."""
    s4b, s2b = math.sin(4 * beta), math.sin(2 * beta)
    cg = math.cos(gamma)
    return (0.5 + 0.25 * s4b * math.sin(gamma) * (cg ** du + cg ** dv)
            - 0.25 * s2b ** 2 * cg ** (du + dv - 2 * t) * (1 - math.cos(2 * gamma) ** t))


def closed_form_energy(n, edges, gamma, beta):
    nb = {q: set() for q in range(n)}
    for u, v in edges:
        nb[u].add(v)
        nb[v].add(u)
    return sum(qaoa_p1_edge(gamma, beta, len(nb[u]) - 1, len(nb[v]) - 1, len(nb[u] & nb[v]))
               for u, v in edges)


@pytest.mark.parametrize("edges,n", [
    (random_regular_graph(6, 3, 1000), 6),
    ([(0, 1), (1, 2), (0, 2), (2, 3), (3, 4)], 5),          # has a triangle
    (random_regular_graph(8, 3, 5), 8),
])
@pytest.mark.parametrize("gamma,beta", [(0.7, 0.3), (2.9, 1.1), (1.8, 2.06)])
def test_noiseless_p1_closed_form(edges, n, gamma, beta):
    pr = make_problem(n, edges, [gamma], [beta], 0.0, 0.0, 4, 1)
    psi = sim.noiseless_state(pr)
    e = sim.energy(psi, n, pr.edges, pr.weights)
    assert abs(e - closed_form_energy(n, pr.edges, gamma, beta)) < 1e-12
    # noiseless limit: rho = |psi><psi| and every trajectory is psi
    rho = sim.density_matrix(pr)
    np.testing.assert_allclose(rho, np.outer(psi, psi.conj()), atol=1e-13)
    ens = sim.ensemble(pr, 9, 0, 4)
    np.testing.assert_allclose(ens["rho_hat"], rho, atol=1e-13)
    assert np.all(ens["idx"] == 0)


def test_dm_invariants_config0():
    pr = config_problem(0)
    rho = sim.density_matrix(pr)
    assert abs(np.trace(rho) - 1) < 1e-12
    np.testing.assert_allclose(rho, rho.conj().T, atol=1e-14)
    assert np.linalg.eigvalsh(rho).min() > -1e-12


def test_dm_invariants_with_ampdamp():
    edges = random_regular_graph(6, 3, 42)
    pr = make_problem(6, edges, [0.4, 1.3], [0.9, 0.2], 0.05, 0.1, 4, 3, gamma_ad=0.2)
    rho = sim.density_matrix(pr)
    assert abs(np.trace(rho) - 1) < 1e-12
    np.testing.assert_allclose(rho, rho.conj().T, atol=1e-14)
    assert np.linalg.eigvalsh(rho).min() > -1e-12
    assert any(c.kind == "ampdamp" for c in pr.channels)


def test_superoperator_equals_kraus_sum():
    edges = [(0, 1), (1, 2)]
    pr = make_problem(3, edges, [0.5], [0.8], 0.1, 0.2, 1, 1, gamma_ad=0.3)
    np.testing.assert_allclose(sim.density_matrix(pr), sim.density_matrix(pr, literal=True), atol=1e-15)


def tiny_problems():
    yield Problem(2, [Gate("h", (0,)), Gate("cx", (0, 1)), Gate("rx", (1,), 0.7)],
                  [Channel(0, "bitflip", (0,), 0.2), Channel(1, "depol2", (0, 1), 0.3),
                   Channel(2, "ampdamp", (1,), 0.25), Channel(2, "depol1", (1,), 0.1)])
    yield Problem(3, [Gate("h", (0,)), Gate("h", (2,)), Gate("zz", (0, 2), 1.1), Gate("ry", (1,), 0.4)],
                  [Channel(0, "depol1", (0,), 0.2), Channel(2, "depol2", (0, 2), 0.15),
                   Channel(3, "bitflip", (1,), 0.3)])


@pytest.mark.parametrize("pr", list(tiny_problems()))
def test_exhaustive_enumeration_equals_dm(pr):
    """Sum over every tuple of Kraus outcomes of prod(q) psi psi^dag equals the
    exact rho: the estimator is unbiased, with no stochastic error."""
    tabs = sim.site_tables(pr)
    sizes = [len(t[0]) for t in tabs]
    acc = 0
    for tup in itertools.product(*[range(s) for s in sizes]):
        w = math.prod(tabs[s][0][j] for s, j in enumerate(tup))
        if w == 0:
            continue
        psi = sim.trajectory(pr, np.array(tup), tabs)
        acc = acc + w * np.outer(psi, psi.conj())
    np.testing.assert_allclose(acc, sim.density_matrix(pr), atol=1e-13)


def test_fig1_bitflip_after_h():
    # Fig. 1: H, then X with probability p.  X|+> = |+>, so rho = |+><+| for any p
    p = 0.3
    pr = Problem(1, [Gate("h", (0,))], [Channel(0, "bitflip", (0,), p)])
    rho = sim.density_matrix(pr)
    np.testing.assert_allclose(rho, 0.5 * np.ones((2, 2)), atol=1e-15)
    ens = sim.ensemble(pr, 3, 0, 50)
    np.testing.assert_allclose(ens["rho_hat"], rho, atol=1e-15)


def test_trajectories_unit_norm_for_pauli_noise():
    pr = config_problem(0, K=40)
    ens = sim.ensemble(pr, pr.seed, 0, 40)
    np.testing.assert_allclose(np.linalg.norm(ens["psi"], axis=1), 1.0, atol=1e-13)
    assert abs(np.trace(ens["rho_hat"]) - 1) < 1e-12
    assert np.linalg.eigvalsh(ens["rho_hat"]).min() > -1e-12
    # sigma_approx is the diagonal of rho_hat
    np.testing.assert_allclose(ens["sigma_approx"], np.diag(ens["rho_hat"]).real, atol=1e-15)


def test_kraus_indices_follow_thresholds():
    pr = config_problem(0)
    from oracle.philox import site_draws
    r = site_draws(pr.seed, 5, 20, len(pr.channels))
    idx = sim.kraus_indices(pr, pr.seed, 5, 20)
    for s, ch in enumerate(pr.channels):
        T = chn.thresholds(chn.selection_probs(ch))
        for k in range(20):
            assert idx[k, s] == chn.select(int(r[k, s]), T)
    # draws depend on k only, not on the range they are requested in
    np.testing.assert_array_equal(sim.kraus_indices(pr, pr.seed, 0, 25)[5:], idx)
