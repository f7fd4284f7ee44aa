"""Statistical pins of the ensemble estimator (CPU only).

* For unit-norm trajectories E||rho_hat - rho||_F^2 = (1 - Tr rho^2) / K exactly
  (the variance of an average of K i.i.d. projectors with mean rho), so the
  Frobenius error falls as K^(-1/2).
* The diagonal infidelity of Eq.(2) is second order in the deviation of
  sigma_approx, so its expectation falls as 1/K (the paper's observation in
  Sec. IV that Error is proportional to 1/K).
* <C>_hat is unbiased for Tr(rho C).
"""
import math

import numpy as np

from oracle import metrics
from oracle import simulate as sim
from workloads import make_problem, random_regular_graph


def strong_noise_problem():
    edges = random_regular_graph(4, 3, 8)
    return make_problem(4, edges, [0.9, 2.1], [0.6, 1.9], 0.08, 0.15, 1, 12345)


def test_frobenius_law_and_slope():
    pr = strong_noise_problem()
    rho = sim.density_matrix(pr)
    purity = float(np.real(np.trace(rho @ rho)))
    R, Kmax = 150, 32
    ens = sim.ensemble(pr, pr.seed, 0, R * Kmax)
    Psi = ens["psi"].reshape(R, Kmax, -1)
    means = {}
    for K in (2, 8, 32):
        errs = []
        for r in range(R):
            P = Psi[r, :K]
            rh = P.T @ P.conj() / K
            errs.append(np.linalg.norm(rh - rho) ** 2)
        errs = np.array(errs)
        pred = (1 - purity) / K
        # mean over R repetitions within 4 standard errors of the exact law
        assert abs(errs.mean() - pred) < 4 * errs.std(ddof=1) / math.sqrt(R) + 1e-12, (K, errs.mean(), pred)
        means[K] = math.sqrt(errs.mean())
    slope = np.polyfit(np.log([2, 8, 32]), np.log([means[2], means[8], means[32]]), 1)[0]
    assert abs(slope + 0.5) < 0.08


def test_paper_error_falls_as_one_over_K():
    pr = strong_noise_problem()
    rho = sim.density_matrix(pr)
    sig = np.diag(rho).real
    R, Kmax = 120, 64
    ens = sim.ensemble(pr, pr.seed + 1, 0, R * Kmax)
    P2 = (np.abs(ens["psi"]) ** 2).reshape(R, Kmax, -1)
    Ks = [4, 16, 64]
    e = [np.mean([metrics.paper_error(P2[r, :K].mean(0), sig) for r in range(R)]) for K in Ks]
    slope = np.polyfit(np.log(Ks), np.log(e), 1)[0]
    assert abs(slope + 1.0) < 0.15, slope


def test_energy_unbiased():
    pr = strong_noise_problem()
    rho = sim.density_matrix(pr)
    exact = sim.energy_exact(rho, pr.n_qubits, pr.edges, pr.weights)
    ens = sim.ensemble(pr, pr.seed + 2, 0, 3000, want_states=False)
    en = ens["energies"]
    assert abs(en.mean() - exact) < 4 * en.std(ddof=1) / math.sqrt(len(en))


def test_uhlmann_paths_agree_and_fidelity_bounds():
    pr = strong_noise_problem()
    rho = sim.density_matrix(pr)
    ens = sim.ensemble(pr, pr.seed + 3, 0, 64)
    f1 = metrics.uhlmann_fidelity(rho, ens["rho_hat"])
    f2 = metrics.uhlmann_fidelity_from_states(rho, ens["psi"], 64)
    assert abs(f1 - f2) < 1e-9 and 0 < f1 <= 1
    assert abs(metrics.uhlmann_fidelity(rho, rho) - 1) < 1e-9
    # pure states: F = |<a|b>|^2; diagonal states: classical fidelity
    a = np.array([1, 1j, 0, 0]) / math.sqrt(2)
    b = np.array([1, 0, 1, 0]) / math.sqrt(2)
    assert abs(metrics.uhlmann_fidelity(np.outer(a, a.conj()), np.outer(b, b.conj())) - 0.25) < 1e-9
    p, q = np.array([0.5, 0.25, 0.25, 0]), np.array([0.25, 0.25, 0.25, 0.25])
    assert abs(metrics.uhlmann_fidelity(np.diag(p), np.diag(q)) - np.sum(np.sqrt(p * q)) ** 2) < 1e-12
    assert abs(metrics.paper_error(p, q) - (1 - np.sum(np.sqrt(p * q)) ** 2)) < 1e-15
    assert metrics.paper_error(p, p) < 1e-15
    assert abs(metrics.paper_error(np.array([1, 0]), np.array([0, 1])) - 1) < 1e-15
    assert abs(metrics.trace_distance(np.diag(p), np.diag(q)) - 0.5 * np.abs(p - q).sum()) < 1e-12


def test_stored_sigma_exact_fixture_is_consistent():
    """tests/golden/config1_sigma_exact.json (the oracle's exact diagonal of the
    n=12 workload, the reference of the rho_hat bench leg's Eq. (2) sweep) is a
    probability vector whose stored energy is its cut-size expectation, with
    the cut size counted here bit by bit."""
    import json
    import os
    from workloads import config_problem
    path = os.path.join(os.path.dirname(__file__), "golden", "config1_sigma_exact.json")
    with open(path) as f:
        g = json.load(f)
    sig = np.array(g["sigma_exact"])
    pr = config_problem(1)
    assert g["n_qubits"] == pr.n_qubits and sig.shape == (1 << pr.n_qubits,)
    assert sig.min() > -1e-15 and abs(sig.sum() - 1.0) < 1e-12 and abs(g["trace"] - 1.0) < 1e-12
    cut = [sum(w for (u, v), w in zip(pr.edges, pr.weights) if ((z >> u) & 1) != ((z >> v) & 1))
           for z in range(1 << pr.n_qubits)]
    assert abs(float(np.dot(sig, cut)) - g["energy_exact"]) < 1e-10
