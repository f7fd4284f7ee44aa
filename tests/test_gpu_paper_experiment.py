"""The paper's own experiment (Sec. IV; Eq. (2); Eq. (3)) on the GPU path.

QAOA p=2 on 4-regular graphs with depolarizing noise on every gate
(lambda_1 = 0.001, lambda_2 = 0.004), n = 5 .. 12, three graphs per n, one
seeded angle pair (the paper's fixed-angle table is not available), ensembles
of K = 10 .. 1,780 circuits.  sigma_approx (Sec. III-G) comes from the GPU
path (whole-state-in-LDS contraction, FP64 sigma accumulation), nested
prefixes of one run per Philox key, eight keys per circuit; sigma_exact is
the diagonal of the oracle's exact density matrix, stored by
tests/golden/make_paper_experiment_sigma.py.  The Eq. (2) error is averaged
per (n, K) over graphs and keys, and log Error = log alpha + delta n -
mu log K is fitted by least squares, as the paper fits Eq. (3).

What is asserted is what the method fixes, not the paper's constants (they
depend on its angles and graphs): the error falls about as 1/K (|mu - 1| <
0.15; the Eq. (2) infidelity is second order in the deviation of
sigma_approx, so its expectation is proportional to 1/K) and grows with n at
fixed K (delta > 0), with a good log-linear fit.  The table, the fit and the
mean fidelities of sigma_approx with the uniform and the noiseless
distributions are printed (and written as JSON when STN_RECORD_DIR is set).
"""
import base64
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_experiment_sigma_exact.json")
REPS = 8


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_15874_amd as stn
    stn.load()
    torch.cuda.set_device(0)


def fidelity(a, b):
    return float(np.dot(np.sqrt(np.clip(a, 0, None)), np.sqrt(np.clip(b, 0, None))) ** 2)


@pytest.mark.timeout(600)
def test_paper_experiment_error_fit():
    import paper_2210_15874_amd as stn
    from oracle import simulate as sim
    from workloads import PAPER_EXPERIMENT, paper_experiment_problem
    with open(GOLDEN) as f:
        gold = json.load(f)
    Ks = list(PAPER_EXPERIMENT["K_values"])
    bounds = [0] + Ks
    err = {}                                  # (n, K) -> list of Eq. (2) errors
    f_uniform, f_noiseless = [], []
    for case in gold["cases"]:
        n, graph = case["n"], case["graph"]
        exact = np.frombuffer(base64.b64decode(case["sigma_exact_b64"]), dtype="<f8")
        pr = paper_experiment_problem(n, graph)
        assert [list(e) for e in pr.edges] == [list(e) for e in case["edges"]]
        assert exact.shape == (1 << n,) and abs(exact.sum() - 1.0) < 1e-12
        noiseless = np.abs(sim.noiseless_state(pr)) ** 2
        pl = stn.Plan(pr, outputs=stn.OUT_DIAG, precision=64)
        assert pl.info()["plan_name"] == "sv_lds"
        for rep in range(REPS):
            seed = paper_experiment_problem(n, graph, rep).seed
            acc_sum = np.zeros(1 << n)
            for a, b in zip(bounds[:-1], bounds[1:]):
                acc = pl.accum()
                bt = pl.sample(seed, a, b - a)
                pl.contract(bt)
                pl.reduce(bt, acc)
                r = acc.read()
                acc_sum += np.asarray(r["diag"]) * r["k_done"]
                acc.close()
                bt.close()
                est = acc_sum / b
                err.setdefault((n, b), []).append(1.0 - fidelity(est, exact))
            f_uniform.append(fidelity(est, np.full(1 << n, 1.0 / (1 << n))))
            f_noiseless.append(fidelity(est, noiseless))
        pl.close()
    cells = sorted(err)
    mean = np.array([np.mean(err[c]) for c in cells])
    X = np.array([[1.0, n, -np.log(K)] for n, K in cells])
    y = np.log(mean)
    coef, *_ = np.linalg.lstsq(X, y, rcond=None)
    fit = X @ coef
    r2 = 1.0 - float(np.sum((y - fit) ** 2) / np.sum((y - y.mean()) ** 2))
    alpha, delta, mu = float(np.exp(coef[0])), float(coef[1]), float(coef[2])
    print("n  " + " ".join(f"{K:>9d}" for K in Ks))
    for n in sorted({c[0] for c in cells}):
        print(f"{n:<3d}" + " ".join(f"{np.mean(err[(n, K)]):9.2e}" for K in Ks))
    print(f"fit: alpha={alpha:.5f} delta={delta:.5f} mu={mu:.5f} R2={r2:.4f} "
          f"(paper, its own angles and graphs: 0.05737, 0.11164, 0.98682, 0.996)")
    print(f"mean F(sigma_approx, uniform)={np.mean(f_uniform):.3f} "
          f"mean F(sigma_approx, noiseless)={np.mean(f_noiseless):.3f} (paper: 0.938, 0.959)")
    if os.environ.get("STN_RECORD_DIR"):
        os.makedirs(os.environ["STN_RECORD_DIR"], exist_ok=True)
        with open(os.path.join(os.environ["STN_RECORD_DIR"], "paper_experiment_fit.json"), "w") as f:
            json.dump(dict(params=PAPER_EXPERIMENT, reps=REPS,
                           cells=[dict(n=c[0], K=c[1], mean_error=float(np.mean(err[c])), samples=len(err[c]))
                                  for c in cells],
                           fit=dict(alpha=alpha, delta=delta, mu=mu, r2=r2),
                           mean_fidelity_uniform=float(np.mean(f_uniform)),
                           mean_fidelity_noiseless=float(np.mean(f_noiseless))), f, indent=1)
    assert abs(mu - 1.0) < 0.15, mu
    assert delta > 0.0, delta
    assert r2 > 0.9, r2
