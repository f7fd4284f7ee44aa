"""Writes tests/golden/paper_experiment_sigma_exact.json: for every circuit of
the paper's own experiment as this repository sets it up (Sec. IV: QAOA p=2
on 4-regular graphs, depolarizing lambda_1 = 0.001 / lambda_2 = 0.004 on
every gate; n = 5 .. 12, three seeded graphs per n), sigma_exact = diag(rho)
of the exact density matrix (Eq. (1)), the reference of the Eq. (2) error.
Values are float64 little-endian, base64-encoded.

Calls only ``oracle`` and ``workloads``.  Run from the repository root:
    python tests/golden/make_paper_experiment_sigma.py [n_procs]
"""
import base64
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import simulate as sim  # noqa: E402
from workloads import PAPER_EXPERIMENT, paper_experiment_problem  # noqa: E402


def one(case):
    n, graph = case
    pr = paper_experiment_problem(n, graph)
    t = time.time()
    rho = sim.density_matrix(pr)
    sigma = np.ascontiguousarray(np.real(np.diag(rho)), dtype="<f8")
    return dict(n=n, graph=graph, edges=pr.edges, trace=float(np.trace(rho).real),
                seconds=time.time() - t, sigma_exact_b64=base64.b64encode(sigma.tobytes()).decode())


if __name__ == "__main__":
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else 3
    lo, hi = PAPER_EXPERIMENT["n_range"]
    cases = [(n, g) for n in range(hi, lo - 1, -1) for g in range(PAPER_EXPERIMENT["graphs"])]
    with Pool(procs) as pool:
        rows = pool.map(one, cases)
    rows.sort(key=lambda r: (r["n"], r["graph"]))
    out = dict(source="oracle.simulate.density_matrix (complex128, operator sum per channel) on "
                      "workloads.paper_experiment_problem", params=PAPER_EXPERIMENT, cases=rows)
    with open(os.path.join(HERE, "paper_experiment_sigma_exact.json"), "w") as f:
        json.dump(out, f)
    print("wrote", len(rows), "cases")
