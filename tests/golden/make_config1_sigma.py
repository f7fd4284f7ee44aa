"""Writes tests/golden/config1_sigma_exact.json: sigma_exact = diag(rho) of
the exact density matrix (Eq. (1), every channel as its operator sum) of the
n=12, p=2 QAOA workload with depolarizing noise and amplitude damping per
layer, and Tr(rho C).  sigma_exact is the reference distribution of the
paper's Eq. (2) error (Sec. III-G).

Calls only ``oracle`` and ``workloads``.  Run from the repository root:
    python tests/golden/make_config1_sigma.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import simulate as sim  # noqa: E402
from workloads import config_problem  # noqa: E402

if __name__ == "__main__":
    pr = config_problem(1)
    t = time.time()
    rho = sim.density_matrix(pr)
    sigma = np.real(np.diag(rho))
    out = dict(source="oracle.simulate.density_matrix (complex128, operator sum per channel) on workload "
                      f"{pr.name}: n={pr.n_qubits}, p={pr.p}",
               n_qubits=pr.n_qubits, trace=float(np.trace(rho).real),
               energy_exact=sim.energy_exact(rho, pr.n_qubits, pr.edges, pr.weights),
               seconds=time.time() - t, sigma_exact=[float(v) for v in sigma])
    with open(os.path.join(HERE, "config1_sigma_exact.json"), "w") as f:
        json.dump(out, f)
    print("wrote sigma_exact of", pr.name, "in", round(out["seconds"], 1), "s")
