"""Writes tests/golden/config2_sampled.json: oracle values of sampled
trajectories of the n=26, p=4, 3-regular QAOA workload (complex128,
literal Kraus insertion, the same Philox draws as the product path).

Calls only ``oracle`` and ``workloads``.  Run from the repository root:
    python tests/golden/make_config2_golden.py [n_procs]
"""
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import simulate as sim  # noqa: E402
from workloads import config_problem  # noqa: E402

KS = [0, 1, 2, 3, 5, 8, 1000, 4095]


def one(k):
    pr = config_problem(2)
    idx = sim.kraus_indices(pr, pr.seed, k, 1)[0]
    t = time.time()
    psi = sim.trajectory(pr, idx)
    n = pr.n_qubits
    e = sim.energy(psi, n, pr.edges, pr.weights)
    zz = sim.edge_zz(psi, n, pr.edges)
    return dict(k=k, n_errors=int((idx != 0).sum()), energy=e, edge_zz=[float(x) for x in zz],
                seconds=time.time() - t)


if __name__ == "__main__":
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    with Pool(procs) as pool:
        rows = pool.map(one, KS)
    pr = config_problem(2)
    out = dict(source="oracle.simulate.trajectory (complex128, literal Kraus insertion) on workload "
                      f"{pr.name}: n={pr.n_qubits}, p={pr.p}, seed={pr.seed}",
               edges=pr.edges, trajectories=rows)
    with open(os.path.join(HERE, "config2_sampled.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", len(rows), "trajectories")
