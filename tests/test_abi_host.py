"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/stn.h declares, plans the workloads, and its integer
selection thresholds are bit-identical to the oracle's (the sampler's
bit-exactness rests on them)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2210_15874_amd", "libstn.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libstn.so not built")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "stn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stn_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name


def test_header_is_plain_c():
    """include/stn.h is a C ABI: it compiles as C99 and as C++."""
    import shutil
    import subprocess
    hdr = os.path.join(ROOT, "include", "stn.h")
    for cc, args in [("gcc", ["-x", "c", "-std=c99"]), ("g++", ["-x", "c++"])]:
        exe = shutil.which(cc)
        if exe is None:
            pytest.skip(f"{cc} not found")
        r = subprocess.run([exe, "-fsyntax-only", "-Wall", "-Werror"] + args + [hdr], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


def test_binding_covers_header():
    from paper_2210_15874_amd.binding import EXPORTS
    assert set(declared_functions()) == set(EXPORTS)


def plan(problem, **kw):
    from paper_2210_15874_amd import Plan
    return Plan(problem, torch_allocator=False, **kw)


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_thresholds_bit_identical_to_oracle(cfg):
    from oracle import channels as chn
    from workloads import config_problem
    pr = config_problem(cfg)
    pl = plan(pr)
    for s, ch in enumerate(pr.channels):
        assert pl.site_thresholds(s) == chn.thresholds(chn.selection_probs(ch)), s


def test_thresholds_random_rates():
    from oracle import channels as chn
    from workloads import Channel, Gate, Problem
    rng = np.random.default_rng(3)
    lams = list(rng.random(40)) + [0.0, 1.0, 1e-4, 0.5, 1 / 3]
    gates = [Gate("h", (0,)), Gate("zz", (0, 1), 0.3)]
    chans = []
    for lam in lams:
        chans += [Channel(1, "depol1", (0,), float(lam)), Channel(1, "depol2", (0, 1), float(lam)),
                  Channel(1, "bitflip", (1,), float(lam)), Channel(1, "ampdamp", (0,), float(lam))]
    pr = Problem(2, gates, chans, [(0, 1)], [1.0])
    pl = plan(pr)
    for s, ch in enumerate(chans):
        assert pl.site_thresholds(s) == chn.thresholds(chn.selection_probs(ch)), (s, ch)


def test_plan_kinds_and_cost_model():
    from workloads import config_problem
    from paper_2210_15874_amd import OUT_ENERGY, OUT_RHO
    i0 = plan(config_problem(0), outputs=OUT_RHO | OUT_ENERGY).info()
    assert i0["plan_name"] == "sv_lds" and i0["n_sites"] == 21
    i2 = plan(config_problem(2)).info()
    assert i2["plan_name"] == "sv_tiled" and i2["n_gates"] == 286 and i2["n_sites"] == 286
    # every pass reads and writes the stored complex64 amplitudes, except the
    # first (generated) and last (reduced to the energy); by the bit-flip
    # symmetry of these circuits half the 2^26 amplitudes are stored
    N = 2 ** 25 * 8
    assert i2["half_state"] == 1
    assert i2["bytes_per_traj"] == (2 * i2["n_passes"] - 2) * N
    assert i2["peak_bytes"] == i2["max_batch"] * (N + 64 * 1024)
    full = plan(config_problem(2), full_state=True).info()
    assert full["half_state"] == 0 and full["n_passes"] == i2["n_passes"]
    assert full["bytes_per_traj"] == 2 * i2["bytes_per_traj"]
    assert plan(config_problem(2), precision=128).info()["half_state"] == 1
    # 15-qubit tiles by default at this size (one launch shape); 14-qubit
    # tiles on request: the same passes and bytes, three launch shapes
    assert i2["tile_bits"] == 15 and i2["variant"] == 0
    i14 = plan(config_problem(2), tile_bits=14).info()
    assert i14["tile_bits"] == 14 and i14["variant"] == 2
    assert (i14["n_passes"], i14["bytes_per_traj"], i14["max_batch"]) == (i2["n_passes"], i2["bytes_per_traj"],
                                                                          i2["max_batch"])


def test_plan_released_before_its_accumulators():
    """The C ABI lets a plan's handle be released before the accumulators
    made from it (they hold the plan until their own destroy), in either
    order; energy-only accumulators touch no device."""
    from workloads import config_problem
    for plan_first in (True, False):
        pl = plan(config_problem(0))
        accs = [pl.accum() for _ in range(3)]
        if plan_first:
            pl.close()
        for a in accs:
            a.close()
        pl.close()


def test_validation_errors():
    from paper_2210_15874_amd import OUT_RHO, StnError
    from workloads import Channel, Gate, Problem, config_problem
    bad_q = Problem(2, [Gate("h", (2,))], [])
    with pytest.raises(StnError, match="INVALID"):
        plan(bad_q, outputs=OUT_RHO)
    non_cptp = Problem(1, [Gate("h", (0,))], [Channel(0, "kraus", (0,), 0.0, ((1, 0, 0, 1), (1, 0, 0, 0)))])
    with pytest.raises(StnError, match="trace preserving"):
        plan(non_cptp, outputs=OUT_RHO)
    order = Problem(2, [Gate("h", (0,)), Gate("h", (1,))],
                    [Channel(1, "depol1", (1,), 0.1), Channel(0, "depol1", (0,), 0.1)])
    with pytest.raises(StnError, match="ordered"):
        plan(order, outputs=OUT_RHO)
    with pytest.raises(StnError, match="UNSUPPORTED"):
        plan(config_problem(2), outputs=OUT_RHO)
    with pytest.raises(StnError, match="INVALID"):
        plan(bad_q)  # ENERGY without edges is fine, bad qubit is not
    for kw in ({"tile_bits": 13}, {"tile_bits": 16}, {"tile_bits": 15, "precision": 128}):
        with pytest.raises(StnError, match="sv_tile_bits"):
            plan(config_problem(2), **kw)


def test_complex128_tiled_plan():
    from workloads import config_problem
    pr = config_problem(2)
    i = plan(pr, precision=128).info()
    assert i["plan_name"] == "sv_tiled"
    # 12-qubit tiles: 3 tiles per layer, alternating order merges layer
    # boundaries, so p = 4 layers cost 4 * (3 - 1) + 1 passes of the stored
    # half, 2^25 * 16 B
    assert i["n_passes"] == 9 and i["half_state"] == 1
    assert i["bytes_per_traj"] == (2 * 9 - 2) * 2 ** 25 * 16
    full = plan(pr, precision=128, full_state=True).info()
    assert full["half_state"] == 0 and full["bytes_per_traj"] == 2 * i["bytes_per_traj"]


def test_lightcone_plans_and_auto_choice():
    from workloads import make_problem, random_regular_graph, uniform_angles
    from paper_2210_15874_amd import PLAN_LIGHTCONE, StnError
    g, b = uniform_angles(1, 5)
    pr = make_problem(40, random_regular_graph(40, 3, 4), g, b, 1e-3, 1e-2, 16, 6)
    i = plan(pr).info()
    # p = 1 on a 3-regular graph: each edge's lightcone touches at most 6 qubits
    assert i["plan_name"] == "lightcone" and i["width"] <= 8 and i["n_steps"] > 0
    g, b = uniform_angles(4, 5)
    pr = make_problem(26, random_regular_graph(26, 3, 7), g, b, 1e-3, 1e-2, 16, 6)
    assert plan(pr).info()["plan_name"] == "sv_tiled"
    with pytest.raises(StnError, match="UNSUPPORTED"):
        plan(pr, plan_kind=PLAN_LIGHTCONE)


def test_new_entry_points_validate_arguments():
    """Argument checks of the multi-batch, resample and graph entry points
    (no device needed: they fail before any device call)."""
    import ctypes as C
    from paper_2210_15874_amd.binding import load
    lib = load()
    INVALID = 1
    assert lib.stn_contract_many(None, None, 0, None) == 0          # nothing to do
    assert lib.stn_contract_many(None, None, 2, None) == INVALID
    null2 = (C.c_void_p * 2)(None, None)
    assert lib.stn_contract_many(null2, null2, 2, None) == INVALID
    assert lib.stn_resample(None, 1, 0, 4, None) == INVALID
    assert lib.stn_plan_set_graphs(None, 1) == INVALID
    from workloads import config_problem
    pl = plan(config_problem(0))
    assert lib.stn_plan_set_graphs(pl.h, 1) == 0
    assert pl.info()["graphs"] == 1
    assert lib.stn_plan_set_graphs(pl.h, 0) == 0
    assert pl.info()["graphs"] == 0 and pl.info()["graph_captures"] == 0
    # bitstring sampling: NULL accumulator, then an energy-only accumulator (no diagonal kept)
    assert lib.stn_accum_sample(None, None, 0, None, None) == INVALID
    from paper_2210_15874_amd import OUT_ENERGY
    pe = plan(config_problem(0), outputs=OUT_ENERGY)
    acc = pe.accum()
    assert lib.stn_accum_sample(acc.h, None, 4, None, None) == INVALID
    assert lib.stn_accum_sample(acc.h, None, 0, None, None) == 5    # STN_E_STATE
    acc.close()


def test_lightcone_slicing_plans():
    """Index slicing (Sec. III-C) on the host: a width-20 network sliced to
    steps of rank 12 and 16; without slicing a rank cap below the width is
    rejected."""
    from workloads import make_problem, random_regular_graph, uniform_angles
    from paper_2210_15874_amd import PLAN_LIGHTCONE, StnError
    g, b = uniform_angles(3, 904)
    pr = make_problem(14, random_regular_graph(14, 3, 903), g, b, 5e-3, 2e-2, 6, 905)
    base = plan(pr, plan_kind=PLAN_LIGHTCONE).info()
    assert base["width"] == 20 and base["lc_slices"] == len(pr.edges) and base["lc_slice_bits"] == 0
    for rank, bits in [(12, 10), (16, 6)]:
        i = plan(pr, plan_kind=PLAN_LIGHTCONE, lc_max_rank=rank, lc_slice_bits=bits).info()
        assert i["width"] <= rank + 1
        assert 0 < i["lc_slice_bits"] <= bits and len(pr.edges) < i["lc_slices"] <= len(pr.edges) << bits
    with pytest.raises(StnError, match="UNSUPPORTED"):
        plan(pr, plan_kind=PLAN_LIGHTCONE, lc_max_rank=12)


def min_degree_order(net):
    """A plain greedy minimum-degree elimination order, written here so that
    the caller-order tests do not depend on the library's min-fill."""
    nv = net["n_vars"]
    adj = [set() for _ in range(nv)]
    for t in net["tensors"]:
        for a in t:
            adj[a].update(b for b in t if b != a)
    done, order = [False] * nv, []
    for _ in range(nv):
        v = min((x for x in range(nv) if not done[x]), key=lambda x: (len(adj[x]), x))
        order.append(v)
        done[v] = True
        nb = list(adj[v])
        for a in nb:
            adj[a].discard(v)
            adj[a].update(y for y in nb if y != a)
        adj[v] = set()
    return order


def test_caller_contraction_order():
    """A caller-supplied elimination order (Sec. III-A/B) replaces min-fill:
    called once per term with that term's network, lowered as given (here one
    that beats min-fill's width); orders that are not permutations, rejected
    orders and orders with slicing are INVALID; an order too wide for the
    rank cap is UNSUPPORTED, and an AUTO plan then takes the statevector."""
    from workloads import make_problem, random_regular_graph, uniform_angles
    from paper_2210_15874_amd import PLAN_LIGHTCONE, StnError
    g, b = uniform_angles(1, 5)
    pr = make_problem(40, random_regular_graph(40, 3, 4), g, b, 1e-3, 1e-2, 16, 6)
    seen = []

    def record(net):
        seen.append(net)
        return min_degree_order(net)
    i = plan(pr, plan_kind=PLAN_LIGHTCONE, lc_order=record).info()
    assert i["plan_name"] == "lightcone" and i["width"] <= 8
    assert [(d["term"], d["u"], d["v"]) for d in seen] == [(t, u, v) for t, (u, v) in enumerate(pr.edges)]
    for d in seen:
        used = sorted({x for t in d["tensors"] for x in t})
        assert used == list(range(d["n_vars"]))
    # n=14, p=3: reversing the variable numbering gives width 15 where min-fill gives 20
    g, b = uniform_angles(3, 904)
    pr3 = make_problem(14, random_regular_graph(14, 3, 903), g, b, 5e-3, 2e-2, 6, 905)
    base = plan(pr3, plan_kind=PLAN_LIGHTCONE).info()["width"]
    rev = plan(pr3, plan_kind=PLAN_LIGHTCONE, lc_order=lambda net: range(net["n_vars"] - 1, -1, -1)).info()
    assert rev["width"] < base
    for bad in (lambda net: [0] * net["n_vars"],                 # not a permutation
                lambda net: list(range(net["n_vars"] - 1)),       # too short (the callback rejects)
                lambda net: 1 / 0):                               # raises (the callback rejects)
        with pytest.raises(StnError, match="INVALID"):
            plan(pr3, plan_kind=PLAN_LIGHTCONE, lc_order=bad)
    with pytest.raises(StnError, match="INVALID"):
        plan(pr3, plan_kind=PLAN_LIGHTCONE, lc_order=min_degree_order, lc_slice_bits=4)
    # the numbering order needs steps above the rank cap at n=20, p=2
    g, b = uniform_angles(2, 5)
    pr2 = make_problem(20, random_regular_graph(20, 3, 11), g, b, 1e-3, 1e-2, 16, 6)
    natural = lambda net: range(net["n_vars"])
    with pytest.raises(StnError, match="UNSUPPORTED"):
        plan(pr2, plan_kind=PLAN_LIGHTCONE, lc_order=natural)
    assert plan(pr2, lc_order=natural).info()["plan_name"] == "sv_tiled"


def test_gate_by_gate_plans():
    """<C> jobs with non-unitary channels above the whole-state-in-LDS size
    have no Pauli frame (so no tiled or lightcone lowering): AUTO takes the
    gate-by-gate HBM statevector, also for sigma above that size; it keeps
    energies and sigma only, for n <= 30."""
    from workloads import make_problem, random_regular_graph, uniform_angles
    from paper_2210_15874_amd import OUT_DIAG, OUT_ENERGY, OUT_RHO, OUT_STATES, PLAN_SV_GATES, StnError
    g, b = uniform_angles(2, 31)
    pr = make_problem(16, random_regular_graph(16, 3, 32), g, b, 1e-3, 1e-2, 8, 33, gamma_ad=0.01)
    i = plan(pr).info()
    assert i["plan_name"] == "sv_gates" and i["width"] == 16
    n_ops = len(pr.gates) + len(pr.channels)
    # consecutive entries are fused into passes over 13-bit tiles: far fewer
    # passes than entries; each reads and writes the state once (the first
    # only writes) and the energy reads it once more
    assert 0 < i["n_passes"] <= n_ops // 8
    assert i["bytes_per_traj"] == 8.0 * (1 << 16) * 2 * i["n_passes"]
    pq = make_problem(16, random_regular_graph(16, 3, 32), g, b, 1e-3, 1e-2, 8, 33)
    assert plan(pq, plan_kind=PLAN_SV_GATES).info()["plan_name"] == "sv_gates"
    # sigma (DIAG) is kept up to n = 30 by this lowering; rho_hat and states are not
    assert plan(pr, outputs=OUT_DIAG | OUT_ENERGY).info()["plan_name"] == "sv_gates"
    assert plan(pq, outputs=OUT_DIAG).info()["plan_name"] == "sv_gates"
    for outs in (OUT_RHO, OUT_STATES | OUT_ENERGY):
        with pytest.raises(StnError, match="UNSUPPORTED"):
            plan(pr, plan_kind=PLAN_SV_GATES, outputs=outs)
        with pytest.raises(StnError, match="UNSUPPORTED"):
            plan(pr, outputs=outs)
    g1, b1 = uniform_angles(1, 34)
    big = make_problem(32, random_regular_graph(32, 3, 35), g1, b1, 1e-3, 1e-2, 8, 36, gamma_ad=0.01)
    with pytest.raises(StnError, match="UNSUPPORTED"):
        plan(big, plan_kind=PLAN_SV_GATES)


def test_server_needs_a_device_and_valid_options():
    from paper_2210_15874_amd import Server, StnError
    with pytest.raises(StnError, match="INVALID"):
        Server(n_streams=0)
    with pytest.raises(StnError, match="INVALID"):
        Server(job_share=0.0)
    with pytest.raises(StnError, match="INVALID"):
        Server(precision=32)
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except ImportError:
        has_gpu = False
    if not has_gpu:
        with pytest.raises(StnError, match="DEVICE"):
            Server()


def test_planning_mixed_workloads():
    """Host planning of every lowering on a spread of inputs (the sanitizer
    run executes this too): random circuits of every gate and channel kind in
    the LDS and gate-by-gate lowerings, Erdos-Renyi QAOA jobs through AUTO
    (lightcone networks with trajectory groups and merged steps, or the tiled
    statevector), complex128 lightcone plans, sliced networks, and the
    paper's 4-regular experiment circuits."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from random_circuits import random_problem
    from workloads import erdos_renyi_graph, make_problem, paper_experiment_problem, uniform_angles
    from paper_2210_15874_amd import OUT_DIAG, OUT_ENERGY, OUT_RHO, PLAN_LIGHTCONE, PLAN_SV_GATES, PLAN_SV_LDS
    for seed in range(12):
        pr = random_problem(seed)
        outs = OUT_RHO | OUT_DIAG | (OUT_ENERGY if pr.edges else 0)
        assert plan(pr, outputs=outs, plan_kind=PLAN_SV_LDS).info()["plan_name"] == "sv_lds"
        big = random_problem(100 + seed, n_range=(14, 20))
        i = plan(big, outputs=OUT_DIAG, plan_kind=PLAN_SV_GATES).info()
        assert i["plan_name"] == "sv_gates" and 0 < i["n_passes"]
    for n, p, kind in [(22, 2, "lightcone"), (29, 2, "lightcone"), (20, 1, "lightcone"), (24, 3, "sv_tiled"),
                       (16, 3, "sv_tiled")]:
        g, b = uniform_angles(p, 5000 + n)
        pr = make_problem(n, erdos_renyi_graph(n, 3.0 / (n - 1), 4000 + n), g, b, 1e-3, 1e-2, 64, 6000 + n)
        i = plan(pr).info()
        assert i["plan_name"] == kind, (n, p, i["plan_name"])
        if kind == "lightcone":
            assert i["lc_group"] in (1, 2, 4, 8, 16) and i["lc_width_lower_bound"] == 0
        i128 = plan(pr, precision=128, plan_kind=PLAN_LIGHTCONE).info() if p <= 2 else None
        if i128:
            assert i128["width"] == i["width"] or kind != "lightcone"
    g, b = uniform_angles(3, 5014)
    pr = make_problem(14, erdos_renyi_graph(14, 3.0 / 13, 4014), g, b, 1e-3, 1e-2, 16, 6014)
    i = plan(pr, plan_kind=PLAN_LIGHTCONE, lc_max_rank=12, lc_slice_bits=10).info()
    assert i["lc_slice_bits"] > 0 and i["width"] <= 13
    for n in (5, 8, 12):
        assert plan(paper_experiment_problem(n, 0), outputs=OUT_DIAG).info()["plan_name"] == "sv_lds"
