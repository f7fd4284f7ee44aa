"""Throughput of the noisy-trajectory ensemble on one MI355X.

Workload (default): QAOA MaxCut p=4 on a seeded random 3-regular graph with
n=26 qubits, depolarizing noise after every gate (1q 1e-3, 2q 1e-2), K=4096
trajectories per job, complex64 contraction with FP64 reductions.  One step is
one whole job: Philox sampling + Pauli frame, contraction of every
trajectory, FP64 reduction and the read of <C> +- SE.  The plan (host
lowering) is built once outside the timed region and reported separately.

Prints one JSON line (value = trajectories/s over the timed steps) with the
dominant kernel's roofline (algorithmic bytes per launch / HIP-event launch
time, against 8 TB/s HBM) and the CPU FP64 oracle timed on a bounded sample.
Untimed legs beside it:
  fp64       the complex128 path on a prefix of the same job: per-trajectory
             and mean error of the complex64 result, and of both against
             stored oracle values;
  plain_loop the same kernels one trajectory per launch, sequentially;
  serving    the job server on the first arrivals of a Poisson stream (mean
             200 jobs/s; n 10..30, p 1..6, K 256..8192, depolarizing rates
             log-uniform in 1e-4..1e-2): p50/p99 latency, trajectories/s, and
             the <C> error of sampled jobs against the complex128 path.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "noisy trajectories/s at n=26 QAOA p=4 (⟨C⟩ err vs FP64); p50/p99 job latency"
HBM_PEAK_GBS = 8000.0


def _cpu_kind_times(args):
    """One worker of the CPU baseline: the oracle's gate application
    (complex128 statevector, one BLAS thread) on a full 2^n state, timed per
    gate kind on gates of the workload's own circuit, and the oracle's energy
    of one trajectory."""
    problem_cfg, reps = args
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import simulate as sim
    from oracle.gates import PAULIS, gate_matrix, pauli_string
    from oracle.statevector import apply_to_state
    from workloads import config_problem
    pr = config_problem(problem_cfg)
    n = pr.n_qubits
    psi = np.full((2,) * n, 1.0 / math.sqrt(2.0 ** n), dtype=np.complex128)
    by_kind = {}
    for g in pr.gates:
        by_kind.setdefault(g.kind, []).append(g)
    out = {}
    with threadpool_limits(1):
        for kind, gs in sorted(by_kind.items()):
            # gates spread over the register (the cost depends on the axis moved)
            pick = [gs[(len(gs) - 1) * i // max(1, reps - 1)] for i in range(reps)]
            t0 = time.perf_counter()
            for g in pick:
                psi = apply_to_state(psi, gate_matrix(g), g.qubits)
            out[kind] = (time.perf_counter() - t0) / len(pick)
        # inserted Paulis of the depolarizing sites: one- and two-qubit products
        t0 = time.perf_counter()
        psi = apply_to_state(psi, PAULIS[1], (n // 2,))
        out["pauli1"] = time.perf_counter() - t0
        e = pr.edges[len(pr.edges) // 2]
        t0 = time.perf_counter()
        psi = apply_to_state(psi, pauli_string([1, 3]), e)
        out["pauli2"] = time.perf_counter() - t0
        # the energy's cost is a fixed part plus one part per edge: timed on 2
        # and on 6 edges of the graph, extrapolated to all of them
        t = []
        for m in (2, 6):
            t0 = time.perf_counter()
            sim.energy(psi.reshape(-1), n, pr.edges[:m], pr.weights[:m])
            t.append(time.perf_counter() - t0)
        per_edge = max(0.0, (t[1] - t[0]) / 4.0)
        out["energy"] = max(0.0, t[0] - 2.0 * per_edge) + per_edge * len(pr.edges)
    return out


def cpu_baseline(problem_cfg, reps=2):
    """The CPU FP64 oracle on the host cores: one process per core (the box's
    CPU share, at most 16), each timing the oracle's own gate application on
    the full 2^26 complex128 state for every gate kind of the circuit (h, zz,
    rx: `reps` gates each, spread over the register), the inserted one- and
    two-qubit Paulis and the energy of one trajectory (timed on 2 and on 6
    edges: a fixed part plus a part per edge), all processes at once
    (so they share the memory bandwidth as a full run would).  Seconds per
    trajectory = sum over kinds of (gates of that kind) x (mean seconds per
    gate) + (expected inserted Paulis) x (their seconds) + energy;
    throughput = processes / that."""
    import multiprocessing as mp

    from oracle import simulate as sim
    from workloads import config_problem
    pr = config_problem(problem_cfg)
    procs = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(procs) as pool:
        rows = pool.map(_cpu_kind_times, [(problem_cfg, reps)] * procs)
    wall = time.perf_counter() - t0
    mean = {k: sum(r[k] for r in rows) / len(rows) for k in rows[0]}
    counts = {}
    for g in pr.gates:
        counts[g.kind] = counts.get(g.kind, 0) + 1
    # expected non-identity insertions per trajectory, from the sites' selection probabilities
    exp1 = exp2 = 0.0
    for q, _, _ in sim.site_tables(pr):
        if len(q) == 4:
            exp1 += 1.0 - q[0]
        elif len(q) == 16:
            exp2 += 1.0 - q[0]
    per_traj = sum(counts[k] * mean[k] for k in counts) + exp1 * mean["pauli1"] + exp2 * mean["pauli2"] + mean["energy"]
    return {"value": procs / per_traj, "unit": "trajectories/s", "cores": procs, "kind": "oracle",
            "seconds_per_trajectory_per_core": per_traj,
            "per_kind_s": {k: round(v, 4) for k, v in mean.items()},
            "gate_counts": counts, "expected_paulis": {"one_qubit": exp1, "two_qubit": exp2},
            "sample": f"{procs} processes at once, each timing {reps} gates of each kind of the n={pr.n_qubits} "
                      f"p={pr.p} circuit, 2 inserted Paulis and the energy (on 2 and 6 edges, extrapolated to "
                      f"{len(pr.edges)}) on a full complex128 state "
                      f"({wall:.0f} s wall); per-trajectory time weighted by the circuit's gate counts"}


def measured_traffic(kernel_source, tile_bits, launch_shape, per_launch):
    """HBM bytes per launch of the tiled pass from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None if the kernel source or the
    planner (pass schedule) has changed since the counters were taken or they
    were taken with another tile width, launch shape or number of
    trajectories per launch."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sv_pass_qaoa_n26_p4_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    # the kernel source and the planner that sets the pass schedule
    for src, key in ((kernel_source, "source_sha256"), (t.get("schedule_source"), "schedule_source_sha256")):
        if not src:
            return None
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != t.get(key):
                return None
    if (t.get("tile_bits") != tile_bits or t.get("launch_shape") != launch_shape
            or t.get("trajectories_per_launch") != per_launch):
        return None
    return t["traffic_bytes_per_launch"] / 1e9


def note(msg):
    """Progress line on stderr (one per leg), so a long run shows where it is."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def fp64_check(energies_by_k, problem):
    """Largest |<C>_k - <C>_k(oracle, FP64)| / m over the stored oracle samples."""
    path = os.path.join(ROOT, "tests", "golden", "config2_sampled.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    m = len(problem.edges)
    errs = [abs(energies_by_k[r["k"]] - r["energy"]) / m for r in g["trajectories"] if r["k"] in energies_by_k]
    return {"max_abs_err_per_edge": max(errs) if errs else None, "trajectories": len(errs),
            "reference": "oracle complex128, same draws (tests/golden/config2_sampled.json)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--K", type=int, default=None, help="trajectories per job (default: the workload's 4096)")
    ap.add_argument("--batch", type=int, default=0, help="trajectories per launch (0: from the HBM budget)")
    ap.add_argument("--hbm-budget-gib", type=float, default=160.0)
    ap.add_argument("--cpu-reps", type=int, default=2, help="gates of each kind timed per CPU process")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fp64-prefix", type=int, default=1024,
                    help="trajectories of the job also run in complex128 (0: skip)")
    ap.add_argument("--plain-traj", type=int, default=16, help="trajectories of the one-per-launch loop (0: skip)")
    ap.add_argument("--serve-jobs", type=int, default=16, help="arrivals of the serving stream (0: skip)")
    ap.add_argument("--serve-window", type=float, default=40.0, help="seconds the serving leg runs")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="mean arrivals per second")
    ap.add_argument("--serve-check-every", type=int, default=4, help="complex128 check of every k-th served job")
    ap.add_argument("--rho-leg", type=int, default=1, help="n=12 rho_hat workload leg (0: skip)")
    ap.add_argument("--gates-leg", type=int, default=1,
                    help="n=20 amplitude-damping <C> job in the gate-by-gate lowering (0: skip)")
    ap.add_argument("--uneven", action="store_true",
                    help="only the uneven-batch leg: 64 jobs (n 10..30, p 1..6, K 256..8192) submitted at once to "
                         "the job server, for --uneven-window seconds")
    ap.add_argument("--uneven-window", type=float, default=900.0)
    ap.add_argument("--uneven-leg-window", type=float, default=60.0,
                    help="seconds of the uneven-batch leg in the default run (0: skip); jobs still running at "
                         "its end are reported as censored")
    ap.add_argument("--job", type=str, default=None,
                    help="only one job n,p,K[,precision[,lc_max_rank,lc_slice_bits]] (QAOA on an Erdos-Renyi graph, "
                         "p_edge 3/(n-1), depolarizing 1e-3/1e-2) through the plan API with the planner's choice of "
                         "lowering, or sliced lightcone networks when slice bits are given")
    ap.add_argument("--dedup", type=int, default=1,
                    help="time one extra headline job contracting each distinct trajectory once (0: skip)")
    ap.add_argument("--tile-bits", type=int, default=0,
                    help="qubits per tile of the headline plan (14 or 15; 0: the planner's default, 15 at n=26)")
    ap.add_argument("--job-tune", action="store_true",
                    help="with --job: autotune the launch shape on 256 sampled trajectories first")
    ap.add_argument("--graph-leg", action="store_true",
                    help="only the contraction-graph leg: many small chunks refilled into one batch, eager "
                         "launches against replayed HIP graphs")
    ap.add_argument("--queue-leg", action="store_true",
                    help="only the multi-batch leg: 64 small jobs (n 6..12, p 1..4, K 16..256) contracted one "
                         "launch per job against one launch draining a device-side queue of all their trajectories")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="copy a buffer of this size once before the timed region (a known-size reference "
                         "for hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the trajectory ensemble shards by trajectory range across GPUs "
              "with one FP64 all-reduce of the partial sums (not built in this repository); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.uneven:
        import paper_2210_15874_amd as stn
        print(json.dumps({"uneven_batch": uneven_leg(stn, args)}))
        return
    if args.job:
        import paper_2210_15874_amd as stn
        print(json.dumps({"job": one_job_leg(stn, args)}))
        return
    if args.queue_leg:
        import paper_2210_15874_amd as stn
        print(json.dumps({"queue": queue_leg(stn)}))
        return
    if args.graph_leg:
        import paper_2210_15874_amd as stn
        print(json.dumps({"graphs": graph_leg(stn)}))
        return

    from workloads import config_problem
    problem = config_problem(2, K=args.K)
    K = problem.K

    if not args.no_cpu:
        note("CPU oracle baseline")
    cpu = None if args.no_cpu else cpu_baseline(2, args.cpu_reps)
    note("plan and autotune")

    import torch

    import paper_2210_15874_amd as stn
    torch.cuda.set_device(0)
    stn.load()
    t0 = time.perf_counter()
    plan = stn.Plan(problem, outputs=stn.OUT_ENERGY, precision=64, max_batch=args.batch,
                    hbm_budget=int(args.hbm_budget_gib * (1 << 30)), tile_bits=args.tile_bits)
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info()
    B = info["max_batch"]
    # launch shape from the autotuner (untimed; results do not depend on it)
    tb = plan.sample(problem.seed, 0, B)
    tune = plan.autotune(tb, reps=1)
    tb.close()

    def job():
        acc = plan.accum()
        for k0 in range(0, K, B):
            b = plan.sample(problem.seed, k0, min(B, K - k0))
            plan.contract(b)
            plan.reduce(b, acc)
            b.close()
        r = acc.read()
        acc.close()
        return r

    if args.copy_probe_gib > 0:
        nbytes = int(args.copy_probe_gib * (1 << 30))
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    note(f"{args.warmup} warm-up and {args.steps} timed steps")
    for _ in range(args.warmup):
        job()
    torch.cuda.synchronize()
    plan.profile(True)
    times = []
    t_all = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        res = job()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    prof = plan.profile_read()
    plan.profile(False)

    value = K * args.steps / wall
    kern = prof["sv_pass"] if prof["sv_pass"]["launches"] else prof["sv_lds"]
    kname = "sv_pass" if prof["sv_pass"]["launches"] else "sv_lds"
    achieved = kern["bytes"] / (kern["ms"] * 1e-3) / 1e9 if kern["ms"] else None
    energies = {k: float(e) for k, e in enumerate(res["energies"])}
    times.sort()

    # the same job with each distinct trajectory contracted once (reported
    # apart from the headline value, which contracts every trajectory)
    dedup = None
    if args.dedup:
        note("de-duplicated job")
        import numpy as np
        unique = 0

        def job_dedup():
            nonlocal unique
            unique = 0
            acc = plan.accum()
            for k0 in range(0, K, B):
                b = plan.sample(problem.seed, k0, min(B, K - k0))
                unique += plan.contract_dedup(b)
                plan.reduce(b, acc)
                b.close()
            r = acc.read()
            acc.close()
            return r

        torch.cuda.synchronize()
        ts = time.perf_counter()
        rd = job_dedup()
        torch.cuda.synchronize()
        td = time.perf_counter() - ts
        dedup = {"distinct_trajectories": unique, "K": K, "seconds": td,
                 "trajectories_per_s": K / td,
                 "same_energies": bool((np.asarray(rd["energies"]) == np.asarray(res["energies"])).all()),
                 "note": "each distinct (gate signs, final frame X) trajectory contracted once; not the headline"}

    plan.close()                    # release the headline workspace before the other legs
    torch.cuda.empty_cache()
    note("complex128 leg")
    fp64 = fp64_leg(stn, problem, res["energies"], args.fp64_prefix) if args.fp64_prefix > 0 else None
    torch.cuda.empty_cache()
    note("plain per-trajectory loop")
    plain = (plain_loop(stn, problem, args.plain_traj, value, tune["chosen"], args.tile_bits)
             if args.plain_traj > 0 else None)
    torch.cuda.empty_cache()
    note("rho_hat leg")
    rho_leg = rho_hat_leg(stn) if args.rho_leg else None
    torch.cuda.empty_cache()
    note("gate-by-gate leg")
    gates = gates_leg(stn) if args.gates_leg else None
    torch.cuda.empty_cache()
    note("serving leg")
    serving = serving_leg(stn, args) if args.serve_jobs > 0 else None
    torch.cuda.empty_cache()
    uneven = None
    if args.uneven_leg_window > 0:
        note("uneven batch leg")
        uneven = uneven_leg(stn, args, args.uneven_leg_window)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": problem.name, "n_qubits": problem.n_qubits, "p": problem.p,
                   "graph": "random 3-regular (seed 1002)", "K": K, "lambda1": 1e-3, "lambda2": 1e-2,
                   "contraction": "complex64 (FP32), FP64 reductions", "plan": info["plan_name"],
                   "trajectories_per_launch": B, "passes_per_trajectory": info["n_passes"],
                   "stored_amplitudes_per_trajectory": 2 ** (problem.n_qubits - info["half_state"]),
                   "tile_qubits": info["tile_bits"],
                   "launch_shape": {"chosen": tune["chosen"], "ms_per_variant": tune["ms"]},
                   "plan_ms": plan_ms},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": measured_traffic("paper_2210_15874_amd/csrc/kernels_sv_tiled.hip", info["tile_bits"],
                                                 tune["chosen"], B)
                     if kname == "sv_pass" else None, "traffic_unit": "GB per launch",
                     "launches": kern["launches"], "avg_launch_ms": kern["ms"] / max(1, kern["launches"]),
                     "bytes_per_launch": kern["bytes"] / max(1, kern["launches"])},
        "kernels": {k: {"launches": v["launches"], "ms": v["ms"]} for k, v in prof.items() if v["launches"]},
        "result": {"energy_mean": res["energy_mean"], "energy_se": res["energy_se"],
                   "fp64_check": fp64_check(energies, problem), "fp64": fp64},
        "job_latency_ms": {"p50": times[len(times) // 2] * 1e3, "max": times[-1] * 1e3},
        "dedup": dedup,
        "plain_loop": plain,
        "rho_hat": rho_leg,
        "sv_gates": gates,
        "serving": serving,
        "uneven_batch": uneven,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def fp64_leg(stn, problem, e64, prefix):
    """The complex128 tiled path on trajectories 0 .. prefix-1 of the job:
    error of the complex64 energies against it (per trajectory and of the
    mean), and of the complex128 energies against the stored oracle values."""
    import numpy as np
    prefix = min(prefix, problem.K)
    pl = stn.Plan(problem, outputs=stn.OUT_ENERGY, precision=128, hbm_budget=160 << 30)
    t0 = time.perf_counter()
    e128 = stn.simulate_batch_ensemble(problem, K=prefix, plan=pl)["energies"]
    dt = time.perf_counter() - t0
    m = len(problem.edges)
    e64 = np.asarray(e64[:prefix])
    d = np.abs(e64 - e128) / m
    out = {"trajectories": prefix, "plan": pl.info()["plan_name"], "seconds": dt,
           "c64_vs_c128_max_abs_err_per_edge": float(d.max()),
           "c64_vs_c128_mean_abs_err_per_edge": float(abs(e64.mean() - e128.mean()) / m),
           "stochastic_se_per_edge": float(e128.std(ddof=1) / math.sqrt(prefix) / m)}
    path = os.path.join(ROOT, "tests", "golden", "config2_sampled.json")
    if os.path.exists(path):
        with open(path) as f:
            g = json.load(f)
        errs = [abs(e128[r["k"]] - r["energy"]) / m for r in g["trajectories"] if r["k"] < prefix]
        out["c128_vs_oracle_max_abs_err_per_edge"] = max(errs) if errs else None
        out["oracle_trajectories"] = len(errs)
    pl.close()
    return out


def plain_loop(stn, problem, n_traj, batched_value, variant=None, tile_bits=0):
    """Plain per-trajectory loop: the same kernels (tiles and launch shape),
    one trajectory per launch, sequential (sample, contract, reduce,
    synchronise)."""
    import torch
    pl = stn.Plan(problem, outputs=stn.OUT_ENERGY, precision=64, max_batch=1, tile_bits=tile_bits)
    if variant is not None:
        pl.set_variant(variant)
    acc = pl.accum()
    b = pl.sample(problem.seed, 0, 1)   # warm: tables, workspace
    pl.contract(b)
    torch.cuda.synchronize()
    b.close()
    t0 = time.perf_counter()
    for k in range(n_traj):
        b = pl.sample(problem.seed, k, 1)
        pl.contract(b)
        pl.reduce(b, acc)
        torch.cuda.synchronize()
        b.close()
    dt = time.perf_counter() - t0
    acc.close()
    pl.close()
    v = n_traj / dt
    return {"value": v, "unit": "trajectories/s", "trajectories": n_traj, "batched_over_plain": batched_value / v}


def gates_leg(stn):
    """n=20 QAOA p=2, 3-regular, depolarizing + amplitude damping per layer,
    K=256 <C>: no Pauli frame, so the gate-by-gate HBM statevector lowering
    (one launch per gate or noise site).  Reports trajectories/s and the
    HBM rate of its passes from the library's own per-class timing."""
    import torch
    from workloads import make_problem, random_regular_graph, uniform_angles
    g, b = uniform_angles(2, 61)
    pr = make_problem(20, random_regular_graph(20, 3, 62), g, b, 1e-3, 1e-2, 256, 63, gamma_ad=0.01)
    pl = stn.Plan(pr, precision=64)
    info = pl.info()
    stn.simulate_batch_ensemble(pr, plan=pl)            # warm
    torch.cuda.synchronize()
    pl.profile(True)
    t0 = time.perf_counter()
    res = stn.simulate_batch_ensemble(pr, plan=pl)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = pl.profile_read()["sv_pass"]
    pl.profile(False)
    gbs = prof["bytes"] / (prof["ms"] * 1e-3) / 1e9 if prof["ms"] else None
    return {"workload": "qaoa-n20-p2-3reg-depol-ad-K256", "plan": info["plan_name"], "K": pr.K,
            "passes_per_trajectory": info["n_passes"], "seconds": dt, "trajectories_per_s": pr.K / dt,
            "pass_ms": prof["ms"], "hbm_GBps": gbs, "hbm_frac": gbs / 8000.0 if gbs else None,
            "energy_mean": res["energy_mean"], "energy_se": res["energy_se"]}


def rho_hat_leg(stn):
    """n=12 QAOA p=2, 3-regular, depolarizing + amplitude damping, K=1024 in
    one launch: complex64 contraction, FP64 rho_hat (4096 x 4096).  Times the
    job, its FP64 matrix-core rank-K update and bitstring draws from sigma."""
    import torch
    from workloads import config_problem
    pr = config_problem(1)
    pl = stn.Plan(pr, outputs=stn.OUT_RHO | stn.OUT_ENERGY, precision=64)
    stn.simulate_batch_ensemble(pr, plan=pl)            # warm
    torch.cuda.synchronize()
    pl.profile(True)
    t0 = time.perf_counter()
    res = stn.simulate_batch_ensemble(pr, plan=pl)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = pl.profile_read()
    pl.profile(False)
    herk = prof["herk"]
    # the same kernels one trajectory per launch, sequential (plain loop)
    n_plain = 64
    acc = pl.accum()
    t1 = time.perf_counter()
    for k in range(n_plain):
        bt = pl.sample(pr.seed, k, 1)
        pl.contract(bt)
        pl.reduce(bt, acc)
        torch.cuda.synchronize()
        bt.close()
    plain = n_plain / (time.perf_counter() - t1)
    # bitstrings drawn from sigma_approx of those trajectories (inverse transform, 2^24 draws)
    m = 1 << 24
    u = torch.rand(m, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    xs = acc.sample(u)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    xs = acc.sample(u, out=xs)
    ev1.record()
    torch.cuda.synchronize()
    sample_s = ev0.elapsed_time(ev1) * 1e-3
    acc.close()
    out = {"workload": pr.name, "K": pr.K, "seconds": dt, "trajectories_per_s": pr.K / dt,
           "sweep": sigma_sweep(stn, pr),
           "plain_loop_trajectories_per_s": plain, "batched_over_plain": pr.K / dt / plain,
           "bitstring_samples_per_s": m / sample_s,
           "kernels_ms": {k: v["ms"] for k, v in prof.items() if v["launches"]},
           "herk_fp64_tflops": herk["flops"] / (herk["ms"] * 1e-3) / 1e12 if herk["ms"] else None,
           "herk_peak_tflops": 78.6, "trace": res["trace"]}
    pl.close()
    return out


def sigma_sweep(stn, pr):
    """Eq. (2) error of sigma_approx (nested prefixes K = 16 .. 1024 of the
    same trajectories, each estimate normalised by its trace) against the
    stored exact diagonal (tests/golden/config1_sigma_exact.json, written by
    the oracle).  Fidelity and trace distance against the full exact density
    matrix are computed by the GPU test of the same sweep."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "config1_sigma_exact.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        exact = np.array(json.load(f)["sigma_exact"])
    pl = stn.Plan(pr, outputs=stn.OUT_DIAG, precision=64)
    edges = [0, 16, 32, 64, 128, 256, 512, 1024]
    acc_sum = np.zeros_like(exact)
    rows = []
    for a, b in zip(edges[:-1], edges[1:]):
        acc = pl.accum()
        bt = pl.sample(pr.seed, a, b - a)
        pl.contract(bt)
        pl.reduce(bt, acc)
        r = acc.read()
        acc_sum += np.asarray(r["diag"]) * r["k_done"]
        acc.close()
        bt.close()
        est = acc_sum / b
        tr = float(est.sum())
        fid = float(np.dot(np.sqrt(np.clip(est / tr, 0, None)), np.sqrt(np.clip(exact, 0, None))) ** 2)
        rows.append({"K": b, "eq2_error": 1.0 - fid, "trace": tr})
    pl.close()
    return rows


def one_job_leg(stn, args):
    """One QAOA job (n, p, K[, precision]) on a seeded Erdos-Renyi graph:
    plan, then sample / contract / reduce in the planner's chunks, timed warm;
    per-kernel event times."""
    import torch
    from workloads import erdos_renyi_graph, make_problem, uniform_angles
    f = [int(x) for x in args.job.split(",")]
    n, p, K = f[:3]
    precision = f[3] if len(f) > 3 else 64
    lc_max_rank, lc_slice_bits = (f[4], f[5]) if len(f) > 5 else (0, 0)
    torch.cuda.set_device(0)
    g, b = uniform_angles(p, 5000 + n)
    pr = make_problem(n, erdos_renyi_graph(n, 3.0 / (n - 1), 4000 + n), g, b, 1e-3, 1e-2, K, 6000 + n,
                      name=f"er-n{n}-p{p}-K{K}")
    t0 = time.perf_counter()
    pl = stn.Plan(pr, outputs=stn.OUT_ENERGY, precision=precision, hbm_budget=int(args.hbm_budget_gib * (1 << 30)),
                  plan_kind=stn.PLAN_LIGHTCONE if lc_slice_bits else stn.PLAN_AUTO, lc_max_rank=lc_max_rank,
                  lc_slice_bits=lc_slice_bits)
    plan_ms = (time.perf_counter() - t0) * 1e3
    tune = None
    if args.job_tune:
        tb = pl.sample(pr.seed, 0, min(K, 256))
        tune = pl.autotune(tb, reps=1)
        tb.close()
    info = pl.info()
    B = info["max_batch"]

    def run():
        acc = pl.accum()
        for k0 in range(0, K, B):
            bt = pl.sample(pr.seed, k0, min(B, K - k0))
            pl.contract(bt)
            pl.reduce(bt, acc)
            bt.close()
        r = acc.read()
        acc.close()
        return r

    run()
    torch.cuda.synchronize()
    pl.profile(True)
    t1 = time.perf_counter()
    r = run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    prof = pl.profile_read()
    pl.close()
    return {"workload": pr.name, "precision": precision, "plan": info["plan_name"], "width": info["width"],
            "lc_slices": info["lc_slices"], "lc_slice_bits": info["lc_slice_bits"], "launch_shape": tune,
            "steps": info["n_steps"], "passes": info["n_passes"], "trajectories_per_launch": B, "plan_ms": plan_ms,
            "seconds": dt, "trajectories_per_s": K / dt, "energy_mean": r["energy_mean"], "energy_se": r["energy_se"],
            "kernels": {k: {"launches": v["launches"], "ms": v["ms"],
                            "gbps": v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] else None}
                        for k, v in prof.items() if v["launches"]}}


def queue_leg(stn, jobs=64, reps=5):
    """Many small jobs (whole state in LDS) on one stream: one launch per job
    against one launch whose persistent workgroups drain a device-side queue
    of every job's trajectories.  Same results, bit for bit."""
    import numpy as np
    import torch
    from workloads import make_problem, random_regular_graph, uniform_angles
    torch.cuda.set_device(0)
    rng = np.random.default_rng(2024)
    probs = []
    for i in range(jobs):
        n = 2 * int(rng.integers(3, 7))
        p = int(rng.integers(1, 5))
        K = int(rng.integers(16, 257))
        g, b = uniform_angles(p, 300 + i)
        probs.append(make_problem(n, random_regular_graph(n, 3, 400 + i), g, b, 1e-3, 1e-2, K, 500 + i,
                                  name=f"small{i}"))
    plans = [stn.Plan(pr, plan_kind=stn.PLAN_SV_LDS, outputs=stn.OUT_ENERGY) for pr in probs]
    batches = [pl.sample(pr.seed, 0, pr.K) for pl, pr in zip(plans, probs)]
    for pl, bt in zip(plans, batches):
        pl.contract(bt)
    alone = [bt.energies() for bt in batches]
    stn.contract_many(plans, batches)
    torch.cuda.synchronize()
    same = all((bt.energies() == e).all() for bt, e in zip(batches, alone))

    def timed(fn):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    t_each = timed(lambda: [pl.contract(bt) for pl, bt in zip(plans, batches)])
    t_queue = timed(lambda: stn.contract_many(plans, batches))
    traj = sum(pr.K for pr in probs)
    for bt in batches:
        bt.close()
    return {"jobs": jobs, "trajectories": traj, "n_range": [min(pr.n_qubits for pr in probs),
                                                              max(pr.n_qubits for pr in probs)],
            "one_launch_per_job_ms": t_each * 1e3, "queue_launch_ms": t_queue * 1e3,
            "one_launch_per_job_traj_per_s": traj / t_each, "queue_traj_per_s": traj / t_queue,
            "speedup": t_each / t_queue, "identical": bool(same)}


def graph_leg(stn, chunks=400):
    """Chunks of small jobs (one batch refilled with stn_resample, then
    contracted) on a side stream, eager against replayed HIP graphs: wall
    time per chunk with the device kept busy, and with a synchronisation
    after every chunk (latency)."""
    import torch
    from workloads import make_problem, random_regular_graph, uniform_angles
    torch.cuda.set_device(0)
    out = {}
    for name, n, p, K in [("sv_lds", 10, 2, 64), ("lightcone", 20, 1, 64), ("sv_tiled", 16, 2, 8)]:
        g, b = uniform_angles(p, 70 + n)
        pr = make_problem(n, random_regular_graph(n, 3, 60 + n), g, b, 1e-3, 1e-2, K, 80 + n)
        row = {"n": n, "p": p, "K": K}
        energies = {}
        for graphs in (False, True):
            pl = stn.Plan(pr, outputs=stn.OUT_ENERGY)
            pl.set_graphs(graphs)
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                bt = pl.sample(pr.seed, 0, K)
                for c in range(3):            # eager, capture, first replay
                    pl.resample(bt, pr.seed, c * K, K)
                    pl.contract(bt)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for c in range(chunks):
                    pl.resample(bt, pr.seed, c * K, K)
                    pl.contract(bt)
                torch.cuda.synchronize()
                busy = (time.perf_counter() - t0) / chunks
                t0 = time.perf_counter()
                for c in range(chunks // 4):
                    pl.resample(bt, pr.seed, c * K, K)
                    pl.contract(bt)
                    s.synchronize()
                lat = (time.perf_counter() - t0) / (chunks // 4)
                energies[graphs] = bt.energies()
            info = pl.info()
            key = "graph" if graphs else "eager"
            row[key + "_us_per_chunk"] = busy * 1e6
            row[key + "_us_per_chunk_synced"] = lat * 1e6
            if graphs:
                row["captures"] = info["graph_captures"]
                row["replays"] = info["graph_replays"]
            row["plan"] = info["plan_name"]
            bt.close()
            pl.close()
        row["identical"] = bool((energies[False] == energies[True]).all())
        out[name] = row
    return out


def uneven_leg(stn, args, window=None):
    """64 QAOA jobs, n ~ U{10..30}, p ~ U{1..6}, Erdos-Renyi p_edge = 3/(n-1),
    K ~ U{256..8192}, submitted at once to the job server; runs until all are
    done or the window ends (jobs still running then are censored)."""
    window = args.uneven_window if window is None else window
    import numpy as np
    import torch
    from workloads import uneven_batch
    torch.cuda.set_device(0)
    jobs = uneven_batch()
    res = {}
    sv = stn.Server(hbm_budget=int(args.hbm_budget_gib * (1 << 30)), job_share=0.5, n_streams=3, max_active=32,
                    drain_on_destroy=False)
    t0 = sv.clock()
    for i, pr in enumerate(jobs):
        sv.submit(pr, tag=i)
    last_chunks, last_print = 0, 0.0
    while sv.clock() - t0 < window and len(res) < len(jobs):
        for r in sv.poll(wait=1.0, cap=4096):
            res[r["tag"]] = r
            print(f"uneven: job {r['tag']} n={jobs[r['tag']].n_qubits} p={jobs[r['tag']].p} K={r['K']} "
                  f"{r['plan_name']} done at {r['t_done'] - t0:.2f} s", file=sys.stderr, flush=True)
        # chunks issued since the last line (long jobs complete rarely)
        st = sv.stats()
        if st["chunks"] > last_chunks and st["clock"] - last_print >= 20.0:
            print(f"uneven: {st['clock'] - t0:.0f} s, {st['completed']} jobs done, {st['chunks']} chunks issued",
                  file=sys.stderr, flush=True)
            last_chunks, last_print = st["chunks"], st["clock"]
    t_end = min(sv.clock() - t0, window)
    st = sv.stats()
    sv.close()
    done = [i for i in res if res[i]["status"] == 0]
    traj = sum(res[i]["K"] for i in done)
    lat = np.array([res[i]["t_done"] - t0 if i in res else np.inf for i in range(len(jobs))])
    by_plan = {}
    for i in done:
        d = by_plan.setdefault(res[i]["plan_name"], {"jobs": 0, "trajectories": 0})
        d["jobs"] += 1
        d["trajectories"] += res[i]["K"]
    censored = [{"n": jobs[i].n_qubits, "p": jobs[i].p, "K": jobs[i].K} for i in range(len(jobs)) if i not in res]
    torch.cuda.synchronize()
    # the batch's work in device-seconds by the library's cost model (the
    # server's admission and scheduling estimate), done and in all
    est = []
    for pr in jobs:
        pl = stn.Plan(pr, outputs=stn.OUT_ENERGY, precision=64, hbm_budget=int(0.5 * args.hbm_budget_gib * (1 << 30)))
        est.append(pl.info()["est_s_per_traj"] * pr.K)
        pl.close()
    return {"jobs": len(jobs), "window_s": window, "completed": len(done),
            "work_device_s": {"all": float(sum(est)), "completed": float(sum(est[i] for i in done))},
            "failed": int(sum(r["status"] != 0 for r in res.values())), "censored": censored,
            "makespan_s": t_end, "trajectories": traj, "trajectories_per_s": traj / t_end if t_end > 0 else None,
            "completion_s": {"p50": float(np.percentile(lat, 50, method="higher"))
                             if np.isfinite(np.percentile(lat, 50, method="higher")) else None,
                             "max_completed": float(lat[np.isfinite(lat)].max()) if np.isfinite(lat).any() else None},
            "by_plan": by_plan, "max_concurrent_jobs": st["max_active_jobs"], "autotuned_shapes": st["autotuned"],
            "plan_cache_hits": st["plan_cache_hits"], "device_bytes_peak": st["bytes_peak"]}


def serving_leg(stn, args):
    """The first `serve_jobs` arrivals of the Poisson stream through the job
    server at their arrival times, for a window of `serve_window` seconds from
    the first arrival; latency = completion - arrival.  Jobs still running at
    the end of the window are counted as censored and abandoned; a percentile
    that falls on a censored job is reported as a lower bound (window end -
    that job's arrival) and flagged.  Offered and achieved load are stated in
    device-seconds of work by the library's cost model."""
    import numpy as np
    import torch
    from workloads import poisson_stream
    arrivals, jobs = poisson_stream(args.serve_jobs, rate_per_s=args.serve_rate)
    res = {}
    sv = stn.Server(hbm_budget=int(args.hbm_budget_gib * (1 << 30)), job_share=0.5, n_streams=3, max_active=16,
                    drain_on_destroy=False)
    t0 = sv.clock()
    for i, (ta, pr) in enumerate(zip(arrivals, jobs)):
        while sv.clock() - t0 < ta:
            time.sleep(min(1e-3, max(0.0, ta - (sv.clock() - t0))))
        sv.submit(pr, tag=i)
    last = sv.clock()
    while sv.clock() - t0 < args.serve_window and len(res) < len(jobs):
        for r in sv.poll(wait=0.5, cap=4096):
            res[r["tag"]] = r
        if sv.clock() - last > 20.0:    # progress for long windows
            last = sv.clock()
            print(f"serving: {last - t0:.0f} s, {len(res)} of {len(jobs)} jobs done", file=sys.stderr, flush=True)
    t_end = min(sv.clock() - t0, args.serve_window)
    st = sv.stats()
    sv.close()                      # abandons unfinished jobs
    lat = np.array([res[i]["t_done"] - t0 - arrivals[i] if i in res else np.inf for i in range(len(jobs))])
    # a job still running when the window closed has latency > (window end - its arrival)
    lat_lb = np.array([lat[i] if i in res else t_end - arrivals[i] for i in range(len(jobs))])
    done = [i for i in res if res[i]["status"] == 0]
    traj = sum(res[i]["K"] for i in done)

    def pct(q):
        """(value, censored): the percentile, or when it falls on a job still
        running at the end of the window, a lower bound of it."""
        v = float(np.percentile(lat, q, method="higher"))
        if math.isfinite(v):
            return v, False
        return float(np.percentile(lat_lb, q, method="higher")), True

    # offered and achieved load in device-seconds of work by the library's cost
    # model (the same estimate the server admits and schedules by), per second
    est = []
    for pr in jobs:
        pl = stn.Plan(pr, outputs=stn.OUT_ENERGY, precision=64,
                      hbm_budget=int(0.5 * args.hbm_budget_gib * (1 << 30)))
        inf = pl.info()
        est.append(inf["est_s_per_traj"] * pr.K)
        pl.close()
    span = max(float(arrivals[-1]), 1.0 / args.serve_rate)
    offered = {"work_device_s": float(sum(est)),
               "per_s_at_rate": float(args.serve_rate * np.mean(est)),
               "per_s_over_trace": float(sum(est) / span),
               "achieved_work_device_s": float(sum(est[i] for i in done)),
               "achieved_per_s": float(sum(est[i] for i in done) / t_end) if t_end > 0 else None,
               "note": "device-seconds of work (cost model) offered per second of arrivals, at the stream's mean "
                       "rate and over this trace's arrival span; achieved = the work of the completed jobs per "
                       "second of the window; a ratio above 1 means the GPU cannot keep up and latency is queueing"}

    checks = []
    # every k-th finished job up to n = 24 (the complex128 path costs ~3x the complex64 one)
    chk = [i for i in range(0, len(jobs), max(1, args.serve_check_every)) if i in done and jobs[i].n_qubits <= 24]
    if chk:
        with stn.Server(hbm_budget=int(args.hbm_budget_gib * (1 << 30)), precision=128) as sv2:
            for i in chk:
                sv2.submit(jobs[i], tag=i)
            sv2.drain(3600)
            ref = {r["tag"]: r for r in sv2.poll(cap=4096)}
        for i in chk:
            m = max(1, len(jobs[i].edges))
            checks.append({"job": i, "n": jobs[i].n_qubits, "p": jobs[i].p, "K": jobs[i].K,
                           "plan": res[i]["plan_name"],
                           "reference": "complex128 path, same draws, through the server (served jobs against "
                                        "the oracle: tests/test_gpu_server.py)",
                           "abs_err_per_edge": abs(res[i]["energy_mean"] - ref[i]["energy_mean"]) / m,
                           "se_per_edge": res[i]["energy_se"] / m})
    torch.cuda.synchronize()
    return {
        "jobs": len(jobs), "rate_per_s": args.serve_rate, "window_s": args.serve_window,
        "completed": len(done), "censored": len(jobs) - len(res),
        "failed": int(sum(r["status"] != 0 for r in res.values())),
        "latency_s": {"p50": pct(50)[0], "p50_is_lower_bound": pct(50)[1],
                      "p99": pct(99)[0], "p99_is_lower_bound": pct(99)[1],
                      "max_completed": float(lat[np.isfinite(lat)].max()) if np.isfinite(lat).any() else None},
        "trajectories_per_s": traj / t_end if t_end > 0 else None, "arrivals_span_s": arrivals[-1],
        "max_concurrent_jobs": st["max_active_jobs"],
        "plans": {k: sum(1 for r in res.values() if r["plan_name"] == k) for k in ("sv_lds", "sv_tiled", "lightcone")},
        "jobs_detail": [{"n": jobs[i].n_qubits, "p": jobs[i].p, "K": jobs[i].K,
                         "latency_s": None if not math.isfinite(lat[i]) else float(lat[i]),
                         "admit_wait_s": res[i]["t_admit"] - t0 - arrivals[i] if i in res else None,
                         "chunks": res[i]["chunks"] if i in res else None,
                         "plan": res[i]["plan_name"] if i in res else None,
                         "est_device_s": est[i]} for i in range(len(jobs))],
        "load": offered,
        "fp64_checks": checks,
    }


if __name__ == "__main__":
    main()
