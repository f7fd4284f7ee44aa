"""Job server (continuous batching of many <C> jobs on one device): results
of served jobs against the same jobs run alone through the plan API (bit
for bit), against the oracle, and the admission / failure behaviour."""
import math
import time

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


def stn_mod():
    import paper_2210_15874_amd as stn
    return stn


def mixed_jobs():
    """Small jobs covering the three lowerings (whole state in LDS, tiled
    HBM statevector, lightcone networks)."""
    from workloads import erdos_renyi_graph, make_problem, random_regular_graph, uniform_angles
    jobs = []
    for i, (n, p, K, lam) in enumerate([(10, 3, 700, (1e-3, 1e-2)), (16, 2, 300, (2e-3, 2e-2)),
                                        (22, 1, 500, (1e-3, 1e-2)), (12, 4, 1200, (1e-4, 5e-3)),
                                        (18, 3, 96, (5e-3, 1e-2)), (20, 1, 64, (1e-2, 1e-2))]):
        if i % 2:
            edges = random_regular_graph(n, 3, 900 + i)
        else:
            edges = erdos_renyi_graph(n, 3.0 / (n - 1), 900 + i)
        g, b = uniform_angles(p, 950 + i)
        jobs.append(make_problem(n, edges, g, b, lam[0], lam[1], K, 7000 + i, name=f"mix{i}"))
    return jobs


def alone(pr, precision=64):
    stn = stn_mod()
    return stn.simulate_batch_ensemble(pr, precision=precision)


def test_served_jobs_equal_plan_api_bit_for_bit():
    stn = stn_mod()
    jobs = mixed_jobs()
    ref = [alone(pr) for pr in jobs]
    with stn.Server(hbm_budget=8 << 30, n_streams=4, max_active=8) as sv:
        ids = [sv.submit(pr, tag=i) for i, pr in enumerate(jobs)]
        sv.drain(300)
        res = {r["tag"]: r for r in sv.poll(cap=64)}
        st = sv.stats()
    assert sorted(res) == list(range(len(jobs)))
    kinds = set()
    for i, pr in enumerate(jobs):
        r = res[i]
        assert r["status"] == 0, r["error"]
        assert r["k_done"] == pr.K
        kinds.add(r["plan_name"])
        assert r["energy_mean"] == ref[i]["energy_mean"], (i, r["energy_mean"], ref[i]["energy_mean"])
        assert r["energy_se"] == ref[i]["energy_se"]
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
    assert kinds == {"sv_lds", "sv_tiled", "lightcone"}
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["trajectories"] == sum(pr.K for pr in jobs)
    assert len(set(ids)) == len(ids)


def test_served_wide_tile_job_equals_plan_api_bit_for_bit():
    """An n=26 p=3 job, planned with 15-qubit tiles: the server runs it in
    chunks sized by its tiles (16 trajectories here), the plan API in one
    batch; the results agree bit for bit."""
    from workloads import make_problem, random_regular_graph, uniform_angles
    stn = stn_mod()
    g, b = uniform_angles(3, 31)
    pr = make_problem(26, random_regular_graph(26, 3, 77), g, b, 1e-3, 1e-2, 40, 5, name="wide")
    pl = stn.Plan(pr)
    info = pl.info()
    assert info["plan_name"] == "sv_tiled" and info["tile_bits"] == 15 and info["max_batch"] >= pr.K
    ref = stn.simulate_batch_ensemble(pr, plan=pl)
    pl.close()
    torch.cuda.empty_cache()
    with stn.Server(hbm_budget=24 << 30, n_streams=2, max_active=2) as sv:
        sv.submit(pr, tag=1)
        sv.drain(300)
        res = sv.poll(cap=4)
    assert len(res) == 1 and res[0]["status"] == 0, res
    r = res[0]
    assert r["plan_name"] == "sv_tiled" and r["k_done"] == pr.K and r["chunks"] >= 2
    assert r["energy_mean"] == ref["energy_mean"] and r["energy_se"] == ref["energy_se"]


def test_same_result_alone_and_in_mix():
    """A job's result does not depend on what else the server runs."""
    stn = stn_mod()
    jobs = mixed_jobs()
    probe = jobs[1]
    with stn.Server(hbm_budget=8 << 30) as sv:
        sv.submit(probe, tag=99)
        sv.drain(120)
        solo = sv.poll(cap=4)[0]
    with stn.Server(hbm_budget=8 << 30, n_streams=3, max_active=6, chunk_max=64) as sv:
        for i, pr in enumerate(jobs):
            sv.submit(pr, tag=i)
            if i == 2:
                sv.submit(probe, tag=99)
        sv.drain(300)
        mixed = [r for r in sv.poll(cap=64) if r["tag"] == 99][0]
    assert mixed["status"] == 0 and solo["status"] == 0
    assert mixed["chunks"] > solo["chunks"]      # smaller chunks in the mix
    assert mixed["energy_mean"] == solo["energy_mean"]
    assert mixed["energy_se"] == solo["energy_se"]


def test_graphs_on_and_off_give_the_same_results():
    """Chunk contractions replayed from HIP graphs against eager launches
    (the default): the same jobs, many chunks each, bit for bit."""
    stn = stn_mod()
    jobs = mixed_jobs()
    out = {}
    for graphs in (False, True):
        with stn.Server(hbm_budget=8 << 30, n_streams=3, max_active=6, chunk_max=64, graphs=graphs) as sv:
            for i, pr in enumerate(jobs):
                sv.submit(pr, tag=i)
            sv.drain(300)
            out[graphs] = {r["tag"]: r for r in sv.poll(cap=64)}
    for i, pr in enumerate(jobs):
        a, b = out[False][i], out[True][i]
        assert a["status"] == 0 and b["status"] == 0, (a["error"], b["error"])
        assert b["chunks"] == a["chunks"] and b["k_done"] == pr.K
        assert b["energy_mean"] == a["energy_mean"] and b["energy_se"] == a["energy_se"]


def test_multi_batch_launches_give_the_same_results():
    """Ready chunks of whole-state-in-LDS jobs gathered into multi-batch
    launches (the default) against one launch per chunk: bit for bit."""
    from workloads import make_problem, random_regular_graph, uniform_angles
    stn = stn_mod()
    jobs = []
    for i in range(12):
        n, p, K = 6 + 2 * (i % 4), 1 + i % 3, 100 + 37 * i
        g, b = uniform_angles(p, 600 + i)
        jobs.append(make_problem(n, random_regular_graph(n, 3, 610 + i), g, b, 2e-3, 1e-2, K, 620 + i,
                                 name=f"lds{i}"))
    out, stats = {}, {}
    for gang in (False, True):
        with stn.Server(hbm_budget=4 << 30, n_streams=3, max_active=16, chunk_max=64, gang=gang) as sv:
            for i, pr in enumerate(jobs):
                sv.submit(pr, tag=i)
            sv.drain(120)
            out[gang] = {r["tag"]: r for r in sv.poll(cap=64)}
            stats[gang] = sv.stats()
    assert stats[False]["gang_launches"] == 0
    assert stats[True]["gang_launches"] > 0 and stats[True]["gang_chunks"] >= 2 * stats[True]["gang_launches"]
    for i, pr in enumerate(jobs):
        a, b = out[False][i], out[True][i]
        assert a["status"] == 0 and b["status"] == 0, (a["error"], b["error"])
        assert a["plan_name"] == b["plan_name"] == "sv_lds"
        assert b["k_done"] == pr.K and b["chunks"] == a["chunks"]
        assert b["energy_mean"] == a["energy_mean"] and b["energy_se"] == a["energy_se"]


def test_served_job_against_oracle():
    from oracle import simulate as sim
    from workloads import make_problem, random_regular_graph, uniform_angles
    stn = stn_mod()
    n, p, K = 10, 2, 48
    g, b = uniform_angles(p, 31)
    pr = make_problem(n, random_regular_graph(n, 3, 30), g, b, 5e-3, 3e-2, K, 32)
    ens = sim.ensemble(pr, pr.seed, 0, K, want_states=False)
    e = np.asarray(ens["energies"])
    for precision, tol in [(64, 1e-5), (128, 1e-11)]:
        with stn.Server(hbm_budget=1 << 30, precision=precision) as sv:
            sv.submit(pr)
            sv.drain(60)
            r = sv.poll(cap=4)[0]
        assert r["status"] == 0, r["error"]
        m = len(pr.edges)
        assert abs(r["energy_mean"] - e.mean()) / m < tol
        assert abs(r["energy_se"] - e.std(ddof=1) / math.sqrt(K)) / m < tol


def test_served_stream_jobs_against_oracle():
    """Jobs of the Poisson serving stream (n <= 16 among its first arrivals;
    random Erdos-Renyi graphs, p 1..6, log-uniform depolarizing rates), each
    cut to its first 6 trajectories, served together in complex64 and
    checked against the oracle's literal-Kraus ensemble of the same
    trajectories (mean and standard error per edge within 1e-5)."""
    from oracle import simulate as sim
    from workloads import poisson_stream
    stn = stn_mod()
    _, jobs = poisson_stream(60)
    sel = [pr for pr in jobs if pr.n_qubits <= 16 and pr.edges][:5]
    assert len(sel) == 5
    for pr in sel:
        pr.K = 6
    with stn.Server(hbm_budget=4 << 30, precision=64) as sv:
        for i, pr in enumerate(sel):
            sv.submit(pr, tag=i)
        sv.drain(120)
        res = {r["tag"]: r for r in sv.poll(cap=16)}
    for i, pr in enumerate(sel):
        r = res[i]
        assert r["status"] == 0, r["error"]
        e = np.asarray(sim.ensemble(pr, pr.seed, 0, pr.K, want_states=False)["energies"])
        m = len(pr.edges)
        err = abs(r["energy_mean"] - e.mean()) / m
        print(f"stream job n={pr.n_qubits} p={pr.p} {r['plan_name']}: |<C> - oracle|/m = {err:.2e}")
        assert err < 1e-5
        assert abs(r["energy_se"] - e.std(ddof=1) / math.sqrt(pr.K)) / m < 1e-5


def test_small_jobs_overtake_a_long_one():
    """Continuous batching: jobs submitted after a long job has started run
    beside it and finish before it."""
    from workloads import make_problem, random_regular_graph, uniform_angles
    stn = stn_mod()
    g, b = uniform_angles(4, 61)
    big = make_problem(24, random_regular_graph(24, 3, 60), g, b, 1e-3, 1e-2, 6144, 62, name="big")
    smalls = mixed_jobs()
    with stn.Server(hbm_budget=48 << 30, job_share=0.5, n_streams=4, max_active=8) as sv:
        sv.submit(big, tag=1000)
        t_wait = time.time() + 30
        while sv.stats()["active"] == 0 and time.time() < t_wait:
            time.sleep(0.01)
        time.sleep(0.2)
        for i, pr in enumerate(smalls):
            sv.submit(pr, tag=i)
        sv.drain(600)
        res = {r["tag"]: r for r in sv.poll(cap=64)}
        st = sv.stats()
    assert all(r["status"] == 0 for r in res.values())
    assert st["max_active_jobs"] >= 2
    tb = res[1000]
    assert tb["chunks"] > 1
    done_first = [i for i in range(len(smalls)) if res[i]["t_done"] < tb["t_done"]]
    assert len(done_first) >= len(smalls) - 1, (done_first, tb)


def test_failed_jobs_reported_and_others_unaffected():
    from workloads import Gate, Problem
    stn = stn_mod()
    jobs = mixed_jobs()[:2]
    bad = Problem(4, [Gate("h", (7,))], [], [(0, 1)], [1.0], [], [], 16, 5, "bad")   # qubit out of range
    with stn.Server(hbm_budget=1 << 30) as sv:
        sv.submit(jobs[0], tag=0)
        sv.submit(bad, tag=1)
        sv.submit(jobs[1], tag=2)
        # larger than the whole budget: rejected, not admitted
        from workloads import make_problem, random_regular_graph, uniform_angles
        g, b = uniform_angles(4, 3)   # p = 4: statevector only, 2 GiB per trajectory
        huge = make_problem(28, random_regular_graph(28, 3, 4), g, b, 1e-3, 1e-2, 64, 5)
        sv.submit(huge, tag=3)
        sv.drain(120)
        res = {r["tag"]: r for r in sv.poll(cap=8)}
    assert res[1]["status"] == 1 and "qubit" in res[1]["error"]
    assert res[3]["status"] == 3
    ref0, ref2 = alone(jobs[0]), alone(jobs[1])
    assert res[0]["status"] == 0 and res[0]["energy_mean"] == ref0["energy_mean"]
    assert res[2]["status"] == 0 and res[2]["energy_mean"] == ref2["energy_mean"]


def test_plan_cache_reuses_plans():
    stn = stn_mod()
    pr = mixed_jobs()[0]
    with stn.Server(hbm_budget=2 << 30, plan_cache=4) as sv:
        for s in range(3):
            sv.submit(pr, seed=100 + s, K=128, tag=s)
            sv.drain(60)
        res = {r["tag"]: r for r in sv.poll(cap=8)}
        st = sv.stats()
    assert st["plan_cache_hits"] == 2 and st["plan_cache_misses"] == 1
    for s in range(3):
        ref = stn.simulate_batch_ensemble(pr, K=128, seed=100 + s)
        assert res[s]["energy_mean"] == ref["energy_mean"]


def test_served_amplitude_damping_job_uses_gate_by_gate_lowering():
    """A <C> job with amplitude damping above the whole-state-in-LDS size is
    served through the gate-by-gate lowering, bit for bit as alone, beside a
    job of another lowering."""
    from workloads import make_problem, random_regular_graph, uniform_angles
    stn = stn_mod()
    g, b = uniform_angles(2, 71)
    ad = make_problem(16, random_regular_graph(16, 3, 72), g, b, 1e-3, 1e-2, 48, 73, gamma_ad=0.02, name="ad16")
    jobs = [ad, mixed_jobs()[0]]
    ref = [alone(pr) for pr in jobs]
    with stn.Server(hbm_budget=8 << 30, n_streams=4, max_active=8) as sv:
        for i, pr in enumerate(jobs):
            sv.submit(pr, tag=i)
        sv.drain(300)
        res = {r["tag"]: r for r in sv.poll(cap=64)}
    assert res[0]["status"] == 0, res[0]["error"]
    assert res[0]["plan_name"] == "sv_gates"
    for i in range(len(jobs)):
        assert res[i]["energy_mean"] == ref[i]["energy_mean"]
        assert res[i]["energy_se"] == ref[i]["energy_se"]
