"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle on
the same seeded inputs and the same Philox draws.

Tolerances: complex128 paths agree with the oracle to rounding (1e-12);
complex64 paths (FP32 arithmetic, FP64 reductions) within 1e-5 max-abs on
rho_hat and on <C>/m (per-edge normalised energy), the reading of the
"1e-5 beyond the stochastic error" target for the FP32 path.  Results that
several draws could produce are compared by what is unique: per-trajectory
states only up to a global phase (the Pauli-frame rewrite and the dropped
phase of Y change it), via |<a|b>|.
"""
import ctypes
import itertools
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2210_15874_amd as stn
    stn.load()  # raises if the library is missing: no fallback
    torch.zeros(1, device="cuda")
    yield


def stn_mod():
    import paper_2210_15874_amd as stn
    return stn


def overlap(a, b):
    return abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))


# ----------------------------------------------------------------------------- sampling

@pytest.mark.parametrize("cfg,K,k0", [(0, 100, 0), (1, 1024, 0), (2, 4096, 0), (2, 64, (1 << 32) - 17)])
def test_sampler_bit_exact(cfg, K, k0):
    from oracle.simulate import kraus_indices
    from workloads import config_problem
    stn = stn_mod()
    pr = config_problem(cfg)
    pl = stn.Plan(pr)
    b = pl.sample(pr.seed, k0, K)
    got = b.indices()
    exp = kraus_indices(pr, pr.seed, k0, K)
    np.testing.assert_array_equal(got, exp)


# ----------------------------------------------------------------------------- whole-state-in-LDS path

def run_states(pr, K, precision, outputs=None, seed=None, batch=None):
    stn = stn_mod()
    outputs = outputs or (stn.OUT_RHO | stn.OUT_DIAG | stn.OUT_ENERGY | stn.OUT_STATES)
    pl = stn.Plan(pr, outputs=outputs, precision=precision)
    acc = pl.accum()
    states, energies = [], []
    step = batch or K
    for k0 in range(0, K, step):
        b = pl.sample(seed if seed is not None else pr.seed, k0, min(step, K - k0))
        pl.contract(b)
        pl.reduce(b, acc)
        if outputs & stn.OUT_STATES:
            states.append(b.states())
        energies.append(b.energies())
    res = acc.read()
    res["states"] = np.concatenate(states) if states else None
    res["batch_energies"] = np.concatenate(energies)
    res["info"] = pl.info()
    return res


@pytest.mark.parametrize("precision,tol", [(128, 1e-12), (64, 1e-5)])
def test_lds_config0_same_draws(precision, tol):
    from oracle import simulate as sim
    from workloads import config_problem
    pr = config_problem(0)
    res = run_states(pr, pr.K, precision)
    assert res["info"]["plan_name"] == "sv_lds"
    ens = sim.ensemble(pr, pr.seed, 0, pr.K)
    for k in range(pr.K):
        assert overlap(res["states"][k], ens["psi"][k]) > 1 - tol, k
    m = len(pr.edges)
    np.testing.assert_allclose(res["batch_energies"] / m, ens["energies"] / m, atol=tol)
    np.testing.assert_allclose(res["rho"], ens["rho_hat"], atol=tol)
    np.testing.assert_allclose(res["diag"], ens["sigma_approx"], atol=tol)
    assert abs(res["energy_mean"] - ens["energies"].mean()) / m < tol
    assert abs(res["energy_se"] - ens["energies"].std(ddof=1) / math.sqrt(pr.K)) < tol
    # rho_hat is Hermitian exactly (mirrored) and PSD; trace 1 for Pauli noise
    np.testing.assert_array_equal(res["rho"], res["rho"].conj().T)
    assert np.linalg.eigvalsh(res["rho"]).min() > -10 * tol
    assert abs(res["trace"] - 1) < 10 * tol


def test_lds_config0_against_exact_density_matrix():
    from oracle import metrics
    from oracle import simulate as sim
    from workloads import config_problem
    pr = config_problem(0)
    res = run_states(pr, pr.K, 128)
    rho = sim.density_matrix(pr)
    exact = sim.energy_exact(rho, pr.n_qubits, pr.edges, pr.weights)
    assert abs(res["energy_mean"] - exact) <= 1e-5 + 4 * res["energy_se"]
    purity = float(np.real(np.trace(rho @ rho)))
    # E||rho_hat - rho||_F^2 = (1 - Tr rho^2)/K; a 5-sigma-ish bound
    assert metrics.frobenius(res["rho"], rho) ** 2 < 5 * (1 - purity) / pr.K
    assert metrics.paper_error(res["diag"], np.diag(rho).real) < 0.05


@pytest.mark.parametrize("precision,tol", [(64, 1e-5), (128, 1e-12)])
def test_lds_config1_same_draws(precision, tol):
    """n=12, p=2, depolarizing + amplitude damping, K=1024 in one launch."""
    from oracle import simulate as sim
    from workloads import config_problem
    stn = stn_mod()
    pr = config_problem(1)
    res = run_states(pr, pr.K, precision, outputs=stn.OUT_RHO | stn.OUT_DIAG | stn.OUT_ENERGY | stn.OUT_STATES)
    ens = sim.ensemble(pr, pr.seed, 0, pr.K)
    m = len(pr.edges)
    np.testing.assert_allclose(res["batch_energies"] / m, ens["energies"] / m, atol=tol)
    for k in range(0, pr.K, 37):
        assert overlap(res["states"][k], ens["psi"][k]) > 1 - tol
        assert abs(np.linalg.norm(res["states"][k]) - np.linalg.norm(ens["psi"][k])) < tol
    assert np.abs(res["rho"] - ens["rho_hat"]).max() < tol
    assert np.abs(res["diag"] - ens["sigma_approx"]).max() < tol
    assert abs(res["trace"] - np.trace(ens["rho_hat"]).real) < tol


def tiny_problems():
    from workloads import Channel, Gate, Problem
    yield Problem(2, [Gate("h", (0,)), Gate("cx", (0, 1)), Gate("rx", (1,), 0.7)],
                  [Channel(0, "bitflip", (0,), 0.2), Channel(1, "depol2", (0, 1), 0.3),
                   Channel(2, "ampdamp", (1,), 0.25), Channel(2, "depol1", (1,), 0.1)], [(0, 1)], [1.0])
    yield Problem(3, [Gate("h", (0,)), Gate("y", (2,)), Gate("zz", (0, 2), 1.1), Gate("ry", (1,), 0.4),
                      Gate("u2", (2, 1), 0.0, tuple(np.linalg.qr(np.arange(16).reshape(4, 4) + 1j)[0].reshape(-1)))],
                  [Channel(0, "depol1", (0,), 0.2), Channel(2, "depol2", (0, 2), 0.15),
                   Channel(3, "bitflip", (1,), 0.3), Channel(4, "ampdamp", (2,), 0.4)], [(0, 1), (1, 2)], [1.0, 0.5])


@pytest.mark.parametrize("precision,tol", [(128, 1e-12), (64, 2e-6)])
@pytest.mark.parametrize("pi", [0, 1])
def test_exhaustive_enumeration_matches_dm(pi, precision, tol):
    """Every outcome tuple fed through stn_batch_from_indices; the
    probability-weighted sum of psi psi^dag equals the exact rho."""
    from oracle import simulate as sim
    stn = stn_mod()
    pr = list(tiny_problems())[pi]
    tabs = sim.site_tables(pr)
    sizes = [len(t[0]) for t in tabs]
    tuples = list(itertools.product(*[range(s) for s in sizes]))
    w = np.array([math.prod(tabs[s][0][j] for s, j in enumerate(t)) for t in tuples])
    pl = stn.Plan(pr, outputs=stn.OUT_STATES | stn.OUT_ENERGY, precision=precision)
    b = pl.batch_from_indices(np.array(tuples, dtype=np.uint8))
    pl.contract(b)
    st = b.states()
    rho = np.einsum("k,ki,kj->ij", w, st, st.conj())
    np.testing.assert_allclose(rho, sim.density_matrix(pr), atol=tol)


# ----------------------------------------------------------------------------- tiled HBM path

def qaoa(n, p, seed, lam1, lam2, K):
    from workloads import make_problem, random_regular_graph, uniform_angles
    edges = random_regular_graph(n, 3 if n % 2 == 0 else 4, seed)   # no 3-regular graph on odd n
    g, b = uniform_angles(p, seed + 1)
    return make_problem(n, edges, g, b, lam1, lam2, K, seed + 2)


@pytest.mark.parametrize("precision,tol", [(64, 1e-5), (128, 1e-12)])
@pytest.mark.parametrize("n,p,K,lam", [(14, 2, 48, (1e-3, 1e-2)), (14, 1, 32, (0.05, 0.2)), (16, 3, 12, (0.02, 0.1)),
                                       (15, 2, 16, (0.02, 0.1)), (12, 2, 20, (0.02, 0.1))])
def test_tiled_energies_same_draws(n, p, K, lam, precision, tol):
    """Pauli-frame rewrite + tiled passes against literal Kraus insertion."""
    from oracle import simulate as sim
    stn = stn_mod()
    pr = qaoa(n, p, 100 + n + p, lam[0], lam[1], K)
    if n < 14 and precision == 64:
        # complex64 tiles hold 14 qubits: the planner must refuse, not run a partial tile
        with pytest.raises(stn.StnError) as ei:
            stn.Plan(pr, plan_kind=stn.PLAN_SV_TILED, max_batch=7, precision=precision)
        assert ei.value.status == 2 and "n >= 14" in str(ei.value)
        return
    pl = stn.Plan(pr, plan_kind=stn.PLAN_SV_TILED, max_batch=7, precision=precision)
    assert pl.info()["plan_name"] == "sv_tiled"
    acc = pl.accum()
    b = pl.sample(pr.seed, 0, K)
    pl.contract(b)
    pl.reduce(b, acc)
    got = b.energies()
    ens = sim.ensemble(pr, pr.seed, 0, K, want_states=False)
    m = len(pr.edges)
    assert (ens["idx"] != 0).any(axis=1).mean() > 0.1  # the frame is exercised
    np.testing.assert_allclose(got / m, ens["energies"] / m, atol=tol)
    r = acc.read()
    assert abs(r["energy_mean"] - got.mean()) < 1e-9


@pytest.mark.parametrize("n,p,K,lam", [(15, 2, 16, (0.02, 0.1)), (16, 3, 12, (0.02, 0.1)), (17, 2, 10, (1e-2, 5e-2))])
def test_tiled15_energies_same_draws(n, p, K, lam):
    """15-qubit tiles (one 1024-thread workgroup per CU, the layouts'
    register bits disjoint): Pauli-frame rewrite and tiled passes against
    literal Kraus insertion.  n = 15 is a single full-state tile; n = 16
    and 17 keep half the state, the second tile holding qubit n-1."""
    from oracle import simulate as sim
    stn = stn_mod()
    pr = qaoa(n, p, 100 + n + p, lam[0], lam[1], K)
    pl = stn.Plan(pr, plan_kind=stn.PLAN_SV_TILED, max_batch=5, precision=64, tile_bits=15)
    info = pl.info()
    assert info["plan_name"] == "sv_tiled" and info["tile_bits"] == 15 and info["half_state"] == (1 if n >= 16 else 0)
    acc = pl.accum()
    b = pl.sample(pr.seed, 0, K)
    pl.contract(b)
    pl.reduce(b, acc)
    got = b.energies()
    ens = sim.ensemble(pr, pr.seed, 0, K, want_states=False)
    m = len(pr.edges)
    assert (ens["idx"] != 0).any(axis=1).mean() > 0.1
    np.testing.assert_allclose(got / m, ens["energies"] / m, atol=1e-5)
    with pytest.raises(stn.StnError) as ei:
        stn.Plan(qaoa(14, 1, 5, 1e-3, 1e-2, 4), plan_kind=stn.PLAN_SV_TILED, precision=64, tile_bits=15)
    assert ei.value.status == 2 and "n >= 15" in str(ei.value)


def test_plan_handle_released_before_batch_and_accumulator():
    """A plan whose handle is released first stays alive until its last
    batch and accumulator are destroyed: their results can still be read,
    and their device buffers are freed through the plan's allocator
    afterwards (C ABI lifetime rule)."""
    stn = stn_mod()
    pr = qaoa(16, 2, 321, 1e-3, 1e-2, 8)
    pl = stn.Plan(pr, plan_kind=stn.PLAN_SV_TILED)
    acc = pl.accum()
    b = pl.sample(pr.seed, 0, pr.K)
    pl.contract(b)
    pl.reduce(b, acc)
    pl.close()
    e = b.energies()
    r = acc.read()
    assert abs(r["energy_mean"] - e.mean()) < 1e-9
    b.close()
    acc.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", [64, 128])
def test_batching_does_not_change_results(precision):
    stn = stn_mod()
    pr = qaoa(14, 2, 7, 0.01, 0.05, 40)
    out = []
    for step in (40, 13, 8):
        pl = stn.Plan(pr, plan_kind=stn.PLAN_SV_TILED, precision=precision)
        acc = pl.accum()
        for k0 in range(0, 40, step):
            b = pl.sample(pr.seed, k0, min(step, 40 - k0))
            pl.contract(b)
            pl.reduce(b, acc)
        out.append(acc.read())
    for r in out[1:]:
        np.testing.assert_array_equal(r["energies"], out[0]["energies"])
        assert r["energy_mean"] == out[0]["energy_mean"] and r["energy_se"] == out[0]["energy_se"]


def test_accumulator_read_buffers_not_shared():
    """rho_hat, sigma and the energies are read back into pinned host
    buffers taken from a pool of released ones: two live accumulators never
    share one, and a buffer released by a closed accumulator serves the next
    one correctly (each read checked against a fresh accumulator's)."""
    stn = stn_mod()
    from workloads import config_problem
    pr = config_problem(0)
    pl = stn.Plan(pr, outputs=stn.OUT_RHO | stn.OUT_DIAG | stn.OUT_ENERGY)

    def run(k0, K):
        acc = pl.accum()
        b = pl.sample(pr.seed, k0, K)
        pl.contract(b)
        pl.reduce(b, acc)
        b.close()
        return acc

    a1, a2 = run(0, 40), run(40, 40)
    r1, r2 = a1.read(), a2.read()
    r1b = a1.read()                       # a2's read must not have overwritten a1's buffers
    for key in ("rho", "diag", "energies"):
        np.testing.assert_array_equal(r1b[key], r1[key])
    assert np.abs(r1["rho"] - r2["rho"]).max() > 1e-6   # different trajectories
    a1.close()
    a3 = run(0, 40)                       # may take a1's released buffers
    r3 = a3.read()
    for key in ("rho", "diag", "energies"):
        np.testing.assert_array_equal(r3[key], r1[key])
    np.testing.assert_array_equal(a2.read()["rho"], r2["rho"])
    a2.close()
    a3.close()
    pl.close()


def test_reduce_same_range_twice_rejected():
    stn = stn_mod()
    from workloads import config_problem
    pr = config_problem(0)
    pl = stn.Plan(pr)
    acc = pl.accum()
    b = pl.sample(pr.seed, 0, 10)
    pl.contract(b)
    pl.reduce(b, acc)
    with pytest.raises(stn.StnError, match="already reduced"):
        pl.reduce(b, acc)
    assert acc.read()["k_done"] == 10


# ----------------------------------------------------------------------------- lightcone networks

LC_CASES = [(14, 1, 24, (0.05, 0.2), 64), (16, 2, 12, (0.02, 0.1), 64), (15, 2, 16, (1e-3, 1e-2), 64),
            (14, 1, 24, (0.05, 0.2), 128), (16, 2, 12, (0.02, 0.1), 128), (15, 1, 16, (1e-3, 1e-2), 128)]


@pytest.mark.parametrize("n,p,K,lam,precision", LC_CASES)
def test_lightcone_energies_same_draws(n, p, K, lam, precision):
    """Per-edge lightcone networks (min-fill bucket elimination, Pauli frame)
    against the full-statevector oracle with literal Kraus insertion."""
    from oracle import simulate as sim
    from workloads import erdos_renyi_graph, make_problem, uniform_angles
    stn = stn_mod()
    if n == 15:
        edges = erdos_renyi_graph(n, 3.0 / (n - 1), 77)
        g, b = uniform_angles(p, 78)
        pr = make_problem(n, edges, g, b, lam[0], lam[1], K, 79)
    else:
        pr = qaoa(n, p, 300 + n + p, lam[0], lam[1], K)
    pl = stn.Plan(pr, plan_kind=stn.PLAN_LIGHTCONE, precision=precision)
    info = pl.info()
    assert info["plan_name"] == "lightcone" and info["width"] <= 14
    b = pl.sample(pr.seed, 0, K)
    pl.contract(b)
    got = b.energies()
    ens = sim.ensemble(pr, pr.seed, 0, K, want_states=False)
    m = max(1, len(pr.edges))
    tol = 1e-5 if precision == 64 else 1e-11
    np.testing.assert_allclose(got / m, ens["energies"] / m, atol=tol)


@pytest.mark.parametrize("n,p,precision,tile_bits", [(15, 2, 64, 14), (17, 3, 64, 14), (27, 2, 64, 14),
                                                     (16, 2, 64, 15), (17, 3, 64, 15), (27, 2, 64, 15),
                                                     (13, 2, 128, 0), (17, 3, 128, 0)])
def test_tiled_half_state_against_full_state(n, p, precision, tile_bits):
    """Half-state plans (only qubit n-1 = 0 stored; the tile holding qubit
    n-1 also covers the complemented tile, stored in reverse) against
    full-state plans on the same draws, in every launch shape.  n = 15 with
    14-qubit tiles, 16 with 15-qubit tiles (complex64) and 13 (complex128)
    have a single tile per pass; n = 27 has three 14-qubit tiles per layer,
    or two 15-qubit tiles with 64-byte runs."""
    stn = stn_mod()
    pr = qaoa(n, p, 700 + n, 2e-2, 1e-1, 10)
    res = {}
    variants = (0, 1, 2) if tile_bits == 14 else (0,)
    for full in (True, False):
        pl = stn.Plan(pr, plan_kind=stn.PLAN_SV_TILED, full_state=full, max_batch=4, precision=precision,
                      tile_bits=tile_bits)
        info = pl.info()
        assert info["half_state"] == (0 if full else 1)
        assert info["tile_bits"] == (tile_bits or 12)
        for variant in variants:
            pl.set_variant(variant)
            b = pl.sample(pr.seed, 0, pr.K)
            pl.contract(b)
            res[(full, variant)] = b.energies()
            b.close()
        pl.close()
        torch.cuda.empty_cache()
    m = len(pr.edges)
    ref = res[(True, variants[-1])]
    for key, e in res.items():
        np.testing.assert_allclose(e / m, ref / m, atol=1e-5 if precision == 64 else 1e-12, err_msg=str(key))


def test_tiled_complex64_against_complex128_n22():
    """Same draws, n = 22: the complex64 passes (14- and 15-qubit tiles)
    against the complex128 twin."""
    stn = stn_mod()
    pr = qaoa(22, 3, 51, 1e-3, 1e-2, 64)
    res = {}
    for precision, tb in ((64, 14), (64, 15), (128, 0)):
        pl = stn.Plan(pr, plan_kind=stn.PLAN_SV_TILED, precision=precision, tile_bits=tb)
        b = pl.sample(pr.seed, 0, pr.K)
        pl.contract(b)
        res[tb] = b.energies()
    m = len(pr.edges)
    for tb in (14, 15):
        np.testing.assert_allclose(res[tb] / m, res[0] / m, atol=1e-5)
        assert np.abs(res[tb] - res[0]).max() > 0     # two different arithmetics


@pytest.mark.parametrize("n,p", [(30, 2), (18, 3), (28, 1)])
def test_tiled_tile_counts_complex64_against_complex128(n, p):
    """14-qubit tiles: 3 (n=28, 30) and 2 (n=18) per layer; 15-qubit tiles:
    3 (n=30) and 2 (n=18, 28; 32-byte runs at 28) per layer; merged layer
    boundaries: energies of the same draws against the complex128 passes
    (12-qubit tiles, another schedule)."""
    stn = stn_mod()
    pr = qaoa(n, p, 60 + n, 2e-3, 2e-2, 6)
    res = {}
    for precision, tile_bits in ((64, 14), (64, 15), (128, 0)):
        pl = stn.Plan(pr, plan_kind=stn.PLAN_SV_TILED, precision=precision, hbm_budget=64 << 30, tile_bits=tile_bits)
        b = pl.sample(pr.seed, 0, pr.K)
        pl.contract(b)
        res[tile_bits] = b.energies()
        b.close()
        pl.close()
        torch.cuda.empty_cache()
    m = len(pr.edges)
    np.testing.assert_allclose(res[14] / m, res[0] / m, atol=1e-5)
    np.testing.assert_allclose(res[15] / m, res[0] / m, atol=1e-5)


def test_lightcone_matches_tiled_statevector():
    stn = stn_mod()
    pr = qaoa(20, 2, 44, 0.01, 0.05, 32)
    res = {}
    for kind in (stn.PLAN_LIGHTCONE, stn.PLAN_SV_TILED):
        pl = stn.Plan(pr, plan_kind=kind)
        b = pl.sample(pr.seed, 0, pr.K)
        pl.contract(b)
        res[kind] = b.energies()
    np.testing.assert_allclose(res[stn.PLAN_LIGHTCONE] / len(pr.edges), res[stn.PLAN_SV_TILED] / len(pr.edges),
                               atol=2e-5)


@pytest.mark.parametrize("n,precision,tol", [(40, 64, 1e-5), (64, 128, 1e-10)])
def test_lightcone_noiseless_p1_closed_form_large_n(n, precision, tol):
    """n beyond any statevector: the noiseless p=1 energy against the closed
    form of Wang, Hadfield, Jiang and Rieffel (PRA 97, 022304)."""
    from test_oracle_density import closed_form_energy
    from workloads import make_problem, random_regular_graph
    stn = stn_mod()
    edges = random_regular_graph(n, 3, 500 + n)
    gamma, beta = 0.83, 2.41
    pr = make_problem(n, edges, [gamma], [beta], 0.0, 0.0, 4, 1)
    pl = stn.Plan(pr, precision=precision)
    assert pl.info()["plan_name"] == "lightcone"
    acc = pl.accum()
    b = pl.sample(pr.seed, 0, 4)
    pl.contract(b)
    pl.reduce(b, acc)
    r = acc.read()
    exact = closed_form_energy(n, pr.edges, gamma, beta)
    assert abs(r["energy_mean"] - exact) / len(pr.edges) < tol
    assert r["energy_se"] < 1e-9


# ----------------------------------------------------------------------------- full-size workload

@pytest.mark.parametrize("tile_bits,variant", [(15, 0), (14, 0), (14, 1), (14, 2)])
def test_full_size_workload_sampled_trajectories(tile_bits, variant):
    """n=26, p=4, K=4096 in the launch configurations the benchmark times
    (trajectories per launch from a 160 GiB budget; 15-qubit tiles, the
    default at this size, and each launch shape of the 14-qubit tiles):
    sampled trajectories against stored oracle values (complex128, literal
    Kraus insertion, same draws), plus properties that hold at any size."""
    import json
    from workloads import config_problem
    stn = stn_mod()
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "golden", "config2_sampled.json")) as f:
        gold = json.load(f)
    pr = config_problem(2)
    assert [list(e) for e in pr.edges] == gold["edges"]
    m = len(pr.edges)
    pl = stn.Plan(pr, outputs=stn.OUT_ENERGY, precision=64, hbm_budget=160 << 30, tile_bits=tile_bits)
    pl.set_variant(variant)
    info = pl.info()
    assert info["plan_name"] == "sv_tiled" and info["variant"] == variant and info["tile_bits"] == tile_bits
    B = info["max_batch"]
    acc = pl.accum()
    for k0 in range(0, pr.K, B):
        b = pl.sample(pr.seed, k0, min(B, pr.K - k0))
        pl.contract(b)
        pl.reduce(b, acc)
        b.close()
    r = acc.read()
    e = np.asarray(r["energies"])
    assert e.shape == (pr.K,)
    for row in gold["trajectories"]:
        assert abs(e[row["k"]] - row["energy"]) / m < 1e-5, row["k"]
    # any trajectory: 0 <= <C>_k <= m; the mean is the mean of the samples
    assert np.all(e >= -1e-4) and np.all(e <= m + 1e-4)
    assert abs(r["energy_mean"] - e.mean()) < 1e-9 * m
    assert abs(r["energy_se"] - e.std(ddof=1) / math.sqrt(pr.K)) < 1e-9 * m


# ----------------------------------------------------------------------------- launch shapes

@pytest.mark.parametrize("kind,n,p,precision", [("sv_lds", 10, 3, 64), ("sv_lds", 12, 2, 128),
                                                ("lightcone", 20, 1, 64), ("lightcone", 16, 1, 128),
                                                ("lightcone", 22, 2, 64), ("sv_tiled", 18, 2, 64)])
def test_launch_shapes_give_identical_results(kind, n, p, precision):
    """Every launch shape the autotuner may pick gives the same energies, bit
    for bit, and autotune keeps the fastest."""
    stn = stn_mod()
    kinds = {"sv_lds": stn.PLAN_SV_LDS, "lightcone": stn.PLAN_LIGHTCONE, "sv_tiled": stn.PLAN_SV_TILED}
    pr = qaoa(n, p, 700 + n, 5e-3, 2e-2, 96)
    pl = stn.Plan(pr, plan_kind=kinds[kind], precision=precision)
    b = pl.sample(pr.seed, 0, pr.K)
    tune = pl.autotune(b, reps=1)
    assert len(tune["ms"]) >= 2 and tune["chosen"] == int(np.argmin(tune["ms"]))
    assert pl.info()["variant"] == tune["chosen"] and pl.info()["tuned"] == 1
    ref = None
    for v in range(len(tune["ms"])):
        pl.set_variant(v)
        pl.contract(b)
        e = b.energies()
        if ref is None:
            ref = e
        np.testing.assert_array_equal(e, ref)
    with pytest.raises(stn.StnError, match="INVALID"):
        pl.set_variant(len(tune["ms"]))


# ----------------------------------------------------------------------------- multi-batch queue launch

@pytest.mark.parametrize("precision", [64, 128])
def test_contract_many_matches_per_batch(precision):
    """Batches of several whole-state-in-LDS plans (different n, depth,
    noise, outputs and K, one of them with amplitude damping) contracted by
    one launch that drains a device-side queue of (batch, trajectory) items,
    against each batch contracted alone: energies and states bit for bit, for
    two launch shapes and a repeated launch."""
    from workloads import config_problem
    stn = stn_mod()
    probs = [qaoa(n, p, 850 + n, lam, 2 * lam, K) for n, p, K, lam in
             [(6, 1, 5, 1e-2), (8, 2, 40, 5e-3), (10, 3, 200, 2e-3), (12, 2, 77, 1e-2), (4, 1, 1, 0.1)]]
    probs.append(config_problem(1, K=64))
    outs = [stn.OUT_ENERGY] * 3 + [stn.OUT_ENERGY | stn.OUT_RHO] + [stn.OUT_ENERGY] + [stn.OUT_ENERGY | stn.OUT_RHO]
    want = []
    for pr, o in zip(probs, outs):
        pl = stn.Plan(pr, plan_kind=stn.PLAN_SV_LDS, outputs=o, precision=precision)
        b = pl.sample(pr.seed, 3, pr.K)
        pl.contract(b)
        want.append((b.energies(), b.states() if o & stn.OUT_RHO else None))
        b.close()
        pl.close()
    plans = [stn.Plan(pr, plan_kind=stn.PLAN_SV_LDS, outputs=o, precision=precision) for pr, o in zip(probs, outs)]
    batches = [pl.sample(pr.seed, 3, pr.K) for pl, pr in zip(plans, probs)]
    for variant in (0, 2, 2):
        plans[0].set_variant(variant)
        stn.contract_many(plans, batches)
        for i, (b, (e, st)) in enumerate(zip(batches, want)):
            np.testing.assert_array_equal(b.energies(), e, err_msg=str(i))
            if st is not None:
                np.testing.assert_array_equal(b.states(), st, err_msg=str(i))
    # one batch alone through the queue
    stn.contract_many(plans[2:3], batches[2:3])
    np.testing.assert_array_equal(batches[2].energies(), want[2][0])
    other = 64 if precision == 128 else 128
    mixed = stn.Plan(probs[1], plan_kind=stn.PLAN_SV_LDS, precision=other)
    mb = mixed.sample(probs[1].seed, 0, 4)
    with pytest.raises(stn.StnError, match="INVALID"):
        stn.contract_many([plans[0], mixed], [batches[0], mb])
    with pytest.raises(stn.StnError, match="INVALID"):
        stn.contract_many([plans[0], plans[0]], [batches[0], batches[0]])
    tiled = stn.Plan(qaoa(16, 1, 870, 1e-3, 1e-2, 4), plan_kind=stn.PLAN_SV_TILED, precision=precision)
    tb = tiled.sample(870, 0, 4)
    with pytest.raises(stn.StnError, match="UNSUPPORTED"):
        stn.contract_many([plans[0], tiled], [batches[0], tb])
    for b in batches + [mb, tb]:
        b.close()


# ----------------------------------------------------------------------------- de-duplicated contraction

@pytest.mark.parametrize("kind,n,p,precision,lam", [("sv_tiled", 18, 2, 64, (1e-3, 5e-3)),
                                                    ("sv_tiled", 16, 2, 128, (2e-3, 1e-2)),
                                                    ("lightcone", 20, 1, 64, (1e-3, 1e-2)),
                                                    ("sv_lds", 10, 2, 128, (1e-3, 1e-2)),
                                                    ("sv_gates", 14, 2, 64, (1e-3, 5e-3))])
def test_dedup_contraction_matches_plain(kind, n, p, precision, lam):
    """Each distinct trajectory contracted once, its energy copied to the
    equal ones: the same energies as contracting every trajectory, bit for
    bit; the distinct count is at most the number of distinct Kraus-index
    rows (different Pauli errors can leave the same signs and frame).  The
    gate-by-gate case carries amplitude damping (no Pauli frame), so its
    trajectories are keyed by their Kraus-index rows."""
    stn = stn_mod()
    kinds = {"sv_lds": stn.PLAN_SV_LDS, "lightcone": stn.PLAN_LIGHTCONE, "sv_tiled": stn.PLAN_SV_TILED,
             "sv_gates": stn.PLAN_SV_GATES}
    if kind == "sv_gates":
        from workloads import make_problem, random_regular_graph, uniform_angles
        g, b = uniform_angles(p, 880 + n)
        pr = make_problem(n, random_regular_graph(n, 3, 881 + n), g, b, lam[0], lam[1], 300, 882 + n,
                          gamma_ad=0.002)
    else:
        pr = qaoa(n, p, 880 + n, lam[0], lam[1], 300)
    pl = stn.Plan(pr, plan_kind=kinds[kind], precision=precision)
    for k0 in (0, 300):
        b = pl.sample(pr.seed, k0, pr.K)
        pl.contract(b)
        want = b.energies()
        rows = len({r.tobytes() for r in b.indices()})
        b.close()
        b2 = pl.sample(pr.seed, k0, pr.K) if k0 == 0 else pl.resample(b2, pr.seed, k0, pr.K)
        u = pl.contract_dedup(b2)
        np.testing.assert_array_equal(b2.energies(), want)
        assert 1 <= u <= rows < pr.K
        if kind in ("sv_lds", "sv_gates"):
            assert u == rows
    b2.close()


# ----------------------------------------------------------------------------- contraction graphs

@pytest.mark.parametrize("kind,n,p,precision", [("sv_lds", 10, 2, 64), ("sv_lds", 12, 2, 128),
                                                ("sv_tiled", 18, 2, 64), ("sv_tiled", 16, 2, 128), ("sv_tiled15", 20, 2, 64),
                                                ("lightcone", 20, 1, 64), ("lightcone", 22, 2, 64)])
def test_contraction_graph_replays_match_eager(kind, n, p, precision):
    """One batch refilled chunk after chunk and contracted through a HIP
    graph (eager, captured, then replayed) against a plan launching eagerly,
    bit for bit, with unrelated eager work and synchronisation between the
    replays; then a change of K and of launch shape, which start over."""
    stn = stn_mod()
    kinds = {"sv_lds": stn.PLAN_SV_LDS, "lightcone": stn.PLAN_LIGHTCONE, "sv_tiled": stn.PLAN_SV_TILED,
             "sv_tiled15": stn.PLAN_SV_TILED}
    tb = 15 if kind == "sv_tiled15" else 0
    pr = qaoa(n, p, 800 + n, 5e-3, 2e-2, 96)
    ref = stn.Plan(pr, plan_kind=kinds[kind], precision=precision, tile_bits=tb)
    pl = stn.Plan(pr, plan_kind=kinds[kind], precision=precision, tile_bits=tb)
    pl.set_graphs(True)
    stream = torch.cuda.Stream()
    K, chunks = 48, 6

    def check(b, k0, K):
        got = b.energies()
        rb = ref.sample(pr.seed, k0, K)
        ref.contract(rb)
        want = rb.energies()
        rb.close()
        np.testing.assert_array_equal(got, want)

    with torch.cuda.stream(stream):
        b = pl.sample(pr.seed, 0, K)
        for c in range(chunks):
            if c:
                pl.resample(b, pr.seed, c * K, K)
            pl.contract(b)
            check(b, c * K, K)
            x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
            assert float((x * 2).sum().item()) == float(2 * sum(range(1 << 20)))
        info = pl.info()
        assert info["graphs"] == 1 and info["graph_captures"] == 1 and info["graph_replays"] == chunks - 2
        # a different K: eager, captured, replayed again
        for c in range(3):
            pl.resample(b, pr.seed, 1000 + c * 17, 17)
            pl.contract(b)
            check(b, 1000 + c * 17, 17)
        info = pl.info()
        assert info["graph_captures"] == 2 and info["graph_replays"] == chunks - 1
        if not kind.startswith("sv_tiled") or pl.info()["tile_bits"] == 14:
            pl.set_variant(1)
            for c in range(3):
                pl.resample(b, pr.seed, 2000 + c * 17, 17)
                pl.contract(b)
                check(b, 2000 + c * 17, 17)
            assert pl.info()["graph_captures"] == 3
        b.close()
    # the NULL stream never captures
    pl2 = stn.Plan(pr, plan_kind=kinds[kind], precision=precision, tile_bits=tb)
    pl2.set_graphs(True)
    b2 = pl2.sample(pr.seed, 0, K, stream=ctypes.c_void_p(0))
    for c in range(3):
        pl2.contract(b2, stream=ctypes.c_void_p(0))
    assert pl2.info()["graph_captures"] == 0
    check(b2, 0, K)
    b2.close()


# ----------------------------------------------------------------------------- sliced lightcone networks

@pytest.mark.parametrize("precision,tol", [(64, 1e-5), (128, 1e-11)])
def test_lightcone_slicing_against_oracle_and_unsliced(precision, tol):
    """Networks of width 20 sliced down to steps of rank 16 (intermediates in
    HBM) and 12 (whole arena in LDS): per-trajectory energies against literal
    Kraus insertion and against the unsliced networks."""
    from oracle import simulate as sim
    stn = stn_mod()
    pr = qaoa(14, 3, 903, 5e-3, 2e-2, 6)
    ens = sim.ensemble(pr, pr.seed, 0, pr.K, want_states=False)
    m = len(pr.edges)
    ref = None
    for kw in [dict(), dict(lc_max_rank=16, lc_slice_bits=6), dict(lc_max_rank=12, lc_slice_bits=10)]:
        pl = stn.Plan(pr, plan_kind=stn.PLAN_LIGHTCONE, precision=precision, **kw)
        info = pl.info()
        if kw:
            assert info["lc_slice_bits"] > 0 and info["lc_slices"] > len(pr.edges)
            assert info["width"] <= kw["lc_max_rank"] + 1
        else:
            assert info["width"] == 20 and info["lc_slices"] == len(pr.edges)
        b = pl.sample(pr.seed, 0, pr.K)
        pl.contract(b)
        got = b.energies()
        b.close()
        np.testing.assert_allclose(got / m, ens["energies"] / m, atol=tol)
        if ref is None:
            ref = got
        else:
            np.testing.assert_allclose(got / m, ref / m, atol=tol)


# ----------------------------------------------------------------------------- lightcone networks in HBM

@pytest.mark.parametrize("precision,tol", [(64, 1e-5), (128, 1e-11)])
def test_lightcone_hbm_tier_against_oracle(precision, tol):
    """Networks of width 20 (intermediates in global-memory arenas of
    persistent workgroups) against literal Kraus insertion."""
    from oracle import simulate as sim
    stn = stn_mod()
    pr = qaoa(14, 3, 903, 5e-3, 2e-2, 6)
    pl = stn.Plan(pr, plan_kind=stn.PLAN_LIGHTCONE, precision=precision)
    assert pl.info()["width"] == 20
    b = pl.sample(pr.seed, 0, pr.K)
    pl.contract(b)
    got = b.energies()
    ens = sim.ensemble(pr, pr.seed, 0, pr.K, want_states=False)
    m = len(pr.edges)
    np.testing.assert_allclose(got / m, ens["energies"] / m, atol=tol)


@pytest.mark.parametrize("n,seed,precision,tol", [(22, 904, 64, 2e-5), (22, 904, 128, 1e-11), (24, 907, 64, 2e-5)])
def test_lightcone_hbm_tier_against_statevector(n, seed, precision, tol):
    stn = stn_mod()
    pr = qaoa(n, 2, seed, 5e-3, 2e-2, 24)
    res = {}
    for kind in (stn.PLAN_LIGHTCONE, stn.PLAN_SV_TILED):
        pl = stn.Plan(pr, plan_kind=kind, precision=precision)
        if kind == stn.PLAN_LIGHTCONE:
            assert pl.info()["width"] >= 17
        b = pl.sample(pr.seed, 0, pr.K)
        pl.contract(b)
        res[kind] = b.energies()
        b.close()
        pl.close()
    m = len(pr.edges)
    np.testing.assert_allclose(res[stn.PLAN_LIGHTCONE] / m, res[stn.PLAN_SV_TILED] / m, atol=tol)


# ----------------------------------------------------------------------------- bitstrings from sigma_approx

@pytest.mark.parametrize("cfg,precision,dense", [(0, 128, "diag"), (1, 64, "rho")])
def test_bitstring_sampling_matches_oracle(cfg, precision, dense):
    """Bitstrings drawn from sigma_approx (Sec. III-G) by inverse transform,
    against the oracle's draws from its own sigma_approx with the same
    uniforms: equal index for index wherever u lies farther than the two
    sides' cumulative-sum difference from a boundary of the oracle's interval,
    and inside the widened interval otherwise.  Two reduced batches, 300001
    draws (more than one grid-stride round, a ragged tail), the end points of
    [0, 1), then m = 0 and m = 1."""
    import torch
    from oracle import simulate as sim
    from oracle.sampling import sample_bitstrings
    from workloads import config_problem
    stn = stn_mod()
    pr = config_problem(cfg)
    outs = (stn.OUT_DIAG | stn.OUT_ENERGY) if dense == "diag" else (stn.OUT_RHO | stn.OUT_DIAG)
    pl = stn.Plan(pr, outputs=outs, precision=precision)
    acc = pl.accum()
    half = pr.K // 2
    for k0, K in ((0, half), (half, pr.K - half)):
        b = pl.sample(pr.seed, k0, K)
        pl.contract(b)
        pl.reduce(b, acc)
        b.close()
    rng = np.random.default_rng(4100 + cfg)
    m = 300001
    u = rng.random(m)
    u[:4] = [0.0, np.nextafter(1.0, 0.0), 0.5, 1e-300]
    x = acc.sample(torch.from_numpy(u).cuda()).cpu().numpy().astype(np.int64)
    torch.cuda.synchronize()
    res = acc.read()
    ens = sim.ensemble(pr, pr.seed, 0, pr.K)
    sigma = ens["sigma_approx"]
    tol = 1e-12 if precision == 128 else 1e-5
    assert np.abs(res["diag"] - sigma).max() < tol
    xo = sample_bitstrings(sigma, u)
    N = 1 << pr.n_qubits
    assert x.min() >= 0 and x.max() < N
    Fo = np.cumsum(sigma) / sigma.sum()
    Fg = np.cumsum(res["diag"]) / res["diag"].sum()
    delta = 2 * np.abs(Fg - Fo).max() + 1e-15
    lo = np.where(xo > 0, Fo[np.maximum(xo - 1, 0)], 0.0)
    hi = Fo[xo]
    near = (np.abs(u - lo) < delta) | (np.abs(u - hi) < delta)
    assert (x[~near] == xo[~near]).all()
    xn = x[near]
    xl = np.where(xn > 0, Fo[np.maximum(xn - 1, 0)], 0.0)
    assert ((xl - delta <= u[near]) & (u[near] < Fo[xn] + delta)).all()
    assert near.mean() < 0.05
    # sample frequencies follow sigma_approx (chi-square over bins of expected count >= 20)
    p = sigma / sigma.sum()
    counts = np.bincount(x, minlength=N)
    big = p * m >= 20
    chi2 = float(((counts[big] - m * p[big]) ** 2 / (m * p[big])).sum())
    dof = int(big.sum())
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    # degenerate sizes
    empty = acc.sample(torch.empty(0, dtype=torch.float64, device="cuda"))
    assert empty.numel() == 0
    one = acc.sample(torch.tensor([0.5], dtype=torch.float64, device="cuda")).cpu().numpy()
    assert one[0] == x[2]
    acc.close()


# ----------------------------------------------------------------------------- caller-supplied contraction order

@pytest.mark.parametrize("precision,tol", [(128, 1e-11), (64, 1e-5)])
def test_caller_contraction_order_same_energies(precision, tol):
    """Lightcone networks contracted in caller-supplied orders (Sec. III-A/B:
    the order changes the cost, not the value): n=14 p=3 in the reversed
    variable numbering (width 15, below min-fill's 20, intermediates in HBM)
    against the full-statevector oracle, and n=20 p=2 in a minimum-degree
    order against the min-fill plan, same draws."""
    from oracle import simulate as sim
    from test_abi_host import min_degree_order
    from workloads import make_problem, random_regular_graph, uniform_angles
    stn = stn_mod()
    g, b = uniform_angles(3, 904)
    pr = make_problem(14, random_regular_graph(14, 3, 903), g, b, 5e-3, 2e-2, 6, 905)
    pl = stn.Plan(pr, plan_kind=stn.PLAN_LIGHTCONE, precision=precision,
                  lc_order=lambda net: range(net["n_vars"] - 1, -1, -1))
    assert pl.info()["width"] == 15
    bt = pl.sample(pr.seed, 0, pr.K)
    pl.contract(bt)
    got = bt.energies()
    ens = sim.ensemble(pr, pr.seed, 0, pr.K, want_states=False)
    m = len(pr.edges)
    np.testing.assert_allclose(got / m, ens["energies"] / m, atol=tol)
    g, b = uniform_angles(2, 5)
    pr2 = make_problem(20, random_regular_graph(20, 3, 11), g, b, 1e-3, 1e-2, 48, 6)
    res = []
    for order in (None, min_degree_order):
        pl2 = stn.Plan(pr2, plan_kind=stn.PLAN_LIGHTCONE, precision=precision, lc_order=order)
        bt = pl2.sample(pr2.seed, 0, pr2.K)
        pl2.contract(bt)
        res.append(bt.energies())
    m2 = len(pr2.edges)
    np.testing.assert_allclose(res[1] / m2, res[0] / m2, atol=tol)


# ----------------------------------------------------------------------------- gate-by-gate HBM statevector

@pytest.mark.parametrize("precision,tol", [(128, 1e-11), (64, 1e-5)])
def test_gate_by_gate_amplitude_damping_against_oracle(precision, tol):
    """<C> with amplitude damping above the whole-state-in-LDS size (n=14,
    p=2, depolarizing + amplitude damping per layer: no Pauli frame, so
    neither the tiled nor the lightcone lowering applies) against the
    oracle's literal-Kraus statevectors, same draws; a second batch at
    k0 = 5 with a ragged size."""
    from oracle import simulate as sim
    from workloads import make_problem, random_regular_graph, uniform_angles
    stn = stn_mod()
    g, b = uniform_angles(2, 31)
    pr = make_problem(14, random_regular_graph(14, 3, 32), g, b, 2e-3, 2e-2, 12, 33, gamma_ad=0.05)
    pl = stn.Plan(pr, precision=precision)
    assert pl.info()["plan_name"] == "sv_gates"
    m = len(pr.edges)
    for k0, K in ((0, 12), (5, 7)):
        bt = pl.sample(pr.seed, k0, K)
        pl.contract(bt)
        got = bt.energies()
        ens = sim.ensemble(pr, pr.seed, k0, K, want_states=False)
        np.testing.assert_allclose(got / m, ens["energies"] / m, atol=tol)
        bt.close()


@pytest.mark.parametrize("precision,tol", [(128, 1e-11), (64, 1e-5)])
def test_gate_by_gate_random_circuits_against_oracle(precision, tol):
    """Random circuits of every gate kind (h, x, y, z, rx, ry, rz, u1, zz, cx,
    u2) with every channel kind (bit flip, depolarizing, amplitude damping,
    explicit Kraus sets on one and two qubits), n = 2..8, in the gate-by-gate
    lowering against the oracle, same draws.  Error per unit weight and per
    unit squared norm of the trajectory: an inserted K_j/sqrt(q_j) of a
    non-unitary channel scales the trajectory, and its energy and rounding
    error with it (Pauli-noise trajectories have norm 1)."""
    from oracle import simulate as sim
    from random_circuits import random_problem
    stn = stn_mod()
    done, worst = 0, 0.0
    for seed in range(40):
        pr = random_problem(seed)
        if pr.n_qubits < 2 or not pr.edges:
            continue
        pl = stn.Plan(pr, plan_kind=stn.PLAN_SV_GATES, precision=precision)
        bt = pl.sample(pr.seed, 0, pr.K)
        pl.contract(bt)
        got = bt.energies()
        ens = sim.ensemble(pr, pr.seed, 0, pr.K, want_states=True)
        norm2 = np.maximum(1.0, (np.abs(ens["psi"]) ** 2).sum(axis=1))
        scale = max(1.0, float(np.sum(pr.weights))) * norm2
        err = np.abs(got - ens["energies"]) / scale
        worst = max(worst, float(err.max()))
        assert err.max() <= tol, f"seed {seed}: {err.max():.3e}"
        done += 1
    print(f"gate-by-gate random circuits, precision {precision}: {done} circuits, "
          f"max error per unit weight and squared norm {worst:.3e}")
    assert done >= 20


def test_gate_by_gate_matches_tiled_and_lds():
    """The same trajectories in other lowerings: n=20 Pauli noise against the
    tiled passes (complex64), n=10 against the whole-state-in-LDS kernel
    (complex128)."""
    stn = stn_mod()
    pr = qaoa(20, 2, 44, 0.01, 0.05, 24)
    res = {}
    for kind in (stn.PLAN_SV_GATES, stn.PLAN_SV_TILED):
        pl = stn.Plan(pr, plan_kind=kind)
        bt = pl.sample(pr.seed, 0, pr.K)
        pl.contract(bt)
        res[kind] = bt.energies()
    m = len(pr.edges)
    np.testing.assert_allclose(res[stn.PLAN_SV_GATES] / m, res[stn.PLAN_SV_TILED] / m, atol=2e-5)
    pr = qaoa(10, 3, 45, 0.01, 0.05, 32)
    res = {}
    for kind in (stn.PLAN_SV_GATES, stn.PLAN_SV_LDS):
        pl = stn.Plan(pr, plan_kind=kind, precision=128)
        bt = pl.sample(pr.seed, 0, pr.K)
        pl.contract(bt)
        res[kind] = bt.energies()
    m = len(pr.edges)
    np.testing.assert_allclose(res[stn.PLAN_SV_GATES] / m, res[stn.PLAN_SV_LDS] / m, atol=1e-12)


def test_gate_by_gate_large_state_matches_tiled():
    """n=24 (2^23 pairs per trajectory: the chunk cap is reached and every
    workgroup loops), K=8: the gate-by-gate lowering against the tiled
    passes on the same trajectories."""
    stn = stn_mod()
    pr = qaoa(24, 1, 46, 0.01, 0.05, 8)
    res = {}
    for kind in (stn.PLAN_SV_GATES, stn.PLAN_SV_TILED):
        pl = stn.Plan(pr, plan_kind=kind)
        bt = pl.sample(pr.seed, 0, pr.K)
        pl.contract(bt)
        res[kind] = bt.energies()
        bt.close()
    m = len(pr.edges)
    np.testing.assert_allclose(res[stn.PLAN_SV_GATES] / m, res[stn.PLAN_SV_TILED] / m, atol=2e-5)


def check_bitstrings(x, u, sigma, diag):
    """Draws x (from the library, with uniforms u) against the oracle's draws
    from its own sigma: equal wherever u lies farther than the two sides'
    cumulative-sum difference from a boundary of the oracle's interval, and
    inside the widened interval otherwise."""
    from oracle.sampling import sample_bitstrings
    xo = sample_bitstrings(sigma, u)
    assert x.min() >= 0 and x.max() < len(sigma)
    Fo = np.cumsum(sigma) / sigma.sum()
    Fg = np.cumsum(diag) / diag.sum()
    delta = 2 * np.abs(Fg - Fo).max() + 1e-15
    lo = np.where(xo > 0, Fo[np.maximum(xo - 1, 0)], 0.0)
    near = (np.abs(u - lo) < delta) | (np.abs(u - Fo[xo]) < delta)
    assert (x[~near] == xo[~near]).all()
    xn = x[near]
    xl = np.where(xn > 0, Fo[np.maximum(xn - 1, 0)], 0.0)
    assert ((xl - delta <= u[near]) & (u[near] < Fo[xn] + delta)).all()
    assert near.mean() < 0.05


@pytest.mark.parametrize("precision,tol", [(128, 1e-11), (64, 1e-5)])
def test_gate_by_gate_sigma_and_bitstrings_against_oracle(precision, tol):
    """sigma_approx above the whole-state-in-LDS size (n=14, amplitude
    damping: the gate-by-gate lowering keeps it) against the oracle, over two
    reduced batches; bitstrings drawn from it (running sums searched in
    device memory: 2^14 states) against the oracle's sampler."""
    import torch
    from oracle import simulate as sim
    from workloads import make_problem, random_regular_graph, uniform_angles
    stn = stn_mod()
    g, b = uniform_angles(2, 31)
    pr = make_problem(14, random_regular_graph(14, 3, 32), g, b, 2e-3, 2e-2, 12, 33, gamma_ad=0.05)
    pl = stn.Plan(pr, outputs=stn.OUT_DIAG | stn.OUT_ENERGY, precision=precision)
    assert pl.info()["plan_name"] == "sv_gates"
    acc = pl.accum()
    for k0, K in ((0, 7), (7, 5)):
        bt = pl.sample(pr.seed, k0, K)
        pl.contract(bt)
        pl.reduce(bt, acc)
        bt.close()
    ens = sim.ensemble(pr, pr.seed, 0, pr.K)
    sigma = ens["sigma_approx"]
    rng = np.random.default_rng(4200)
    u = rng.random(200001)
    u[:3] = [0.0, np.nextafter(1.0, 0.0), 0.5]
    x = acc.sample(torch.from_numpy(u).cuda()).cpu().numpy().astype(np.int64)
    torch.cuda.synchronize()
    res = acc.read()
    assert np.abs(res["diag"] - sigma).max() < tol * sigma.max()
    m = len(pr.edges)
    assert abs(res["energy_mean"] - ens["energies"].mean()) / m < tol
    check_bitstrings(x, u, sigma, res["diag"])
    acc.close()


@pytest.mark.timeout(900)
def test_rho_hat_converges_to_exact_density_matrix_n12():
    """n=12, p=2 with amplitude damping (the rho_hat workload): nested
    prefixes K = 16 .. 1024 of the GPU ensemble against the oracle's exact
    density matrix (Eq. (1)), estimate normalised by its trace.  At every K:
    Uhlmann fidelity (from the trajectories' states: the singular values of
    sqrt(rho) Psi / sqrt(K)), trace distance, Frobenius distance and the
    Eq. (2) error.  Frobenius falls about as K^(-1/2), the Eq. (2) error
    about as K^(-1) (Sec. IV), the fidelity rises and the trace distance
    falls.  The table is printed, and written as JSON when STN_RECORD_DIR is
    set."""
    import json
    from oracle import metrics, simulate as sim
    from workloads import config_problem
    stn = stn_mod()
    pr = config_problem(1)
    rho = sim.density_matrix(pr)
    N = rho.shape[0]
    w, V = np.linalg.eigh((rho + rho.conj().T) / 2)
    sqrt_rho = (V * np.sqrt(np.clip(w, 0.0, None))) @ V.conj().T
    pl = stn.Plan(pr, outputs=stn.OUT_RHO | stn.OUT_STATES, precision=64)
    edges = [0, 16, 32, 64, 128, 256, 512, 1024]
    acc_sum = np.zeros((N, N), dtype=np.complex128)
    proj = np.zeros((N, 0), dtype=np.complex128)     # sqrt(rho) Psi^T, columns in trajectory order
    rows = []
    for a, b in zip(edges[:-1], edges[1:]):
        acc = pl.accum()
        bt = pl.sample(pr.seed, a, b - a)
        pl.contract(bt)
        pl.reduce(bt, acc)
        r = acc.read()
        proj = np.concatenate([proj, sqrt_rho @ bt.states().T], axis=1)
        acc_sum += r["rho"] * r["k_done"]
        acc.close()
        bt.close()
        est = acc_sum / b
        tr = np.trace(est).real
        est = est / tr
        # F(rho, est) = (sum of singular values of sqrt(rho) Psi^T / sqrt(K))^2 / Tr(rho_hat)
        fid = float(np.sum(np.linalg.svd(proj / np.sqrt(b), compute_uv=False)) ** 2 / tr)
        rows.append(dict(K=b, uhlmann_F=fid, trace_distance=metrics.trace_distance(rho, est),
                         frobenius=metrics.frobenius(rho, est),
                         eq2_error=metrics.paper_error(np.diag(est).real, np.diag(rho).real), trace=tr))
        print("K=%(K)d F=%(uhlmann_F).4f TD=%(trace_distance).4f Frob=%(frobenius).4f Eq2=%(eq2_error).2e "
              "Tr=%(trace).6f" % rows[-1], flush=True)
    # the state-based fidelity equals the matrix definition on the final estimate; the matrix
    # form takes square roots of the rounding-level eigenvalues in the null space of the
    # rank-1024 estimate (about 3000 of them), which adds up to about 1e-5
    assert abs(rows[-1]["uhlmann_F"] - metrics.uhlmann_fidelity(rho, est)) < 1e-4
    if os.environ.get("STN_RECORD_DIR"):
        os.makedirs(os.environ["STN_RECORD_DIR"], exist_ok=True)
        with open(os.path.join(os.environ["STN_RECORD_DIR"], "rho_hat_sweep_n12.json"), "w") as f:
            json.dump(dict(workload="qaoa-n12-p2-3reg-ad-K1024", rows=rows), f, indent=1)
    first, last = rows[0], rows[-1]
    assert last["frobenius"] < first["frobenius"] / 4          # 64x the trajectories: about 8x smaller
    assert last["eq2_error"] < first["eq2_error"] / 16         # about 64x smaller
    assert last["trace_distance"] < first["trace_distance"]
    assert last["uhlmann_F"] > first["uhlmann_F"]
    # the trends hold across the sweep, not only at its ends (stochastic, so over doublings of 4x)
    for lo, hi in zip(rows[:-2], rows[2:]):
        assert hi["frobenius"] < lo["frobenius"]
        assert hi["uhlmann_F"] > lo["uhlmann_F"] - 0.02
