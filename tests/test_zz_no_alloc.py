"""stn_accum_sample_noalloc: the bitstring sampler with its running sums in
the library's fixed device buffer (for callers that cannot allocate) against
stn_accum_sample, which keeps them in memory its accumulator allocates.  The
draws are integer indices, so the two must agree exactly, on two calls in a
row (the second on a smaller plan with fewer draws, so the buffer still holds
the first call's larger contents), with no device allocation by the call."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def reduced_accum(stn, cfg, outputs):
    from workloads import config_problem
    pr = config_problem(cfg)
    pl = stn.Plan(pr, outputs=outputs, precision=64)
    acc = pl.accum()
    half = pr.K // 2
    for k0, K in ((0, half), (half, pr.K - half)):
        b = pl.sample(pr.seed, k0, K)
        pl.contract(b)
        pl.reduce(b, acc)
        b.close()
    return pl, acc


def allocations():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.memory_stats().get("allocation.all.allocated", 0)


def test_noalloc_sampler_matches_allocating_sampler():
    import torch
    import paper_2210_15874_amd as stn
    torch.cuda.set_device(0)
    rng = np.random.default_rng(4242)
    # first call: n = 12 (running sums in two chunks), 300001 draws
    # second call: n = 6 (one partial chunk), 1001 draws
    for cfg, outputs, m in ((1, stn.OUT_RHO | stn.OUT_DIAG, 300001), (0, stn.OUT_DIAG | stn.OUT_ENERGY, 1001)):
        pl, acc = reduced_accum(stn, cfg, outputs)
        u_h = rng.random(m)
        u_h[:3] = [0.0, np.nextafter(1.0, 0.0), 0.5]
        u = torch.from_numpy(u_h).cuda()
        ref = acc.sample(u).cpu().numpy()
        out = torch.full((m,), -1, dtype=torch.int32, device="cuda")
        before = allocations()
        got = acc.sample(u, out=out, no_alloc=True)
        after = allocations()
        assert after == before, (before, after)
        got = got.cpu().numpy()
        print(f"n={pl.n} m={m}: {int((got == ref).sum())} of {m} draws equal")
        assert got.min() >= 0 and got.max() < (1 << pl.n)
        np.testing.assert_array_equal(got, ref)
        # m = 0 does nothing
        empty = torch.empty(0, dtype=torch.float64, device="cuda")
        assert acc.sample(empty, no_alloc=True).numel() == 0
        acc.close()
        pl.close()


def test_noalloc_sampler_rejects_plans_above_its_buffer():
    """n = 21 needs 2^21 running sums, more than the fixed buffer holds: the
    call fails on the host with UNSUPPORTED before any kernel runs."""
    import torch
    import paper_2210_15874_amd as stn
    from workloads import Gate, Problem
    torch.cuda.set_device(0)
    n = 21
    pr = Problem(n, [Gate("h", (q,)) for q in range(n)], [], [(0, 1)], [1.0])
    pl = stn.Plan(pr, outputs=stn.OUT_DIAG, precision=64, plan_kind=stn.PLAN_SV_GATES)
    acc = pl.accum()
    u = torch.full((4,), 0.5, dtype=torch.float64, device="cuda")
    with pytest.raises(stn.StnError, match="UNSUPPORTED"):
        acc.sample(u, no_alloc=True)
    acc.close()
    pl.close()
