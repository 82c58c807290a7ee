"""The continuous-batching server on a small request stream (GPU).

* every request completes; admission never exceeds the slots or the HBM budget
  (the budget is set tight, so requests queue for memory);
* each request's final populations are bitwise the same when it is served
  alone and when it is served in the mix;
* served FP64 results match the CPU oracle (1e-12 on rho, u, theta) for a
  stream in which members join and leave mid-run at uneven step counts, so
  members at different buffer parities share launches;
* served FP32 results agree with the plain single-grid kernel run alone to a
  few units of the storage precision;
* a request whose initial state is not finite fails alone, the others finish;
* p50/p99 latency and aggregate MLUPS are reported.
"""
import pytest
import torch

from _parity import gpu_moments, oracle_run, rel_err
from paper_2302_04741_amd import serve

pytestmark = pytest.mark.gpu


def restored(wl, pops, storage, steps):
    """A handle holding a served request's final state (for its moments)."""
    from paper_2302_04741_amd import sim

    s = sim.from_workload(wl, storage=storage)
    s.set_populations(pops.to("cuda"))
    s.step_count = steps
    return s


def small_stream(n=20, seed=11):
    return serve.make_requests(n=n, rate=200.0, seed=seed, steps=120, lmin=16, lmax=160)


def test_mix_equals_alone_bitwise_and_budget_respected():
    reqs = small_stream()
    keep = {2, 7, 13}
    budget = 3 * max(serve.request_bytes(r, "f32") for r in reqs)
    srv = serve.Server(storage="f32", max_slots=6, budget_bytes=budget, chunk_steps=25,
                       keep_populations=lambda rid: rid in keep)
    out = srv.run(reqs, realtime=True)
    assert out["requests"] == len(reqs) and out["failed"] == 0
    assert out["max_concurrent"] <= 6
    assert srv.adm.used == 0 and srv.adm.slots == 0
    mixed = {r.rid: r.populations for r in out["results"] if r.rid in keep}
    print("p50 %.3f s p99 %.3f s aggregate %.0f MLUPS, max concurrent %d"
          % (out["p50_latency_s"], out["p99_latency_s"], out["aggregate_mlups"],
             out["max_concurrent"]), flush=True)
    for r in reqs:
        if r.rid not in keep:
            continue
        alone = serve.Server(storage="f32", max_slots=1, budget_bytes=budget, chunk_steps=25,
                             keep_populations=lambda rid: True).run([r], realtime=False)
        ref = alone["results"][0].populations
        assert ref.numel() == mixed[r.rid].numel()
        assert bool((ref == mixed[r.rid]).all()), r.rid


def test_failed_request_does_not_disturb_others():
    reqs = small_stream(n=8, seed=5)
    bad = reqs[3]
    theta = bad.workload.theta.copy()
    theta[0] = float("nan")
    bad.workload.theta = theta
    out = serve.Server(storage="f32", max_slots=8, chunk_steps=40, check_every=1).run(
        reqs, realtime=False)
    status = {r.rid: r.ok for r in out["results"]}
    assert status[bad.rid] is False
    assert all(ok for rid, ok in status.items() if rid != bad.rid)
    assert out["failed"] == 1


def test_served_fp64_matches_oracle_with_midrun_joins(oracle_mod):
    """FP64 stream with a budget for three members at a time: requests join as
    others finish, at chunk boundaries that fall at odd and even step counts,
    and leave at uneven lengths; every served result against the oracle."""
    reqs = serve.make_requests(n=10, rate=1000.0, seed=21, steps=200, lmin=16, lmax=64)
    for k, r in enumerate(reqs):
        r.steps = 150 + 13 * k
    budget = 3 * max(serve.request_bytes(r, "f64") for r in reqs)
    srv = serve.Server(storage="f64", max_slots=4, budget_bytes=budget, chunk_steps=25,
                       keep_populations=lambda rid: True)
    out = srv.run(reqs, realtime=False)
    assert out["requests"] == 10 and out["failed"] == 0
    assert out["max_concurrent"] <= 4 and srv.adm.used == 0
    res = {r.rid: r for r in out["results"]}
    assert sum(1 for r in res.values() if r.admitted_chunk > 0) >= 5  # joined mid-run
    worst = (0.0, 0.0, 0.0)
    for r in reqs:
        got = res[r.rid]
        assert got.steps == r.steps
        s = restored(r.workload, got.populations, "f64", r.steps)
        m = gpu_moments(s)
        s.close()
        o = oracle_run(oracle_mod, r.workload, r.steps)
        e = rel_err(m, o.moments())
        worst = tuple(max(a, b) for a, b in zip(worst, e))
        assert all(x <= 1e-12 for x in e), (r.rid, r.workload.dims, e)
    print("served FP64 vs oracle, worst rho %.1e u %.1e theta %.1e" % worst, flush=True)


def test_served_fp32_matches_plain_kernel():
    """Served FP32 populations against the same request stepped alone with
    the plain single-grid kernel: the same cell update inlined into two
    kernels, so at most a few units of FP32 rounding apart."""
    from paper_2302_04741_amd import sim

    reqs = small_stream(n=8, seed=3)
    srv = serve.Server(storage="f32", max_slots=3, chunk_steps=25,
                       keep_populations=lambda rid: True)
    out = srv.run(reqs, realtime=False)
    assert out["failed"] == 0
    worst = 0.0
    for got in out["results"]:
        r = reqs[[q.rid for q in reqs].index(got.rid)]
        p = sim.from_workload(r.workload, storage="f32")
        p.step(r.steps)
        ref = p.get_populations().cpu().view(torch.float32)
        d = (got.populations.view(torch.float32) - ref).abs().max().item()
        worst = max(worst, d)
        p.close()
        assert d <= 2e-6, (r.rid, d)
    print("served FP32 vs plain kernel: max stored-value difference %.1e" % worst, flush=True)
