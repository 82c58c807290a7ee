"""The continuous-batching server on a small request stream (GPU).

* every request completes; admission never exceeds the slots or the HBM budget
  (the budget is set tight, so requests queue for memory);
* each request's final populations are bitwise the same when it is served
  alone and when it is served in the mix;
* a request whose initial state is not finite fails alone, the others finish;
* p50/p99 latency and aggregate MLUPS are reported.
"""
import pytest

from paper_2302_04741_amd import serve

pytestmark = pytest.mark.gpu


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
