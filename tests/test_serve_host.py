"""Host-side logic of the serving loop (CPU only): the request generator and the
slot / HBM-budget admission accounting."""

import numpy as np
import pytest

from paper_2302_04741_amd import serve


def test_request_stream_matches_the_serving_recipe():
    reqs = serve.make_requests(n=256)
    assert len(reqs) == 256
    t = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 20.0) < 0.01  # Poisson at 20/s
    L = np.array([r.workload.dims[0] for r in reqs])
    assert L.min() >= 64 and L.max() <= 1024
    assert all(r.workload.dims[0] == r.workload.dims[1] for r in reqs)
    for r in reqs:
        wl = r.workload
        g = np.asarray(wl.force[1])
        assert 1e-6 <= np.hypot(*g) <= 1e-4
        assert 0.55 <= wl.tau_hat <= 1.0 and r.steps == 2000
    # the stream is reproducible from its seed
    again = serve.make_requests(n=256)
    assert [r.arrival for r in again] == [r.arrival for r in reqs]


def test_admission_by_slots_and_budget():
    a = serve.Admission(max_slots=3, budget_bytes=100)
    assert a.fits(60)
    a.take(60)
    assert not a.fits(50)  # budget
    assert a.fits(40)
    a.take(40)
    a.release(60)
    assert a.used == 40 and a.slots == 1
    a.take(10)
    a.take(10)
    assert not a.fits(1)  # slots
    with pytest.raises(AssertionError):
        a.take(1)


def test_request_bytes_is_the_workspace_of_the_handle():
    from paper_2302_04741_amd import _lib, workloads

    r = serve.make_requests(n=1, seed=2)[0]
    p = _lib.make_params(r.workload.lattice, r.workload.dims, r.workload.tau_hat, "f32")
    assert serve.request_bytes(r, "f32") == _lib.workspace_bytes(p) + 256
    # a full force field and plates need more workspace, and are budgeted for
    wl = workloads.random_smooth("D2Q37", (64, 40, 1), seed=1, force_kind="field")
    wl.walls = (1.0, 1.1, 0.0, 0.0)
    big = serve.Request(0, 0.0, wl, 10)
    pf = _lib.make_params("D2Q37", (64, 40, 1), wl.tau_hat, "f32", force_field=True, walls=True)
    assert serve.request_bytes(big, "f32") == _lib.workspace_bytes(pf) + 256
