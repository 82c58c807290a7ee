"""The resident kernel (small grids, many steps per launch in one workgroup).

Grids of at most lbm_set_resident_limit cells (default 0, off) step in one
workgroup that loops over the steps with a barrier between them; larger grids
take one launch per step.  Both are held to the oracle, and to
each other: the per-cell arithmetic is the same source compiled into two
kernels (the compiler may contract and schedule them differently), so they
agree to rounding: FP64 1e-13, FP32 and F16 storage at the tolerances of the
short parity runs.
"""
import numpy as np
import pytest
import torch

from _parity import gpu_moments, oracle_run, rel_err, to_host
from paper_2302_04741_amd import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
BIG = 1 << 40


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2302_04741_amd import sim

    return sim


def smooth(lat, dims, seed=3, fo=4, mu=0.0, walls=None, kind="uniform"):
    wl = workloads.random_smooth(lat, dims, seed=seed, force_kind=kind, g_amp=2e-4,
                                 force_order=fo, amp_u=0.03)
    wl.mu = mu
    wl.walls = walls
    return wl


def run(sim_mod, wl, steps, storage, limit, block=0, **kw):
    s = sim_mod.from_workload(wl, storage=storage, **kw)
    s.set_resident_limit(limit)
    if block:
        s.set_block(block)
    s.step(steps)
    return s


CASES = [
    ("D2Q37", (20, 24, 1), 0.0, None, "field"),
    ("D2Q37", (3, 5, 1), 0.0, None, "uniform"),     # 15 cells: one partial wavefront
    ("D2Q37", (3, 150, 1), 0.15, (0.7, 1.4, 0.0, 0.0), "uniform"),  # the channel
    ("D3Q39", (6, 8, 5), 0.0, None, "field"),
    ("D3Q39", (4, 16, 5), 0.05, (0.9, 1.2, 0.02, -0.03), "uniform"),
]


@pytest.mark.parametrize("lat,dims,mu,walls,kind", CASES)
def test_resident_against_oracle_fp64(sim_mod, oracle_mod, lat, dims, mu, walls, kind):
    wl = smooth(lat, dims, mu=mu, walls=walls, kind=kind)
    steps = 201
    ora = oracle_run(oracle_mod, wl, steps).moments()
    for limit in (BIG, 0):
        s = run(sim_mod, wl, steps, "f64", limit, rho0=0.0)
        errs = rel_err(gpu_moments(s), ora)
        print("%s %s mu=%g walls=%s resident=%s err rho %.2e u %.2e theta %.2e"
              % (lat, dims, mu, walls, limit > 0, *errs), flush=True)
        assert max(errs) <= TOL64, errs
        s.close()


# (bound on each path's error against the FP64 oracle, slack of the resident
# path over the per-step path); u is relative to max|u| (about 0.03)
@pytest.mark.parametrize("storage,tol", [("f64", (1e-12, 1e-13)), ("f32", (5e-5, 1e-6)),
                                         ("f16dev", (1e-2, 1e-4))])
@pytest.mark.parametrize("lat,dims,mu,walls,kind", CASES)
def test_resident_matches_per_step_kernel(sim_mod, oracle_mod, lat, dims, mu, walls, kind,
                                          storage, tol):
    """After an odd number of steps, with and without the resident kernel (every
    storage, with and without plates and per-cell tau): both near the oracle, the
    resident path no further from it than the per-step path (to a rounding-level
    slack), and FP64 within 1e-13 of each other."""
    wl = smooth(lat, dims, mu=mu, walls=walls, kind=kind)
    ora = oracle_run(oracle_mod, wl, 101).moments()
    a = run(sim_mod, wl, 101, storage, BIG)
    b = run(sim_mod, wl, 101, storage, 0)
    ma, mb = gpu_moments(a), gpu_moments(b)
    ea, eb, ab = rel_err(ma, ora), rel_err(mb, ora), rel_err(ma, mb)
    print("%s %s %s vs oracle: resident rho %.1e u %.1e theta %.1e, per-step rho %.1e u %.1e "
          "theta %.1e; between them %.1e %.1e %.1e" % (lat, dims, storage, *ea, *eb, *ab),
          flush=True)
    bound, slack = tol
    assert max(ea) <= bound and max(eb) <= bound, (ea, eb)
    assert all(x <= 1.5 * y + slack for x, y in zip(ea, eb)), (ea, eb)
    if storage == "f64":
        assert max(ab) <= 1e-13, ab
    a.close()
    b.close()


def test_resident_chunks_and_launch_shapes(sim_mod):
    """Runs longer than one launch's step cap, and every workgroup size, give
    bitwise the same populations (each cell's arithmetic does not depend on
    which lane computes it)."""
    wl = smooth("D2Q37", (20, 30, 1), mu=0.1)  # 600 cells: 1 to 10 per lane
    ref = to_host(run(sim_mod, wl, 4096 + 5, "f32", BIG).get_populations())
    split = run(sim_mod, wl, 1000, "f32", BIG)
    split.step(3096)
    split.step(5)
    assert np.array_equal(to_host(split.get_populations()), ref)
    for block in (64, 128, 256, 512):
        s = run(sim_mod, wl, 4096 + 5, "f32", BIG, block=block)
        assert np.array_equal(to_host(s.get_populations()), ref), block
    per_step = to_host(run(sim_mod, wl, 4096 + 5, "f64", 0).get_populations())
    res = to_host(run(sim_mod, wl, 4096 + 5, "f64", BIG).get_populations())
    d = np.abs(per_step.view(np.float64) - res.view(np.float64)).max()
    print("4101 steps FP64 resident vs per-step: max |dh| %.2e" % d, flush=True)
    assert d < 1e-13


def test_resident_graph_replays(sim_mod):
    """A captured loop over the resident kernel replays to the same state as
    direct calls, replay after replay, with eager work in between."""
    wl = smooth("D2Q37", (3, 150, 1), mu=0.15, walls=(0.7, 1.4, 0.0, 0.0))
    stream = torch.cuda.Stream()
    s = sim_mod.from_workload(wl, storage="f64", stream=stream)
    ref = sim_mod.from_workload(wl, storage="f64", stream=stream)
    s.set_resident_limit(BIG)
    ref.set_resident_limit(BIG)
    g = sim_mod.Graph(s, 50)
    for rep in range(4):
        g.launch(1)
        ref.step(50)
        _ = s.totals()
        stream.synchronize()
        assert np.array_equal(to_host(s.get_populations()), to_host(ref.get_populations())), rep
    g.close()
    # a changed limit invalidates the capture
    g = sim_mod.Graph(s, 2)
    s.set_resident_limit(0)
    with pytest.raises(Exception):
        g.launch(1)
    g.close()
    s.close()
    ref.close()


def test_limit_boundary(sim_mod):
    """A limit of 4096 cells: 4096 cells take the resident kernel, 4097 not (and
    by default neither does); all agree to rounding."""
    for dims in ((64, 64, 1), (17, 241, 1)):  # 4096 and 4097 cells
        wl = smooth("D2Q37", dims)
        a = run(sim_mod, wl, 11, "f64", 4096)
        b = run(sim_mod, wl, 11, "f64", 0)
        c = sim_mod.from_workload(wl, storage="f64")
        c.step(11)
        for m in (gpu_moments(b), gpu_moments(c)):
            errs = rel_err(gpu_moments(a), m)
            assert max(errs) < 1e-13, errs
