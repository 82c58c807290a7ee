"""Plates (lbm_set_walls) on the GPU against the oracle's plates.

The channel flow of Sec. 3 runs between two plates; the wall condition is the
library's own design (the paper does not publish its own), implemented
independently in the oracle (push, per-column sums after a full collision
pass) and on the GPU (pull; a per-column density kernel, the fused step over
every row, then the rows next to the plates again with the plates' emission).
FP64 bar as in the periodic parity tests (1e-12; the deviation form against
the oracle's 80-bit build, the literal form against its binary64 build).
"""
import numpy as np
import pytest
import torch

from _parity import gpu_moments, oracle_run, rel_err, to_host
from paper_2302_04741_amd import workloads

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_SHORT = (2e-6, 5e-5, 2e-6)
TOL16_SHORT = (2e-4, 2e-3, 2e-4)


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2302_04741_amd import sim

    return sim


def channel(lat, dims, seed=1, walls=(0.9, 1.2, 0.02, -0.03), fo=4, mu=0.0, g_amp=2e-4,
            kind="uniform"):
    wl = workloads.random_smooth(lat, dims, seed=seed, force_kind=kind, g_amp=g_amp,
                                 force_order=fo, amp_u=0.03)
    wl.walls = walls
    wl.mu = mu
    return wl


def check(sim_mod, oracle_mod, wl, steps, storage="f64", rho0=None, prec="f64", tol=TOL64):
    s = sim_mod.from_workload(wl, storage=storage, rho0=rho0)
    s.step(steps)
    gpu = gpu_moments(s)
    ora = oracle_run(oracle_mod, wl, steps, prec=prec)
    errs = rel_err(gpu, ora.moments())
    print("%s walls=%s steps=%d storage=%s rho0=%s oracle=%s err rho %.2e u %.2e theta %.2e"
          % (wl.name, wl.walls, steps, storage, rho0, prec, *errs), flush=True)
    tols = tol if isinstance(tol, tuple) else (tol,) * 3
    assert all(e <= t for e, t in zip(errs, tols)), errs
    return s, ora


@pytest.mark.parametrize("lat,dims", [("D2Q37", (5, 24, 1)), ("D2Q37", (70, 9, 1)),
                                      ("D3Q39", (4, 16, 5))])
def test_parity_with_plates(sim_mod, oracle_mod, lat, dims):
    wl = channel(lat, dims)
    check(sim_mod, oracle_mod, wl, 200, rho0=0.0)
    check(sim_mod, oracle_mod, wl, 200, rho0=1.0, prec="ld")


@pytest.mark.parametrize("ny", [1, 2, 5, 6, 7])
def test_parity_narrow_channels(sim_mod, oracle_mod, ny):
    # every row touches a plate when ny <= 6; ny = 7 leaves one interior row
    wl = channel("D2Q37", (6, ny, 1), seed=ny)
    check(sim_mod, oracle_mod, wl, 60, rho0=0.0)


def test_parity_channel_of_the_paper_kind(sim_mod, oracle_mod):
    # per-cell tau = mu/(rho theta), plates at rest at different temperatures,
    # gravity along and across the channel, force orders 4 and 2
    for fo in (4, 2):
        wl = channel("D2Q37", (3, 40, 1), seed=3, walls=(0.8, 1.3, 0.0, 0.0), fo=fo, mu=0.15,
                     g_amp=1e-3)
        check(sim_mod, oracle_mod, wl, 300, rho0=0.0)


def test_initial_state_and_heat_flux(sim_mod, oracle_mod):
    wl = channel("D2Q37", (7, 12, 1), seed=5, kind="field")
    s = sim_mod.from_workload(wl)
    ora = oracle_run(oracle_mod, wl, 0)
    assert max(rel_err(gpu_moments(s), ora.moments())) < 1e-14
    s.step(20)
    ora.step(20)
    q, qo = to_host(s.heat_flux()), ora.heat_flux()
    assert np.abs(q - qo).max() / np.abs(qo).max() < 1e-11


@pytest.mark.parametrize("storage,tol", [("f32", TOL32_SHORT), ("f16dev", TOL16_SHORT)])
def test_reduced_storage_with_plates(sim_mod, oracle_mod, storage, tol):
    check(sim_mod, oracle_mod, channel("D2Q37", (70, 9, 1)), 25, storage=storage, tol=tol)
    check(sim_mod, oracle_mod, channel("D3Q39", (9, 7, 8)), 25, storage=storage, tol=tol)


def test_mass_conserved_with_plates(sim_mod):
    wl = channel("D2Q37", (16, 40, 1), seed=9, walls=(0.8, 1.3, 0.05, -0.05), g_amp=1e-3)
    s = sim_mod.from_workload(wl)
    m0 = s.totals()[0]
    s.step(500)
    assert abs(s.totals()[0] / m0 - 1) < 1e-13


def test_graph_replay_with_plates(sim_mod):
    wl = channel("D2Q37", (8, 20, 1), seed=2)
    stream = torch.cuda.Stream()
    ref = sim_mod.from_workload(wl, stream=stream)
    s = sim_mod.from_workload(wl, stream=stream)
    g = sim_mod.Graph(s, 4)
    for _ in range(3):
        g.launch(1)
        ref.step(4)
        assert torch.equal(s.get_populations(), ref.get_populations())


def test_plate_argument_checks(sim_mod):
    from paper_2302_04741_amd._lib import LbmError

    wl = channel("D2Q37", (4, 8, 1))
    plain = sim_mod.Sim(wl.lattice, wl.dims, wl.tau_hat, wl.rho, wl.u, wl.theta)
    with pytest.raises(LbmError):
        plain.set_walls(1.0, 1.0)  # no LBM_FLAG_WALLS
    s = sim_mod.Sim(wl.lattice, wl.dims, wl.tau_hat, wl.rho, wl.u, wl.theta, walls=True)
    with pytest.raises(LbmError):
        s.set_walls(-1.0, 1.0)
    s.set_walls(1.0, 1.1)
    b = sim_mod.Batch(2)
    with pytest.raises(LbmError):
        b.set([s])  # batches are periodic
    s.step(1)
    with pytest.raises(LbmError):
        s.set_walls(1.0, 1.0)  # after the first step


def test_restored_state_with_plates(sim_mod):
    """A state written from outside (lbm_set_populations) gets the plates' row sums
    of that state before the next step, on every path: direct steps, a graph
    captured before the restore, and the resident kernel.  They are recomputed by
    the column pass instead of taken from the producing step, so the runs agree
    with the uninterrupted one to rounding."""
    wl = channel("D2Q37", (8, 20, 1), seed=4, mu=0.1)
    stream = torch.cuda.Stream()
    a = sim_mod.from_workload(wl, stream=stream)
    a.step(37)
    snap = a.get_populations().clone()
    a.step(50)
    ref = gpu_moments(a)
    b = sim_mod.from_workload(wl, stream=stream)
    g = sim_mod.Graph(b, 10)  # captured on the initial state's buffer parity
    b.set_populations(snap)
    g.launch(5)
    c = sim_mod.from_workload(wl, stream=stream)
    c.set_populations(snap)
    c.step(50)
    d = sim_mod.from_workload(wl, stream=stream)
    d.set_resident_limit(1 << 40)
    d.set_populations(snap)
    d.step(50)
    for s in (b, c, d):
        errs = rel_err(gpu_moments(s), ref)
        assert max(errs) < 1e-13, errs
    g.close()
