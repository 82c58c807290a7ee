"""Bitwise determinism, checkpoint/resume and launch-shape independence (GPU).

The step has no atomics and no cross-thread reductions, so every launch shape
must give the same bits, and exporting/importing the populations must resume a
run bitwise.  The totals use a fixed partition and order, so they repeat
bitwise too.
"""
import numpy as np
import pytest
import torch

from paper_2302_04741_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2302_04741_amd import sim

    return sim


@pytest.mark.parametrize("lat,dims,storage", [("D2Q37", (200, 9, 1), "f64"),
                                              ("D3Q39", (130, 6, 5), "f32"),
                                              ("D3Q39", (70, 9, 6), "f16dev")])
def test_block_shape_does_not_change_bits(sim_mod, lat, dims, storage):
    wl = workloads.random_smooth(lat, dims, seed=2, force_kind="axis", g_amp=1e-3)
    pops = []
    for block in (64, 128, 256, 1024):
        s = sim_mod.from_workload(wl, storage=storage)
        s.set_block(block)
        s.step(7)
        pops.append(s.get_populations().cpu())
        s.close()
    for p in pops[1:]:
        assert torch.equal(p, pops[0])


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_resume_from_checkpoint_is_bitwise(sim_mod, storage):
    """With F16 storage the step number keys the stochastic rounding:
    setting the step count restores it."""
    wl = workloads.random_smooth("D3Q39", (12, 10, 8), seed=3, force_kind="uniform", g_amp=1e-3)
    a = sim_mod.from_workload(wl, storage=storage)
    a.step(9)
    ref = a.get_populations().clone()
    b = sim_mod.from_workload(wl, storage=storage)
    b.step(4)
    ck = b.get_populations().clone()
    c = sim_mod.from_workload(wl, storage=storage)
    c.set_populations(ck)
    c.step_count = 4
    c.step(5)
    assert c.step_count == 9
    assert torch.equal(c.get_populations(), ref)


@pytest.mark.parametrize("plates", [False, True])
def test_nan_canary_every_output_written(sim_mod, plates):
    """Every slot of the output buffer is written by a step (the single-grid
    kernel, the kernel with plates)."""
    wl = workloads.random_smooth("D2Q37", (67, 7, 1), seed=5, force_kind="uniform")
    if plates:
        wl.walls = (0.9, 1.1, 0.0, 0.0)
    s = sim_mod.from_workload(wl)
    s.step(1)
    # fill the state with NaN, then restore a valid state and step: every
    # element of the output buffer must be overwritten by finite values
    good = s.get_populations().clone()
    bad = torch.full_like(good.view(torch.float64), float("nan")).view(torch.uint8)
    s.set_populations(bad)
    s.step(1)  # writes the other buffer from NaN input: all NaN
    s.set_populations(good)
    s.step(1)
    p = s.get_populations().view(torch.float64)
    assert torch.isfinite(p).all()


def test_totals_repeat_bitwise(sim_mod):
    wl = workloads.random_smooth("D3Q39", (20, 9, 7), seed=6, force_kind="uniform")
    s = sim_mod.from_workload(wl)
    s.step(3)
    t1 = s.totals()
    t2 = s.totals()
    assert np.array_equal(t1, t2)


def test_nonfinite_state_is_reported(sim_mod):
    from paper_2302_04741_amd._lib import LBM_ENONFINITE, LbmError

    wl = workloads.random_smooth("D2Q37", (16, 16, 1), seed=7, force_kind="uniform")
    s = sim_mod.from_workload(wl)
    bad = torch.full((s.population_bytes() // 8,), float("inf"), dtype=torch.float64,
                     device="cuda")
    s.set_populations(bad.view(torch.uint8))
    with pytest.raises(LbmError) as ei:
        s.totals()
    assert ei.value.status == LBM_ENONFINITE


def test_force_errors_on_gpu(sim_mod):
    from paper_2302_04741_amd._lib import LBM_EINVAL, LbmError

    s = sim_mod.Sim("D2Q37", (8, 6), 0.8, 1.0, np.zeros((2, 48)), 1.0)
    with pytest.raises(LbmError) as ei:
        s.set_force(field=np.zeros((2, 48)))  # no LBM_FLAG_FORCE_FIELD at creation
    assert ei.value.status == LBM_EINVAL
    with pytest.raises(LbmError):
        s.set_force(axis=0, profile=np.zeros((2, 7)))  # length 7 != nx = 8
    with pytest.raises(LbmError):
        s.set_force(axis=2, profile=np.zeros((2, 1)))  # no z axis in 2-D
    with pytest.raises(LbmError):
        s.set_force([float("nan"), 0.0])
    with pytest.raises(LbmError):
        s.set_block(96)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_pattern_pass_leaves_the_state(sim_mod, storage):
    """The access-pattern diagnostic writes only the idle buffer: the state and
    every later step are bitwise those of a run without it."""
    wl = workloads.random_smooth("D3Q39", (70, 9, 6), seed=11, force_kind="axis")
    a = sim_mod.from_workload(wl, storage=storage)
    b = sim_mod.from_workload(wl, storage=storage)
    a.step(3)
    b.step(3)
    before = a.get_populations().clone()
    a.pattern_pass(2)
    assert torch.equal(a.get_populations(), before)
    assert a.step_count == 3
    a.step(4)
    b.step(4)
    assert torch.equal(a.get_populations(), b.get_populations())
    with pytest.raises(Exception):
        a.pattern_pass(-1)


def test_f16_stochastic_rounding_is_unbiased(sim_mod):
    """F16 storage rounds stochastically: on a uniform gas at rest
    (rho = 1.003, theta = 1, no force) every step stores h_i = w_i (rho - 1),
    a value binary16 cannot hold.  Round-to-nearest would make the same error
    in every cell, and the total mass would drift by N times it per step;
    with zero-mean rounding the mass performs a random walk whose standard
    deviation after n steps is at most sqrt(n sum over stored values of
    (ulp/2)^2) (each value's rounding variance is p(1 - p) ulp^2 <= ulp^2/4).
    The measured drift must stay within 6 of those deviations, a bound the
    nearest rounding of these values would exceed many times over."""
    from paper_2302_04741_amd import _lib

    n, steps, drho = 256, 100, 3e-3
    N = n * n
    s = sim_mod.Sim("D2Q37", (n, n), 0.8, np.full(N, 1.0 + drho), np.zeros((2, N)),
                    np.ones(N), storage="f16dev")
    m0 = s.totals()[0]
    s.step(steps)
    m1 = s.totals()[0]
    _, w, _ = _lib.lattice_table("D2Q37")
    k = np.round(-np.log2(w))
    # the values stored each step (scaled), their half spacing, and the
    # spacing in units of f
    v = np.abs(w * drho * 2.0 ** k)
    ulp = 2.0 ** (np.floor(np.log2(v)) - 10)
    sigma = np.sqrt(steps * N * ((ulp * 2.0 ** -k / 2.0) ** 2).sum())
    # what round-to-nearest would do: the same error in every cell, every step
    rn = np.abs(np.float16(v) - v)  # |RN(v) - v| in scaled units (v > 0)
    rn_drift = steps * N * np.abs((np.sign(np.float16(v) - v) * rn * 2.0 ** -k).sum())
    drift = abs(m1 - m0)
    print("mass drift %.3e, SR bound 6 sigma %.3e, RN drift would be %.3e"
          % (drift, 6 * sigma, rn_drift), flush=True)
    assert drift <= 6.0 * sigma
    assert rn_drift >= 20.0 * 6.0 * sigma
