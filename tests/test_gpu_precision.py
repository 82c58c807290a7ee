"""Reduced-precision storage: FP32 deviations and F16 deviations (FP32 arithmetic).

Errors after 2000 steps against FP64: on the 256^2 thermal shear workload the
FP64 reference is the CPU oracle itself; on the full-size workloads it is the
GPU FP64 path, whose parity with the oracle the parity tests establish.

The a3_F heat-flux correction of the paper (Sec. 2, q_err: the heat flux that
dropping the third-moment force term adds) is measured as
dq = q(force order 2) - q(force order 4), two runs from the same initial
state, projected on the Fourier modes the workload drives (sin/cos(2 pi y/L);
in 3-D also their products with sin/cos(2 pi z/L), where the Kolmogorov
case's correction lives), at step 2000 and averaged over 8 snapshots 25 steps
apart from there (the time average takes out rounding noise that decorrelates
between snapshots; FP64 is averaged the same way).

Bars (FP32 about 5x the values measured on an MI355X):
  FP32: rho 2e-4, u 2e-3, theta 5e-4 relative (as in the parity tests), q 1e-2
        relative to max|q|; the dominant dq mode within 10% of FP64's.
  F16 (stochastic rounding): rho 3e-3, u 2e-2, theta 2e-3.  q pointwise is
        not bounded: the half rounding of deviations that reach ~25% of w_i
        leaves noise of 1e-2..5e-1 of max|q| in single cells.  The dq mode is
        a sum of that noise over the grid, so its error is random: over
        independent rounding realizations (the step counter that keys the
        random bits offset by k * 10^6) its relative error, time-averaged as
        above, had standard deviation 17% on the 256^2 shear (16 realizations,
        mean +1.6%), 2.9% on 1024^2 (12, mean +0.6%) and 0.10% on the
        Kolmogorov flow (8, mean +0.09%).  Asserted: a single run within 10% on
        1024^2 and 256^3 (3.4 and 100 standard deviations); on 256^2 the mean
        of 32 realizations within 10% (3.3 standard deviations of that mean),
        their spread below 35%, and a single run within 70% (4 standard
        deviations); on 1024^2 also the mean of 12 realizations within 5% and
        their spread below 8%.  With round-to-nearest stores (measured with a library
        variant) the shear workloads' dq came out 37-217% off, twice with the
        wrong sign.
"""
import math

import numpy as np
import pytest

from _parity import gpu_moments, oracle_run, rel_err, to_host
from paper_2302_04741_amd import workloads

pytestmark = pytest.mark.gpu

STEPS = 2000
TOL = {"f32": (2e-4, 2e-3, 5e-4), "f16dev": (3e-3, 2e-2, 2e-3)}
TOL_Q32 = 1e-2


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2302_04741_amd import sim

    return sim


SNAPS, EVERY = 8, 25


def run(sim_mod, wl, storage, force_order, offset=0):
    """Moments and heat flux at STEPS, and the heat-flux modes averaged over
    SNAPS snapshots EVERY steps apart from STEPS on.  offset: the step counter
    starts there (F16: another realization of the stochastic rounding)."""
    wl.force_order = force_order
    s = sim_mod.from_workload(wl, storage=storage)
    if offset:
        s.step_count = offset
    s.step(STEPS)
    m = gpu_moments(s)
    q = to_host(s.heat_flux())
    avg = modes(q, wl)
    for _ in range(SNAPS - 1):
        s.step(EVERY)
        avg = avg + modes(to_host(s.heat_flux()), wl)
    s.close()
    return m, q, avg / SNAPS


def oracle_runs(oracle_mod, wl):
    """The same quantities from the CPU oracle."""
    o = oracle_run(oracle_mod, wl, STEPS)
    m, q = o.moments(), o.heat_flux()
    avg = modes(q, wl)
    for _ in range(SNAPS - 1):
        o.step(EVERY)
        avg = avg + modes(o.heat_flux(), wl)
    return m, q, avg / SNAPS


def modes(q, wl):
    """Amplitudes of the lowest Fourier modes the workloads drive: sin and
    cos(2 pi y/ny) of every component, and in 3-D also their products with
    sin and cos(2 pi z/nz) (the Kolmogorov force varies in z, the temperature
    in y, so its a3_F heat flux lives on the product modes)."""
    nx, ny, nz = wl.dims
    cell = np.arange(wl.ncell)
    y = (cell // nx) % ny
    z = cell // (nx * ny)
    basis = [f(2 * math.pi * y / ny) for f in (np.sin, np.cos)]
    if nz > 1:
        basis += [f(2 * math.pi * y / ny) * g(2 * math.pi * z / nz)
                  for f in (np.sin, np.cos) for g in (np.sin, np.cos)]
    out = []
    for a in range(q.shape[0]):
        for b in basis:
            out.append((q[a] * b).sum() / (b * b).sum())
    return np.array(out)


WORKLOADS = {
    "shear256": lambda fo: workloads.thermal_shear_2d(n=256, tau_hat=0.6, dtheta=0.1, mach=0.2,
                                                      force_order=fo),
    "shear1024": lambda fo: workloads.thermal_shear_2d(n=1024, tau_hat=0.6, dtheta=0.1, mach=0.2,
                                                       force_order=fo),
    "kolmogorov256": lambda fo: workloads.kolmogorov_3d(n=256, force_order=fo),
}


# bar on the time-averaged a3_F dq mode of one run, relative to FP64 (F16 on
# 256^2: four standard deviations of its rounding noise; the mean over
# realizations is held to 10% by test_f16_dq_over_realizations)
TOL_DQ = {("f32", "shear256"): 0.10, ("f32", "shear1024"): 0.10, ("f32", "kolmogorov256"): 0.10,
          ("f16dev", "shear256"): 0.70, ("f16dev", "shear1024"): 0.10,
          ("f16dev", "kolmogorov256"): 0.10}
OFFSET = 10 ** 6  # step-counter offset between realizations


@pytest.fixture(scope="module")
def references(sim_mod, oracle_mod):
    refs = {}
    for name, make in WORKLOADS.items():
        if name == "shear256":
            m4, q4, a4 = oracle_runs(oracle_mod, make(4))
            _, q2, a2 = oracle_runs(oracle_mod, make(2))
        else:
            m4, q4, a4 = run(sim_mod, make(4), "f64", 4)
            _, q2, a2 = run(sim_mod, make(2), "f64", 2)
        refs[name] = ((m4, q4), modes(q2 - q4, make(4)), a2 - a4)
    return refs


@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_reduced_precision_errors(sim_mod, references, name, storage):
    (ref_m, ref_q), ref_dq, ref_avg = references[name]
    m, q, a4 = run(sim_mod, WORKLOADS[name](4), storage, 4)
    errs = rel_err(m, ref_m)
    eq = np.abs(q - ref_q).max() / np.abs(ref_q).max()
    _, q2, a2 = run(sim_mod, WORKLOADS[name](2), storage, 2)
    dq = modes(q2 - q, WORKLOADS[name](4))
    k = int(np.argmax(np.abs(ref_dq)))
    edq = abs(dq[k] - ref_dq[k]) / abs(ref_dq[k])
    ka = int(np.argmax(np.abs(ref_avg)))
    edq_avg = abs((a2 - a4)[ka] - ref_avg[ka]) / abs(ref_avg[ka])
    print("%s %s after %d steps: rho %.2e u %.2e theta %.2e q %.2e | a3_F dq mode %.3e vs %.3e "
          "(rel %.2e); averaged over %d snapshots %.3e vs %.3e (rel %.2e)"
          % (name, storage, STEPS, *errs, eq, dq[k], ref_dq[k], edq, SNAPS, (a2 - a4)[ka],
             ref_avg[ka], edq_avg), flush=True)
    assert all(e <= t for e, t in zip(errs, TOL[storage])), errs
    if storage == "f32":
        assert eq <= TOL_Q32
        assert edq <= 0.10  # the a3_F correction is resolved at one snapshot
    assert edq_avg <= TOL_DQ[(storage, name)]  # and on the time average


# realizations, bar on the error of their mean, bar on their spread (standard
# deviation of the relative error; measured 14-17% on 256^2, 2.9% on 1024^2)
REALIZATION_CASES = {"shear256": (32, 0.10, 0.35), "shear1024": (12, 0.05, 0.08)}


@pytest.mark.parametrize("name", list(REALIZATION_CASES))
def test_f16_dq_over_realizations(sim_mod, references, name):
    """The rounding noise of the F16 a3_F dq mode, measured over independent
    stochastic-rounding realizations: the rounding is unbiased (the mean over
    realizations converges to FP64's value) and its spread stays at the
    documented budget (one run on 256^2 scatters by about 17%, on 1024^2 by
    about 3%)."""
    count, tol_mean, tol_std = REALIZATION_CASES[name]
    wl = WORKLOADS[name]
    ref_avg = references[name][2]
    ka = int(np.argmax(np.abs(ref_avg)))
    vals = []
    for k in range(count):
        _, _, a4 = run(sim_mod, wl(4), "f16dev", 4, offset=k * OFFSET)
        _, _, a2 = run(sim_mod, wl(2), "f16dev", 2, offset=k * OFFSET)
        vals.append((a2 - a4)[ka])
    rel = (np.array(vals) - ref_avg[ka]) / abs(ref_avg[ka])
    err_mean = abs(np.mean(vals) - ref_avg[ka]) / abs(ref_avg[ka])
    print("%s f16dev, %d realizations: dq mode error mean %+.4f (of the mean %.4f), "
          "std %.4f, max %.3f" % (name, count, rel.mean(), err_mean, rel.std(ddof=1),
                                  np.abs(rel).max()), flush=True)
    assert err_mean <= tol_mean
    assert rel.std(ddof=1) <= tol_std
