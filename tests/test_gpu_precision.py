"""Reduced-precision storage: FP32 deviations and F16 deviations (FP32 arithmetic).

Errors after 2000 steps against FP64: on the 256^2 thermal shear workload the
FP64 reference is the CPU oracle itself; on the full-size workloads it is the
GPU FP64 path, whose parity with the oracle the parity tests establish.

The a3_F heat-flux correction of the paper (Sec. 2, q_err: the heat flux that
dropping the third-moment force term adds) is measured as
dq = q(force order 2) - q(force order 4), projected on the sin/cos(2 pi y/L)
modes; FP32 storage must reproduce the dominant FP64 mode within 10%.

Bars (about 5x the values measured on an MI355X):
  FP32: rho 2e-4, u 2e-3, theta 5e-4 relative (as in the parity tests), q 1e-2
        relative to max|q|.
  F16 : rho 3e-3, u 2e-2, theta 2e-3; q is not bounded: with 11-bit half
        rounding of deviations that reach ~25% of w_i, q is off by 1e-2..3e-1
        and dq is not resolved (recorded, not asserted).
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


def run(sim_mod, wl, storage, force_order):
    wl.force_order = force_order
    s = sim_mod.from_workload(wl, storage=storage)
    s.step(STEPS)
    m = gpu_moments(s)
    q = to_host(s.heat_flux())
    s.close()
    return m, q


def modes(q, wl):
    nx, ny, nz = wl.dims
    y = (np.arange(wl.ncell) // nx) % ny
    out = []
    for a in range(q.shape[0]):
        for f in (np.sin, np.cos):
            out.append(2.0 / wl.ncell * (q[a] * f(2 * math.pi * y / ny)).sum())
    return np.array(out)


WORKLOADS = {
    "shear256": lambda fo: workloads.thermal_shear_2d(n=256, tau_hat=0.6, dtheta=0.1, mach=0.2,
                                                      force_order=fo),
    "shear1024": lambda fo: workloads.thermal_shear_2d(n=1024, tau_hat=0.6, dtheta=0.1, mach=0.2,
                                                       force_order=fo),
    "kolmogorov256": lambda fo: workloads.kolmogorov_3d(n=256, force_order=fo),
}


@pytest.fixture(scope="module")
def references(sim_mod, oracle_mod):
    refs = {}
    for name, make in WORKLOADS.items():
        if name == "shear256":
            wl = make(4)
            o = oracle_run(oracle_mod, wl, STEPS)
            ref4 = (o.moments(), o.heat_flux())
            o2 = oracle_run(oracle_mod, make(2), STEPS)
            q2 = o2.heat_flux()
        else:
            ref4 = run(sim_mod, make(4), "f64", 4)
            q2 = run(sim_mod, make(2), "f64", 2)[1]
        refs[name] = (ref4, modes(q2 - ref4[1], make(4)))
    return refs


@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_reduced_precision_errors(sim_mod, references, name, storage):
    (ref_m, ref_q), ref_dq = references[name]
    m, q = run(sim_mod, WORKLOADS[name](4), storage, 4)
    errs = rel_err(m, ref_m)
    eq = np.abs(q - ref_q).max() / np.abs(ref_q).max()
    _, q2 = run(sim_mod, WORKLOADS[name](2), storage, 2)
    dq = modes(q2 - q, WORKLOADS[name](4))
    k = int(np.argmax(np.abs(ref_dq)))
    edq = abs(dq[k] - ref_dq[k]) / abs(ref_dq[k])
    print("%s %s after %d steps: rho %.2e u %.2e theta %.2e q %.2e | a3_F dq mode %.3e vs %.3e "
          "(rel %.2e)" % (name, storage, STEPS, *errs, eq, dq[k], ref_dq[k], edq), flush=True)
    assert all(e <= t for e, t in zip(errs, TOL[storage])), errs
    if storage == "f32":
        assert eq <= TOL_Q32
        assert edq <= 0.10  # the a3_F correction is resolved
