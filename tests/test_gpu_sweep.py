"""The D2Q37 1024^2 thermal-shear sweep (GPU): tau-hat in {0.6, 0.9}, dtheta in
{0.02, 0.1}, Ma in {0.05, 0.2}, uniform g = (0, -1e-5), 5000 steps, FP64 and
FP32 storage.

Per configuration:
  * MLUPS of both storages (HIP events on the simulation's stream);
  * FP32 against FP64 after 5000 steps: rho, u, theta (relative, as in the
    parity tests) and the heat flux (relative to max|q|);
  * the paper's central claim at full size: from the 5000-step state, two
    branches run 50 more steps with the full force term (order 4) and without
    its third-moment part (order 2, the Guo-type scheme); their heat-flux
    difference must equal the Chapman-Enskog q_err of Sec. 2,
    -rho tau/2 [(|u|^2 + (theta - 1)(D + 2)) g + 2 (g.u) u], tau = tau-hat - 1/2,
    evaluated on the branch's moments.  Compared on the dominant Fourier mode
    in y (the flow varies in y only); pointwise the CE estimate also carries
    O(gradient) corrections.
  * FP32 resolves that difference: its mode within 3% of FP64's.
  * The scheme without a3_F (force order 2) run as its own 5000-step
    simulation from the same initial state, in FP64 and FP32: FP32 against
    FP64 within the same bars as the full scheme.  The full-size difference of
    the two schemes after 5000 steps (rho, u, theta and q, FP64) is printed.
    Its temperature part (2.5e-7 to 1.6e-6 of theta at dtheta 0.02, 1.2e-5 to
    1.4e-5 at dtheta 0.1) is resolved by FP32 only where it is comparable to
    FP32's own coherent theta drift over the run (7e-6 to 1.4e-4): where the
    scheme difference is at least 0.4x that drift (tau-hat 0.9, dtheta 0.1) the
    FP32 difference of the two schemes on its dominant y-mode is within 15% of
    FP64's (measured 0.9-1.4%); elsewhere the drift is 2.5x to 60x the
    difference and the mode is not resolved (5-95%, depending on how the
    rounding of each run falls), which the test records as the scheme
    difference staying below 3x the FP32 error.

Measured values are printed; the bars are about 3x above the largest of them.
"""
import itertools
import math

import numpy as np
import pytest
import torch

from _parity import gpu_moments, rel_err, to_host
from paper_2302_04741_amd import workloads

pytestmark = pytest.mark.gpu

STEPS, BRANCH = 5000, 50
CONFIGS = list(itertools.product((0.6, 0.9), (0.02, 0.1), (0.05, 0.2)))
# measured maxima over the sweep: rho 9.9e-5, u 1.0e-3, theta 1.3e-4, q 4.8e-3,
# CE 1.5e-3 (3.1e-4 at tau-hat 0.6), FP32 dq mode 8.6e-3
TOL32 = (3e-4, 3e-3, 4e-4)  # rho, u, theta after 5000 steps
TOL_Q32 = 1.5e-2
TOL_CE = 5e-3
TOL_DQ32 = 3e-2


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2302_04741_amd import sim

    return sim


def q_err(m, g, tau_hat):
    rho, u, th = m
    tau = tau_hat - 0.5
    u2 = (u * u).sum(0)
    gu = (g[:, None] * u).sum(0)
    return -0.5 * rho * tau * ((u2 + (th - 1.0) * 4.0) * g[:, None] + 2.0 * gu * u)


def ymode(f, n):
    """Amplitudes of sin and cos(2 pi k y / n), k = 1, 2, of each component."""
    y = np.arange(f.shape[-1]) // n
    out = []
    for k in (1, 2):
        for fn in (np.sin, np.cos):
            w = fn(2 * math.pi * k * y / n)
            out.append(2.0 / f.shape[-1] * (f * w).sum(-1))
    return np.stack(out, -1)


def run_plain(sim_mod, tau, dth, ma, storage, stream, force_order):
    """A 5000-step run of one scheme from the initial state: MLUPS, moments, q."""
    wl = workloads.thermal_shear_2d(n=1024, tau_hat=tau, dtheta=dth, mach=ma, steps=STEPS,
                                    force_order=force_order)
    s = sim_mod.from_workload(wl, storage=storage, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(STEPS)
    e1.record(stream)
    e1.synchronize()
    mlups = wl.ncell * STEPS / e0.elapsed_time(e1) / 1e3
    m = gpu_moments(s)
    q = to_host(s.heat_flux())
    s.close()
    return mlups, m, q


def run(sim_mod, tau, dth, ma, storage, stream):
    wl = workloads.thermal_shear_2d(n=1024, tau_hat=tau, dtheta=dth, mach=ma, steps=STEPS)
    s = sim_mod.from_workload(wl, storage=storage, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(STEPS)
    e1.record(stream)
    e1.synchronize()
    mlups = wl.ncell * STEPS / e0.elapsed_time(e1) / 1e3
    m = gpu_moments(s)
    q = to_host(s.heat_flux())
    snap = s.get_populations()
    dq = {}
    for fo in (4, 2):
        b = sim_mod.from_workload(
            workloads.thermal_shear_2d(n=1024, tau_hat=tau, dtheta=dth, mach=ma, force_order=fo),
            storage=storage, stream=stream)
        b.set_populations(snap)
        b.step(BRANCH)
        dq[fo] = (to_host(b.heat_flux()), gpu_moments(b))
        b.close()
    s.close()
    return wl, mlups, m, q, dq[2][0] - dq[4][0], dq[4][1]


@pytest.mark.parametrize("tau,dth,ma", CONFIGS)
def test_thermal_shear_1024_sweep(sim_mod, tau, dth, ma):
    stream = torch.cuda.Stream()
    wl, r64, m64, q64, dq64, mb64 = run(sim_mod, tau, dth, ma, "f64", stream)
    _, r32, m32, q32, dq32, _ = run(sim_mod, tau, dth, ma, "f32", stream)
    e = rel_err(m32, m64)
    eq = np.abs(q32 - q64).max() / np.abs(q64).max()
    g = np.asarray(wl.force[1])[:2]
    qe = q_err(mb64, g, tau)
    a_dq, a_qe, a_dq32 = ymode(dq64[1], 1024), ymode(qe[1], 1024), ymode(dq32[1], 1024)
    k = np.argmax(np.abs(a_qe))
    ce = abs(a_dq[k] / a_qe[k] - 1.0)
    p32 = abs(a_dq32[k] / a_dq[k] - 1.0)
    print("tau %.1f dth %.2f Ma %.2f | MLUPS f64 %.0f f32 %.0f | FP32 vs FP64: rho %.1e u %.1e "
          "theta %.1e q %.1e | dq mode %.3e, q_err mode %.3e (CE %.1e) | FP32 dq mode %.1e"
          % (tau, dth, ma, r64, r32, *e, eq, a_dq[k], a_qe[k], ce, p32), flush=True)
    assert all(x <= t for x, t in zip(e, TOL32)), e
    assert eq <= TOL_Q32
    assert ce <= TOL_CE
    assert p32 <= TOL_DQ32

    # the scheme without a3_F as its own 5000-step run
    r64_2, m64_2, q64_2 = run_plain(sim_mod, tau, dth, ma, "f64", stream, 2)
    r32_2, m32_2, q32_2 = run_plain(sim_mod, tau, dth, ma, "f32", stream, 2)
    e2 = rel_err(m32_2, m64_2)
    eq2 = np.abs(q32_2 - q64_2).max() / np.abs(q64_2).max()
    # the two schemes after 5000 steps (FP64), relative like the parity metric
    d_sch = rel_err(m64_2, m64)
    dq_sch = np.abs(q64_2 - q64).max() / np.abs(q64).max()
    dth64 = m64_2[2] - m64[2]
    dth32 = m32_2[2] - m32[2]
    a64, a32 = ymode(dth64[None], 1024)[0], ymode(dth32[None], 1024)[0]
    j = np.argmax(np.abs(a64))
    p_th = abs(a32[j] / a64[j] - 1.0)
    err32_th = max(np.abs(m32_2[2] - m64_2[2]).max(), np.abs(m32[2] - m64[2]).max())
    print("  order 2, 5000 steps | MLUPS f64 %.0f f32 %.0f | FP32 vs FP64: rho %.1e u %.1e "
          "theta %.1e q %.1e | order 2 vs 4 (FP64): rho %.1e u %.1e theta %.1e q %.1e, "
          "max|dtheta| %.2e | FP32 dtheta mode %.1e, FP32 theta error %.1e"
          % (r64_2, r32_2, *e2, eq2, *d_sch, dq_sch, np.abs(dth64).max(), p_th, err32_th),
          flush=True)
    assert all(x <= t for x, t in zip(e2, TOL32)), e2
    assert eq2 <= TOL_Q32
    assert np.abs(dth64).max() > 0.0
    if np.abs(dth64).max() >= 0.4 * err32_th:
        assert p_th <= 0.15
    else:
        # below FP32's resolution over 5000 steps (the 50-step heat-flux
        # branches above resolve the correction itself)
        assert np.abs(dth64).max() <= 3.0 * err32_th
