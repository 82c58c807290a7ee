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
