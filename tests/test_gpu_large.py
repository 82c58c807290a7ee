"""A grid whose population planes exceed 2 GiB (GPU).

The kernels address a plane with 32-bit byte offsets (every plane is < 4 GiB,
checked at creation); the benchmark grids keep planes far below 2^31 bytes, so
offsets past 2^31 are exercised only here: D3Q39 FP32 on 1024 x 1024 x 520
(545 M cells, 2.18e9 bytes per plane, ~170 GB of populations).  The fields are
analytic (separable sines) and built on the device; after 2 steps the moments at
sampled cells, those at the end of the planes included, are recomputed by the
oracle on a periodic window of half-width 7 around each cell.
"""
import math

import numpy as np
import pytest
import torch

from _parity import LAT_ID

pytestmark = pytest.mark.gpu

NX, NY, NZ = 1024, 1024, 520
STEPS = 2
TOL32 = (2e-6, 5e-5, 2e-6)


def fields_at(x, y, z):
    """rho, u (3, n), theta at integer coordinates (numpy or torch, broadcast)."""
    lib = torch if isinstance(x, torch.Tensor) else np
    rho = 1.0 + 0.01 * lib.sin(2 * math.pi * z / NZ) + 0 * x + 0 * y
    th = 1.0 + 0.05 * lib.sin(2 * math.pi * y / NY) + 0 * x + 0 * z
    ux = 0.02 * lib.sin(2 * math.pi * z / NZ) + 0 * x + 0 * y
    uy = 0.01 * lib.sin(2 * math.pi * x / NX) + 0 * y + 0 * z
    uz = 0.015 * lib.cos(2 * math.pi * y / NY) + 0 * x + 0 * z
    return rho, (ux, uy, uz), th


def gx_profile():
    return 1e-5 * np.sin(2 * np.pi * np.arange(NZ) / NZ)


def test_planes_beyond_2gib(oracle_mod):
    from paper_2302_04741_amd import sim

    N = NX * NY * NZ
    assert 1024 * NY * NZ * 4 > (1 << 31)
    dev = torch.device("cuda")
    z = torch.arange(NZ, device=dev, dtype=torch.float64).view(NZ, 1, 1)
    y = torch.arange(NY, device=dev, dtype=torch.float64).view(1, NY, 1)
    x = torch.arange(NX, device=dev, dtype=torch.float64).view(1, 1, NX)
    rho, u, th = fields_at(x, y, z)
    shape = (NZ, NY, NX)
    rho = rho.expand(shape).reshape(N).contiguous()
    th = th.expand(shape).reshape(N).contiguous()
    uu = torch.stack([c.expand(shape).reshape(N) for c in u]).contiguous()
    del u
    s = sim.Sim("D3Q39", (NX, NY, NZ), 0.8, rho, uu, th, storage="f32")
    del rho, uu, th
    prof = np.zeros((3, NZ))
    prof[0] = gx_profile()
    s.set_force(axis=2, profile=prof)
    s.step(STEPS)
    r_g, u_g, t_g = s.moments()
    samples = [(0, 0, 0), (NX - 1, NY - 1, NZ - 1), (NX - 2, NY - 1, NZ - 1), (5, NY - 3, NZ - 2),
               (NX // 2, NY // 2, NZ // 2), (1000, 17, 300), (0, NY - 1, NZ - 1)]
    idx = torch.tensor([(zz * NY + yy) * NX + xx for xx, yy, zz in samples], device=dev)
    rg, ug, tg = r_g[idx].cpu().numpy(), u_g[:, idx].cpu().numpy(), t_g[idx].cpu().numpy()
    del r_g, u_g, t_g
    s.close()
    torch.cuda.empty_cache()
    R = 3 * STEPS + 1
    n = 2 * R + 1
    offs = np.arange(-R, R + 1)
    worst = np.zeros(3)
    for k, (cx, cy, cz) in enumerate(samples):
        Z, Y, X = np.meshgrid((cz + offs) % NZ, (cy + offs) % NY, (cx + offs) % NX, indexing="ij")
        X, Y, Z = (a.reshape(-1).astype(np.float64) for a in (X, Y, Z))
        r0, u0, t0 = fields_at(X, Y, Z)
        g = np.zeros((3, n ** 3))
        g[0] = gx_profile()[Z.astype(int)]
        o = oracle_mod.OracleSim(LAT_ID["D3Q39"], (n, n, n), 0.8, r0, np.stack(u0), t0, g)
        o.step(STEPS)
        ro, uo, to = o.moments()
        mid = n ** 3 // 2
        e = np.array([abs(rg[k] - ro[mid]) / 1.01,
                      np.sqrt(((ug[:, k] - uo[:, mid]) ** 2).sum()) / 0.0206,
                      abs(tg[k] - to[mid]) / 1.05])
        worst = np.maximum(worst, e)
    print("D3Q39 FP32 %dx%dx%d (plane %.2e B), %d samples: worst rho %.2e u %.2e theta %.2e"
          % (NX, NY, NZ, 4.0 * NX * NY * NZ, len(samples), *worst), flush=True)
    assert all(w <= t for w, t in zip(worst, TOL32)), worst
