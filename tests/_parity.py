"""Helpers of the GPU-vs-oracle parity tests."""
import numpy as np

LAT_ID = {"D2Q37": 0, "D3Q39": 1}


def rel_err(gpu, ora):
    """Per-field parity metric: for rho and theta max|a - b| / max|b|; for u the
    Euclidean norm per cell, max_x |u_a - u_b|_2 / max_x |u_b|_2."""
    rho_g, u_g, th_g = gpu
    rho_o, u_o, th_o = ora
    e_rho = np.abs(rho_g - rho_o).max() / np.abs(rho_o).max()
    e_th = np.abs(th_g - th_o).max() / np.abs(th_o).max()
    nu = np.sqrt((u_o ** 2).sum(axis=0)).max()
    e_u = np.sqrt(((u_g - u_o) ** 2).sum(axis=0)).max() / nu if nu > 0 else \
        np.sqrt(((u_g - u_o) ** 2).sum(axis=0)).max()
    return e_rho, e_u, e_th


def to_host(t):
    return t.detach().cpu().numpy()


def gpu_moments(sim):
    r, u, t = sim.moments()
    return to_host(r), to_host(u), to_host(t)


def oracle_run(oracle_mod, wl, steps, nthreads=0, prec="f64"):
    sim = oracle_mod.OracleSim(LAT_ID[wl.lattice], wl.dims, wl.tau_hat, wl.rho, wl.u, wl.theta,
                               wl.force_field(), eq_order=wl.eq_order,
                               force_order=wl.force_order, nthreads=nthreads, prec=prec,
                               mu=wl.mu, walls=wl.walls)
    sim.step(steps)
    return sim


def window_indices(dims, center, radius, D):
    """Flat global cell indices of the periodic window of half-width `radius`
    around `center`, ordered like a (2R+1)^D grid (x fastest)."""
    nx, ny, nz = dims
    cx, cy, cz = center
    offs = np.arange(-radius, radius + 1)
    xs = (cx + offs) % nx
    ys = (cy + offs) % ny
    zs = (cz + offs) % nz if D == 3 else np.array([0])
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return ((Z * ny + Y) * nx + X).reshape(-1)


def oracle_window_moments(oracle_mod, wl, center, steps, g_field=None):
    """Moments at `center` after `steps` steps, from an oracle run on the
    periodic window of half-width 3*steps around it (information travels at
    most 3 nodes per step, so the window edge cannot reach the centre)."""
    D = wl.D
    R = 3 * steps + 1
    idx = window_indices(wl.dims, center, R, D)
    n = 2 * R + 1
    wdims = (n, n, n if D == 3 else 1)
    g = wl.force_field() if g_field is None else g_field
    sim = oracle_mod.OracleSim(LAT_ID[wl.lattice], wdims, wl.tau_hat, wl.rho[idx],
                               np.ascontiguousarray(wl.u[:, idx]), wl.theta[idx],
                               np.ascontiguousarray(g[:, idx]), eq_order=wl.eq_order,
                               force_order=wl.force_order, mu=wl.mu)
    sim.step(steps)
    r, u, t = sim.moments()
    mid = len(idx) // 2
    return r[mid], u[:, mid], t[mid]
