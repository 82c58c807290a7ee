"""The C-ABI library on the host: it loads, exports every symbol include/lbm.h
declares, validates arguments before touching the GPU, and compiles in the same
quadrature rules the oracle derives independently (CPU only; no compute call)."""
import ctypes
import itertools
import os
import re

import numpy as np
import pytest

from paper_2302_04741_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2302_04741_amd import build

        build.build()
    return _lib.load()


def declared_symbols():
    text = open(HEADER).read()
    return re.findall(r"^LBM_API[^(]*?\b(lbm_\w+)\(", text, flags=re.M)


def test_header_declares_the_binding_api():
    assert sorted(declared_symbols()) == sorted(_lib.API_SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_only_declared_symbols_are_exported():
    import subprocess

    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert exported == set(declared_symbols())


def test_version(lib):
    assert lib.lbm_version().decode().startswith("lbm-gfx950")


def params(**kw):
    base = dict(lattice="D2Q37", dims=(64, 64, 1), tau_hat=0.8)
    base.update(kw)
    return _lib.make_params(**base)


def create(lib, p, ws=0x100000, nbytes=None, fields=(0x200000, 0x300000, 0x400000)):
    """lbm_create with fake (never dereferenced) device pointers."""
    h = ctypes.c_void_p()
    if nbytes is None:
        nbytes = _lib.workspace_bytes(p) if p is not None else 0
    pp = ctypes.byref(p) if p is not None else None
    st = lib.lbm_create(pp, ctypes.c_void_p(ws), ctypes.c_size_t(nbytes), None,
                        *[ctypes.c_void_p(f) if f else None for f in fields], ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(tau_hat=0.5), _lib.LBM_EINVAL),
    (dict(tau_hat=0.3), _lib.LBM_EINVAL),
    (dict(tau_hat=float("nan")), _lib.LBM_EINVAL),
    (dict(dims=(0, 64, 1)), _lib.LBM_EINVAL),
    (dict(dims=(64, -1, 1)), _lib.LBM_EINVAL),
    (dict(dims=(64, 64, 2)), _lib.LBM_EINVAL),
    (dict(dims=(64, 70000, 1)), _lib.LBM_EUNSUPPORTED),
    (dict(eq_order=1), _lib.LBM_EINVAL),
    (dict(eq_order=-1), _lib.LBM_EINVAL),
    (dict(eq_order=5), _lib.LBM_EUNSUPPORTED),
    (dict(lattice="D3Q39", dims=(8, 8, 8), eq_order=4), _lib.LBM_EUNSUPPORTED),
    (dict(force_order=0), _lib.LBM_EINVAL),
    (dict(force_order=5), _lib.LBM_EINVAL),
    (dict(rho0=-1.0), _lib.LBM_EINVAL),
    (dict(rho0=float("inf")), _lib.LBM_EINVAL),
])
def test_invalid_parameters(lib, kw, status):
    p = params(**kw)
    assert _lib.workspace_bytes(p) == 0
    st, h = create(lib, p, nbytes=1 << 30)
    assert st == status and not h.value
    assert lib.lbm_last_error().decode() != ""


def test_unknown_lattice_storage_and_struct_size(lib):
    p = params()
    p.lattice = 7
    assert create(lib, p, nbytes=1 << 30)[0] == _lib.LBM_EINVAL
    p = params()
    p.storage = 9
    assert create(lib, p, nbytes=1 << 30)[0] == _lib.LBM_EINVAL
    p = params()
    p.struct_size = 8
    assert create(lib, p, nbytes=1 << 30)[0] == _lib.LBM_EINVAL
    p = params()
    p.flags = 0x80
    assert create(lib, p, nbytes=1 << 30)[0] == _lib.LBM_EINVAL
    assert lib.lbm_workspace_bytes(None) == 0
    assert create(lib, None)[0] == _lib.LBM_EINVAL


def test_workspace_and_field_checks(lib):
    p = params()
    need = _lib.workspace_bytes(p)
    assert create(lib, p, ws=0)[0] == _lib.LBM_EINVAL
    assert create(lib, p, ws=0x100010)[0] == _lib.LBM_EINVAL  # not 256-byte aligned
    assert create(lib, p, nbytes=need - 1)[0] == _lib.LBM_ENOSPACE
    assert create(lib, p, fields=(0, 0x300000, 0x400000))[0] == _lib.LBM_EINVAL
    assert create(lib, p, fields=(0x200000, 0, 0x400000))[0] == _lib.LBM_EINVAL
    h = ctypes.c_void_p()
    assert lib.lbm_create(ctypes.byref(p), ctypes.c_void_p(0x100000), need, None, None, None,
                          None, None) == _lib.LBM_EINVAL


@pytest.mark.parametrize("lattice,dims,storage,sbytes,Q,D", [
    ("D2Q37", (64, 64, 1), "f64", 8, 37, 2),
    ("D2Q37", (1024, 1024, 1), "f32", 4, 37, 2),
    ("D3Q39", (256, 256, 256), "f32", 4, 39, 3),
    ("D3Q39", (32, 32, 32), "f64", 8, 39, 3),
    ("D2Q37", (1017, 33, 1), "f32", 4, 37, 2),
    ("D3Q39", (5, 7, 3), "f16dev", 2, 39, 3),
])
def test_workspace_size(lattice, dims, storage, sbytes, Q, D):
    def up(v):
        return (v + 255) // 256 * 256

    p = _lib.make_params(lattice, dims, 0.8, storage)
    N = int(np.prod(dims))
    # population rows are padded to a multiple of 64 values
    P = (dims[0] + 63) // 64 * 64 * dims[1] * dims[2]
    abytes = 8 if storage == "f64" else 4
    expect = 2 * up(Q * P * sbytes) + up(D * max(dims) * abytes) + up(512 * Q * 8) + up(64)
    assert _lib.workspace_bytes(p) == expect
    pf = _lib.make_params(lattice, dims, 0.8, storage, force_field=True)
    expect_f = 2 * up(Q * P * sbytes) + up(D * N * abytes) + up(512 * Q * 8) + up(64)
    assert _lib.workspace_bytes(pf) == expect_f
    # plates: partial sums per buffer, plate, row and (x, z) column; emission tables
    pw = _lib.make_params(lattice, dims, 0.8, storage, walls=True)
    expect_w = expect + up(2 * 2 * 3 * dims[0] * dims[2] * 8) + up(2 * (Q + 1) * 8)
    assert _lib.workspace_bytes(pw) == expect_w


def test_null_handle_calls(lib):
    lib.lbm_destroy(None)  # no-op
    assert lib.lbm_step(None, 1) == _lib.LBM_EINVAL
    assert lib.lbm_moments(None, None, None, None) == _lib.LBM_EINVAL
    assert lib.lbm_set_force(None, 0, None, 0, 0) == _lib.LBM_EINVAL
    assert lib.lbm_totals(None, None) == _lib.LBM_EINVAL
    assert lib.lbm_heat_flux(None, None) == _lib.LBM_EINVAL
    assert lib.lbm_pattern_pass(None, 1) == _lib.LBM_EINVAL
    assert lib.lbm_get_populations(None, None) == _lib.LBM_EINVAL
    assert lib.lbm_set_populations(None, None) == _lib.LBM_EINVAL
    assert lib.lbm_set_step_count(None, 0) == _lib.LBM_EINVAL
    assert lib.lbm_set_block(None, 64) == _lib.LBM_EINVAL
    assert lib.lbm_set_stream(None, None) == _lib.LBM_EINVAL
    assert lib.lbm_set_viscosity(None, 0.1) == _lib.LBM_EINVAL
    assert lib.lbm_set_walls(None, 1, 1.0, 1.0, 0.0, 0.0) == _lib.LBM_EINVAL
    assert lib.lbm_step_count(None) == -1
    assert lib.lbm_population_bytes(None) == 0
    assert lib.lbm_lattice_table(5, None, None, None) == _lib.LBM_EINVAL


@pytest.mark.parametrize("lattice,lat,deg", [("D2Q37", 0, 9), ("D3Q39", 1, 7)])
def test_compiled_rule_is_gauss_hermite(lib, lattice, lat, deg):
    c, w, r = _lib.lattice_table(lattice)
    D = 2 if lat == 0 else 3
    xi = r * c[:, :D].astype(np.float64)
    for tot in range(deg + 1):
        for p in itertools.product(range(tot + 1), repeat=D):
            if sum(p) != tot:
                continue
            m = np.sum(w * np.prod(xi ** np.asarray(p), axis=1))
            ref = 0.0 if any(k % 2 for k in p) else float(np.prod(
                [np.prod(np.arange(k - 1, 0, -2)) if k else 1 for k in p]))
            assert abs(m - ref) < 1e-13 * max(1, ref)
    # velocities come as rest, then +c/-c pairs
    assert np.all(c[0] == 0)
    assert np.all(c[1::2] == -c[2::2])


@pytest.mark.parametrize("lattice,lat", [("D2Q37", 0), ("D3Q39", 1)])
def test_compiled_rule_equals_oracle_derivation(lib, oracle_mod, lattice, lat):
    c, w, r = _lib.lattice_table(lattice)
    oc, ow, orr, _ = oracle_mod.lattice(lat)
    assert abs(r - orr) < 1e-15
    mine = {tuple(v): wv for v, wv in zip(c, w)}
    theirs = {tuple(v): wv for v, wv in zip(oc, ow)}
    assert set(mine) == set(theirs)
    for k in mine:
        assert abs(mine[k] - theirs[k]) < 1e-16 * max(1.0, 10 * theirs[k])


def test_batch_and_graph_argument_checks(lib):
    assert lib.lbm_batch_workspace_bytes(0) == 0
    need = lib.lbm_batch_workspace_bytes(4)
    assert need > 0
    h = ctypes.c_void_p()
    assert lib.lbm_batch_create(4, None, need, None, ctypes.byref(h)) == _lib.LBM_EINVAL
    assert lib.lbm_batch_create(4, ctypes.c_void_p(0x100010), need, None,
                                ctypes.byref(h)) == _lib.LBM_EINVAL
    assert lib.lbm_batch_create(4, ctypes.c_void_p(0x100000), need - 1, None,
                                ctypes.byref(h)) == _lib.LBM_ENOSPACE
    assert lib.lbm_batch_create(0, ctypes.c_void_p(0x100000), need, None,
                                ctypes.byref(h)) == _lib.LBM_EINVAL
    # a batch handle needs no GPU until members are set
    assert lib.lbm_batch_create(4, ctypes.c_void_p(0x100000), need, None,
                                ctypes.byref(h)) == _lib.LBM_OK
    assert lib.lbm_batch_step(h, 1) == _lib.LBM_EINVAL  # no members
    assert lib.lbm_batch_set(h, None, 1) == _lib.LBM_EINVAL
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.lbm_batch_set(h, arr, 1) == _lib.LBM_EINVAL  # NULL member
    assert lib.lbm_batch_set(h, arr, 5) == _lib.LBM_EINVAL  # more than max_sims
    assert lib.lbm_batch_set_launch(h, 0, -1) == _lib.LBM_EINVAL
    assert lib.lbm_batch_set_launch(h, 100, 0) == _lib.LBM_EINVAL
    assert lib.lbm_batch_set_launch(h, 512, 0) == _lib.LBM_EINVAL
    assert lib.lbm_batch_set_launch(h, 0, 1 << 31) == _lib.LBM_EINVAL
    for threads in (0, 64, 128, 256):  # no members yet: nothing to rebuild
        assert lib.lbm_batch_set_launch(h, threads, 1024) == _lib.LBM_OK
    assert lib.lbm_batch_set_launch(None, 0, 0) == _lib.LBM_EINVAL
    g = ctypes.c_void_p()
    assert lib.lbm_graph_create(None, None, 2, ctypes.byref(g)) == _lib.LBM_EINVAL
    assert lib.lbm_graph_create(None, h, 2, ctypes.byref(g)) == _lib.LBM_EINVAL  # no members
    assert lib.lbm_graph_launch(None, 1) == _lib.LBM_EINVAL
    lib.lbm_batch_destroy(h)
    lib.lbm_batch_destroy(None)
    lib.lbm_graph_destroy(None)


@pytest.mark.parametrize("storage,sbytes", [("f32", 4), ("f64", 8), ("f16dev", 2)])
def test_largest_plane(lib, storage, sbytes):
    """One population plane (rows padded to 64 values) must stay below 4 GiB so
    that 32-bit byte offsets address it: the largest accepted grids and the
    first refused ones, including a grid refused only because of the padding."""
    cap = (1 << 32) // sbytes  # values per plane at the limit
    ny = 1024
    nz = cap // (1024 * ny)     # nx = 1024: plane exactly at the limit
    ok = params(lattice="D3Q39", dims=(1024, ny, nz - 1), storage=storage)
    assert _lib.workspace_bytes(ok) > 2 * 39 * 1024 * ny * (nz - 1) * sbytes
    at = params(lattice="D3Q39", dims=(1024, ny, nz), storage=storage)
    assert _lib.workspace_bytes(at) == 0
    st, _ = create(lib, at, nbytes=1 << 40)
    assert st == _lib.LBM_EUNSUPPORTED
    # 1000 values per row are stored as 1024: refused although 1000*ny*nz fits
    padded = params(lattice="D3Q39", dims=(1000, ny, nz), storage=storage)
    assert 1000 * ny * nz * sbytes < (1 << 32)
    assert _lib.workspace_bytes(padded) == 0


def test_batch_step_noalloc_argument_checks(lib):
    """Argument errors of the no-allocation batch step are found before any
    member is read or any HIP call is made."""
    cap = _lib.NOALLOC_MAX_SIMS
    step = lib.lbm_batch_step_noalloc
    assert step(None, 1, 1, None) == _lib.LBM_EINVAL
    arr = (ctypes.c_void_p * (cap + 1))()
    assert step(arr, 0, 1, None) == _lib.LBM_EINVAL
    assert step(arr, cap + 1, 1, None) == _lib.LBM_EINVAL
    assert "[1, %d]" % cap in lib.lbm_last_error().decode()
    assert step(arr, 1, -1, None) == _lib.LBM_EINVAL
    assert step(arr, 1, 1, None) == _lib.LBM_EINVAL  # a NULL member
    assert "NULL" in lib.lbm_last_error().decode()


def test_round_f16_stochastic_argument_checks(lib):
    """Argument errors of the rounding entry point are found before any HIP
    call; n = 0 does nothing, whatever the pointers."""
    rnd = lib.lbm_round_f16_stochastic
    assert rnd(None, None, None, 0, None) == _lib.LBM_OK
    assert rnd(None, None, None, -1, None) == _lib.LBM_EINVAL
    assert ">= 0" in lib.lbm_last_error().decode()
    assert rnd(None, None, None, 5, None) == _lib.LBM_EINVAL
    assert "NULL" in lib.lbm_last_error().decode()
