"""The batch step for callers that cannot allocate (lbm_batch_step_noalloc),
called through the C ABI, against the existing entry point lbm_batch_step on
the same seeded members: bitwise the same populations and step counts, on two
calls in a row, the second with fewer and smaller members (the fixed tile
table keeps the first call's contents, which must not leak into the second),
and for a member count above the table's capacity a clear error."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2302_04741_amd import _lib, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2302_04741_amd import sim

    return sim


def members(lattice, dims_list, seed):
    rng = np.random.default_rng(seed)
    wls = []
    for k, dims in enumerate(dims_list):
        kind = ["uniform", "axis", "field"][k % 3]
        wl = workloads.random_smooth(lattice, dims, seed=seed * 100 + k, force_kind=kind,
                                     g_amp=1e-3, tau_hat=float(rng.uniform(0.6, 1.0)))
        if k == 1:
            wl.mu = 0.15  # one member with the per-cell relaxation time
        wls.append(wl)
    return wls


def via_batch(sim_mod, wls, storage, steps):
    sims = [sim_mod.from_workload(wl, storage=storage) for wl in wls]
    b = sim_mod.Batch(len(sims))
    b.set(sims)
    b.step(steps)
    out = [(s.step_count, s.get_populations().cpu()) for s in sims]
    b.close()
    for s in sims:
        s.close()
    return out


def via_noalloc(sim_mod, wls, storage, steps):
    sims = [sim_mod.from_workload(wl, storage=storage) for wl in wls]
    stream = torch.cuda.current_stream()
    arr = (ctypes.c_void_p * len(sims))(*[s.handle.value for s in sims])
    _lib.check(_lib.load().lbm_batch_step_noalloc(arr, len(sims), int(steps),
                                                  ctypes.c_void_p(stream.cuda_stream)))
    out = [(s.step_count, s.get_populations().cpu()) for s in sims]
    for s in sims:
        s.close()
    return out


# first call: more and larger members; second call: fewer, smaller ones
CASES = [
    ("D2Q37", "f32", [(256, 256, 1), (100, 37, 1), (1024, 16, 1), (64, 64, 1), (3, 5, 1),
                      (130, 70, 1)], [(64, 48, 1), (9, 7, 1)]),
    ("D3Q39", "f64", [(40, 9, 23), (16, 16, 16), (64, 64, 32), (7, 5, 3)], [(12, 10, 14)]),
    ("D3Q39", "f16dev", [(64, 64, 32), (40, 9, 23), (33, 17, 5)], [(16, 16, 16), (5, 4, 3)]),
]


@pytest.mark.parametrize("lattice,storage,first,second", CASES)
def test_noalloc_equals_batch_step_twice(sim_mod, lattice, storage, first, second):
    for call, dims_list, steps in ((1, first, 13), (2, second, 6)):
        print("noalloc case %s %s call %d dims %s steps %d" % (lattice, storage, call, dims_list,
                                                               steps), flush=True)
        wls = members(lattice, dims_list, seed=call)
        ref = via_batch(sim_mod, wls, storage, steps)
        got = via_noalloc(sim_mod, wls, storage, steps)
        for (n_ref, p_ref), (n_got, p_got), dims in zip(ref, got, dims_list):
            assert n_got == n_ref == steps, dims
            assert torch.equal(p_got, p_ref), (call, dims)


def test_noalloc_many_members_and_capacity(sim_mod):
    """More members than one table-fill launch carries (16), then the limit:
    a count above LBM_NOALLOC_MAX_SIMS is refused before anything runs."""
    dims_list = [(8 + 3 * k, 5 + k % 4, 1) for k in range(37)]
    wls = members("D2Q37", dims_list, seed=5)
    ref = via_batch(sim_mod, wls, "f32", 5)
    got = via_noalloc(sim_mod, wls, "f32", 5)
    for (n_ref, p_ref), (n_got, p_got) in zip(ref, got):
        assert n_got == n_ref == 5
        assert torch.equal(p_got, p_ref)
    s = sim_mod.from_workload(wls[0], storage="f32")
    L = _lib.load()
    cap = _lib.NOALLOC_MAX_SIMS
    arr = (ctypes.c_void_p * (cap + 1))(*([s.handle.value] * (cap + 1)))
    st = L.lbm_batch_step_noalloc(arr, cap + 1, 1, None)
    assert st == _lib.LBM_EINVAL
    assert str(cap) in L.lbm_last_error().decode()
    assert s.step_count == 0
    s.close()


def test_noalloc_python_wrapper_streams(sim_mod):
    """The binding orders the call after members living on another stream."""
    wls = members("D2Q37", [(64, 64, 1), (100, 37, 1)], seed=9)
    ref = via_batch(sim_mod, wls, "f32", 8)
    side = torch.cuda.Stream()
    sims = [sim_mod.from_workload(wl, storage="f32", stream=side) for wl in wls]
    sim_mod.batch_step_noalloc(sims, 8)
    for s, (n_ref, p_ref) in zip(sims, ref):
        assert s.step_count == n_ref
        assert torch.equal(s.get_populations().cpu(), p_ref)
        s.close()
