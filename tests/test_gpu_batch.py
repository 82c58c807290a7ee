"""Batched multi-grid stepping and captured step loops (GPU).

* A batch of uneven grids (different sizes, relaxation times and forces) is
  advanced by the persistent multi-grid kernel, one launch per step.  Each
  member equals the same simulation run as a batch of one, bitwise: nothing is
  reduced across cells, so a member's result cannot depend on the others.
* Against the plain single-grid kernel the batch agrees to rounding: the same
  cell update is inlined into two kernels and the compiler may fuse
  multiply-adds differently (measured: <= 1 ulp of the stored value per step).
* FP64 batch members match the CPU oracle (1e-12).
* HIP-graph replays of a step loop equal the same number of eager steps,
  checked after every replay with eager work and synchronisation in between.
* Stale batches and graphs are refused.
"""
import numpy as np
import pytest
import torch

from _parity import gpu_moments, oracle_run, rel_err
from paper_2302_04741_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2302_04741_amd import sim

    return sim


def mix(lattice, storage, seed=0):
    rng = np.random.default_rng(seed)
    dims_list = ([(64, 64, 1), (100, 37, 1), (256, 256, 1), (1024, 16, 1), (3, 5, 1)]
                 if lattice == "D2Q37" else [(16, 16, 16), (40, 9, 23), (64, 64, 32), (7, 5, 3)])
    wls = []
    for k, dims in enumerate(dims_list):
        kind = ["uniform", "axis", "field"][k % 3]
        wl = workloads.random_smooth(lattice, dims, seed=seed * 100 + k, force_kind=kind,
                                     g_amp=1e-3, tau_hat=float(rng.uniform(0.6, 1.0)))
        if k == 1:
            wl.mu = 0.15  # one member with the per-cell relaxation time
        wls.append(wl)
    return wls


@pytest.mark.parametrize("lattice,storage", [("D2Q37", "f32"), ("D3Q39", "f32"),
                                             ("D2Q37", "f64"), ("D3Q39", "f16dev")])
def test_batch_member_independent_of_mix_bitwise(sim_mod, lattice, storage):
    wls = mix(lattice, storage)
    alone = []
    for wl in wls:
        s = sim_mod.from_workload(wl, storage=storage)
        b1 = sim_mod.Batch(1)
        b1.set([s])
        b1.step(13)
        alone.append(s.get_populations().cpu())
        b1.close()
        s.close()
    sims = [sim_mod.from_workload(wl, storage=storage) for wl in wls]
    b = sim_mod.Batch(len(sims))
    b.set(sims)
    b.step(6)
    b.step(7)  # odd counts: the buffer parity is carried between calls
    for s, ref in zip(sims, alone):
        assert s.step_count == 13
        assert torch.equal(s.get_populations().cpu(), ref)


# (threads per block, blocks: 0 = one wavefront per tile, else a persistent grid)
LAUNCHES = [(256, 0), (64, 0), (128, 0), (256, 3), (64, 1000)]


@pytest.mark.parametrize("lattice,storage", [("D2Q37", "f32"), ("D3Q39", "f64")])
def test_batch_launch_shapes_bitwise(sim_mod, lattice, storage):
    wls = mix(lattice, storage, seed=4)
    out = []
    for threads, blocks in LAUNCHES:
        sims = [sim_mod.from_workload(wl, storage=storage) for wl in wls]
        b = sim_mod.Batch(len(sims))
        b.set_launch(threads, blocks)
        b.set(sims)
        b.step(7)
        out.append([s.get_populations().cpu() for s in sims])
        b.close()
        for s in sims:
            s.close()
    for k in range(1, len(LAUNCHES)):
        for a, c in zip(out[0], out[k]):
            assert torch.equal(a, c), LAUNCHES[k]
    # a new launch shape between steps continues from the current state
    sims = [sim_mod.from_workload(wl, storage=storage) for wl in wls]
    b = sim_mod.Batch(len(sims))
    b.set(sims)
    b.step(3)
    b.set_launch(64, 0)
    b.step(4)
    for s, ref in zip(sims, out[0]):
        assert s.step_count == 7
        assert torch.equal(s.get_populations().cpu(), ref)


# stored-value difference allowed between the plain and the batched kernel after
# 13 steps: a few units of the storage precision on values of size <= 1e-2
PLAIN_VS_BATCH = {"f32": 1e-6, "f64": 1e-14, "f16dev": 1e-5}


@pytest.mark.parametrize("lattice,storage", [("D2Q37", "f32"), ("D3Q39", "f64")])
def test_batch_matches_plain_kernel(sim_mod, lattice, storage):
    dt = {"f32": torch.float32, "f64": torch.float64}[storage]
    wls = mix(lattice, storage, seed=2)
    sims = [sim_mod.from_workload(wl, storage=storage) for wl in wls]
    b = sim_mod.Batch(len(sims))
    b.set(sims)
    b.step(13)
    for wl, s in zip(wls, sims):
        p = sim_mod.from_workload(wl, storage=storage)
        p.step(13)
        d = (s.get_populations().view(dt) - p.get_populations().view(dt)).abs().max().item()
        assert d <= PLAIN_VS_BATCH[storage], (wl.dims, d)


def test_batch_fp64_matches_oracle(sim_mod, oracle_mod):
    wls = mix("D2Q37", "f64", seed=3)[:3]
    sims = [sim_mod.from_workload(wl) for wl in wls]
    b = sim_mod.Batch(4)
    b.set(sims)
    b.step(40)
    for wl, s in zip(wls, sims):
        errs = rel_err(gpu_moments(s), oracle_run(oracle_mod, wl, 40).moments())
        assert max(errs) < 1e-12, errs


def test_batch_rejects_stale_and_mixed_members(sim_mod):
    from paper_2302_04741_amd._lib import LbmError

    wls = mix("D2Q37", "f32")[:2]
    a, c = (sim_mod.from_workload(wl, storage="f32") for wl in wls)
    b = sim_mod.Batch(2)
    b.set([a, c])
    a.step(1)  # stepped outside the batch
    with pytest.raises(LbmError):
        b.step(1)
    b.set([a, c])
    b.step(1)
    c.set_force([1e-4, 0.0])
    with pytest.raises(LbmError):
        b.step(1)
    d = sim_mod.from_workload(wls[0], storage="f64")
    with pytest.raises(LbmError):
        b.set([a, d])  # different storage
    with pytest.raises(LbmError):
        b.set([a, a])  # duplicate


@pytest.mark.parametrize("storage", ["f32", "f64", "f16dev"])
def test_graph_replays_equal_eager_steps(sim_mod, storage):
    wl = workloads.random_smooth("D3Q39", (24, 20, 18), seed=4, force_kind="axis", g_amp=1e-3)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ref = sim_mod.from_workload(wl, storage=storage)
        s = sim_mod.from_workload(wl, storage=storage)
        g = sim_mod.Graph(s, 4)
        for rep in range(4):
            g.launch(1)
            ref.step(4)
            torch.cuda.synchronize()
            _ = (ref.get_populations().float().sum()).item()  # eager work between replays
            assert s.step_count == 4 * (rep + 1)
            assert torch.equal(s.get_populations(), ref.get_populations()), rep
        s.step(1)  # odd eager step: the graph's buffers no longer match
        from paper_2302_04741_amd._lib import LbmError

        with pytest.raises(LbmError):
            g.launch(1)
    torch.cuda.synchronize()


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_batch_graph_replays(sim_mod, storage):
    wls = mix("D2Q37", storage, seed=7)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        refs = [sim_mod.from_workload(wl, storage=storage) for wl in wls]
        bref = sim_mod.Batch(len(refs))
        bref.set(refs)
        sims = [sim_mod.from_workload(wl, storage=storage) for wl in wls]
        b = sim_mod.Batch(len(sims))
        b.set(sims)
        g = sim_mod.Graph(b, 6)
        for rep in range(3):
            g.launch(1)
            bref.step(6)  # the same kernel, launched eagerly
            torch.cuda.synchronize()
            for s, r in zip(sims, refs):
                assert torch.equal(s.get_populations(), r.get_populations())
        from paper_2302_04741_amd._lib import LbmError

        b.set_launch(128, 0)  # a new launch shape makes the captured graph stale
        with pytest.raises(LbmError):
            g.launch(1)
    torch.cuda.synchronize()


def test_autotuner_picks_and_caches_launch_shapes(sim_mod, tmp_path, monkeypatch):
    from paper_2302_04741_amd import autotune

    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    b = autotune.tune_block("D3Q39", (64, 48, 40), storage="f32", steps=4)
    assert b in autotune.BLOCK_CANDIDATES
    dims_list = [(100, 37, 1), (64, 64, 1), (257, 9, 1)]
    launch = autotune.tune_batch_launch("D2Q37", dims_list, storage="f32", steps=4)
    assert launch in autotune.BATCH_CANDIDATES
    import json

    cache = json.loads((tmp_path / "tune.json").read_text())
    assert len(cache) == 2 and all("ms_per_step" in v for v in cache.values())
    # kept per device architecture and library build
    assert all("/gfx950/lbm-gfx950 " in k for k in cache), list(cache)
    # a second call is served from the cache (no timing run)
    assert autotune.tune_batch_launch("D2Q37", dims_list, storage="f32") == launch
    # the tuned shape gives the same populations as the default shape
    wls = [workloads.random_smooth("D2Q37", d, seed=k) for k, d in enumerate(dims_list)]
    out = []
    for shape in (None, launch):
        sims = [sim_mod.from_workload(wl, storage="f32") for wl in wls]
        bt = sim_mod.Batch(len(sims))
        if shape:
            bt.set_launch(*shape)
        bt.set(sims)
        bt.step(5)
        out.append([s.get_populations().cpu() for s in sims])
    assert all(torch.equal(a, c) for a, c in zip(*out))
