"""The F16 storage's stochastic rounding (lbm_round_f16_stochastic, the
conversion the step uses for every F16 store), checked against its definition:

* normal half range: exactly the bit-level rule -- add the seed's top 13 bits
  to the FP32 pattern below the 13 bits binary16 drops, then drop them --
  computed here in numpy from the definition;
* values a half holds exactly (zero, normal and subnormal halves) come back
  unchanged for every seed;
* below 2^-14: every result is one of the two neighbouring multiples of 2^-24,
  and the up-rounding frequency over many seeds equals the value's fraction of
  the spacing (within 5 standard deviations), so the error has zero mean;
* the same inputs give the same bits (the step's determinism rests on it).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sim_mod():
    from paper_2302_04741_amd import sim

    return sim


def run(sim_mod, v, seed):
    vt = torch.from_numpy(v).cuda()
    st = torch.from_numpy(seed.view(np.int32)).cuda()
    out = sim_mod.round_f16_stochastic(vt, st)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_normal_range_equals_bit_rule(sim_mod):
    rng = np.random.default_rng(4741)
    n = 1 << 18
    e = rng.integers(-14, 15, n)  # |v| in [2^-14, 2^15): results stay finite
    mant = rng.integers(0, 1 << 23, n, dtype=np.uint32)
    sign = rng.integers(0, 2, n, dtype=np.uint32) << np.uint32(31)
    bits = sign | ((e + 127).astype(np.uint32) << np.uint32(23)) | mant
    v = bits.view(np.float32)
    seed = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    mag = ((bits & np.uint32(0x7FFFFFFF)) + (seed >> np.uint32(19))) & np.uint32(0xFFFFE000)
    want = (mag | sign).view(np.float32).astype(np.float16)  # exact: a half already
    got = run(sim_mod, v, seed)
    bad = np.flatnonzero(got.view(np.uint16) != want.view(np.uint16))
    assert bad.size == 0, (bad[:5], v[bad[:5]], seed[bad[:5]], got[bad[:5]], want[bad[:5]])
    assert np.array_equal(run(sim_mod, v, seed).view(np.uint16), got.view(np.uint16))


def test_representable_values_unchanged(sim_mod):
    rng = np.random.default_rng(7)
    halves = np.concatenate([
        np.array([0.0, 1.0, -1.0, 2.0 ** -24, -(2.0 ** -24), 2.0 ** -14, 65504.0], np.float16),
        rng.integers(0, 0x7C00, 4096, dtype=np.uint16).view(np.float16),  # finite positive
        (rng.integers(0, 0x7C00, 4096, dtype=np.uint16) | np.uint16(0x8000)).view(np.float16),
    ])
    v = np.repeat(halves.astype(np.float32), 16)
    seed = rng.integers(0, 1 << 32, v.size, dtype=np.uint64).astype(np.uint32)
    got = run(sim_mod, v, seed)
    assert np.array_equal(got.astype(np.float32), v)


def test_subnormal_range_unbiased(sim_mod):
    rng = np.random.default_rng(11)
    q = 2.0 ** -24
    # 24 values below 2^-14 at spread fractions of the spacing, both signs
    k = rng.integers(0, 1 << 10, 24)
    frac = np.linspace(0.03, 0.97, 24)
    vals = ((k + frac) * q * np.where(np.arange(24) % 2 == 0, 1.0, -1.0)).astype(np.float32)
    reps = 1 << 15
    v = np.repeat(vals, reps)
    seed = rng.integers(0, 1 << 32, v.size, dtype=np.uint64).astype(np.uint32)
    got = run(sim_mod, v, seed).astype(np.float64).reshape(24, reps)
    for j, x in enumerate(vals.astype(np.float64)):
        lo, hi = np.floor(abs(x) / q) * q, np.ceil(abs(x) / q) * q
        mags = np.abs(got[j])
        assert np.all((mags == lo) | (mags == hi)), (x, np.unique(mags)[:4])
        assert np.all(np.sign(got[j][mags > 0]) == np.sign(x))
        f = (abs(x) - lo) / q
        p_up = float((mags == hi).mean())
        sigma = np.sqrt(f * (1 - f) / reps)
        assert abs(p_up - f) <= 5 * sigma, (x, f, p_up, sigma)
