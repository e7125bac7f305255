"""Seeded input generator: published SplitMix64 values, an independent numpy
re-implementation, distributions, the derived a3 and bnd arrays, batch sizes."""
import numpy as np
import pytest

from paper_2002_12115_amd import inputs

GAMMA = np.uint64(0x9E3779B97F4A7C15)


def np_mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def np_uniform(seed, fid, n):
    state = np_mix(np.uint64(seed)) ^ (np.uint64(fid) << np.uint64(56))
    with np.errstate(over="ignore"):
        x = np_mix(state + (np.asarray(n, np.uint64) + np.uint64(1)) * GAMMA)
    return (x >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def test_splitmix64_published_sequence():
    # SplitMix64 started from state 0 (reference implementation by Vigna,
    # after Steele, Lea and Flood 2014): first three outputs.
    assert inputs.bits(0, 0, 0) == 0xE220A8397B1DCDAF
    assert inputs.bits(0, 0, 1) == 0x6E789E6AA1B965F4
    assert inputs.bits(0, 0, 2) == 0x06C45D188009454F


def test_mix_matches_numpy():
    for z in (0, 1, 12345, 2**63 + 17, 2**64 - 1):
        assert inputs.mix(z) == int(np_mix(np.uint64(z)))


@pytest.mark.parametrize("seed", [2002, 1, 7])
def test_uniform_fields_match_numpy(seed):
    shape = (5, 6, 7)
    n = np.arange(np.prod(shape))
    u = np_uniform(seed, 0, n).reshape(shape)
    assert np.array_equal(inputs.field(seed, "p", shape), u)
    a1 = 0.9 + 0.2 * np_uniform(seed, 2, n).reshape(shape)
    assert np.array_equal(inputs.field(seed, "a1", shape), a1)
    b2 = -0.05 + 0.1 * np_uniform(seed, 7, n).reshape(shape)
    assert np.array_equal(inputs.field(seed, "b2", shape), b2)


def test_normals_box_muller():
    shape = (4, 4, 6)
    n = np.arange(np.prod(shape))
    m = n // 2
    u0 = np_uniform(2002, 12, 2 * m)
    u1 = np_uniform(2002, 12, 2 * m + 1)
    r = np.sqrt(-2.0 * np.log(1.0 - u0))
    t = 2 * np.pi * u1
    z = np.where(n % 2 == 1, r * np.sin(t), r * np.cos(t)) * 0.01
    got = inputs.field(2002, "wrk1", shape).ravel()
    np.testing.assert_allclose(got, z, rtol=1e-14, atol=1e-18)


def test_distributions():
    shape = (40, 40, 40)
    f = inputs.fields(2002, shape)
    p = f["p"]
    assert 0.0 <= p.min() and p.max() < 1.0
    assert abs(p.mean() - 0.5) < 0.005 and abs(p.var() - 1 / 12) < 0.002
    for name in ("a0", "a1", "a2", "c0", "c1", "c2"):
        assert 0.9 <= f[name].min() and f[name].max() < 1.1
        assert abs(f[name].mean() - 1.0) < 0.002
    for name in ("b0", "b1", "b2"):
        assert -0.05 <= f[name].min() and f[name].max() < 0.05
        assert abs(f[name].mean()) < 0.001
    w = f["wrk1"]
    assert abs(w.mean()) < 2e-4 and abs(w.std() - 0.01) < 2e-4
    # distinct fields are distinct streams
    assert not np.array_equal(f["a0"], f["a1"])


def test_a3_and_bnd_derived():
    shape = (6, 7, 9)
    f = inputs.fields(7, shape)
    sa = (f["a0"] + f["a1"]) + f["a2"]
    sc = (f["c0"] + f["c1"]) + f["c2"]
    sb = (np.abs(f["b0"]) + np.abs(f["b1"])) + np.abs(f["b2"])
    a3 = 1.0 / (((sa + sc) + 4.0 * sb) + 0.1)
    assert np.array_equal(f["a3"], a3)
    bnd = np.zeros(shape)
    bnd[1:-1, 1:-1, 1:-1] = 1.0
    assert np.array_equal(f["bnd"], bnd)
    rb = inputs.field(7, "bnd", shape, bnd_mode=1)
    assert np.all(rb[bnd == 0] == 0) and set(np.unique(rb[1:-1, 1:-1, 1:-1])) <= {0.0, 1.0}
    assert 0 < rb.sum() < bnd.sum()


def test_f32_is_rne_of_f64():
    shape = (5, 5, 9)
    for name in inputs.INPUTS:
        d = inputs.field(2002, name, shape)
        s = inputs.field(2002, name, shape, dtype=np.float32)
        assert np.array_equal(s, d.astype(np.float32))


def test_deterministic():
    a = inputs.fields(1, (8, 9, 10))
    b = inputs.fields(1, (8, 9, 10))
    for n in a:
        assert np.array_equal(a[n], b[n])


def test_batch_shapes():
    shapes, seeds = inputs.batch_shapes(2002, 64)
    assert len(shapes) == 64 and len(set(seeds)) == 64
    for nx, ny, nz in shapes:
        assert 17 <= nx <= 129 and 17 <= ny <= 129 and 33 <= nz <= 257
    assert shapes == inputs.batch_shapes(2002, 64)[0]
    assert len(set(shapes)) > 50


def test_bad_field_rejected():
    with pytest.raises(ValueError):
        inputs.field(1, 13, (3, 3, 3))
