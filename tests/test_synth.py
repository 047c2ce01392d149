"""The seeded generators: SplitMix64 against its published definition, determinism,
ranges and distributions of the workloads' inputs."""
import numpy as np

import synth

MASK = (1 << 64) - 1


def splitmix64_ref(seed, count):
    """SplitMix64 with Python integers (Steele, Lea, Flood 2014)."""
    out = []
    state = seed & MASK
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & MASK
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        out.append(z ^ (z >> 31))
    return out


def test_splitmix64_matches_definition():
    # first output of the stream seeded with 0 (the generator's usual test vector)
    assert int(synth.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF
    for seed in (0, 1, 12345, 2 ** 63 + 17):
        got = [int(v) for v in synth.splitmix64(seed, 50)]
        assert got == splitmix64_ref(seed, 50)
    # counter-based: any window equals the same outputs of the full stream
    full = synth.splitmix64(99, 1000)
    assert np.array_equal(synth.splitmix64(99, 100, start=400), full[400:500])


def test_deterministic_and_chunk_independent():
    a = synth.uniform_pm1((300, 50), 7)
    b = synth.uniform_pm1((300, 50), 7)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, synth.uniform_pm1((300, 50), 8))
    old = synth._CHUNK
    try:
        synth._CHUNK = 997
        c = synth.uniform_pm1((300, 50), 7)
        w1 = synth.wide_range((40, 30), 3)
    finally:
        synth._CHUNK = old
    assert np.array_equal(a, c)
    assert np.array_equal(w1, synth.wide_range((40, 30), 3))


def test_uniform_range_and_moments():
    x = synth.uniform_pm1((200000,), 1)
    assert x.min() >= -1.0 and x.max() < 1.0
    assert abs(x.mean()) < 0.01
    assert abs(x.var() - 1.0 / 3.0) < 0.01


def test_wide_range_exponents_cover_the_interval():
    x = synth.wide_range((100000,), 2)
    nz = x[x != 0]
    m, e = np.frexp(np.abs(nz))
    # |u| in [0,1) times 2^e, e in [-20, 20]: frexp exponent at most 20
    assert e.max() == 20
    assert np.all(np.abs(x) < 2.0 ** 20)
    # the raw exponents are uniform: check the share of |x| >= 2^19 (needs e = 20
    # and |u| >= 1/2): 1/41 * 1/2
    share = np.mean(np.abs(x) >= 2.0 ** 19)
    assert abs(share - 0.5 / 41) < 0.003


def test_integer_valued_and_log_uniform():
    v = synth.integer_valued((50000,), 3, 8)
    assert np.all(v == np.round(v)) and v.min() == -8 and v.max() == 8
    s = synth.log_uniform_int(20000, 4, 16, 1024)
    assert s.min() >= 16 and s.max() <= 1024
    # log-uniform: about half the mass below the geometric midpoint 128
    assert abs(np.mean(s < 128) - np.log2(128 / 16) / np.log2(1025 / 16)) < 0.02
