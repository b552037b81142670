"""The seeded input generators: determinism and the constraints the workloads state."""

import numpy as np

import synth


def test_splitmix64_reference_outputs():
    # SplitMix64 with state 0: the first outputs of the published generator.
    z = synth.splitmix64(0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_direction_numbers_odd_and_bounded():
    m = synth.sobol_direction_init(64, 0).astype(np.uint64)
    assert np.all(m & np.uint64(1) == 1)
    for k in range(synth.MAX_DEGREE):
        assert np.all(m[:, k] < np.uint64(1 << (k + 1)))
    assert np.array_equal(m, synth.sobol_direction_init(64, 0).astype(np.uint64))


def test_lattice_vectors_odd_in_range_without_duplicates_or_mirrors():
    for s, bits in ((32, 20), (64, 30)):
        g = synth.lattice_vector(s, bits, 3).astype(np.int64)
        assert np.all(g % 2 == 1) and np.all(g >= 1) and np.all(g < 1 << bits)
        n = 1 << bits
        assert np.unique(g).size == s
        mirrored = set(int(n - v) for v in g)
        assert not mirrored & set(int(v) for v in g)


def test_count_maps():
    c = synth.counts_pow2(1920, 1080, 5)
    assert c.size == 1920 * 1080
    assert set(np.unique(c)) <= {1 << k for k in range(9)}
    assert len(np.unique(c)) == 9
    cp = synth.counts_progressive(3840, 2160, 5)
    assert cp.min() >= 64 and cp.max() <= 1024 and np.all(cp % 64 == 0)


def test_parameter_ranges():
    pp = synth.genz_params(1000, 4)
    assert pp.dtype == np.float32 and np.all((pp[:, :8] >= 0) & (pp[:, :8] < 1))
    assert np.all((pp[:, 8:] >= 2) & (pp[:, 8:] <= 20))
    th = synth.lobe_params(64, 8, 6)
    assert th.size == 64 * 17 and th.dtype == np.float32
    sig = np.exp(th[64 * 8:128 * 8].astype(np.float64))
    assert np.all((sig > 0.0999) & (sig < 0.5001))
    idx = synth.pick(1088, 16, 8)
    assert idx.size == 16 and np.unique(idx).size == 16 and idx.max() < 1088
