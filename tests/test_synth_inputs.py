"""The seeded input generators (synth): the counter-based generator the
library's initialisers also draw from, against its published outputs."""
import numpy as np

import synth


def test_splitmix64_published_outputs():
    """splitmix64 from state 0 (Steele, Lea & Flood, OOPSLA 2014; the
    reference generator used to seed the xoshiro family) yields
    0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F; synth takes
    the top 53 bits of output c + 1 as cell c's uniform value."""
    u = synth.splitmix_uniform(3, 0)
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [int(v * 2.0 ** 53) for v in u] == [w >> 11 for w in want]


def test_splitmix_noise_range_and_independence_of_cells():
    n = 100000
    u = synth.splitmix_uniform(n, synth.SEED)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5e-3 and abs(u.var() - 1.0 / 12.0) < 5e-3
    assert abs(np.corrcoef(u[:-1], u[1:])[0, 1]) < 2e-2
    # counter-based: a prefix is the same whatever the length drawn
    assert np.array_equal(synth.splitmix_uniform(10, 7), synth.splitmix_uniform(1000, 7)[:10])
    x = synth.splitmix_noise((2, 3, 5), 1e-3, 11)
    assert x.shape == (2, 3, 5) and np.abs(x).max() < 1e-3
