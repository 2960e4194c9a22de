"""The seeded input generators are deterministic and have the documented shapes."""
import math

import numpy as np

import workloads


def test_named_workloads_shapes_and_determinism():
    for name, n, nrhs in [("2d_n63_const", 63, 1), ("2d_n511_lens", 31, 3), ("3d_n63_lens", 9, 2),
                          ("2d_n1023_random", 47, 2)]:
        a = workloads.workload(name, n=n, nrhs=nrhs)
        b = workloads.workload(name, n=n, nrhs=nrhs)
        assert a["c"].shape == (n,) * a["d"]
        assert a["f"].shape == (nrhs, n ** a["d"]) and a["f"].dtype == np.complex128
        assert np.array_equal(a["c"], b["c"]) and np.array_equal(a["f"], b["f"])
        assert np.all(a["c"] > 0)


def test_field_ranges_and_source_peak():
    c = workloads.velocity_random(64, 2, seed=3)
    assert abs(c.min() - 0.8) < 1e-12 and abs(c.max() - 1.2) < 1e-12
    lens = workloads.velocity_lens2d(63)
    assert lens.min() > 2 / 3 - 1e-9 and lens.max() < 4 / 3
    n = 63
    f = workloads.gaussian_source(n, 2, 2 * math.pi * 8, (32 / 64, 16 / 64))
    assert f[31, 15] == 1.0 and f.max() == 1.0
    # column-major flattening: first index fastest
    a = np.arange(6).reshape(2, 3)
    assert list(workloads.flat(a)) == [0, 3, 1, 4, 2, 5]
