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


def test_paper_recipes():
    """The stand-ins for the paper's figure-only fields and forces: the
    waveguide is slowest on x1 = 1/2 and constant along x2; the packet peaks
    at its centre with unit modulus and its phase advances along (1, 1)."""
    import math

    n = 63
    c = workloads.velocity_waveguide2d(n)
    h = 1.0 / (n + 1)
    assert np.allclose(c, c[:, :1])                       # no x2 dependence
    assert abs(c[31, 0] - (4 / 3) * (1 - 0.5)) < 1e-12    # x1 = 32 h = 1/2
    w = workloads.paper_workload("lens", n)
    assert w["omega"] == 2 * math.pi * 8 and w["gamma"] == 9 and w["b"] == 8
    assert w["restart"] == 40 and w["tol"] == 1e-3 and w["f"].shape == (2, n * n)
    fb = w["f"][1].reshape(n, n, order="F")
    i0 = round(0.125 / h) - 1                              # grid point at 1/8
    assert abs(abs(fb[i0, i0]) - 1.0) < 1e-12
    ph = np.angle(fb[i0 + 1, i0 + 1] / fb[i0, i0])
    assert abs(ph - w["omega"] * 2 * h / math.sqrt(2)) < 1e-9


def test_variation_widths():
    """Unequal layer widths recipe: NARROW/WIDE layers tiling the physical
    lines; wide layers across the lens (where c varies along the sweep axis),
    narrow ones where it does not (the waveguide is constant along it)."""
    for field in workloads.PAPER_FIELDS:
        w = workloads.paper_workload(field, 127)
        ws = workloads.variation_widths(w["c"], 9, 4, 16)
        assert sum(ws) == 127 - 16 and all(1 <= x <= 16 for x in ws)
        assert all(x in (4, 16) for x in ws[:-1])
    lens = workloads.variation_widths(workloads.velocity_lens2d(127), 9, 4, 16)
    assert 16 in lens and lens[0] == 4 and lens[-2] == 4
    guide = workloads.variation_widths(workloads.velocity_waveguide2d(127), 9, 4, 16)
    assert guide[:-1] == [4] * (len(guide) - 1)
