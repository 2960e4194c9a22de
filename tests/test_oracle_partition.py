"""Pins of oracle.partition: the layer sizes printed with the experiments
(Sections 3.2, 4.2), the index sets printed in Sections 2.1 and 3.1 (under
the paper's assumption n = 2 gamma + m b - 2), and structural invariants."""
import json
import os

import pytest

from oracle import partition

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_printed_first_and_last_layer_sizes():
    data = json.load(open(os.path.join(GOLDEN, "paper_layer_sizes.json")))
    for case in data["cases"]:
        for n in case["n"]:
            X = partition.layers(n, case["b"], case["gamma"])
            assert X[0][1] - X[0][0] + 1 == case["first"], (case, n)
            assert X[-1][1] - X[-1][0] + 1 == case["last"], (case, n)


@pytest.mark.parametrize("gamma,b,m", [(9, 8, 6), (12, 4, 9), (5, 3, 3), (2, 1, 4)])
def test_printed_index_sets(gamma, b, m):
    n = 2 * gamma + m * b - 2
    X = partition.layers(n, b, gamma)
    assert len(X) == m
    # Section 2 / 3.1: X_1, X_p, X_m
    assert X[0] == (1, gamma + b - 1)
    for p in range(2, m):
        assert X[p - 1] == (gamma + (p - 1) * b, gamma + p * b - 1)
    assert X[-1] == (gamma + (m - 1) * b, 2 * gamma + m * b - 2)
    subs = partition.subproblems(n, b, gamma)
    # X^M_q = {(q-1)b+1 <= i <= 2 gamma + q b - 2}  (Section 2.1)
    for s in subs["M"]:
        q = s.p
        assert (s.lo, s.hi) == ((q - 1) * b + 1, 2 * gamma + q * b - 2)
    # X^R_p = {gamma + (p-1)b <= i <= 2 gamma + p b - 2}, p = 2..m
    assert [s.p for s in subs["R"]] == list(range(2, m + 1))
    for s in subs["R"]:
        p = s.p
        assert (s.lo, s.hi) == (gamma + (p - 1) * b, 2 * gamma + p * b - 2)
        # left boundary of D^R_p is at x = eta + ((p-1)b - 1)h, i.e. the last line of X_{p-1}
        assert s.lo - 1 == gamma + (p - 1) * b - 1 == X[p - 2][1]
    # X^L_p = {(p-1)b+1 <= i <= gamma + p b - 1}, p = 1..m-1
    assert [s.p for s in subs["L"]] == list(range(1, m))
    for s in subs["L"]:
        p = s.p
        assert (s.lo, s.hi) == ((p - 1) * b + 1, gamma + p * b - 1)
        # right boundary of D^L_p is at x = eta + p b h, i.e. the first line of X_{p+1}
        assert s.hi + 1 == gamma + p * b == X[p][0]
    # X^R_m = X_m and X^L_1 = X_1
    assert (subs["R"][-1].lo, subs["R"][-1].hi) == X[-1]
    assert (subs["L"][0].lo, subs["L"][0].hi) == X[0]


@pytest.mark.parametrize("n", [63, 64, 65, 66, 127, 511, 1023, 31, 39, 79, 159])
@pytest.mark.parametrize("gamma,b", [(12, 4), (9, 8), (8, 4), (9, 4), (3, 5)])
def test_partition_invariants(n, gamma, b):
    if n - 2 * (gamma - 1) < 1:
        pytest.skip("grid too small for the PML")
    X = partition.layers(n, b, gamma)
    m = len(X)
    # contiguous, disjoint, covering 1..n
    assert X[0][0] == 1 and X[-1][1] == n
    for a, c in zip(X, X[1:]):
        assert c[0] == a[1] + 1
    # every layer holds physical lines; interior layers exactly b of them
    g = gamma - 1
    for p, (s_p, e_p) in enumerate(X, start=1):
        phi, psi = partition.physical(n, gamma, (s_p, e_p))
        assert 1 <= psi - phi + 1 <= b
        if 1 < p < m:
            assert e_p - s_p + 1 == b
    subs = partition.subproblems(n, b, gamma)
    for s in subs["M"] + subs["R"] + subs["L"]:
        assert 1 <= s.lo <= s.hi <= n
        s_p, e_p = X[s.p - 1]
        assert s.lo <= s_p and e_p <= s.hi       # the extended grid contains X_p
    for s in subs["M"]:
        assert s.L == (s.psi - s.phi + 1) + 2 * g
    for s in subs["R"]:
        assert s.lo - 1 == X[s.p - 2][1]
    for s in subs["L"]:
        assert s.hi + 1 == X[s.p][0]


def test_single_layer_and_invalid():
    X = partition.layers(30, 8, 12)     # n_phys = 8 <= b
    assert X == [(1, 30)]
    subs = partition.subproblems(30, 8, 12)
    assert [(s.lo, s.hi) for s in subs["M"]] == [(1, 30)]
    assert subs["R"] == [] and subs["L"] == []
    for bad in [(20, 4, 12), (63, 0, 12), (63, 4, 1)]:
        with pytest.raises(ValueError):
            partition.layers(*bad)


@pytest.mark.parametrize("n,gamma,gamma_aux,b", [(63, 9, 5, 4), (127, 9, 5, 8), (66, 12, 4, 4),
                                                 (40, 6, 2, 5)])
def test_thin_auxiliary_pads(n, gamma, gamma_aux, b):
    """Thinner auxiliary PML (Section 3.1 remarks): a pad facing a neighbouring
    layer has gamma_aux - 1 lines and width gamma_aux, a pad at the boundary of
    the domain is the boundary PML (gamma - 1 lines, width gamma); the zero
    regions and the layers do not change."""
    g, ga = gamma - 1, gamma_aux - 1
    base = partition.subproblems(n, b, gamma)
    thin = partition.subproblems(n, b, gamma, gamma_aux)
    m = len(partition.layers(n, b, gamma))
    for kind in "MRL":
        for s0, s in zip(base[kind], thin[kind]):
            assert (s.kind, s.p, s.phi, s.psi) == (s0.kind, s0.p, s0.phi, s0.psi)
    for s in thin["M"]:
        assert s.phi - s.lo == (g if s.p == 1 else ga)
        assert s.hi - s.psi == (g if s.p == m else ga)
        assert (s.gamma_lo, s.gamma_hi) == (gamma if s.p == 1 else gamma_aux,
                                            gamma if s.p == m else gamma_aux)
    for s in thin["R"]:
        assert s.lo == s.phi + 1 and s.hi - s.psi == (g if s.p == m else ga)
        assert s.gamma_hi == (gamma if s.p == m else gamma_aux)
    for s in thin["L"]:
        assert s.hi == s.psi - 1 and s.phi - s.lo == (g if s.p == 1 else ga)
        assert s.gamma_lo == (gamma if s.p == 1 else gamma_aux)
    # gamma_aux = gamma is the default partition
    same = partition.subproblems(n, b, gamma, gamma)
    for kind in "MRL":
        assert [(s.lo, s.hi, s.phi, s.psi) for s in same[kind]] == \
               [(s.lo, s.hi, s.phi, s.psi) for s in base[kind]]


def test_thin_auxiliary_sizes_at_the_3d_settings():
    """Section 4.2's 3D settings (eta = 9h, eta_aux = 5h, b = 4): interior
    M-problems span b + 2 (gamma_aux - 1) = 12 lines, interior R/L problems 8,
    the first M-problem g + b + 4 = 16."""
    n = 79
    subs = partition.subproblems(n, 4, 9, 5)
    assert subs["M"][0].L == 16 and all(s.L == 12 for s in subs["M"][1:-2])
    assert all(s.L == 8 for s in subs["R"][:-1]) and all(s.L == 8 for s in subs["L"][1:])
    with pytest.raises(ValueError):
        partition.subproblems(n, 4, 9, 10)


@pytest.mark.parametrize("n,b,gamma", [(63, 4, 12), (127, 8, 9), (100, 4, 12), (30, 8, 12),
                                       (2 * 9 + 6 * 8 - 2, 8, 9)])
def test_uniform_widths_list_is_the_uniform_partition(n, b, gamma):
    """Arbitrary widths (Section 3.1 remarks) with the list (b, ..., b, r)
    reproduce the uniform partition, whose index sets are pinned above."""
    w = partition.widths(n, b, gamma)
    assert w[:-1] == [b] * (len(w) - 1) and 1 <= w[-1] <= b and sum(w) == n - 2 * (gamma - 1)
    assert partition.layers(n, w, gamma) == partition.layers(n, b, gamma)
    for kind in "MRL":
        assert partition.subproblems(n, w, gamma)[kind] == partition.subproblems(n, b, gamma)[kind]


@pytest.mark.parametrize("n,gamma,w", [(40, 6, [3, 7, 1, 5, 6, 8]), (63, 12, [1, 1, 9, 2, 4, 24]),
                                       (30, 5, [22]), (31, 9, [1, 14])])
def test_arbitrary_layer_widths(n, gamma, w):
    """Layers of the given physical widths tile [1, n]; layer 1 also holds the
    lower PML, layer m the upper one; the auxiliary grids follow the same
    definitions as for equal widths (zero regions on each layer's physical part)."""
    g = gamma - 1
    X = partition.layers(n, w, gamma)
    assert len(X) == len(w) and X[0][0] == 1 and X[-1][1] == n
    for p in range(1, len(X)):
        assert X[p][0] == X[p - 1][1] + 1
    for p, (s, e) in enumerate(X):
        phi, psi = partition.physical(n, gamma, (s, e))
        assert psi - phi + 1 == w[p]
    assert X[0][1] - X[0][0] + 1 == w[0] + g * (1 if len(w) > 1 else 2)
    subs = partition.subproblems(n, w, gamma)
    m = len(X)
    for s in subs["M"]:
        assert (s.phi, s.psi) == partition.physical(n, gamma, X[s.p - 1])
        assert (s.phi - s.lo, s.hi - s.psi) == (g, g)
    for s in subs["R"]:
        assert s.lo == X[s.p - 1][0] and s.phi == s.lo - 1
    for s in subs["L"]:
        assert s.hi == X[s.p - 1][1] and s.psi == s.hi + 1
    assert len(subs["R"]) == len(subs["L"]) == m - 1


@pytest.mark.parametrize("n,gamma,w", [(40, 6, [3, 7, 1, 5, 6, 7]), (40, 6, [3, 0, 27]),
                                       (40, 6, []), (40, 6, [31, -1])])
def test_bad_layer_widths(n, gamma, w):
    with pytest.raises(ValueError):
        partition.layers(n, w, gamma)
