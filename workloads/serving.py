"""Seeded request streams for served solves.

A stream is a list of request descriptions ordered by arrival time:

* arrivals form a Poisson process of the given rate (exponential gaps, NumPy
  PCG64 with a fixed seed);
* with probability ``repeat`` a request reuses the problem (velocity, omega, n)
  of a uniformly drawn earlier request; otherwise it draws a problem not seen
  before: a dimension (uniform over those present in ``sizes``), a grid of that
  dimension, omega = 2 pi n / 8, a velocity family from constant / lens /
  random (a random field gets a fresh seed; a draw equal to an earlier problem
  is drawn again);
* the number of right-hand sides is uniform on 1..max_rhs; each right-hand side
  is a Gaussian point source at a seeded point of [0.2, 0.8]^d.

Descriptions are plain dicts; ``materialize`` builds the velocity and sources
of one of them.  Nothing here knows about PML, layers or solvers.
"""
import math

import numpy as np

from .fields import (flat, gaussian_source, seeded_centres, velocity_constant,
                     velocity_lens2d, velocity_lens3d, velocity_random)

FAMILIES = ("constant", "lens", "random")


def request_stream(count=2000, rate=50.0, seed=5, sizes=((2, 127), (2, 255), (2, 511), (2, 1023),
                                                        (3, 31), (3, 63)),
                   max_rhs=32, repeat=0.5, pml_gamma=None, layer_b=4):
    """``count`` request descriptions with keys rid, arrival (s), key, d, n, omega,
    family, velocity_seed, nrhs, source_seed, gamma, b."""
    rng = np.random.default_rng(seed)
    dims = sorted({d for d, _ in sizes})
    by_dim = {d: [n for dd, n in sizes if dd == d] for d in dims}
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    problems, seen = [], set()
    out = []
    for rid in range(count):
        if problems and rng.random() < repeat:
            prob = problems[int(rng.integers(len(problems)))]
        else:
            while True:       # a new problem: redraw while it equals an earlier one
                d = dims[int(rng.integers(len(dims)))]
                n = by_dim[d][int(rng.integers(len(by_dim[d])))]
                fam = FAMILIES[int(rng.integers(len(FAMILIES)))]
                vseed = int(rng.integers(1 << 30)) if fam == "random" else 0
                gamma = pml_gamma if pml_gamma is not None else (12 if d == 2 else 8)
                prob = dict(d=d, n=n, omega=2 * math.pi * n / 8, family=fam, velocity_seed=vseed,
                            gamma=gamma, b=layer_b)
                if _key(prob) not in seen:
                    break
            seen.add(_key(prob))
            problems.append(prob)
        nrhs = int(rng.integers(1, max_rhs + 1))
        out.append(dict(prob, rid=rid, arrival=float(arrivals[rid]), key=_key(prob), nrhs=nrhs,
                        source_seed=int(rng.integers(1 << 30))))
    return out


def _key(prob):
    return (prob["d"], prob["n"], prob["omega"], prob["family"], prob["velocity_seed"],
            prob["gamma"], prob["b"])


def velocity_of(desc):
    d, n, fam = desc["d"], desc["n"], desc["family"]
    if fam == "constant":
        return velocity_constant(n, d)
    if fam == "lens":
        return velocity_lens2d(n) if d == 2 else velocity_lens3d(n)
    if fam == "random":
        return velocity_random(n, d, desc["velocity_seed"])
    raise ValueError(f"unknown velocity family {fam!r}")


def sources_of(desc):
    """(nrhs, n**d) complex128 Gaussian sources, each row column-major."""
    d, n = desc["d"], desc["n"]
    cents = seeded_centres(desc["nrhs"], d, desc["source_seed"])
    out = np.zeros((len(cents), n ** d), dtype=np.complex128)
    t = np.arange(1, n + 1, dtype=np.float64) / (n + 1)
    a = 4.0 * desc["omega"] / math.pi
    for k, x0 in enumerate(cents):
        # gaussian_source's factors and products, built with the last axis
        # outermost so that C order is the column-major order of the grid
        g = np.exp(-(a * a) * (t - x0[0]) ** 2)
        for c in x0[1:d]:
            g = np.multiply.outer(np.exp(-(a * a) * (t - c) ** 2), g)
        out[k].real = g.reshape(-1)
    return out


def materialize(desc):
    """(velocity (n,)*d float64, sources (nrhs, n**d) complex128)."""
    return velocity_of(desc), sources_of(desc)
