"""Velocity fields and sources for the synthetic Helmholtz workloads.

The paper shows its velocity fields (a converging Gaussian lens, a Gaussian
waveguide, a random field) only as figures and gives no formulas for them
(Sections 3.2 and 4.2), so the fields below are explicit, seeded stand-ins:

* constant:   c = 1
* lens (2D):  c = (4/3) (1 - 0.5 exp(-32 |x - (1/2, 1/2)|^2))
* lens (3D):  c = 1 + 0.3 exp(-32 |x - (1/2, 1/2, 1/2)|^2)
* random:     i.i.d. N(0,1) samples on the grid (NumPy PCG64, fixed seed),
              Gaussian-smoothed with standard deviation ``width`` grid cells
              (reflecting boundary, truncated at 4 standard deviations), then
              mapped affinely so that min -> 0.8 and max -> 1.2
* waveguide (2D): c = (4/3) (1 - 0.5 exp(-32 (x1 - 1/2)^2)), a slow channel
              along x2 (the vertical axis of the paper's figures)
* paper 3D fields: lens c = (4/3) (1 - 0.5 exp(-32 |x - (1/2, 1/2, 1/2)|^2)),
              waveguide c = (4/3) (1 - 0.5 exp(-32 ((x1 - 1/2)^2 + (x2 - 1/2)^2)))
              (a slow channel along x3), random as above with a correlation
              width of (n + 1) / 16 cells
* source:     f = exp(-(4 omega / pi)^2 |x - x0|^2), a Gaussian point source
              whose width shrinks with the wavelength.
* packet:     f = exp(-|x - x0|^2 / (2 lambda^2)) exp(i omega d.(x - x0)) with
              lambda = 2 pi / omega (one wavelength), a Gaussian wave packet
              travelling along the unit vector d.

Nothing here knows about PML, layers or solvers.
"""
import math

import numpy as np


def grid_coords(n, d):
    """Coordinates of the interior grid points, one array per axis, shape (n,)*d.

    Point (i1, ..., id) sits at (i1*h, ..., id*h) with h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    t = np.arange(1, n + 1, dtype=np.float64) * h
    return np.meshgrid(*([t] * d), indexing="ij")


def flat(a):
    """Column-major flattening (first index fastest)."""
    return np.asarray(a).reshape(-1, order="F")


def velocity_constant(n, d, value=1.0):
    return np.full((n,) * d, float(value))


def velocity_lens2d(n):
    x1, x2 = grid_coords(n, 2)
    r2 = (x1 - 0.5) ** 2 + (x2 - 0.5) ** 2
    return (4.0 / 3.0) * (1.0 - 0.5 * np.exp(-32.0 * r2))


def velocity_lens3d(n):
    x1, x2, x3 = grid_coords(n, 3)
    r2 = (x1 - 0.5) ** 2 + (x2 - 0.5) ** 2 + (x3 - 0.5) ** 2
    return 1.0 + 0.3 * np.exp(-32.0 * r2)


def velocity_random(n, d, seed, width=8.0, lo=0.8, hi=1.2):
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n,) * d)
    z = gaussian_filter(z, sigma=width, mode="reflect", truncate=4.0)
    zmin, zmax = float(z.min()), float(z.max())
    return lo + (hi - lo) * (z - zmin) / (zmax - zmin)


def velocity_waveguide2d(n):
    x1, _ = grid_coords(n, 2)
    return (4.0 / 3.0) * (1.0 - 0.5 * np.exp(-32.0 * (x1 - 0.5) ** 2))


def variation_widths(c, gamma, narrow, wide, quantile=0.5):
    """Unequal layer widths (Section 3.1 remarks: wider layers where the
    velocity varies strongly).  v(t) is the largest relative change of c
    between physical sweep lines t and t + 1 (the sweep axis is the last
    index).  From the first physical line on, a layer takes ``wide`` lines if
    v exceeds its ``quantile`` anywhere in those lines, else ``narrow``; the
    last layer takes what remains.  Returns the list of physical lines per
    layer (summing to n - 2(gamma - 1))."""
    c = np.asarray(c, dtype=np.float64)
    n, g = c.shape[-1], gamma - 1
    phys = c[..., g:n - g]
    n_phys = phys.shape[-1]
    diff = np.abs(np.diff(phys, axis=-1)) / float(np.mean(phys))
    v = diff.reshape(-1, n_phys - 1).max(axis=0) if n_phys > 1 else np.zeros(0)
    v = np.append(v, 0.0)
    thr = float(np.quantile(v, quantile))
    w, t = [], 0
    while t < n_phys:
        k = wide if v[t:t + wide].max() > thr else narrow
        k = min(k, n_phys - t)
        w.append(int(k))
        t += k
    return w


def wave_packet(n, d, omega, centre, direction):
    xs = grid_coords(n, d)
    lam = 2.0 * math.pi / omega
    r2 = sum((x - c0) ** 2 for x, c0 in zip(xs, centre))
    phase = sum(dk * (x - c0) for x, c0, dk in zip(xs, centre, direction))
    return np.exp(-r2 / (2.0 * lam * lam)) * np.exp(1j * omega * phase)


def gaussian_source(n, d, omega, centre):
    """exp(-(4 omega / pi)^2 |x - centre|^2) on the (n,)*d grid, formed as the
    product of its one-dimensional factors (n^d products instead of n^d
    exponentials; equal to the direct form up to rounding)."""
    t = np.arange(1, n + 1, dtype=np.float64) / (n + 1)
    a = 4.0 * omega / math.pi
    out = np.exp(-(a * a) * (t - centre[0]) ** 2)
    for c0 in centre[1:d]:
        out = np.multiply.outer(out, np.exp(-(a * a) * (t - c0) ** 2))
    return out


def seeded_centres(count, d, seed, lo=0.2, hi=0.8):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(count, d))


# Named workloads.  Each entry: dimension, interior points per side, angular
# frequency, PML width gamma (eta = gamma*h), PML constant C, lines per
# interior layer b, number of right-hand sides, GMRES restart and tolerance.
WORKLOADS = {
    "2d_n63_const": dict(d=2, n=63, omega=2 * math.pi * 8, gamma=12, C=25.0, b=4,
                         nrhs=1, restart=20, tol=1e-6, velocity="constant",
                         centres="fixed"),
    "2d_n511_lens": dict(d=2, n=511, omega=2 * math.pi * 64, gamma=12, C=25.0, b=4,
                         nrhs=8, restart=20, tol=1e-6, velocity="lens",
                         centres=2),
    "2d_n1023_random": dict(d=2, n=1023, omega=2 * math.pi * 128, gamma=12, C=25.0,
                            b=4, nrhs=64, restart=20, tol=1e-6, velocity="random",
                            velocity_seed=3, centres=33),
    "3d_n63_lens": dict(d=3, n=63, omega=2 * math.pi * 8, gamma=8, C=25.0, b=4,
                        nrhs=16, restart=20, tol=1e-6, velocity="lens",
                        centres=4),
}


def _velocity(spec):
    d, n, kind = spec["d"], spec["n"], spec["velocity"]
    if kind == "constant":
        return velocity_constant(n, d)
    if kind == "lens":
        return velocity_lens2d(n) if d == 2 else velocity_lens3d(n)
    if kind == "random":
        return velocity_random(n, d, spec.get("velocity_seed", 3))
    raise ValueError(f"unknown velocity family {kind!r}")


# The settings of the paper's 2D experiments (Section 3.2): PML width
# gamma = 9, layers of b = 8 lines, 8 points per wavelength (omega / 2 pi =
# (n + 1) / 8), GMRES(40) to a relative residual of 1e-3.  Two right-hand sides
# per problem: force (a), a Gaussian point source at (1/2, 1/8), and force (b),
# a wave packet at (1/8, 1/8) travelling along (1, 1) / sqrt 2.
PAPER_2D = dict(d=2, gamma=9, C=25.0, b=8, restart=40, tol=1e-3)
PAPER_FIELDS = ("lens", "waveguide", "random")
PAPER_SIZES = (127, 255, 511, 1023, 2047)


def paper_workload(field, n):
    """A problem of the paper's 2D experiments (Tables 1-3) with the field
    ``field`` in PAPER_FIELDS on an n x n grid; same keys as ``workload``."""
    spec = dict(PAPER_2D, n=n, nrhs=2, omega=2 * math.pi * (n + 1) / 8, velocity=field)
    if field == "lens":
        c = velocity_lens2d(n)
    elif field == "waveguide":
        c = velocity_waveguide2d(n)
    elif field == "random":
        c = velocity_random(n, 2, 3)
    else:
        raise ValueError(f"unknown paper field {field!r}")
    w = spec["omega"]
    fa = gaussian_source(n, 2, w, (0.5, 0.125))
    s2 = 1.0 / math.sqrt(2.0)
    fb = wave_packet(n, 2, w, (0.125, 0.125), (s2, s2))
    f = np.stack([flat(fa).astype(np.complex128), flat(fb).astype(np.complex128)])
    spec.update(c=c, f=f, name=f"paper2d_{field}_n{n}")
    return spec


# The settings of the paper's 3D experiments (Section 4.2): boundary PML
# gamma = 9, auxiliary PML gamma_aux = 5, layers of b = 4 lines, 8 points per
# wavelength, GMRES(40) to 1e-3.  Force (a): a Gaussian point source at
# (1/2, 1/2, 1/4); force (b): a wave packet at (1/2, 1/4, 1/4) travelling along
# (0, 1, 1) / sqrt 2.
PAPER_3D = dict(d=3, gamma=9, gamma_aux=5, C=25.0, b=4, restart=40, tol=1e-3)
PAPER_SIZES_3D = (39, 79)


def paper_workload3d(field, n):
    """A problem of the paper's 3D experiments (Tables 4-6) with the field
    ``field`` in PAPER_FIELDS on an n^3 grid; same keys as ``workload``."""
    spec = dict(PAPER_3D, n=n, nrhs=2, omega=2 * math.pi * (n + 1) / 8, velocity=field)
    x1, x2, x3 = grid_coords(n, 3)
    if field == "lens":
        c = (4.0 / 3.0) * (1.0 - 0.5 * np.exp(-32.0 * ((x1 - 0.5) ** 2 + (x2 - 0.5) ** 2 +
                                                        (x3 - 0.5) ** 2)))
    elif field == "waveguide":
        c = (4.0 / 3.0) * (1.0 - 0.5 * np.exp(-32.0 * ((x1 - 0.5) ** 2 + (x2 - 0.5) ** 2)))
    elif field == "random":
        c = velocity_random(n, 3, 3, width=(n + 1) / 16.0)
    else:
        raise ValueError(f"unknown paper field {field!r}")
    w = spec["omega"]
    fa = gaussian_source(n, 3, w, (0.5, 0.5, 0.25))
    s2 = 1.0 / math.sqrt(2.0)
    fb = wave_packet(n, 3, w, (0.5, 0.25, 0.25), (0.0, s2, s2))
    f = np.stack([flat(fa).astype(np.complex128), flat(fb).astype(np.complex128)])
    spec.update(c=c, f=f, name=f"paper3d_{field}_n{n}")
    return spec


def workload(name, n=None, nrhs=None):
    """Materialise a named workload.

    ``n`` and ``nrhs`` optionally shrink the workload (same recipe, smaller
    grid or fewer right-hand sides); omega then scales with n so that the
    number of points per wavelength is unchanged.

    Returns a dict with keys d, n, omega, gamma, C, b, restart, tol,
    c (float64, shape (n,)*d) and f (complex128, shape (nrhs, n**d), each row
    column-major)."""
    spec = dict(WORKLOADS[name])
    if n is not None and n != spec["n"]:
        spec["omega"] = spec["omega"] * (n + 1) / (spec["n"] + 1)
        spec["n"] = n
    if nrhs is not None:
        spec["nrhs"] = nrhs
    d, n = spec["d"], spec["n"]
    c = _velocity(spec)
    if spec["centres"] == "fixed":
        cents = np.array([[0.5, 0.25]] * spec["nrhs"])
    else:
        cents = seeded_centres(spec["nrhs"], d, spec["centres"])
    f = np.stack([flat(gaussian_source(n, d, spec["omega"], x0)) for x0 in cents])
    spec.update(c=c, f=f.astype(np.complex128), centres_xy=cents, name=name)
    return spec
