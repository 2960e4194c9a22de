"""CPU FP64 oracle for the additive sweeping preconditioner (Liu & Ying).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the method, written from the paper.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or run it.  The product path (the HIP library and its Python binding)
never imports it and shares no code with it; the only thing both sides
consume is the seeded input generator in ``workloads``.

Modules and the passages they restate:

* ``pml``        -- the PML profile sigma and s = (1 + i sigma/omega)^-1
                    (Section 2, PML definition; auxiliary profiles of 2.1).
* ``partition``  -- the layer partition X_1..X_m and the extended grids
                    X^M_q, X^R_p, X^L_p (Sections 2, 3.1 "Auxiliary domains",
                    4.1 "Auxiliary domains").
* ``operator``   -- the centered-difference PML operator, eq. (1D), (2D),
                    (3D), in symmetric form (Section 3.1 remark 4).
* ``subproblem`` -- assembly and LU factorization of H^M, H^R, H^L and the
                    auxiliary Green's operators G~ (Sections 3.1, 4.1;
                    Algorithms 1 and 3).
* ``sweep``      -- the preconditioner apply, Algorithms 2 and 4, and the
                    O(m^2) per-component recursion of Section 2.1 it must equal.
* ``gmres``      -- textbook right-preconditioned restarted GMRES (the outer
                    solver of Sections 3.2 and 4.2).
* ``direct``     -- the exact discrete solution u = A^-1 f.

Precision is FP64 / complex128 throughout (the paper states none).
"""
from . import pml, partition, operator, subproblem, sweep, gmres, direct  # noqa: F401
