"""FP64 CPU oracle for the lattice-H-matrix product — TEST INFRASTRUCTURE.

This package is a plain, slow, deliberately unoptimised statement of what
the GPU path computes.  It is used only by ``tests/``, by the smoke check
in ``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of
``bench.py``.  The product library never imports, links or calls it, and
the two share no code: the only common module is ``synth`` (seeded mesh
and random-input generators, which contain none of the method's
arithmetic).

Modules and the parts of the paper they follow:

* ``greens``   — element stiffness entries (section 2.1, eqs. 3-6), full-space
                 kernel for coplanar rectangular elements.
* ``cluster``  — binary cluster tree, admissibility and block partition
                 (section 3.1.1, eq. 17), lattice structure (section 3.2).
* ``aca``      — adaptive cross approximation (section 3.1.2, eqs. 18-19).
* ``hmatrix``  — H-matrix build and H-matrix-vector product
                 (section 3.1.3, eq. 20).
* ``dense``    — the plain definition y = A x (eqs. 5-6): explicit matrix,
                 rows one by one, and an exact FFT form for equal-square
                 planar grids.

Parity status of each function is stated in its module docstring.
"""
