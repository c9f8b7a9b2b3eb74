"""Oracle for the Voronoi diagram restricted to a box -- TEST INFRASTRUCTURE ONLY.

Only tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import this
package.  It shares no code with the GPU path and imports nothing from it.

* ``cdiagram``  -- exact half-plane clipping in C (``vor_oracle.c``), multi-threaded.
* ``ref``       -- independent exact-rational reference (Python ``Fraction``), small n.
* ``brute``     -- brute-force enumeration of candidate vertices, n <= 8.
* ``checks``    -- invariant checkers (symmetry, Euler, equidistance, exact area).
* ``paper_forms`` -- closed forms printed in the paper (integer rectangle, constants of the
  uniform-distribution theorem).
"""
