"""Seeded synthetic point-set generators shared by the tests, the benchmark and the oracle runs.

This module draws inputs only; it holds none of the Voronoi arithmetic.  Every generator is
deterministic given its seed (numpy PCG64) and returns int32 structure-of-arrays coordinates plus
the box X = [x0, x1] x [y0, y1].  Sites are distinct and lie strictly inside X, the setting of the
paper's problem statement (Section 2, the definition of the Voronoi diagram): any draw that would
put a coordinate on the boundary or repeat an earlier site is redrawn from the same stream.
``boundary_points`` / ``with_boundary_sites`` add sites on the boundary of X (sides and corners),
the extension of the definition to such sites that the problem statement mentions.
"""
from .generators import (  # noqa: F401
    PointSet,
    uniform,
    clustered,
    lattice,
    batch_sizes,
    batch_sets,
    request_stream,
    small_integer_set,
    convex_polygon,
    inside_polygon,
    in_polygon,
    boundary_points,
    with_boundary_sites,
)
