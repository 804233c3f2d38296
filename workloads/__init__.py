"""Seeded synthetic right-hand sides for the 2-D Poisson workloads.

This module only builds inputs.  It contains none of the multigrid arithmetic
(no smoother, residual, transfer or solve) and imports neither the CPU oracle
nor the HIP library, so both sides can be fed from it without sharing code.

Grid convention (shared by every caller): a square grid of ``n`` nodes per
side on the unit square, ``n - 1 = 4 * 2**k``, spacing ``h = 1/(n-1)``, stored
row-major as ``a[i, j]`` with ``i`` the y index (row) and ``j`` the x index
(column).  Zero-Dirichlet grids carry their boundary nodes (always 0).
Periodic grids carry a duplicated seam: row/column ``n-1`` repeats row/column
0, so the unique nodes are ``0 .. n-2`` in each direction.

The paper solves the pressure-Poisson equation whose source is a derivative of
a turbulent velocity field (Section 2.3, Eq. for the pressure-Poisson source;
Section 2.5 on the training data).  Its fields come from a Navier-Stokes run
that is not available, so these generators stand in for them: the source is
the divergence of a random velocity field with a Kolmogorov-like spectrum.
"""

from .rhs import (  # noqa: F401
    SIZES_BATCHED,
    TWOLEVEL_BATCH,
    TWOLEVEL_N,
    batch_sizes,
    grid_unknowns,
    initial_grid_periodic,
    manufactured_solution,
    rhs_divu_dirichlet,
    rhs_divu_periodic,
    rhs_manufactured_dirichlet,
    rhs_twolevel_periodic,
    twolevel_batch,
    velocity_periodic,
    workload,
)
