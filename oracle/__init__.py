"""CPU oracle for the geometric-multigrid V-cycle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` use it.  It shares no code with the HIP library
(no kernels, headers, helpers or tables); the two only see the same seeded
inputs from ``paper_1904_08684_amd.workloads``.

What it computes
----------------
The paper (Sec. 1) places its solvers in the ExaStencils line of work:
whole programs that solve PDEs iteratively on regular grids whose operators
are stencils.  The ExaSlang vocabulary listed with the paper's listings names
the parts of such a solver: fields on ``Node`` or ``Cell`` positions, a
``Stencil`` per level with ``coarser``/``coarsest`` levels, ``restriction``
and ``prolongation`` operators, ``jacobi`` and ``color``-ed ``relax``-ation,
a ``solve`` on the coarsest level, ``repeat ... until`` a criterion,
``StencilField`` coefficients, ``ghost`` layers and ``reduction``-s.  The
paper states no algorithm for these parts, so each function here writes out
the textbook definition (Trottenberg, Oosterlee and Schueller, *Multigrid*,
Academic Press 2001, chapters 2-4 and 5.7) in plain NumPy, FP64 unless an
array of another dtype is passed in (float32 arrays emulate the
single-precision inner cycle exactly, operation by operation).

Floating-point evaluation order is written out explicitly in every formula
(left to right, neighbours in the order x-, x+, y-, y+, z-, z+), never fused
multiply-adds, so that the order is a documented part of the definition.

Readings of points the paper leaves open are listed in ``readings.py``.

Files
-----
``node.py``   node-centred constant-coefficient Poisson operator, damped
              Jacobi, red-black Gauss-Seidel, full weighting, linear
              interpolation (2-D and 3-D).
``cell.py``   cell-centred variable-coefficient operator with harmonic-mean
              face coefficients and mirror ghosts, its smoothers and
              transfers.
``cycle.py``  level hierarchy, coarsest direct solve, V-cycle, solve to a
              tolerance, and the mixed-precision iterative refinement.
"""
from . import node, cell, cycle, readings  # noqa: F401
from .cycle import (Hierarchy, build_hierarchy, vcycle, solve, mixed_solve,  # noqa: F401
                    residual_norm, residual)
