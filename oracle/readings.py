"""Readings taken where the paper is silent, ambiguous or garbled.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper describes no multigrid algorithm (its method is a quadrature-free
DG discretisation of the shallow water equations, Sec. 2); the V-cycle
vocabulary comes from the ExaSlang keyword lists that accompany its
listings (``coarsest``, ``restriction``, ``prolongation``, ``jacobi``,
``color``, ``relax``, ``solve``, ``repeat ... until``, ``StencilField``).
Each reading below fixes one constant of the textbook method; the GPU
library is configured with the same values in its tests.
"""

READINGS = {
    "R0": "V-cycle, smoothers and transfers follow the textbook definitions (gamma = 1).",
    "R1": "'coarsest 3x3' / '3^3 coarse solve' = 3^d interior unknowns, i.e. 5^d nodes "
          "(513 -> ... -> 5 is 8 grids, matching the stated 8 levels).",
    "R2": "Full weighting sums to 1 and linear interpolation is P = 2^d R^T.",
    "R3": "Coarse operators are rediscretised (same stencil, coarse 1/H^2) by default; the Galerkin "
          "option uses R A P on every coarser level and keeps the finest 5/7-point stencil.",
    "R4": "Boundary nodes are not unknowns and hold 0 on every level for u, r and e.",
    "R5": "Red = even index sum (boundary index 0), updated first in pre- and post-smoothing.",
    "R6": "Initial guess 0 where unstated; the 2-D case uses U[-1,1] on interior nodes.",
    "R7": "The variable-coefficient case uses red-black GS V(3,3) and zero Dirichlet walls.",
    "R8": "'257^3 cells' is read as 256^3 cells (257 vertices per axis).",
    "R9": "Coarse face coefficient = mean of the fine faces that tile the coarse face.",
    "R10": "Mixed precision: one single-precision V-cycle per FP64 refinement step, "
           "scale 2^floor(log2 m), m = max|r| of the previous step's residual (the first "
           "step's own); any power of two gives the same iterates away from FP32 under/overflow.",
    "R11": "Norm = unweighted 2-norm over the unknowns; relative to the initial residual.",
    "R12": "Stopping counts may differ by one cycle when ||r|| crosses tol within rounding; "
           "parity is judged on iterates at equal cycle counts.",
    "R13": "Seeds: NumPy PCG64, 0 (2-D u0), 1 (3-D f), 2 (variable-coefficient f), "
           "3/4 (arrivals/sizes), 1000+id (request f).",
    "R14": "Served 2-D requests use damped Jacobi V(2,2); 3-D requests use red-black GS V(3,3).",
    "R15": "FMG: the right-hand side goes to every level by the cycle's restriction, each finer "
           "level starts from the interpolated coarser result, a level directly above the "
           "coarsest gets its cycles too.",
    "R16": "Preconditioned CG: the preconditioner is one cycle from zero with nu1 = nu2 and the "
           "adjoint post-smoother (red-black GS: reversed colours); the stopping test uses CG's "
           "recurrence residual.",
    "R17": "Neumann walls (cell grids): f is projected to zero mean at the start and after every "
           "restriction, the finest iterate after every cycle; the coarsest solve returns the "
           "zero-mean (minimum-norm) solution.",
    "R18": "DG volume terms: the element basis is |det B_e|^(-1/2) phi^_i o F_e^-1 (orthonormal on the "
           "element); the paper's algebraic forms carry 1/|det B_e| and 1/|det B_e|^(3/2), which this "
           "scaling produces, while its definition line omits the factor.",
    "R19": "The y-momentum volume term (the paper's 'similar expression') uses the third flux row "
           "(V u, V v + g xi (H + h_b)/2): V in place of U and d/dx2 for the pressure terms.",
    "R20": "The bathymetry h_b is a P^k field on every element, like xi; the algebraic form, which "
           "takes h_b outside the integral, is the case of a field with only the constant mode, and "
           "the linear h_b of the convergence test is exact for k >= 1.  det B_e keeps its sign "
           "(|det B_e| for counter-clockwise elements).",
    "R21": "DG edge terms: the Lax-Friedrichs wave speed is one value per edge, the larger of "
           "|u_mean . n| + sqrt(g H_mean) over the two elements (element means).",
    "R22": "Dirichlet boundaries: the exterior state of a boundary edge is a prescribed polynomial "
           "in the owning element's basis (in the convergence test the L2 projection of the exact "
           "xi, U, V and of u = U/H, v = V/H onto that element), entering the Lax-Friedrichs flux "
           "like a neighbour with the element's own bathymetry.",
    "R23": "Source and time stepping: tau_bf and f_c are constants (zero in the convergence test, "
           "which states neither); the body force enters as the coefficients of its L2 projection; "
           "the integrator is the three-stage SSP Runge-Kutta method of Shu and Osher with the "
           "velocity projected from every stage state.",
    "R24": "Gravity in the convergence test: the paper states no value of g.  With g = 9.81 the "
           "momentum errors are 4-7 times the table's and a step of 0.5 is unstable on the finest "
           "meshes; one column (k = 1, every mesh, step 0.5) run once with g = 1 is stable and gives "
           "xi errors within 11 % and U, V errors within 0.9-2.1 times the table's, so the table "
           "is read as computed with g = 1 (a nondimensional gravity); the library takes g as an "
           "argument and nothing in it depends on this reading.",
}
