"""Kernel-level parity: every level operation of the HIP library against the
oracle routine it implements, one application on seeded random fields, at
sizes spanning one to many tiles with ragged tails, node and cell grids,
FP64 and the single-precision hierarchy.  The library is compiled without
FMA contraction and evaluates the oracle's formulas in the same order, so
the expected agreement is to the last bit; the test bar is 1e-14 relative
(FP64) and 1e-6 relative (FP32)."""
import numpy as np
import pytest

from oracle import cell, cycle, node
from paper_1904_08684_amd import workloads as W

pytestmark = pytest.mark.gpu

NODE_CASES = [(2, 9), (2, 17), (2, 129), (2, 257), (3, 9), (3, 17), (3, 33), (3, 65), (3, 129), (3, 257)]
CELL_CASES = [(2, 8), (2, 16), (2, 128), (3, 8), (3, 16), (3, 32)]


def tol(prec):
    return 1e-14 if prec == 0 else 1e-6


def close(got, ref, prec, what):
    scale = max(np.max(np.abs(ref)), 1e-300)
    err = np.max(np.abs(got - ref)) / scale
    exact = np.array_equal(got, ref)
    print(f"{what}: max rel diff {err:.3e} bit-exact {exact}", flush=True)
    assert err <= tol(prec), (what, err)


def make(mg, dim, n, cent, prec, smoother=None):
    k = W.varcoef_k(n, dim) if cent == mg.MG_CELL else None
    s = mg.Solver(dim, n, centering=cent, smoother=mg.MG_JACOBI if smoother is None else smoother,
                  omega=0.8, nu1=1, nu2=1, precision=mg.MG_MIXED if prec else mg.MG_FP64, k=k)
    p = cycle.Params(centering="cell" if cent else "node", dim=dim, n=n,
                     coarsest=4 if cent else 5, smoother="jacobi", omega=0.8, k=k)
    return s, cycle.build_hierarchy(p)


def rand(n, dim, cent, seed, dtype):
    a = W.cell_uniform(n, dim, seed) if cent else W.interior_uniform(n, dim, seed)
    return a.astype(dtype)


def cases():
    out = []
    for d, n in NODE_CASES:
        out.append((d, n, 0))
    for d, n in CELL_CASES:
        out.append((d, n, 1))
    return out


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim,n,cent", cases())
def test_smoothers_and_residual(mg, dim, n, cent, prec):
    s, h = make(mg, dim, n, cent, prec)
    dt = np.float64 if prec == 0 else np.float32
    u = rand(n, dim, cent, 100 + n, dt)
    f = rand(n, dim, cent, 200 + n, dt) * dt(n * n)
    beta = h.beta_as(0, dt) if cent else None
    tag = f"{dim}d n={n} {'cell' if cent else 'node'} prec={prec}"

    for colour, op in ((0, mg.MG_OP_GS_RED), (1, mg.MG_OP_GS_BLACK)):
        s.level_set(0, mg.MG_FIELD_U, u, prec)
        s.level_set(0, mg.MG_FIELD_F, f, prec)
        s.apply(op, 0, prec)
        got = s.level_get(0, mg.MG_FIELD_U, prec)
        ref = u.copy()
        if cent:
            cell.gs_colour(ref, f, beta, colour)
        else:
            node.gs_colour(ref, f, colour)
        close(got, ref.astype(np.float64), prec, f"gs colour {colour} {tag}")

    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.apply(mg.MG_OP_JACOBI, 0, prec)
    got = s.level_get(0, mg.MG_FIELD_U, prec)
    ref = cell.jacobi(u, f, beta, 0.8) if cent else node.jacobi(u, f, 0.8)
    close(got, ref.astype(np.float64), prec, f"jacobi {tag}")

    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.apply(mg.MG_OP_RESIDUAL, 0, prec)
    got = s.level_get(0, mg.MG_FIELD_R, prec)
    ref = cell.residual(u, f, beta) if cent else node.residual(u, f)
    close(got, ref.astype(np.float64), prec, f"residual {tag}")
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,nu", [(129, 2), (129, 3), (97, 2), (257, 4), (1025, 2)])
def test_presmoothing_residual_restriction_in_one_launch(mg, n, nu, prec):
    """2-D damped Jacobi: the last two pre-smoothing sweeps, the residual and
    its full weighting in one launch (LDS tiles with a halo of four) give
    the iterate and the coarse right-hand side of the separate sweeps and
    residual + restriction bitwise, and the oracle's."""
    def solver():
        return mg.Solver(2, n, coarsest=4 if n == 97 else 5, smoother=mg.MG_JACOBI, omega=0.8, nu1=nu, nu2=nu,
                         precision=mg.MG_MIXED if prec else mg.MG_FP64)
    dt = np.float64 if prec == 0 else np.float32
    u = rand(n, 2, 0, 1500 + n, dt)
    f = rand(n, 2, 0, 1600 + n, dt) * dt(n * n)
    s = solver()
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(0, mg.MG_FIELD_F, f, prec)
    s.apply(mg.MG_OP_PRESMOOTH_RESTRICT, 0, prec)
    uf, ff = s.level_get(0, mg.MG_FIELD_U, prec), s.level_get(1, mg.MG_FIELD_F, prec)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    for _ in range(nu):
        s.apply(mg.MG_OP_JACOBI, 0, prec)
    s.apply(mg.MG_OP_RESIDUAL, 0, prec)
    s.apply(mg.MG_OP_RESTRICT, 0, prec)
    us, fs = s.level_get(0, mg.MG_FIELD_U, prec), s.level_get(1, mg.MG_FIELD_F, prec)
    s.close()
    print(f"presmooth+restrict n={n} nu={nu} prec={prec}: bitwise {np.array_equal(uf, us)} {np.array_equal(ff, fs)}",
          flush=True)
    assert np.array_equal(uf, us) and np.array_equal(ff, fs)
    ref = u.copy()
    for _ in range(nu):
        ref = node.jacobi(ref, f, 0.8)
    assert np.array_equal(uf, ref)
    close(ff, node.restrict_fw(node.residual(ref, f)).astype(np.float64), prec, f"presmooth+restrict n={n}")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,nu", [(129, 2), (129, 3), (257, 2), (97, 2), (1025, 4)])
def test_two_jacobi_sweeps_per_launch_equal_single_sweeps(mg, n, nu, prec):
    """On 2-D levels a smoothing step runs two damped-Jacobi sweeps per
    launch (tiles with a halo of two in LDS): bitwise equal to the same
    number of single sweeps, at power-of-two (129, 257, 1025) and other (97)
    scales, and to the oracle's sweeps."""
    s = mg.Solver(2, n, coarsest=4 if n == 97 else 5, smoother=mg.MG_JACOBI, omega=0.8, nu1=nu, nu2=nu,
                  precision=mg.MG_MIXED if prec else mg.MG_FP64)
    dt = np.float64 if prec == 0 else np.float32
    u = rand(n, 2, 0, 1300 + n, dt)
    f = rand(n, 2, 0, 1400 + n, dt) * dt(n * n)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(0, mg.MG_FIELD_F, f, prec)
    s.apply(mg.MG_OP_PRESMOOTH, 0, prec)
    fused = s.level_get(0, mg.MG_FIELD_U, prec)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    for _ in range(nu):
        s.apply(mg.MG_OP_JACOBI, 0, prec)
    single = s.level_get(0, mg.MG_FIELD_U, prec)
    s.close()
    print(f"two sweeps per launch n={n} nu={nu} prec={prec}: bitwise {np.array_equal(fused, single)}", flush=True)
    assert np.array_equal(fused, single)
    ref = u.copy()
    for _ in range(nu):
        ref = node.jacobi(ref, f, 0.8)
    assert np.array_equal(fused, ref)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim,n", [(2, 65), (2, 97), (3, 33), (3, 49)])
def test_jacobi_sweep_bitwise_at_both_kinds_of_scale(mg, dim, n, prec):
    """A damped-Jacobi sweep equals the oracle's (omega r) / (2d s) bitwise
    whether s = (n - 1)^2 is a power of two (65, 33: the kernels multiply by
    the exact reciprocal) or not (97, 49: they divide)."""
    s = mg.Solver(dim, n, coarsest=4 if n in (97, 49) else 5, smoother=mg.MG_JACOBI, omega=0.8, nu1=2, nu2=2,
                  precision=mg.MG_MIXED if prec else mg.MG_FP64)
    dt = np.float64 if prec == 0 else np.float32
    u = rand(n, dim, 0, 300 + n, dt)
    f = rand(n, dim, 0, 400 + n, dt) * dt(n * n)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(0, mg.MG_FIELD_F, f, prec)
    s.apply(mg.MG_OP_JACOBI, 0, prec)
    got = s.level_get(0, mg.MG_FIELD_U, prec)
    s.close()
    ref = node.jacobi(u, f, 0.8)
    print(f"jacobi {dim}d n={n} prec={prec}: bitwise {np.array_equal(got, ref)}", flush=True)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n,bc", [(128, "dirichlet"), (256, "dirichlet"), (128, "neumann")])
def test_cell_faces_from_k_bitwise(mg, n, bc):
    """On the finest 3-D cell level with n >= 128 the FP64 half-sweeps and
    the residual form each face coefficient from k as they go (column
    marching): every value bit for bit the oracle's, which reads harmonic
    means stored per face."""
    k = W.varcoef_k(n, 3)
    s = mg.Solver(3, n, centering=mg.MG_CELL, smoother=mg.MG_RBGS, nu1=1, nu2=1, k=k,
                  bc=mg.MG_NEUMANN0 if bc == "neumann" else mg.MG_DIRICHLET0)
    beta = cell.harmonic_faces(k)
    u = rand(n, 3, 1, 300 + n, np.float64)
    f = rand(n, 3, 1, 400 + n, np.float64) * float(n * n)
    for colour, op in ((0, mg.MG_OP_GS_RED), (1, mg.MG_OP_GS_BLACK)):
        s.level_set(0, mg.MG_FIELD_U, u, 0)
        s.level_set(0, mg.MG_FIELD_F, f, 0)
        s.apply(op, 0, 0)
        got = s.level_get(0, mg.MG_FIELD_U, 0)
        ref = u.copy()
        cell.gs_colour(ref, f, beta, colour, bc)
        print(f"k-path gs colour {colour} n={n} {bc}: bitwise {np.array_equal(got, ref)}", flush=True)
        assert np.array_equal(got, ref)
    s.level_set(0, mg.MG_FIELD_U, u, 0)
    s.apply(mg.MG_OP_RESIDUAL, 0, 0)
    got = s.level_get(0, mg.MG_FIELD_R, 0)
    ref = cell.residual(u, f, beta, bc)
    print(f"k-path residual n={n} {bc}: bitwise {np.array_equal(got, ref)}", flush=True)
    assert np.array_equal(got, ref)
    s.close()


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim,n,cent", [c for c in cases() if c[1] > (4 if c[2] else 5)])
def test_transfers(mg, dim, n, cent, prec):
    s, h = make(mg, dim, n, cent, prec)
    dt = np.float64 if prec == 0 else np.float32
    nc = s.level_size(1)
    tag = f"{dim}d n={n} {'cell' if cent else 'node'} prec={prec}"
    r = rand(n, dim, cent, 300 + n, dt)
    s.level_set(0, mg.MG_FIELD_R, r, prec)
    s.apply(mg.MG_OP_RESTRICT, 0, prec)
    got = s.level_get(1, mg.MG_FIELD_F, prec)
    ref = cell.restrict_mean(r) if cent else node.restrict_fw(r)
    close(got, ref.astype(np.float64), prec, f"restrict {tag}")

    u = rand(n, dim, cent, 400 + n, dt)
    e = rand(nc, dim, cent, 500 + n, dt)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(1, mg.MG_FIELD_U, e, prec)
    s.apply(mg.MG_OP_PROLONG, 0, prec)
    got = s.level_get(0, mg.MG_FIELD_U, prec)
    ref = cell.correct(u, e) if cent else node.correct(u, e)
    close(got, ref.astype(np.float64), prec, f"prolong {tag}")
    s.close()


@pytest.mark.parametrize("n,bc,prec", [(128, "dirichlet", 0), (128, "dirichlet", 1), (256, "dirichlet", 0),
                                       (256, "dirichlet", 1), (128, "neumann", 0)])
def test_cell_prolongation_on_column_levels(mg, n, bc, prec):
    """Large 3-D cell levels interpolate along columns (each coarse value
    formed once for two fine planes): the correction equals the oracle's
    cell-centred trilinear interpolation with mirror ghosts (Neumann walls
    are FP64-only)."""
    k = W.varcoef_k(n, 3)
    s = mg.Solver(3, n, centering=mg.MG_CELL, smoother=mg.MG_RBGS, nu1=3, nu2=3, k=k,
                  bc=mg.MG_NEUMANN0 if bc == "neumann" else mg.MG_DIRICHLET0,
                  precision=mg.MG_MIXED if prec else mg.MG_FP64)
    dt = np.float64 if prec == 0 else np.float32
    u = rand(n, 3, 1, 900 + n, dt)
    e = rand(n // 2, 3, 1, 950 + n, dt)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(1, mg.MG_FIELD_U, e, prec)
    s.apply(mg.MG_OP_PROLONG, 0, prec)
    got = s.level_get(0, mg.MG_FIELD_U, prec)
    s.close()
    close(got, cell.correct(u, e, bc).astype(np.float64), prec, f"cell prolong n={n} {bc} prec={prec}")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("dim,cent", [(2, 0), (3, 0), (2, 1), (3, 1)])
def test_coarsest_solve(mg, dim, cent, prec):
    n = 17 if not cent else 16
    s, h = make(mg, dim, n, cent, prec)
    dt = np.float64 if prec == 0 else np.float32
    L = s.levels() - 1
    nc = s.level_size(L)
    fc = rand(nc, dim, cent, 600, dt)
    s.level_set(L, mg.MG_FIELD_F, fc, prec)
    s.apply(mg.MG_OP_COARSE, L, prec)
    got = s.level_get(L, mg.MG_FIELD_U, prec)
    ref = cycle.coarse_solve(h, fc)
    # the oracle factors with LAPACK, the library with its own Cholesky: agreement to rounding
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref)) / scale
    print(f"coarse {dim}d cent={cent} prec={prec}: max rel diff {err:.3e}", flush=True)
    assert err <= (1e-13 if prec == 0 else 1e-6)
    s.close()


def test_mixed_hierarchy_rejects_missing_fp64_levels(mg):
    s = mg.Solver(3, 17, smoother=mg.MG_RBGS, precision=mg.MG_MIXED)
    with pytest.raises(mg.MGError):
        s.apply(mg.MG_OP_RESTRICT, 0, mg.MG_PREC_FP64)
    s.close()


def test_repeat_is_bitwise_deterministic(mg):
    """Same inputs, same launches: bitwise identical outputs (catches races in
    the in-place colour sweeps)."""
    n = 65
    f = W.interior_uniform(n, 3, 1)
    outs = []
    for _ in range(2):
        s = mg.Solver(3, n, smoother=mg.MG_RBGS, nu1=3, nu2=3)
        s.set_rhs(f)
        s.set_initial(None)
        s.vcycle(3)
        outs.append(s.solution())
        s.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("case", [("node", 2, 129, "dirichlet", 0), ("node", 2, 129, "dirichlet", 1),
                                  ("node", 2, 1025, "dirichlet", 0), ("cell", 3, 128, "dirichlet", 0),
                                  ("cell", 3, 256, "dirichlet", 0), ("cell", 3, 128, "neumann", 0),
                                  ("cell", 3, 128, "dirichlet", 1), ("cell", 3, 32, "neumann", 0),
                                  ("cell", 3, 64, "dirichlet", 1), ("cell", 2, 64, "dirichlet", 0),
                                  ("cell", 2, 32, "dirichlet", 1)])
def test_one_pass_residual_restriction_equals_the_two_ops(mg, case):
    """The one-pass residual + restriction of 2-D node levels (each coarse
    point forms its nine fine residuals), of the finest 3-D cell level
    (residuals of both colours and two rows per thread, faces from k, summed
    into the 8-child mean) and of small cell levels with stored faces
    (each coarse cell forms its children's residuals) equal the
    residual then the restriction bitwise, and the oracle's restriction of
    its residual."""
    kind, dim, n, bc, prec = case
    cent = mg.MG_CELL if kind == "cell" else mg.MG_NODE
    k = W.varcoef_k(n, dim) if kind == "cell" else None
    s = mg.Solver(dim, n, centering=cent, smoother=mg.MG_RBGS, nu1=3, nu2=3, k=k,
                  bc=mg.MG_NEUMANN0 if bc == "neumann" else mg.MG_DIRICHLET0,
                  precision=mg.MG_MIXED if prec else mg.MG_FP64)
    dt = np.float64 if prec == 0 else np.float32
    cflag = 1 if kind == "cell" else 0
    u = rand(n, dim, cflag, 700 + n, dt)
    f = rand(n, dim, cflag, 800 + n, dt) * dt(n * n)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(0, mg.MG_FIELD_F, f, prec)
    s.apply(mg.MG_OP_RESIDUAL_RESTRICT, 0, prec)
    fused = s.level_get(1, mg.MG_FIELD_F, prec)
    s.level_set(1, mg.MG_FIELD_F, np.zeros_like(fused).astype(dt), prec)
    s.apply(mg.MG_OP_RESIDUAL, 0, prec)
    s.apply(mg.MG_OP_RESTRICT, 0, prec)
    two = s.level_get(1, mg.MG_FIELD_F, prec)
    s.close()
    print(f"one-pass residual+restriction {case}: bitwise {np.array_equal(fused, two)}", flush=True)
    assert np.array_equal(fused, two)
    if kind == "cell":
        beta = cell.harmonic_faces(k)
        ref = cell.restrict_mean(cell.residual(u, f, beta, bc))
    else:
        ref = node.restrict_fw(node.residual(u, f))
    close(fused, ref.astype(np.float64), prec, f"one-pass residual+restriction {case} vs oracle")


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [33, 129, 257, 513])
def test_fused_residual_restriction(mg, n, prec):
    """f_coarse = R (f - A u) in one pass (fused on 3-D levels with n >= 129)
    equals restriction of the oracle's residual."""
    s, h = make(mg, 3, n, 0, prec, smoother=mg.MG_RBGS)
    dt = np.float64 if prec == 0 else np.float32
    u = rand(n, 3, 0, 700 + n, dt)
    f = rand(n, 3, 0, 800 + n, dt) * dt(n * n)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(0, mg.MG_FIELD_F, f, prec)
    s.apply(mg.MG_OP_RESIDUAL_RESTRICT, 0, prec)
    got = s.level_get(1, mg.MG_FIELD_F, prec)
    ref = node.restrict_fw(node.residual(u, f))
    close(got, ref.astype(np.float64), prec, f"residual+restrict 3d n={n} prec={prec}")
    s.close()


@pytest.mark.parametrize("n,bc,nu,post", [(128, "dirichlet", 2, 0), (256, "dirichlet", 3, 0),
                                         (256, "dirichlet", 3, 1), (128, "neumann", 3, 1),
                                         (256, "neumann", 1, 0)])
def test_cell_smoothing_step_equals_half_sweeps(mg, n, bc, nu, post):
    """A smoothing step of the finest 3-D cell level (faces formed from k by
    the column-marching sweeps) equals the same number of separate red-black
    half-sweeps bitwise, and the oracle's sweeps bitwise."""
    k = W.varcoef_k(n, 3)
    s = mg.Solver(3, n, centering=mg.MG_CELL, smoother=mg.MG_RBGS, nu1=nu, nu2=nu, post_order=post, k=k,
                  bc=mg.MG_NEUMANN0 if bc == "neumann" else mg.MG_DIRICHLET0)
    u = rand(n, 3, 1, 500 + n + nu, np.float64)
    f = rand(n, 3, 1, 600 + n + nu, np.float64) * float(n * n)
    s.level_set(0, mg.MG_FIELD_U, u, 0)
    s.level_set(0, mg.MG_FIELD_F, f, 0)
    s.apply(mg.MG_OP_POSTSMOOTH if post else mg.MG_OP_PRESMOOTH, 0, 0)
    fused = s.level_get(0, mg.MG_FIELD_U, 0)
    s.level_set(0, mg.MG_FIELD_U, u, 0)
    first, second = (mg.MG_OP_GS_BLACK, mg.MG_OP_GS_RED) if post else (mg.MG_OP_GS_RED, mg.MG_OP_GS_BLACK)
    for _ in range(nu):
        s.apply(first, 0, 0)
        s.apply(second, 0, 0)
    halves = s.level_get(0, mg.MG_FIELD_U, 0)
    s.close()
    print(f"cell smoothing step n={n} {bc} nu={nu} post={post}: bitwise {np.array_equal(fused, halves)}", flush=True)
    assert np.array_equal(fused, halves)
    beta = cell.harmonic_faces(k)
    ref = u.copy()
    for _ in range(nu):
        cell.gs_colour(ref, f, beta, post, bc)
        cell.gs_colour(ref, f, beta, 1 - post, bc)
    assert np.array_equal(fused, ref)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nu,post", [(1, 0), (2, 0), (3, 0), (3, 1), (4, 0), (5, 1)])
def test_fused_sweeps_equal_half_sweeps(mg, prec, nu, post):
    """On 3-D node levels with n >= 257 the smoother runs up to three red-black
    sweeps as one temporally blocked pass: bitwise equal to the separate
    half-sweeps on the same level, and to the oracle's sweeps to the op bar."""
    n = 257
    s = mg.Solver(3, n, smoother=mg.MG_RBGS, nu1=nu, nu2=nu, post_order=post,
                  precision=mg.MG_MIXED if prec else mg.MG_FP64)
    dt = np.float64 if prec == 0 else np.float32
    u = rand(n, 3, 0, 900 + 10 * nu + post, dt)
    f = rand(n, 3, 0, 950 + 10 * nu + post, dt) * dt(n * n)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(0, mg.MG_FIELD_F, f, prec)
    s.apply(mg.MG_OP_POSTSMOOTH if post else mg.MG_OP_PRESMOOTH, 0, prec)
    fused = s.level_get(0, mg.MG_FIELD_U, prec)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    first, second = (mg.MG_OP_GS_BLACK, mg.MG_OP_GS_RED) if post else (mg.MG_OP_GS_RED, mg.MG_OP_GS_BLACK)
    for _ in range(nu):
        s.apply(first, 0, prec)
        s.apply(second, 0, prec)
    halves = s.level_get(0, mg.MG_FIELD_U, prec)
    s.close()
    assert np.array_equal(fused, halves), f"nu={nu} post={post} prec={prec}"
    ref = u.copy()
    for _ in range(nu):
        node.gs_colour(ref, f, post)
        node.gs_colour(ref, f, 1 - post)
    close(fused, ref.astype(np.float64), prec, f"fused {nu} sweeps 3d n={n} post={post} prec={prec}")


@pytest.mark.parametrize("prec,nu", [(0, 3), (0, 2), (1, 1)])
def test_fused_sweeps_513(mg, prec, nu):
    """The fused passes at the full 513^3 size (five regions across x, the
    last one partly outside the grid; two z chunks): bitwise equal to the
    separate half-sweeps, and the FP64 three-sweep pass equal to the
    oracle's sweeps to the op bar."""
    n = 513
    s = mg.Solver(3, n, smoother=mg.MG_RBGS, nu1=nu, nu2=nu, precision=mg.MG_MIXED if prec else mg.MG_FP64)
    dt = np.float64 if prec == 0 else np.float32
    u = rand(n, 3, 0, 700 + nu, dt)
    f = rand(n, 3, 0, 750 + nu, dt) * dt(n * n)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(0, mg.MG_FIELD_F, f, prec)
    s.apply(mg.MG_OP_PRESMOOTH, 0, prec)
    fused = s.level_get(0, mg.MG_FIELD_U, prec)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    for _ in range(nu):
        s.apply(mg.MG_OP_GS_RED, 0, prec)
        s.apply(mg.MG_OP_GS_BLACK, 0, prec)
    halves = s.level_get(0, mg.MG_FIELD_U, prec)
    s.close()
    print(f"513^3 fused nu={nu} prec={prec}: bitwise {np.array_equal(fused, halves)}", flush=True)
    assert np.array_equal(fused, halves)
    if prec == 0 and nu == 3:
        ref = u.copy()
        for _ in range(nu):
            node.gs_colour(ref, f, 0)
            node.gs_colour(ref, f, 1)
        close(fused, ref, prec, f"fused {nu} sweeps 3d n={n} against the oracle")


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_paths_with_non_power_of_two_scale(mg, prec):
    """385^3 nodes with a 4-node coarsest level: s = 384^2 is not a power of
    two, so the fused sweeps divide by s instead of multiplying by 1/s; the
    fused pass still equals the half-sweeps bitwise and the oracle's sweeps,
    and the fused residual + restriction equals the oracle's."""
    n = 385
    s = mg.Solver(3, n, coarsest=4, smoother=mg.MG_RBGS, nu1=3, nu2=3,
                  precision=mg.MG_MIXED if prec else mg.MG_FP64)
    dt = np.float64 if prec == 0 else np.float32
    u = rand(n, 3, 0, 1200, dt)
    f = rand(n, 3, 0, 1201, dt) * dt(n * n)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.level_set(0, mg.MG_FIELD_F, f, prec)
    s.apply(mg.MG_OP_PRESMOOTH, 0, prec)
    fused = s.level_get(0, mg.MG_FIELD_U, prec)
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    for _ in range(3):
        s.apply(mg.MG_OP_GS_RED, 0, prec)
        s.apply(mg.MG_OP_GS_BLACK, 0, prec)
    halves = s.level_get(0, mg.MG_FIELD_U, prec)
    assert np.array_equal(fused, halves)
    ref = u.copy()
    for _ in range(3):
        node.gs_colour(ref, f, 0)
        node.gs_colour(ref, f, 1)
    close(fused, ref.astype(np.float64), prec, f"fused 3 sweeps n={n} prec={prec}")
    s.level_set(0, mg.MG_FIELD_U, u, prec)
    s.apply(mg.MG_OP_RESIDUAL_RESTRICT, 0, prec)
    got = s.level_get(1, mg.MG_FIELD_F, prec)
    s.close()
    close(got, node.restrict_fw(node.residual(u, f)).astype(np.float64), prec, f"residual+restrict n={n} prec={prec}")
