// Runtime of the multigrid library: workspace plan, level hierarchy, the
// V-cycle driver, solve-to-tolerance, FP64 iterative refinement around
// single-precision cycles, level access and profiling, behind the C ABI of
// include/mg.h.
//
// The V-cycle is the textbook recursion (gamma = 1) over rediscretised
// per-level stencils, the structure that ExaSlang's coarser/coarsest levels,
// restriction/prolongation, relax and solve keywords describe (paper's
// listing vocabulary; the algorithm itself is not stated in the paper).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mg.h"
#include "mg_internal.h"
#include "mg_kernels.h"
#include "mg_runtime.h"

using namespace mg;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }
int round_up(int v, int m) { return (v + m - 1) / m * m; }

Geom make_geom(int dim, int n, int cell) {
    Geom g;
    g.dim = dim;
    g.n = n;
    g.cell = cell;
    g.nz = dim == 3 ? n : 1;
    g.ny = n;
    g.half = cell ? n / 2 : (n + 1) / 2;
    g.pitch = round_up(g.half, 8);
    g.plane = (long long)g.ny * g.pitch;
    g.cs = (long long)g.nz * g.plane;
    g.fpitch = round_up(n + 1, 8);
    g.fplane = (long long)(n + 1) * g.fpitch;
    g.fsize = (dim == 3 ? (long long)(n + 1) : 1LL) * g.fplane;
    g.neu = 0;
    return g;
}

// ----------------------------------------------------------- validation
int validate(const mg_grid* g, const mg_stencil* st, const mg_opts* o, std::string* why) {
    auto bad = [&](const char* m) {
        if (why) *why = m;
        return MG_EINVAL;
    };
    if (!g || !o) return bad("null grid or options");
    if (g->dim != 2 && g->dim != 3) return bad("dim must be 2 or 3");
    if (g->centering != MG_NODE && g->centering != MG_CELL) return bad("unknown centering");
    for (int a = 1; a < g->dim; ++a)
        if (g->n[a] != g->n[0]) return bad("all axes must have the same size");
    const int n = g->n[0], c = g->coarsest_n;
    if (g->centering == MG_NODE) {
        if (c < 3) return bad("node coarsest_n must be >= 3");
        if (n < c || (n - 1) % (c - 1)) return bad("node n must be (coarsest_n - 1) * 2^L + 1");
        const int q = (n - 1) / (c - 1);
        if (q & (q - 1)) return bad("node n must be (coarsest_n - 1) * 2^L + 1");
    } else {
        if (c < 2) return bad("cell coarsest_n must be >= 2");
        if (n < c || n % c) return bad("cell n must be coarsest_n * 2^L");
        const int q = n / c;
        if (q & (q - 1)) return bad("cell n must be coarsest_n * 2^L");
        if (c % 2) return bad("cell coarsest_n must be even");
    }
    long long m = 1;
    const int side = g->centering == MG_NODE ? c - 2 : c;
    for (int a = 0; a < g->dim; ++a) m *= side;
    if (m > 64) return bad("coarsest level has more than 64 unknowns");
    if (st) {
        if (st->kind != MG_LAPLACE && st->kind != MG_VARCOEF) return bad("unknown stencil kind");
        if (st->kind == MG_VARCOEF && g->centering != MG_CELL)
            return bad("variable coefficients need a cell-centred grid");
        if (st->kind == MG_VARCOEF && !st->k) return bad("variable coefficients need k");
    }
    if (o->smoother != MG_JACOBI && o->smoother != MG_RBGS) return bad("unknown smoother");
    if (o->precision != MG_FP64 && o->precision != MG_MIXED) return bad("unknown precision");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1) return bad("need nu1, nu2 >= 0 and nu1 + nu2 >= 1");
    if (!(o->omega > 0.0) || !(o->omega < 2.0)) return bad("omega must be in (0, 2)");
    if (o->max_cycles < 1) return bad("max_cycles must be >= 1");
    if (o->post_order != 0 && o->post_order != 1) return bad("post_order must be 0 or 1");
    if (o->cycle != MG_CYCLE_V && o->cycle != MG_CYCLE_W && o->cycle != MG_CYCLE_F) return bad("unknown cycle type");
    if (o->krylov != 0 && o->krylov != 1) return bad("krylov must be 0 or 1");
    if (o->krylov && o->precision != MG_FP64) return bad("krylov vectors need an FP64 context");
    if (o->coarse_op != MG_COARSE_REDISCRETISE && o->coarse_op != MG_COARSE_GALERKIN)
        return bad("unknown coarse operator");
    if (o->coarse_op == MG_COARSE_GALERKIN &&
        (g->centering != MG_NODE || o->smoother != MG_JACOBI || o->precision != MG_FP64))
        return bad("Galerkin coarse operators need a node grid, damped Jacobi and FP64");
    return MG_OK;
}

std::vector<int> ladder(const mg_grid* g) {
    std::vector<int> s{g->n[0]};
    int n = g->n[0];
    while (n > g->coarsest_n) {
        n = g->centering == MG_NODE ? (n - 1) / 2 + 1 : n / 2;
        s.push_back(n);
    }
    return s;
}

}  // namespace

// =================================================================== plan
namespace mg {

size_t plan_workspace(const mg_grid* g, const mg_stencil* st, const mg_opts* o, Plan* out, bool staging) {
    Plan p;
    const int cell = g->centering == MG_CELL;
    const bool varcoef = cell;   // cell grids always carry face coefficients
    const bool mixed = o->precision == MG_MIXED;
    const bool jac = o->smoother == MG_JACOBI;
    (void)st;
    std::vector<int> sizes = ladder(g);
    p.L = (int)sizes.size();
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(bytes);
        return at;
    };
    for (int l = 0; l < p.L; ++l) {
        LevelPlan lp;
        lp.g = make_geom(g->dim, sizes[l], cell);
        for (int pr = 0; pr < 2; ++pr) {
            const bool has = pr == 0 ? (!mixed || l == 0) : mixed;
            lp.has[pr] = has;
            if (!has) continue;
            const size_t es = pr == 0 ? 8 : 4;
            const size_t fb = (size_t)(2 * lp.g.cs) * es;
            lp.u[pr] = take(fb);
            lp.f[pr] = take(fb);
            lp.r[pr] = take(fb);
            // a second iterate: Jacobi's output, or the out-of-place target of
            // fused red-black sweeps on large 3-D node levels
            const bool smoothed = !(mixed && pr == 0);
            // (mixed FP64 finest level that marches columns: the out-of-place
            // target of the fused update, residual and cast)
            const bool fused_update = mixed && pr == 0 && l == 0 && !cell && use_zmarch(lp.g);
            const bool need_tmp = (smoothed && (jac || (!cell && use_tb(lp.g)))) || fused_update;
            lp.utmp[pr] = need_tmp ? take(fb) : SIZE_MAX;
            for (int a = 0; a < 3; ++a)
                lp.beta[pr][a] = (varcoef && a < g->dim) ? take((size_t)lp.g.fsize * es) : SIZE_MAX;
        }
        // the finest 3-D cell level's kernels form its faces from k
        if (l == 0 && cell && lp.has[0] && use_cell_zm(lp.g)) lp.k = take((size_t)(2 * lp.g.cs) * 8);
        p.lv.push_back(lp);
    }
    const Geom& g0 = p.lv[0].g;
    p.partial_pairs = residual_blocks(g0);
    p.partials = take((size_t)p.partial_pairs * 16);
    p.reduce_scratch = take((size_t)reduce_scratch_pairs(p.partial_pairs) * 16);
    p.red = take(64);   // [sum r^2, max |r|, sigma, scale basis, projection sum, next sigma, -, -]
    const Geom& gc = p.lv.back().g;
    const int side = cell ? gc.n : gc.n - 2;
    p.m = side * side * (g->dim == 3 ? side : 1);
    p.chol = take((size_t)p.m * p.m * 8);
    const long long nat = (long long)g0.n * g0.n * (g->dim == 3 ? g0.n : 1);
    p.staging = staging ? take((size_t)nat * 8) : SIZE_MAX;
    if (o->krylov) {
        const size_t fb = (size_t)(2 * g0.cs) * 8;
        p.pcg = take(5 * align_up(fb) + (size_t)(dot_blocks(fb) + reduce_scratch_pairs(dot_blocks(fb))) * 16 + 64);
    }
    p.total = off;
    if (out) *out = p;
    return off;
}

}  // namespace mg

// ============================================================ host numerics
namespace {

// Face coefficients of the finest cell level from cell values k (FP64):
// interior face 2 ka kb / (ka + kb) evaluated as ((2 ka) kb) / (ka + kb) with
// ka the lower cell, wall face the adjacent cell's k.  Stored in the device
// face layout [z][y][x] with row pitch fpitch and plane fplane.
void harmonic_faces(const Geom& g, const double* k, std::vector<double> beta[3]) {
    const int N = g.n, d = g.dim;
    const int nz = d == 3 ? N : 1;
    for (int a = 0; a < d; ++a) beta[a].assign((size_t)g.fsize, 0.0);
    auto K = [&](int x, int y, int z) { return k[((size_t)z * N + y) * N + x]; };
    auto at = [&](std::vector<double>& b, int x, int y, int z) -> double& {
        return b[(size_t)z * g.fplane + (size_t)y * g.fpitch + x];
    };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x <= N; ++x) {
                double v;
                if (x == 0) v = K(0, y, z);
                else if (x == N) v = K(N - 1, y, z);
                else {
                    const double ka = K(x - 1, y, z), kb = K(x, y, z);
                    v = ((2.0 * ka) * kb) / (ka + kb);
                }
                at(beta[0], x, y, z) = v;
            }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y <= N; ++y)
            for (int x = 0; x < N; ++x) {
                double v;
                if (y == 0) v = K(x, 0, z);
                else if (y == N) v = K(x, N - 1, z);
                else {
                    const double ka = K(x, y - 1, z), kb = K(x, y, z);
                    v = ((2.0 * ka) * kb) / (ka + kb);
                }
                at(beta[1], x, y, z) = v;
            }
    if (d == 3)
        for (int z = 0; z <= N; ++z)
            for (int y = 0; y < N; ++y)
                for (int x = 0; x < N; ++x) {
                    double v;
                    if (z == 0) v = K(x, y, 0);
                    else if (z == N) v = K(x, y, N - 1);
                    else {
                        const double ka = K(x, y, z - 1), kb = K(x, y, z);
                        v = ((2.0 * ka) * kb) / (ka + kb);
                    }
                    at(beta[2], x, y, z) = v;
                }
}

// Coarse face = mean of the 2^(d-1) fine faces that tile it: fine face 2I
// along the face's axis, index pairs (2J, 2J+1) along the others, summed
// with the lower array axis slowest, then scaled by 1 / 2^(d-1).
void coarsen_faces(const Geom& gf, const std::vector<double> bf[3], const Geom& gc, std::vector<double> bc[3]) {
    const int d = gf.dim, Nc = gc.n;
    const double sc = d == 3 ? 0.25 : 0.5;
    auto F = [&](const std::vector<double>& b, int x, int y, int z) {
        return b[(size_t)z * gf.fplane + (size_t)y * gf.fpitch + x];
    };
    for (int a = 0; a < d; ++a) bc[a].assign((size_t)gc.fsize, 0.0);
    const int ncz = d == 3 ? Nc : 1;
    // x faces: others are (z, y) in 3-D, (y) in 2-D
    for (int z = 0; z < ncz; ++z)
        for (int y = 0; y < Nc; ++y)
            for (int x = 0; x <= Nc; ++x) {
                double acc;
                if (d == 3)
                    acc = ((F(bf[0], 2 * x, 2 * y, 2 * z) + F(bf[0], 2 * x, 2 * y + 1, 2 * z)) +
                           F(bf[0], 2 * x, 2 * y, 2 * z + 1)) + F(bf[0], 2 * x, 2 * y + 1, 2 * z + 1);
                else
                    acc = F(bf[0], 2 * x, 2 * y, 0) + F(bf[0], 2 * x, 2 * y + 1, 0);
                bc[0][(size_t)z * gc.fplane + (size_t)y * gc.fpitch + x] = acc * sc;
            }
    // y faces: others are (z, x) in 3-D, (x) in 2-D
    for (int z = 0; z < ncz; ++z)
        for (int y = 0; y <= Nc; ++y)
            for (int x = 0; x < Nc; ++x) {
                double acc;
                if (d == 3)
                    acc = ((F(bf[1], 2 * x, 2 * y, 2 * z) + F(bf[1], 2 * x + 1, 2 * y, 2 * z)) +
                           F(bf[1], 2 * x, 2 * y, 2 * z + 1)) + F(bf[1], 2 * x + 1, 2 * y, 2 * z + 1);
                else
                    acc = F(bf[1], 2 * x, 2 * y, 0) + F(bf[1], 2 * x + 1, 2 * y, 0);
                bc[1][(size_t)z * gc.fplane + (size_t)y * gc.fpitch + x] = acc * sc;
            }
    // z faces: others are (y, x)
    if (d == 3)
        for (int z = 0; z <= Nc; ++z)
            for (int y = 0; y < Nc; ++y)
                for (int x = 0; x < Nc; ++x) {
                    const double acc = ((F(bf[2], 2 * x, 2 * y, 2 * z) + F(bf[2], 2 * x + 1, 2 * y, 2 * z)) +
                                        F(bf[2], 2 * x, 2 * y + 1, 2 * z)) + F(bf[2], 2 * x + 1, 2 * y + 1, 2 * z);
                    bc[2][(size_t)z * gc.fplane + (size_t)y * gc.fpitch + x] = acc * sc;
                }
}

// Dense FP64 matrix of the coarsest level over its unknowns in C order.
// Stencil index of the offset (oz, oy, ox), z slowest (2-D: oz = 0, 9 entries).
int st_index(int d, int oz, int oy, int ox) { return (d == 3 ? 9 * (oz + 1) : 0) + 3 * (oy + 1) + (ox + 1); }

// The 5/7-point Laplacian of a node level as a 3^d stencil: 2d s at the
// centre, -s at the axis neighbours, s = (n - 1)^2.
Stencil27 laplacian27(const Geom& g) {
    Stencil27 W{};
    const int d = g.dim;
    const double s = (double)(g.n - 1) * (g.n - 1);
    W.w[st_index(d, 0, 0, 0)] = 2.0 * d * s;
    W.w[st_index(d, 0, 0, -1)] = -s;
    W.w[st_index(d, 0, 0, 1)] = -s;
    W.w[st_index(d, 0, -1, 0)] = -s;
    W.w[st_index(d, 0, 1, 0)] = -s;
    if (d == 3) {
        W.w[st_index(d, -1, 0, 0)] = -s;
        W.w[st_index(d, 1, 0, 0)] = -s;
    }
    return W;
}

// Galerkin coarse stencil R A P of a constant fine stencil: full weighting
// R (weights prod (2 - |a_k|) / 4 over offsets a) and linear interpolation P
// (weight prod phi(v_k), phi(0) = 1, phi(+-1) = 1/2), so that the coarse
// entry at offset J is sum_a R_a sum_b W_b phi(a + b - 2 J).
Stencil27 galerkin_coarse(const Stencil27& Wf, int d) {
    auto phi = [](int v) { return v == 0 ? 1.0 : (v == 1 || v == -1 ? 0.5 : 0.0); };
    auto rho = [](int a) { return a == 0 ? 0.5 : 0.25; };
    const int zl = d == 3 ? -1 : 0, zh = d == 3 ? 1 : 0;
    Stencil27 Wc{};
    for (int jz = zl; jz <= zh; ++jz)
        for (int jy = -1; jy <= 1; ++jy)
            for (int jx = -1; jx <= 1; ++jx) {
                double acc = 0.0;
                for (int az = zl; az <= zh; ++az)
                    for (int ay = -1; ay <= 1; ++ay)
                        for (int ax = -1; ax <= 1; ++ax) {
                            double inner = 0.0;
                            for (int bz = zl; bz <= zh; ++bz)
                                for (int by = -1; by <= 1; ++by)
                                    for (int bx = -1; bx <= 1; ++bx) {
                                        const double ph = phi(ax + bx - 2 * jx) * phi(ay + by - 2 * jy) *
                                                          (d == 3 ? phi(az + bz - 2 * jz) : 1.0);
                                        inner += Wf.w[st_index(d, bz, by, bx)] * ph;
                                    }
                            acc += rho(ax) * rho(ay) * (d == 3 ? rho(az) : 1.0) * inner;
                        }
                Wc.w[st_index(d, jz, jy, jx)] = acc;
            }
    return Wc;
}

// With Neumann walls the matrix is singular (constants); a 1 1^T with a the
// mean diagonal over m is added, which makes it SPD and leaves the solution
// for a zero-mean right-hand side that of A itself with zero mean.  With a
// Galerkin stencil W the node-grid matrix is assembled from W.
std::vector<double> coarse_matrix(const Geom& g, const std::vector<double>* beta, const Stencil27* W) {
    const int d = g.dim;
    const int side = g.cell ? g.n : g.n - 2, off = g.cell ? 0 : 1;
    const int m = side * side * (d == 3 ? side : 1);
    std::vector<double> A((size_t)m * m, 0.0);
    auto idx = [&](int x, int y, int z) { return ((z - (d == 3 ? off : 0)) * side + (y - off)) * side + (x - off); };
    const double s = g.cell ? (double)g.n * g.n : (double)(g.n - 1) * (g.n - 1);
    const int zlo = d == 3 ? off : 0, zhi = d == 3 ? off + side : 1;
    for (int z = zlo; z < zhi; ++z)
        for (int y = off; y < off + side; ++y)
            for (int x = off; x < off + side; ++x) {
                const int i = idx(x, y, z);
                if (!g.cell && W) {
                    for (int oz = (d == 3 ? -1 : 0); oz <= (d == 3 ? 1 : 0); ++oz)
                        for (int oy = -1; oy <= 1; ++oy)
                            for (int ox = -1; ox <= 1; ++ox) {
                                const int X = x + ox, Y = y + oy, Z = z + oz;
                                if (X < 1 || X > g.n - 2 || Y < 1 || Y > g.n - 2) continue;
                                if (d == 3 && (Z < 1 || Z > g.n - 2)) continue;
                                A[(size_t)i * m + idx(X, Y, Z)] = W->w[st_index(d, oz, oy, ox)];
                            }
                } else if (!g.cell) {
                    A[(size_t)i * m + i] = (double)(2 * d) * s;
                    const int nbx[6] = {x - 1, x + 1, x, x, x, x}, nby[6] = {y, y, y - 1, y + 1, y, y},
                              nbz[6] = {z, z, z, z, z - 1, z + 1};
                    for (int q = 0; q < 2 * d; ++q) {
                        const int X = nbx[q], Y = nby[q], Z = nbz[q];
                        if (X < 1 || X > g.n - 2 || Y < 1 || Y > g.n - 2) continue;
                        if (d == 3 && (Z < 1 || Z > g.n - 2)) continue;
                        A[(size_t)idx(X, Y, Z) * m + i] = (0.0 - 1.0) * s;
                    }
                } else {
                    const int N = g.n;
                    auto B = [&](int a, int X, int Y, int Z) {
                        return beta[a][(size_t)Z * g.fplane + (size_t)Y * g.fpitch + X];
                    };
                    // faces in the order x-, x+, y-, y+, z-, z+
                    const double bf[6] = {B(0, x, y, z), B(0, x + 1, y, z), B(1, x, y, z), B(1, x, y + 1, z),
                                          d == 3 ? B(2, x, y, z) : 0.0, d == 3 ? B(2, x, y, z + 1) : 0.0};
                    const bool wall[6] = {x == 0, x == N - 1, y == 0, y == N - 1, z == 0, z == N - 1};
                    const int nbx[6] = {x - 1, x + 1, x, x, x, x}, nby[6] = {y, y, y - 1, y + 1, y, y},
                              nbz[6] = {z, z, z, z, z - 1, z + 1};
                    double dg = 0.0;
                    const double ww = g.neu ? 0.0 : 2.0;
                    for (int q = 0; q < 2 * d; ++q) {
                        const double t = wall[q] ? ww * bf[q] : bf[q];
                        dg = q == 0 ? t : dg + t;
                    }
                    A[(size_t)i * m + i] = (dg * 1.0 - 0.0) * s;
                    for (int q = 0; q < 2 * d; ++q) {
                        if (wall[q]) continue;
                        A[(size_t)idx(nbx[q], nby[q], nbz[q]) * m + i] = (0.0 - bf[q]) * s;
                    }
                }
            }
    if (g.neu) {
        double tr = 0.0;
        for (int i = 0; i < m; ++i) tr += A[(size_t)i * m + i];
        const double a = tr / m / m;
        for (double& v : A) v += a;
    }
    return A;
}

// Textbook Cholesky A = L L^T (row-oriented); false if A is not SPD.
bool cholesky(std::vector<double>& A, int m) {
    std::vector<double> L((size_t)m * m, 0.0);
    for (int j = 0; j < m; ++j) {
        double dsum = A[(size_t)j * m + j];
        for (int k = 0; k < j; ++k) dsum -= L[(size_t)j * m + k] * L[(size_t)j * m + k];
        if (!(dsum > 0.0)) return false;
        const double ljj = std::sqrt(dsum);
        L[(size_t)j * m + j] = ljj;
        for (int i = j + 1; i < m; ++i) {
            double v = A[(size_t)i * m + j];
            for (int k = 0; k < j; ++k) v -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
            L[(size_t)i * m + j] = v / ljj;
        }
    }
    A.swap(L);
    return true;
}

}  // namespace

// ============================================================ the context
namespace mg {

int Ctx::fail(int code, const std::string& msg) {
    err = msg;
    return code;
}

int Ctx::dev(hipError_t e, const char* what) {
    if (e == hipSuccess) return MG_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return MG_EDEVICE;
}

void* Ctx::at(size_t off) const { return off == SIZE_MAX ? nullptr : static_cast<char*>(base) + off; }

Faces Ctx::faces(int l, int pr) const {
    Faces f;
    for (int a = 0; a < 3; ++a) f.b[a] = lv[l].beta[pr][a];
    f.k = pr == 0 ? lv[l].k : nullptr;
    return f;
}

double Ctx::scale(int l) const {
    const Geom& g = lv[l].g;
    return g.cell ? (double)g.n * g.n : (double)(g.n - 1) * (g.n - 1);
}

int Ctx::record(int kclass, int level, hipError_t e, hipEvent_t e0, const char* what) {
    if (prof) {
        hipEvent_t e1 = event();
        (void)hipEventRecord(e1, stream);
        recs.push_back({kclass, level, e0, e1});
    }
    return dev(e, what);
}

hipEvent_t Ctx::begin() {
    if (!prof) return nullptr;
    hipEvent_t e0 = event();
    (void)hipEventRecord(e0, stream);
    return e0;
}

hipEvent_t Ctx::event() {
    if (ev_used == ev_pool.size()) {
        hipEvent_t e;
        (void)hipEventCreate(&e);
        ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
}

// ------------------------------------------------------------- recording
// In recording mode (rec != null) the level ops below append batched-op
// descriptors instead of launching; the serving path records one refinement
// step of a request this way, so a served request runs exactly the op
// sequence and operands of a stand-alone mixed-precision solve.
BItem Ctx::item(int op, int l) const {
    BItem it;
    std::memset(&it, 0, sizeof(it));
    it.op = op;
    it.dim = grid.dim;
    it.g = lv[l].g;
    it.s = scale(l);
    it.omega = opts.omega;
    it.red = red;
    return it;
}

int Ctx::push(BItem it) {
    if (!(it.tiles > 0)) it.tiles = it.sp.blocks();
    if (it.w < 1) it.w = 1;
    rec->push_back(it);
    return MG_OK;
}

int Ctx::rec_check(int pr, bool want_fp32) {
    if (grid.centering != MG_NODE) return fail(MG_EINVAL, "batched execution supports node grids");
    if (want_fp32 != (pr == 1)) return fail(MG_EINVAL, "batched execution runs FP32 cycles only");
    return MG_OK;
}

// ------------------------------------------------------------- level ops
int Ctx::gs(int l, int pr, int colour, bool zero) {
    Level& L = lv[l];
    if (rec) {
        if (int rc = rec_check(pr, true)) return rc;
        const bool march = !zero && use_zmarch(L.g) && 64 * kZRows == 256;
        BItem it = item(march ? BOP_GS_M : (zero ? BOP_GS_ZERO : BOP_GS), l);
        it.sp = level_space(L.g, 1, colour);
        if (march) {
            it.zs = make_zspace(L.g);
            it.tiles = it.zs.blocks();
            it.w = it.zs.zc;
            it.m = colour;
        }
        it.a = static_cast<float*>(L.u[pr]) + (long long)colour * L.g.cs;
        it.b = static_cast<float*>(L.u[pr]) + (long long)(1 - colour) * L.g.cs;
        it.c = static_cast<float*>(L.f[pr]) + (long long)colour * L.g.cs;
        return push(it);
    }
    hipEvent_t e0 = begin();
    return record(MG_K_SMOOTH, l, launch_gs(L.g, pr, colour, zero, L.u[pr], L.f[pr], faces(l, pr), scale(l), stream),
                  e0, "gs");
}

int Ctx::jacobi(int l, int pr, bool zero) {
    Level& L = lv[l];
    if (rec) {
        if (int rc = rec_check(pr, true)) return rc;
        const bool march = use_ymarch_batched(L.g);
        BItem it = item(march ? (zero ? BOP_JAC_ZERO_M : BOP_JAC_M) : (zero ? BOP_JAC_ZERO : BOP_JAC), l);
        it.sp = level_space(L.g, 2, 0);
        if (march) {
            it.ys = make_yspace(L.g);
            it.tiles = it.ys.blocks();
            it.w = 2 * it.ys.yc;
        }
        it.a = L.u[pr];
        it.b = L.f[pr];
        it.c = L.utmp[pr];
        push(it);
        std::swap(L.u[pr], L.utmp[pr]);
        return MG_OK;
    }
    hipEvent_t e0 = begin();
    int rc = record(MG_K_SMOOTH, l,
                    L.gal ? launch_jacobi27(L.g, zero, L.u[pr], L.f[pr], L.utmp[pr], L.W, opts.omega, stream)
                          : launch_jacobi(L.g, pr, zero, L.u[pr], L.f[pr], L.utmp[pr], faces(l, pr), scale(l),
                                          opts.omega, stream),
                    e0, "jacobi");
    if (rc) return rc;
    std::swap(L.u[pr], L.utmp[pr]);
    return MG_OK;
}

int Ctx::smooth(int l, int pr, int sweeps, bool from_zero, int first_colour) {
    Level& L = lv[l];
    if (sweeps == 0 && from_zero && rec) {
        BItem it = item(BOP_ZERO, l);
        it.a = L.u[pr];
        it.n = (long long)(L.field_bytes[pr] / 16);
        it.tiles = (it.n + 255) / 256;
        push(it);
    } else if (sweeps == 0 && from_zero) {
        hipEvent_t e0 = begin();
        int rc = record(MG_K_COPY, l, launch_zero(L.u[pr], L.field_bytes[pr], stream), e0, "zero");
        if (rc) return rc;
    }
    int done = 0;
    if (opts.smoother == MG_RBGS && !rec && sweeps > 1 && L.utmp[pr] && use_tb(L.g)) {
        // two or three sweeps per fused pass, out of place (a lone sweep
        // runs faster as two half-sweeps)
        for (int left = sweeps; left > 1;) {
            const int k = left == 4 ? 2 : (left < 3 ? left : 3);
            hipEvent_t e0 = begin();
            int rc = record(MG_K_SMOOTH, l,
                            launch_gs_tb(L.g, pr, k, first_colour, from_zero && done == 0, L.u[pr], L.f[pr],
                                         L.utmp[pr], scale(l), stream),
                            e0, "gs_tb");
            if (rc) return rc;
            std::swap(L.u[pr], L.utmp[pr]);
            left -= k;
            done += k;
        }
    }
    if (opts.smoother == MG_JACOBI && !rec && grid.centering == MG_NODE && !L.gal && L.utmp[pr] &&
        fused_point_transfers(L.g)) {
        // 2-D point levels: two sweeps per launch (tiles with a halo of two)
        for (; done + 2 <= sweeps; done += 2) {
            hipEvent_t e0 = begin();
            int rc = record(MG_K_SMOOTH, l,
                            launch_jacobi2(L.g, nullptr, pr, from_zero && done == 0, L.u[pr], nullptr, L.f[pr],
                                           L.utmp[pr], nullptr, scale(l), opts.omega, stream),
                            e0, "jacobi x2");
            if (rc) return rc;
            std::swap(L.u[pr], L.utmp[pr]);
        }
    }
    for (int k = done; k < sweeps; ++k) {
        const bool z = from_zero && k == 0;
        int rc;
        if (opts.smoother == MG_RBGS) {
            rc = gs(l, pr, first_colour, z);
            if (!rc) rc = gs(l, pr, 1 - first_colour, false);
        } else {
            rc = jacobi(l, pr, z);
        }
        if (rc) return rc;
    }
    return MG_OK;
}

int Ctx::residual(int l, int pr, bool norm, bool store, bool reduce) {
    Level& L = lv[l];
    if (rec) {
        if (pr == 0 && !(norm && store)) return fail(MG_EINVAL, "batched FP64 residual carries its norm");
        if (pr == 1 && norm) return fail(MG_EINVAL, "batched FP32 residual has no norm");
        if (grid.centering != MG_NODE) return fail(MG_EINVAL, "batched execution supports node grids");
        const bool zm = use_zmarch(L.g) && 64 * kZRows == 256, ym = use_ymarch_batched(L.g);
        BItem it = item(zm || ym ? (pr == 0 ? BOP_RES64_M : BOP_RES32_M) : (pr == 0 ? BOP_RES64 : BOP_RES32), l);
        it.sp = level_space(L.g, 2, 0);
        if (zm) {
            it.zs = make_zspace(L.g);
            it.tiles = it.zs.blocks();
            it.w = 2 * it.zs.zc;
        } else if (ym) {
            it.ys = make_yspace(L.g);
            it.tiles = it.ys.blocks();
            it.w = 2 * it.ys.yc;
        } else {
            it.tiles = it.sp.blocks();
        }
        it.a = L.u[pr];
        it.b = L.f[pr];
        it.c = L.r[pr];
        it.part = partials;
        push(it);
        last_partials = it.tiles;
        return pr == 0 && reduce ? reduce_norm(l) : MG_OK;
    }
    long long nb = 0;
    hipEvent_t e0 = begin();
    int rc = record(MG_K_RESIDUAL, l,
                    L.gal ? launch_residual27(L.g, L.u[pr], L.f[pr], L.r[pr], L.W, norm, store, partials, &nb, stream)
                          : launch_residual(L.g, pr, L.u[pr], L.f[pr], L.r[pr], faces(l, pr), scale(l), norm, store,
                                            partials, &nb, stream),
                    e0, "residual");
    last_partials = nb;
    if (rc || !norm || !reduce) return rc;
    return reduce_norm(l);
}

// (sum r^2, max |r|) of the last residual's partials into red[0..1]; for the
// finest FP64 residual of a mixed-precision context the maximum is also
// kept in red[3] as the scale basis of the next refinement step's cast.
int Ctx::reduce_norm(int l) {
    const bool basis = opts.precision == MG_MIXED && l == 0;
    if (rec) {
        BItem rd = item(BOP_REDUCE, l);
        rd.part = partials;
        rd.n = last_partials;
        rd.res = rec_res;
        rd.tiles = 1;
        rd.m = basis ? 1 : 0;
        return push(rd);
    }
    hipEvent_t e0 = begin();
    int rc = record(MG_K_REDUCE, l,
                    launch_reduce(partials, last_partials, reduce_scratch, red, stream, basis ? red + 3 : nullptr), e0,
                    "reduce");
    if (!rc && basis) scale_known = true;
    return rc;
}

// The FP64 residual of a refinement step and its cast to the right-hand
// side of the single-precision cycle, fl32(r / sigma), sigma the power of
// two of the previous residual's maximum (red[3]; stored to red[2] for the
// update); the norms go to red[0..1] and the maximum to red[3].  Without a
// previous residual (first: a new right-hand side or iterate) the step's own
// maximum is reduced first and taken.  On 3-D node levels
// that march columns the residual is cast as it is formed (no FP64 residual
// is stored); elsewhere r64 is stored, cast, and reduced.
int Ctx::residual_cast(bool first) {
    Level& L0 = lv[0];
    if (!rec && grid.centering == MG_NODE && !L0.gal && use_zmarch(L0.g)) {
        if (first) {
            if (int rc = residual(0, 0, true, false)) return rc;
        }
        long long nb = 0;
        hipEvent_t e0 = begin();
        int rc = record(MG_K_RESIDUAL, 0,
                        launch_residual_cast(L0.g, L0.u[0], L0.f[0], static_cast<float*>(L0.f[1]), scale(0), red + 3,
                                             red + 2, partials, &nb, stream),
                        e0, "residual+cast");
        last_partials = nb;
        return rc ? rc : reduce_norm(0);
    }
    int rc = residual(0, 0, true, true, false);
    if (!rc && first) rc = reduce_norm(0);
    if (rc) return rc;
    if (rec) {
        BItem ca = item(BOP_CAST, 0);
        ca.n = field_quads(L0.g);
        ca.tiles = (ca.n + 255) / 256;
        ca.a = L0.r[0];
        ca.b = L0.f[1];
        push(ca);
    } else {
        hipEvent_t e0 = begin();
        rc = record(MG_K_CAST, 0,
                    launch_cast(L0.g, static_cast<const double*>(L0.r[0]), static_cast<float*>(L0.f[1]), red + 3,
                                red + 2, stream),
                    e0, "cast");
    }
    if (!rc && !first) rc = reduce_norm(0);
    return rc;
}

// Whether a refinement step's update can run fused with the next residual
// and cast (update_residual_cast).
bool Ctx::fused_update() const {
    const Level& L0 = lv[0];
    return opts.precision == MG_MIXED && !rec && grid.centering == MG_NODE && !L0.gal && use_zmarch(L0.g) &&
           L0.utmp[0] != nullptr;
}

// The deferred update of a refinement step, u64 + sigma fl64(c) written to
// the second FP64 iterate (which then becomes the iterate), and the next
// step's residual, cast and norms, in one pass; the reduction then moves
// the new sigma from red[5] to red[2].
int Ctx::update_residual_cast() {
    Level& L0 = lv[0];
    long long nb = 0;
    hipEvent_t e0 = begin();
    int rc = record(MG_K_RESIDUAL, 0,
                    launch_update_residual_cast(L0.g, static_cast<const double*>(L0.u[0]),
                                                static_cast<const float*>(L0.u[1]), static_cast<const double*>(L0.f[0]),
                                                static_cast<double*>(L0.utmp[0]), static_cast<float*>(L0.f[1]),
                                                scale(0), red, partials, &nb, stream),
                    e0, "update+residual+cast");
    if (rc) return rc;
    std::swap(L0.u[0], L0.utmp[0]);
    last_partials = nb;
    hipEvent_t e1 = begin();
    return record(MG_K_REDUCE, 0, launch_reduce(partials, last_partials, reduce_scratch, red, stream, red + 3, red + 5,
                                                red + 2),
                  e1, "reduce");
}

int Ctx::restrict_to(int l, int pr) {
    if (rec) {
        if (int rc = rec_check(pr, true)) return rc;
        BItem it = item(BOP_RESTRICT, l);
        it.gc = lv[l + 1].g;
        it.sp = level_space(lv[l + 1].g, 2, 0);
        it.a = lv[l].r[pr];
        it.b = lv[l + 1].f[pr];
        return push(it);
    }
    hipEvent_t e0 = begin();
    return record(MG_K_RESTRICT, l, launch_restrict(lv[l].g, lv[l + 1].g, pr, lv[l].r[pr], lv[l + 1].f[pr], stream),
                  e0, "restrict");
}

int Ctx::prolong(int l, int pr, int mask) {
    if (rec) {
        if (int rc = rec_check(pr, true)) return rc;
        BItem it = item(BOP_PROLONG, l);
        it.gc = lv[l + 1].g;
        it.sp = level_space(lv[l].g, mask == 3 ? 2 : 1, mask == 2 ? 1 : 0);
        it.a = lv[l].u[pr];
        it.b = lv[l + 1].u[pr];
        return push(it);
    }
    hipEvent_t e0 = begin();
    return record(MG_K_PROLONG, l,
                  launch_prolong(lv[l].g, lv[l + 1].g, pr, lv[l].u[pr], lv[l + 1].u[pr], mask, stream), e0,
                  "prolong");
}

int Ctx::coarse(int pr) {
    const int l = L - 1;
    if (rec) {
        if (int rc = rec_check(pr, true)) return rc;
        BItem it = item(BOP_COARSE, l);
        it.a = lv[l].f[pr];
        it.b = lv[l].u[pr];
        it.L = chol;
        it.m = m;
        it.tiles = 1;
        return push(it);
    }
    hipEvent_t e0 = begin();
    return record(MG_K_COARSE, l, launch_coarse(lv[l].g, pr, lv[l].f[pr], lv[l].u[pr], chol, m, stream), e0,
                  "coarse");
}

// One V(nu1, nu2)-cycle on level l of hierarchy pr.  from_zero: the level's
// current iterate is zero (coarse levels, and the single-precision finest
// level inside refinement), so the first sweep reads no neighbour values and
// no zero fill is needed.
int Ctx::vcycle(int l, int pr, bool from_zero) { return cycle(l, pr, from_zero, opts.cycle); }

// Full multigrid: f restricted to every level, the coarsest solved exactly,
// each finer level started from the interpolated coarser solution and given
// cpl cycles of the context's type.  FP64 contexts.
int Ctx::fmg(int cpl) {
    const int pr = 0;
    for (int l = 0; l + 1 < L; ++l) {
        hipEvent_t e0 = begin();
        int rc = record(MG_K_RESTRICT, l,
                        launch_restrict(lv[l].g, lv[l + 1].g, pr, lv[l].f[pr], lv[l + 1].f[pr], stream), e0,
                        "restrict f");
        if (!rc && neu) rc = project(l + 1, lv[l + 1].f[pr]);
        if (rc) return rc;
    }
    int rc = coarse(pr);
    for (int l = L - 2; l >= 0 && !rc; --l) {
        hipEvent_t e0 = begin();
        rc = record(MG_K_COPY, l, launch_zero(lv[l].u[pr], lv[l].field_bytes[pr], stream), e0, "zero");
        if (!rc) rc = prolong(l, pr, 3);
        for (int k = 0; k < cpl && !rc; ++k) rc = cycle(l, pr, false, opts.cycle);
    }
    return rc;
}

// The levels small enough to keep their fields in one workgroup's LDS run a
// V-cycle as one launch (k_tail): the largest level from which the iterate,
// a second buffer and the right-hand side of every level down to the
// coarsest, and the coarsest factor, fit in kTailLdsBytes (rediscretised
// operators, Dirichlet walls,
// Jacobi or red-black smoothing, at most kTailMax levels; cell levels read
// their face coefficients from device memory).
void Ctx::plan_tail() {
    for (int pr = 0; pr < 2; ++pr) {
        tail_l[pr] = -1;
        if (neu || m > 64) continue;
        if (opts.smoother != MG_JACOBI && opts.smoother != MG_RBGS) continue;
        const long long esz = pr ? 4 : 8;
        for (int l0 = std::max(0, L - kTailMax); l0 <= L - 2; ++l0) {
            bool ok = true;
            long long elems = 0;
            for (int l = l0; l < L; ++l) {
                if (lv[l].gal || !lv[l].has[pr]) ok = false;
                elems += 3 * ((2 * tail_geom(lv[l].g).cs + 3) / 4 * 4);
            }
            if (!ok || (elems * esz + 7) / 8 * 8 + 8LL * m * m > kTailLdsBytes) continue;
            // 2-D damped Jacobi: levels above 17^2 run faster as the
            // two-sweep tile launches than inside the one workgroup
            if (grid.dim == 2 && opts.smoother == MG_JACOBI && lv[l0].g.n > kTail2DJacobiMax) continue;
            TailPlan& P = tail[pr];
            P = TailPlan{};
            P.nl = L - l0;
            P.rbgs = opts.smoother == MG_RBGS ? 1 : 0;
            P.nu1 = opts.nu1;
            P.nu2 = opts.nu2;
            P.post_order = opts.post_order;
            P.m = m;
            P.omega = opts.omega;
            P.chol = chol;
            P.g0 = lv[l0].g;
            int mask = 3;
            if (opts.smoother == MG_RBGS && opts.nu2 > 0) mask = opts.post_order == 0 ? 2 : 1;
            int off = 0;
            P.p2 = 1;
            for (int i = 0; i < P.nl; ++i) {
                const Geom lg = tail_geom(lv[l0 + i].g);
                const int fe = (int)((2 * lg.cs + 3) / 4 * 4);
                P.lg[i] = lg;
                P.one[i][0] = level_space(lg, 1, 0);
                P.one[i][1] = level_space(lg, 1, 1);
                P.all[i] = level_space(lg, 2, 0);
                P.pro[i] = level_space(lg, mask == 3 ? 2 : 1, mask == 2 ? 1 : 0);
                P.oa[i] = off;
                P.ob[i] = off + fe;
                P.of[i] = off + 2 * fe;
                off += 3 * fe;
                P.s[i] = scale(l0 + i);
                P.rs[i] = 1.0 / P.s[i];
                if (!pow2_scale(P.s[i])) P.p2 = 0;
                for (int a = 0; a < 3; ++a) P.beta[i][a] = lv[l0 + i].beta[pr][a];
            }
            P.elems = off;
            tail_l[pr] = l0;
            break;
        }
    }
}

int Ctx::tail_cycle(int l, int pr, bool from_zero) {
    TailPlan P = tail[pr];
    P.from_zero = from_zero ? 1 : 0;
    hipEvent_t e0 = begin();
    return record(MG_K_COARSE, l, launch_tail(P, pr, lv[l].f[pr], lv[l].u[pr], stream), e0, "coarse levels");
}

// Residual of level l restricted into level l + 1's right-hand side: one
// pass where a fused kernel exists (3-D node levels that march columns, 2-D
// node point levels, the finest cell level with k), else the two operations.
int Ctx::residual_restrict(int l, int pr) {
    const Geom& g = lv[l].g;
    const char* what = "residual+restrict";
    if (!rec && grid.centering == MG_NODE && !lv[l].gal && fused_transfers(g)) {
        // fine residual and full weighting in one pass; r is not written
        hipEvent_t e0 = begin();
        return record(MG_K_RESTRICT, l,
                      launch_residual_restrict(g, lv[l + 1].g, pr, lv[l].u[pr], lv[l].f[pr], lv[l + 1].f[pr],
                                               scale(l), stream),
                      e0, what);
    }
    if (!rec && grid.centering == MG_CELL && pr == 0 && faces(l, pr).k && cell_res_restrict_fused(g)) {
        // the finest cell level: residual and 8-child mean in one pass
        hipEvent_t e0 = begin();
        return record(MG_K_RESTRICT, l,
                      launch_cell_res_restrict(g, lv[l + 1].g, lv[l].u[pr], lv[l].f[pr], faces(l, pr).k,
                                               lv[l + 1].f[pr], scale(l), stream),
                      e0, what);
    }
    if (!rec && grid.centering == MG_CELL && !faces(l, pr).k && g.n <= 64) {
        // small cell levels with stored faces (launch-bound): each coarse
        // cell forms the residuals of its children; on larger levels the
        // separate kernels measured as fast (256^3 FP32: 123 against
        // 105 + 17 us)
        hipEvent_t e0 = begin();
        return record(MG_K_RESTRICT, l,
                      launch_cell_res_restrict_pt(g, lv[l + 1].g, pr, lv[l].u[pr], lv[l].f[pr], faces(l, pr),
                                                  lv[l + 1].f[pr], scale(l), stream),
                      e0, what);
    }
    if (!rec && grid.centering == MG_NODE && !lv[l].gal && fused_point_transfers(g)) {
        // 2-D point levels: each coarse point forms its fine residuals
        hipEvent_t e0 = begin();
        return record(MG_K_RESTRICT, l,
                      launch_residual_restrict_pt(g, lv[l + 1].g, pr, lv[l].u[pr], lv[l].f[pr], lv[l + 1].f[pr],
                                                  scale(l), stream),
                      e0, what);
    }
    int rc = residual(l, pr, false, true);
    return rc ? rc : restrict_to(l, pr);
}

// The first half of a cycle on level l: pre-smoothing, then the residual
// restricted into level l + 1 (2-D node levels with damped Jacobi and
// nu1 >= 2: the last two sweeps, the residual and the restriction in one
// launch).
int Ctx::presmooth_restrict(int l, int pr, bool from_zero) {
    Level& P = lv[l];
    if (!rec && opts.smoother == MG_JACOBI && opts.nu1 >= 2 && grid.centering == MG_NODE && !P.gal && P.utmp[pr] &&
        fused_point_transfers(P.g)) {
        const int k = opts.nu1 - 2;
        int rc = smooth(l, pr, k, from_zero, 0);
        if (rc) return rc;
        hipEvent_t e0 = begin();
        rc = record(MG_K_SMOOTH, l,
                    launch_jacobi2(P.g, &lv[l + 1].g, pr, from_zero && k == 0, P.u[pr], nullptr, P.f[pr],
                                   P.utmp[pr], lv[l + 1].f[pr], scale(l), opts.omega, stream),
                    e0, "jacobi x2 + residual + restrict");
        if (!rc) std::swap(P.u[pr], P.utmp[pr]);
        return rc;
    }
    int rc = smooth(l, pr, opts.nu1, from_zero, 0);
    return rc ? rc : residual_restrict(l, pr);
}

// One cycle of the given type on level l (see mg_opts).
int Ctx::cycle(int l, int pr, bool from_zero, int kind) {
    if (l == L - 1) return coarse(pr);
    if (!rec && kind == MG_CYCLE_V && l == tail_l[pr]) return tail_cycle(l, pr, from_zero);
    int rc = presmooth_restrict(l, pr, from_zero);
    if (!rc && neu) rc = project(l + 1, lv[l + 1].f[pr]);
    if (!rc) rc = cycle(l + 1, pr, true, kind);
    if (!rc && l + 2 < L && kind != MG_CYCLE_V)
        rc = cycle(l + 1, pr, false, kind == MG_CYCLE_W ? MG_CYCLE_W : MG_CYCLE_V);
    if (rc) return rc;
    // With red-black smoothing that starts with colour c, the corrections of
    // colour c are overwritten before anything reads them: prolong onto the
    // other colour only.
    int mask = 3;
    if (opts.smoother == MG_RBGS && opts.nu2 > 0) mask = opts.post_order == 0 ? 2 : 1;
    Level& F = lv[l];
    if (!rec && opts.smoother == MG_JACOBI && opts.nu2 > 0 && grid.centering == MG_NODE && !F.gal && F.utmp[pr] &&
        fused_point_transfers(F.g)) {
        // 2-D point levels: the first post-smoothing sweep (or two) reads the
        // corrected iterate as the interpolation forms it
        const int k = opts.nu2 >= 2 ? 2 : 1;
        hipEvent_t e0 = begin();
        rc = record(MG_K_SMOOTH, l,
                    k == 2 ? launch_jacobi2(F.g, &lv[l + 1].g, pr, false, F.u[pr], lv[l + 1].u[pr], F.f[pr],
                                            F.utmp[pr], nullptr, scale(l), opts.omega, stream)
                           : launch_prolong_jacobi(F.g, lv[l + 1].g, pr, F.u[pr], lv[l + 1].u[pr], F.f[pr],
                                                   F.utmp[pr], scale(l), opts.omega, stream),
                    e0, "prolong+jacobi");
        if (rc) return rc;
        std::swap(F.u[pr], F.utmp[pr]);
        rc = smooth(l, pr, opts.nu2 - k, false, opts.post_order);
    } else {
        rc = prolong(l, pr, mask);
        if (!rc) rc = smooth(l, pr, opts.nu2, false, opts.post_order);
    }
    if (!rc && neu && l == 0) rc = project(0, lv[0].u[pr]);
    return rc;
}

// Zero-mean projection of a cell-grid FP64 field of level l (Neumann walls).
int Ctx::project(int l, void* a) {
    hipEvent_t e0 = begin();
    return record(MG_K_REDUCE, l,
                  launch_project(lv[l].g, static_cast<double*>(a), partials, reduce_scratch, red + 4, stream), e0,
                  "project");
}

// One FP64 refinement step around a single-precision V-cycle from zero,
// whose right-hand side residual_cast prepared: u64 += sigma fl64(c)
// (deferred: left to update_residual_cast).
int Ctx::refine_step(bool defer) {
    Level& L0 = lv[0];
    if (int rc = vcycle(0, 1, true)) return rc;
    if (defer) return MG_OK;
    if (rec) {
        BItem up = item(BOP_UPDATE, 0);
        up.n = field_quads(L0.g);
        up.tiles = (up.n + 255) / 256;
        up.a = L0.u[0];
        up.b = L0.u[1];
        return push(up);
    }
    hipEvent_t e0 = begin();
    return record(MG_K_UPDATE, 0,
                  launch_update(L0.g, static_cast<double*>(L0.u[0]), static_cast<const float*>(L0.u[1]), red + 2,
                                stream),
                  e0, "update");
}

int Ctx::read_red(double* sq, double* mx) {
    double h[2];
    int rc = dev(hipMemcpyAsync(h, red, 16, hipMemcpyDeviceToHost, stream), "read norm");
    if (!rc) rc = dev(hipStreamSynchronize(stream), "sync");
    if (rc) return rc;
    *sq = h[0];
    *mx = h[1];
    return MG_OK;
}

int Ctx::norm(double* out) {
    int rc = residual(0, 0, true, false);
    double sq, mx;
    if (!rc) rc = read_red(&sq, &mx);
    if (rc) return rc;
    *out = std::sqrt(sq);
    return MG_OK;
}

int Ctx::step(int k) {
    for (int i = 0; i < k; ++i)
        if (int rc = step_once()) return rc;
    return MG_OK;
}

std::vector<void*> Ctx::buffers() const {
    std::vector<void*> b;
    for (const Level& v : lv)
        for (int pr = 0; pr < 2; ++pr) {
            b.push_back(v.u[pr]);
            b.push_back(v.utmp[pr]);
        }
    return b;
}

void Ctx::set_buffers(const std::vector<void*>& b) {
    size_t i = 0;
    for (Level& v : lv)
        for (int pr = 0; pr < 2; ++pr) {
            v.u[pr] = b[i++];
            v.utmp[pr] = b[i++];
        }
}

const Ctx::Graph* Ctx::capture(int kind) {
    if (graphs.size() >= 8) return nullptr;
    if (!cap_stream) {
        if (hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking) != hipSuccess) {
            cap_stream = nullptr;
            return nullptr;
        }
        if (hipHostMalloc(reinterpret_cast<void**>(&h_red), 16, hipHostMallocDefault) != hipSuccess) {
            h_red = nullptr;
            return nullptr;
        }
    }
    const bool mixed = opts.precision == MG_MIXED;
    const std::vector<void*> pre = buffers();
    if (hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    hipStream_t user = stream;
    stream = cap_stream;
    int rc;
    // (mixed: the scale basis of the previous residual is known here)
    if (kind == 0 && fused_update()) {
        rc = refine_step(true);
        if (!rc) rc = update_residual_cast();
        if (!rc) rc = dev(hipMemcpyAsync(h_red, red, 16, hipMemcpyDeviceToHost, stream), "norm copy");
    } else if (kind == 0) {
        rc = mixed ? refine_step() : vcycle(0, 0, false);
        if (!rc) rc = mixed ? residual_cast(false) : residual(0, 0, true, false);
        if (!rc) rc = dev(hipMemcpyAsync(h_red, red, 16, hipMemcpyDeviceToHost, stream), "norm copy");
    } else {
        rc = mixed ? residual_cast(false) : MG_OK;
        if (!rc) rc = mixed ? refine_step() : vcycle(0, 0, false);
    }
    stream = user;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cap_stream, &g);
    Graph gr;
    gr.kind = kind;
    gr.pre = pre;
    gr.post = buffers();
    // nothing ran yet: the host-side buffer assignment goes back to `pre`
    set_buffers(pre);
    bool ok = rc == MG_OK && ec == hipSuccess && g != nullptr &&
              hipGraphInstantiate(&gr.exec, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!ok) {
        if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
        err.clear();
        return nullptr;
    }
    graphs.push_back(std::move(gr));
    return &graphs.back();
}

void Ctx::add_times(const std::vector<Rec>& rs) {
    for (const Rec& r : rs) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.e0, r.e1) != hipSuccess) continue;
        const int lvl = r.level < 0 ? kMaxLevels - 1 : r.level;
        agg_ms[r.kclass][lvl] += t;
        agg_n[r.kclass][lvl] += 1;
    }
}

// the graph of `kind` for the current buffer assignment (captured on first
// use), or null when launches are to be issued one by one
const Ctx::Graph* Ctx::replayable(int kind) {
    if (prof || graphs_off) return nullptr;
    const std::vector<void*> cur = buffers();
    for (const Graph& x : graphs)
        if (x.kind == kind && x.pre == cur) return &x;
    const Graph* gr = capture(kind);
    if (!gr) graphs_off = true;   // capture unavailable: issue launches from now on
    return gr;
}

int Ctx::step_once() {
    if (opts.precision == MG_MIXED && !scale_known) {
        // a new right-hand side or iterate: the first step scales by its own residual
        if (int rc = residual(0, 0, true, false)) return rc;
    }
    if (const Graph* gr = replayable(1)) {
        int rc = dev(hipGraphLaunch(gr->exec, stream), "graph launch");
        if (rc) return rc;
        ++graph_launches;
        set_buffers(gr->post);
        return MG_OK;
    }
    if (opts.precision == MG_MIXED) {
        int rc = residual_cast(false);
        return rc ? rc : refine_step();
    }
    return vcycle(0, 0, false);
}

int Ctx::iterate(double* nr) {
    {
        const Graph* gr = replayable(0);
        if (gr) {
            int rc = dev(hipGraphLaunch(gr->exec, stream), "graph launch");
            if (!rc) rc = dev(hipStreamSynchronize(stream), "sync");
            if (rc) return rc;
            ++graph_launches;
            set_buffers(gr->post);
            *nr = std::sqrt(h_red[0]);
            return MG_OK;
        }
    }
    if (opts.precision == MG_MIXED) {
        const bool fu = fused_update();
        int rc = refine_step(fu);
        if (!rc) rc = fu ? update_residual_cast() : residual_cast(false);
        double sq, mx;
        if (!rc) rc = read_red(&sq, &mx);
        if (!rc) *nr = std::sqrt(sq);
        return rc;
    }
    int rc = vcycle(0, 0, false);
    if (!rc) rc = norm(nr);
    return rc;
}

Ctx::~Ctx() {
    for (Graph& g : graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (h_red) (void)hipHostFree(h_red);
}

// Preconditioned conjugate gradients; r lives in the finest f (so the
// preconditioner is a cycle from zero on that level, z in the finest u).
int Ctx::pcg(double tol, int max_it, int* its_out, double* relres_out) {
    Level& L0 = lv[0];
    const size_t fb = L0.field_bytes[0];
    double* x = static_cast<double*>(pcg_v[0]);
    double* p = static_cast<double*>(pcg_v[1]);
    double* q = static_cast<double*>(pcg_v[2]);
    double* fs = static_cast<double*>(pcg_v[3]);
    const double* zero = static_cast<const double*>(pcg_v[4]);
    const long long nd = dot_blocks(fb);
    auto dotp = [&](const void* a, const void* b, double* out) -> int {
        hipEvent_t e0 = begin();
        int rc = record(MG_K_REDUCE, 0, launch_dot(static_cast<const double*>(a), static_cast<const double*>(b), fb,
                                                   pcg_part, stream), e0, "dot");
        return rc ? rc : dev(launch_reduce(pcg_part, nd, pcg_scratch, out, stream), "dot reduce");
    };
    auto residual_into = [&](const void* u, const void* f, void* r) -> int {
        long long nb = 0;
        hipEvent_t e0 = begin();
        return record(MG_K_RESIDUAL, 0,
                      launch_residual(L0.g, 0, u, f, r, faces(0, 0), scale(0), false, true, partials, &nb, stream),
                      e0, "residual");
    };
    auto host = [&](const double* d, double* h) -> int {
        int rc = dev(hipMemcpyAsync(h, d, 8, hipMemcpyDeviceToHost, stream), "read scalar");
        return rc ? rc : dev(hipStreamSynchronize(stream), "sync");
    };
    hist.clear();
    int rc = dev(launch_copy(fs, L0.f[0], fb, stream), "save f");
    if (!rc) rc = dev(launch_copy(x, L0.u[0], fb, stream), "iterate");
    if (!rc) rc = residual_into(x, fs, L0.f[0]);                  // r = f - A x
    double rr0 = 0.0;
    if (!rc) rc = dotp(L0.f[0], L0.f[0], pcg_s + 6);
    if (!rc) rc = host(pcg_s + 6, &rr0);
    if (rc) return rc;
    const double r0 = std::sqrt(rr0);
    if (!std::isfinite(r0)) return fail(MG_ENONFINITE, "initial residual is not finite");
    hist.push_back(1.0);
    int its = 0, status = MG_OK;
    double rel = 1.0;
    if (r0 > 0.0 && rel > tol) {
        rc = vcycle(0, 0, true);                                    // z = M r
        if (!rc) rc = dev(launch_copy(p, L0.u[0], fb, stream), "p = z");
        if (!rc) rc = dotp(L0.f[0], L0.u[0], pcg_s + 0);            // rho = r . z
        while (!rc) {
            if (its == max_it) {
                status = MG_ENOTCONV;
                err = "max_it reached";
                break;
            }
            rc = residual_into(p, zero, q);                          // q = -A p
            if (!rc) rc = dotp(p, q, pcg_s + 2);
            if (!rc) rc = dev(launch_pcg_step(x, p, static_cast<double*>(L0.f[0]), q, pcg_s, fb, stream), "x, r");
            double rr = 0.0;
            if (!rc) rc = dotp(L0.f[0], L0.f[0], pcg_s + 6);
            if (!rc) rc = host(pcg_s + 6, &rr);
            if (rc) break;
            ++its;
            rel = std::sqrt(rr) / r0;
            hist.push_back(rel);
            if (!std::isfinite(rel)) {
                status = fail(MG_ENONFINITE, "residual norm is not finite");
                break;
            }
            if (rel <= tol) break;
            rc = vcycle(0, 0, true);                                 // z = M r
            if (!rc) rc = dotp(L0.f[0], L0.u[0], pcg_s + 4);         // rho_new = r . z
            if (!rc) rc = dev(launch_pcg_dir(p, static_cast<const double*>(L0.u[0]), pcg_s, fb, stream), "p");
            if (!rc) rc = dev(launch_scalar_copy(pcg_s + 0, pcg_s + 4, stream), "rho");
        }
    }
    // the solution becomes the iterate, f is restored
    if (!rc) rc = dev(launch_copy(L0.u[0], x, fb, stream), "solution");
    if (!rc) rc = dev(launch_copy(L0.f[0], fs, fb, stream), "restore f");
    if (!rc) rc = dev(hipStreamSynchronize(stream), "sync");
    if (rc) return rc;
    if (its_out) *its_out = its;
    if (relres_out) *relres_out = r0 == 0.0 ? 0.0 : rel;
    return status;
}

int Ctx::solve(double tol, int* cycles_out, double* relres_out) {
    hist.clear();
    double r0;
    int rc = norm(&r0);   // in mixed mode this also leaves max|r| as the first step's scale basis
    // mixed: the first step's single-precision right-hand side
    if (!rc && opts.precision == MG_MIXED && r0 > 0.0 && std::isfinite(r0)) rc = residual_cast(false);
    if (rc) return rc;
    if (!std::isfinite(r0)) return fail(MG_ENONFINITE, "initial residual is not finite");
    hist.push_back(1.0);
    int cycles = 0, grow = 0;
    double rel = 1.0;
    int status = MG_OK;
    while (r0 > 0.0 && rel > tol) {
        if (cycles == opts.max_cycles) {
            status = MG_ENOTCONV;
            err = "max_cycles reached";
            break;
        }
        double nr;
        rc = iterate(&nr);
        if (rc) return rc;
        ++cycles;
        const double prev = rel;
        rel = nr / r0;
        hist.push_back(rel);
        if (!std::isfinite(rel)) {
            status = fail(MG_ENONFINITE, "residual norm is not finite");
            break;
        }
        grow = rel > prev ? grow + 1 : 0;
        if (grow >= 3 && rel > 1.0) {
            status = fail(MG_EDIVERGED, "residual grew in 3 consecutive cycles");
            break;
        }
    }
    if (r0 == 0.0) rel = 0.0;
    if (cycles_out) *cycles_out = cycles;
    if (relres_out) *relres_out = rel;
    return status;
}

}  // namespace mg

namespace mg {

int setup_ctx(const mg_grid* g, const mg_stencil* st, const mg_opts* o, void* d_workspace, size_t bytes,
              hipStream_t stream, bool staging, Ctx** out, std::string* errmsg, int bc_kind) {
    *out = nullptr;
    std::string why;
    int rc = validate(g, st, o, &why);
    if (rc) {
        *errmsg = why;
        return rc;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        *errmsg = "no HIP device";
        return MG_EDEVICE;
    }
    Plan plan;
    const size_t need = plan_workspace(g, st, o, &plan, staging);
    if (!d_workspace || bytes < need) {
        *errmsg = "workspace too small: need " + std::to_string(need) + " bytes";
        return MG_ENOMEM;
    }
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256) {
        *errmsg = "workspace must be 256-byte aligned";
        return MG_EINVAL;
    }
    Ctx* c = new (std::nothrow) Ctx();
    if (!c) return MG_ENOMEM;
    c->grid = *g;
    c->opts = *o;
    c->kind = st ? st->kind : MG_LAPLACE;
    c->neu = bc_kind == MG_NEUMANN0;
    c->base = d_workspace;
    c->bytes = bytes;
    c->stream = stream;
    c->L = plan.L;
    c->m = plan.m;
    c->partial_pairs = plan.partial_pairs;
    c->partials = static_cast<double*>(c->at(plan.partials));
    c->reduce_scratch = static_cast<double*>(c->at(plan.reduce_scratch));
    c->red = static_cast<double*>(c->at(plan.red));
    c->chol = static_cast<double*>(c->at(plan.chol));
    if (plan.pcg != SIZE_MAX) {
        const size_t fb = align_up((size_t)(2 * plan.lv[0].g.cs) * 8);
        char* b = static_cast<char*>(c->at(plan.pcg));
        for (int i = 0; i < 5; ++i) c->pcg_v[i] = b + i * fb;
        c->pcg_part = reinterpret_cast<double*>(b + 5 * fb);
        c->pcg_scratch = c->pcg_part + 2 * dot_blocks((size_t)(2 * plan.lv[0].g.cs) * 8);
        c->pcg_s = c->pcg_scratch + 2 * reduce_scratch_pairs(dot_blocks((size_t)(2 * plan.lv[0].g.cs) * 8));
    }
    c->staging = static_cast<double*>(c->at(plan.staging));
    for (int l = 0; l < plan.L; ++l) {
        const LevelPlan& lp = plan.lv[l];
        Level lvv;
        lvv.g = lp.g;
        lvv.g.neu = bc_kind == MG_NEUMANN0 ? 1 : 0;
        for (int pr = 0; pr < 2; ++pr) {
            lvv.has[pr] = lp.has[pr];
            lvv.u[pr] = c->at(lp.u[pr]);
            lvv.f[pr] = c->at(lp.f[pr]);
            lvv.r[pr] = c->at(lp.r[pr]);
            lvv.utmp[pr] = c->at(lp.utmp[pr]);
            lvv.field_bytes[pr] = (size_t)(2 * lp.g.cs) * (pr == 0 ? 8 : 4);
            for (int a = 0; a < 3; ++a) lvv.beta[pr][a] = c->at(lp.beta[pr][a]);
        }
        lvv.k = c->at(lp.k);
        c->lv.push_back(lvv);
    }
    // zero every field (boundary nodes and padding stay zero for good)
    rc = c->dev(launch_zero(d_workspace, plan.total, c->stream), "zero workspace");
    // face coefficients
    if (!rc && g->centering == MG_CELL) {
        const Geom& g0 = c->lv[0].g;
        const long long ncell = (long long)g0.n * g0.n * (g0.dim == 3 ? g0.n : 1);
        std::vector<double> k((size_t)ncell, 1.0);
        if (c->kind == MG_VARCOEF) {
            if (st->k_on_device)
                rc = c->dev(hipMemcpy(k.data(), st->k, (size_t)ncell * 8, hipMemcpyDeviceToHost), "read k");
            else
                std::memcpy(k.data(), st->k, (size_t)ncell * 8);
            for (long long i = 0; !rc && i < ncell; ++i)
                if (!(k[(size_t)i] > 0.0) || !std::isfinite(k[(size_t)i])) {
                    rc = c->fail(MG_EINVAL, "k must be positive and finite");
                }
        }
        std::vector<double> bf[3], bc2[3];
        if (!rc) harmonic_faces(g0, k.data(), bf);
        if (!rc && c->lv[0].k) {
            // k in colour-split layout for the column-marching finest-level kernels
            std::vector<double> ks((size_t)(2 * g0.cs), 0.0);
            const int N = g0.n;
            for (int z = 0; z < N; ++z)
                for (int y = 0; y < N; ++y)
                    for (int x = 0; x < N; ++x)
                        ks[(size_t)(((x + y + z) & 1) * g0.cs + (long long)z * g0.plane + (long long)y * g0.pitch +
                                    (x >> 1))] = k[((size_t)z * N + y) * N + x];
            rc = c->dev(hipMemcpyAsync(c->lv[0].k, ks.data(), ks.size() * 8, hipMemcpyHostToDevice, c->stream),
                        "upload k");
            if (!rc) rc = c->dev(hipStreamSynchronize(c->stream), "sync");
        }
        std::vector<float> tmp32;
        for (int l = 0; !rc && l < c->L; ++l) {
            const Geom& gl = c->lv[l].g;
            if (l > 0) {
                coarsen_faces(c->lv[l - 1].g, bf, gl, bc2);
                for (int a = 0; a < 3; ++a) bf[a].swap(bc2[a]);
            }
            for (int a = 0; !rc && a < gl.dim; ++a) {
                if (c->lv[l].has[0])
                    rc = c->dev(hipMemcpyAsync(c->lv[l].beta[0][a], bf[a].data(), (size_t)gl.fsize * 8,
                                               hipMemcpyHostToDevice, c->stream),
                                "upload faces");
                if (!rc && c->lv[l].has[1]) {
                    tmp32.assign(bf[a].begin(), bf[a].end());
                    rc = c->dev(hipMemcpyAsync(c->lv[l].beta[1][a], tmp32.data(), (size_t)gl.fsize * 4,
                                               hipMemcpyHostToDevice, c->stream),
                                "upload faces");
                    if (!rc) rc = c->dev(hipStreamSynchronize(c->stream), "sync");
                }
            }
            if (!rc) rc = c->dev(hipStreamSynchronize(c->stream), "sync");
        }
        if (!rc) c->coarse_beta_host.assign(bf, bf + 3);
    }
    // Galerkin stencils of the coarser levels
    if (!rc && o->coarse_op == MG_COARSE_GALERKIN) {
        Stencil27 W = laplacian27(c->lv[0].g);
        for (int l = 1; l < c->L; ++l) {
            W = galerkin_coarse(W, c->lv[l].g.dim);
            c->lv[l].gal = true;
            c->lv[l].W = W;
        }
    }
    // coarsest matrix, Cholesky factor
    if (!rc) {
        std::vector<double> A = coarse_matrix(c->lv.back().g,
                                              c->coarse_beta_host.empty() ? nullptr : c->coarse_beta_host.data(),
                                              c->lv.back().gal ? &c->lv.back().W : nullptr);
        if (!cholesky(A, c->m)) rc = c->fail(MG_EINVAL, "coarsest matrix is not SPD");
        if (!rc)
            rc = c->dev(hipMemcpyAsync(c->chol, A.data(), A.size() * 8, hipMemcpyHostToDevice, c->stream),
                        "upload factor");
        if (!rc) rc = c->dev(hipStreamSynchronize(c->stream), "sync");
    }
    c->coarse_beta_host.clear();
    if (!rc) c->plan_tail();
    if (rc) {
        *errmsg = c->err;
        delete c;
        return rc;
    }
    *out = c;
    return MG_OK;
}

}  // namespace mg

// =================================================================== C ABI
using mg::Ctx;

extern "C" {

const char* mg_version(void) { return "mg 0.1.0 (gfx950, colour-split storage)"; }

void mg_default_opts(mg_opts* o) {
    if (!o) return;
    o->smoother = MG_RBGS;
    o->omega = 0.8;
    o->nu1 = 2;
    o->nu2 = 2;
    o->precision = MG_FP64;
    o->max_cycles = 100;
    o->post_order = 0;
    o->cycle = MG_CYCLE_V;
    o->krylov = 0;
    o->coarse_op = MG_COARSE_REDISCRETISE;
}

int mg_workspace_bytes(const mg_grid* g, const mg_stencil* st, const mg_opts* o, size_t* bytes) {
    if (!bytes) return MG_EINVAL;
    int rc = validate(g, st, o, nullptr);
    if (rc) return rc;
    *bytes = mg::plan_workspace(g, st, o, nullptr, true);
    return MG_OK;
}

static thread_local std::string g_setup_error;

int mg_setup(const mg_grid* g, const mg_stencil* st, const mg_bc* bc, const mg_opts* o, void* d_workspace,
             size_t bytes, void* hip_stream, mg_ctx** out) {
    if (!out) return MG_EINVAL;
    *out = nullptr;
    const int kind = bc ? bc->kind : MG_DIRICHLET0;
    if (kind != MG_DIRICHLET0 && kind != MG_NEUMANN0) {
        g_setup_error = "unknown boundary kind";
        return MG_EINVAL;
    }
    if (kind == MG_NEUMANN0 && g && o &&
        (g->centering != MG_CELL || o->precision != MG_FP64 || o->krylov != 0)) {
        g_setup_error = "Neumann walls need a cell grid, FP64 precision and no Krylov vectors";
        return MG_EINVAL;
    }
    Ctx* c = nullptr;
    const int rc = mg::setup_ctx(g, st, o, d_workspace, bytes, static_cast<hipStream_t>(hip_stream), true, &c,
                                 &g_setup_error, kind);
    if (rc) return rc;
    *out = reinterpret_cast<mg_ctx*>(c);
    return MG_OK;
}

void mg_destroy(mg_ctx* h) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return;
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

static int copy_in(Ctx* c, const mg::Geom& g, int pr, void* field, const double* a, int on_device) {
    const long long tot = (long long)g.n * g.n * (g.dim == 3 ? g.n : 1);
    const double* src = a;
    if (!on_device && !c->staging) return c->fail(MG_EINVAL, "this context takes device arrays only");
    if (!on_device) {
        int rc = c->dev(hipMemcpyAsync(c->staging, a, (size_t)tot * 8, hipMemcpyHostToDevice, c->stream), "upload");
        if (rc) return rc;
        src = c->staging;
    }
    hipEvent_t e0 = c->begin();
    int rc = c->record(MG_K_COPY, -1, mg::launch_pack(g, pr, src, field, c->stream), e0, "pack");
    if (!rc && !on_device) rc = c->dev(hipStreamSynchronize(c->stream), "sync");
    return rc;
}

static int copy_out(Ctx* c, const mg::Geom& g, int pr, const void* field, double* a, int on_device) {
    const long long tot = (long long)g.n * g.n * (g.dim == 3 ? g.n : 1);
    if (!on_device && !c->staging) return c->fail(MG_EINVAL, "this context takes device arrays only");
    double* dst = on_device ? a : c->staging;
    hipEvent_t e0 = c->begin();
    int rc = c->record(MG_K_COPY, -1, mg::launch_unpack(g, pr, field, dst, c->stream), e0, "unpack");
    if (!rc && !on_device)
        rc = c->dev(hipMemcpyAsync(a, c->staging, (size_t)tot * 8, hipMemcpyDeviceToHost, c->stream), "download");
    if (!rc && !on_device) rc = c->dev(hipStreamSynchronize(c->stream), "sync");
    return rc;
}

int mg_set_rhs(mg_ctx* h, const double* f, int on_device) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !f) return MG_EINVAL;
    c->scale_known = false;   // the next refinement step scales by its own residual
    int rc = copy_in(c, c->lv[0].g, 0, c->lv[0].f[0], f, on_device);
    if (!rc && c->neu) rc = c->project(0, c->lv[0].f[0]);
    return rc;
}

int mg_set_initial(mg_ctx* h, const double* u0, int on_device) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return MG_EINVAL;
    c->scale_known = false;   // the next refinement step scales by its own residual
    if (!u0) {
        hipEvent_t e0 = c->begin();
        return c->record(MG_K_COPY, 0, mg::launch_zero(c->lv[0].u[0], c->lv[0].field_bytes[0], c->stream), e0,
                         "zero");
    }
    return copy_in(c, c->lv[0].g, 0, c->lv[0].u[0], u0, on_device);
}

int mg_get_solution(mg_ctx* h, double* u, int on_device) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !u) return MG_EINVAL;
    return copy_out(c, c->lv[0].g, 0, c->lv[0].u[0], u, on_device);
}

int mg_vcycle(mg_ctx* h, int ncycles) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || ncycles < 0) return MG_EINVAL;
    return c->step(ncycles);
}

int mg_fmg(mg_ctx* h, int cycles_per_level) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || cycles_per_level < 1) return MG_EINVAL;
    if (c->opts.precision != MG_FP64) return c->fail(MG_EINVAL, "full multigrid runs in FP64 contexts");
    return c->fmg(cycles_per_level);
}

int mg_pcg(mg_ctx* h, double tol, int max_it, int* its_out, double* relres_out) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !(tol >= 0.0) || max_it < 1) return MG_EINVAL;
    if (!c->pcg_s) return c->fail(MG_EINVAL, "mg_pcg needs a context set up with krylov = 1");
    const mg_opts& o = c->opts;
    if (o.nu1 != o.nu2 || (o.smoother == MG_RBGS && o.post_order != 1))
        return c->fail(MG_EINVAL, "the preconditioner must be symmetric: nu1 = nu2, and post_order = 1 with RB-GS");
    return c->pcg(tol, max_it, its_out, relres_out);
}

int mg_solve(mg_ctx* h, double tol, int* cycles_out, double* relres_out) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !(tol >= 0.0)) return MG_EINVAL;
    return c->solve(tol, cycles_out, relres_out);
}

int mg_residual_norm(mg_ctx* h, double* out) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !out) return MG_EINVAL;
    return c->norm(out);
}

int mg_history(const mg_ctx* h, double* buf, int cap, int* n) {
    const Ctx* c = reinterpret_cast<const Ctx*>(h);
    if (!c || !n || (cap > 0 && !buf)) return MG_EINVAL;
    *n = (int)c->hist.size();
    for (int i = 0; i < cap && i < *n; ++i) buf[i] = c->hist[(size_t)i];
    return MG_OK;
}

int mg_levels(const mg_ctx* h, int* nlevels) {
    const Ctx* c = reinterpret_cast<const Ctx*>(h);
    if (!c || !nlevels) return MG_EINVAL;
    *nlevels = c->L;
    return MG_OK;
}

int mg_level_size(const mg_ctx* h, int level, int* n) {
    const Ctx* c = reinterpret_cast<const Ctx*>(h);
    if (!c || !n || level < 0 || level >= c->L) return MG_EINVAL;
    *n = c->lv[level].g.n;
    return MG_OK;
}

static void* field_ptr(Ctx* c, int level, int field, int pr) {
    if (level < 0 || level >= c->L || pr < 0 || pr > 1 || !c->lv[level].has[pr]) return nullptr;
    mg::Level& L = c->lv[level];
    switch (field) {
        case MG_FIELD_U: return L.u[pr];
        case MG_FIELD_F: return L.f[pr];
        case MG_FIELD_R: return L.r[pr];
        default: return nullptr;
    }
}

int mg_level_set(mg_ctx* h, int level, int field, int prec, const double* a, int on_device) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !a) return MG_EINVAL;
    c->scale_known = false;   // the next refinement step scales by its own residual
    void* p = field_ptr(c, level, field, prec);
    if (!p) return c->fail(MG_EINVAL, "no such level field");
    return copy_in(c, c->lv[level].g, prec, p, a, on_device);
}

int mg_level_get(mg_ctx* h, int level, int field, int prec, double* a, int on_device) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || !a) return MG_EINVAL;
    void* p = field_ptr(c, level, field, prec);
    if (!p) return c->fail(MG_EINVAL, "no such level field");
    return copy_out(c, c->lv[level].g, prec, p, a, on_device);
}

int mg_apply(mg_ctx* h, int op, int level, int prec) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return MG_EINVAL;
    c->scale_known = false;   // the next refinement step scales by its own residual
    if (level < 0 || level >= c->L || prec < 0 || prec > 1 || !c->lv[level].has[prec])
        return c->fail(MG_EINVAL, "no such level in this precision");
    const bool has_next = level + 1 < c->L && c->lv[level + 1].has[prec];
    switch (op) {
        case MG_OP_GS_RED:
        case MG_OP_GS_BLACK:
            if (c->lv[level].gal) return c->fail(MG_EINVAL, "Galerkin levels have no red-black sweep");
            return c->gs(level, prec, op == MG_OP_GS_RED ? 0 : 1, false);
        case MG_OP_JACOBI:
            if (!c->lv[level].utmp[prec]) return c->fail(MG_EINVAL, "Jacobi needs a Jacobi context");
            return c->jacobi(level, prec, false);
        case MG_OP_RESIDUAL: return c->residual(level, prec, false, true);
        case MG_OP_RESTRICT:
            if (!has_next) return c->fail(MG_EINVAL, "no coarser level");
            return c->restrict_to(level, prec);
        case MG_OP_PROLONG:
            if (!has_next) return c->fail(MG_EINVAL, "no coarser level");
            return c->prolong(level, prec, 3);
        case MG_OP_COARSE:
            if (level != c->L - 1) return c->fail(MG_EINVAL, "not the coarsest level");
            return c->coarse(prec);
        case MG_OP_RESIDUAL_RESTRICT:
            if (!has_next) return c->fail(MG_EINVAL, "no coarser level");
            return c->residual_restrict(level, prec);
        case MG_OP_VCYCLE:
            if (level < c->L - 1 && !has_next) return c->fail(MG_EINVAL, "no coarser level");
            return c->vcycle(level, prec, false);
        case MG_OP_PRESMOOTH: return c->smooth(level, prec, c->opts.nu1, false, 0);
        case MG_OP_POSTSMOOTH: return c->smooth(level, prec, c->opts.nu2, false, c->opts.post_order);
        case MG_OP_PRESMOOTH_RESTRICT:
            if (!has_next) return c->fail(MG_EINVAL, "no coarser level");
            return c->presmooth_restrict(level, prec, false);
        default: return c->fail(MG_EINVAL, "unknown op");
    }
}

int mg_profile(mg_ctx* h, int enable) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return MG_EINVAL;
    int rc = c->dev(hipStreamSynchronize(c->stream), "sync");
    c->prof = enable != 0;
    c->recs.clear();
    c->ev_used = 0;
    std::memset(c->agg_ms, 0, sizeof(c->agg_ms));
    std::memset(c->agg_n, 0, sizeof(c->agg_n));
    return rc;
}

int mg_profile_read(mg_ctx* h, int kclass, int level, int* count, double* ms) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c || kclass < 0 || kclass >= MG_K_COUNT || level < -1 || level >= mg::kMaxLevels) return MG_EINVAL;
    int rc = c->dev(hipStreamSynchronize(c->stream), "sync");
    if (rc) return rc;
    c->add_times(c->recs);
    c->recs.clear();
    c->ev_used = 0;
    double s = 0.0;
    int n = 0;
    for (int l = 0; l < mg::kMaxLevels; ++l)
        if (level < 0 || l == level) {
            s += c->agg_ms[kclass][l];
            n += c->agg_n[kclass][l];
        }
    if (count) *count = n;
    if (ms) *ms = s;
    return MG_OK;
}

int mg_graph_launches(const mg_ctx* h, long long* n) {
    const Ctx* c = reinterpret_cast<const Ctx*>(h);
    if (!c || !n) return MG_EINVAL;
    *n = c->graph_launches;
    return MG_OK;
}

const char* mg_strerror(int code) {
    switch (code) {
        case MG_OK: return "ok";
        case MG_EINVAL: return "invalid argument";
        case MG_ENOMEM: return "out of memory (workspace or budget)";
        case MG_EDEVICE: return "HIP device error";
        case MG_ENOTCONV: return "not converged within max_cycles";
        case MG_ENONFINITE: return "non-finite residual";
        case MG_EDIVERGED: return "diverged";
        case MG_EBUSY: return "busy";
        case MG_ECANCELED: return "cancelled";
        case MG_ETIMEDOUT: return "deadline passed";
        default: return "unknown error";
    }
}

const char* mg_last_error(const mg_ctx* h) {
    const Ctx* c = reinterpret_cast<const Ctx*>(h);
    if (!c) return g_setup_error.c_str();
    return c->err.c_str();
}

}  // extern "C"
