// Volume terms of the quadrature-free DG shallow-water scheme (see dg.h):
// exact reference integrals on the host, one GPU thread per element.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "dg.h"
#include "mg.h"


// The allocation-free RK step (dg_ssp_rk3_step_noalloc) keeps the saved
// state and the right-hand side (6 K ne doubles) in this fixed device array
// instead of caller scratch: 64 MiB, held on every device the library runs
// on until the process ends.  In host code the name stands for a host-side
// shadow: only the address from hipGetSymbolAddress (one per device) may be
// passed to kernels or copies.
constexpr long long kDgScratchDoubles = 1LL << 23;
static __device__ __align__(256) double scratch[kDgScratchDoubles];

namespace {

constexpr int kMaxK = 10;
constexpr int kDeg = 10;   // monomial degrees kept per variable (products stay below 9)

// The paper's ten orthonormal polynomials on the reference triangle:
// sqrt(scale) * sum of coef * x^a y^b over the monomials 1, x, y, x^2, xy,
// y^2, x^3, x^2 y, x y^2, y^3.
const int kMono[10][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {1, 1}, {0, 2}, {3, 0}, {2, 1}, {1, 2}, {0, 3}};
const long long kScale[10] = {2, 1, 12, 6, 3, 45, 8, 24, 40, 56};
const double kCoef[10][10] = {
    {1, 0, 0, 0, 0, 0, 0, 0, 0, 0},
    {2, -6, 0, 0, 0, 0, 0, 0, 0, 0},
    {1, -1, -2, 0, 0, 0, 0, 0, 0, 0},
    {1, -8, 0, 10, 0, 0, 0, 0, 0, 0},
    {-1, -4, 12, 5, 0, -15, 0, 0, 0, 0},
    {1, -4, -4, 3, 8, 3, 0, 0, 0, 0},
    {-1, 15, 0, -45, 0, 0, 35, 0, 0, 0},
    {-1, 13, 2, -33, -24, 0, 21, 42, 0, 0},
    {-1, 9, 6, -15, -48, -6, 7, 42, 42, 0},
    {-1, 3, 12, -3, -24, -30, 1, 12, 30, 20},
};

// Polynomials with integer coefficients (the basis without its square-root
// factor), so that products and integrals are exact.
struct Poly {
    long long c[kDeg][kDeg];   // c[a][b] multiplies x^a y^b
};

Poly basis_poly(int p) {
    Poly q;
    std::memset(&q, 0, sizeof(q));
    for (int t = 0; t < 10; ++t) q.c[kMono[t][0]][kMono[t][1]] = (long long)kCoef[p][t];
    return q;
}

Poly deriv(const Poly& a, int axis) {
    Poly q;
    std::memset(&q, 0, sizeof(q));
    for (int i = 0; i < kDeg; ++i)
        for (int j = 0; j < kDeg; ++j) {
            if (axis == 0 && i > 0) q.c[i - 1][j] = i * a.c[i][j];
            if (axis == 1 && j > 0) q.c[i][j - 1] = j * a.c[i][j];
        }
    return q;
}

Poly mul(const Poly& a, const Poly& b) {
    Poly q;
    std::memset(&q, 0, sizeof(q));
    for (int i = 0; i < kDeg; ++i)
        for (int j = 0; j < kDeg; ++j) {
            if (a.c[i][j] == 0) continue;
            for (int k = 0; i + k < kDeg; ++k)
                for (int l = 0; j + l < kDeg; ++l) q.c[i + k][j + l] += a.c[i][j] * b.c[k][l];
        }
    return q;
}

// int over the reference triangle of x^a y^b = a! b! / (a + b + 2)!, summed
// exactly over a common denominator D! and rounded once; then times the
// square root of the product of the basis scale factors (an integer).
double integrate(const Poly& a, long long scale) {
    constexpr int D = kDeg + 2;
    __int128 fact[D + 1];
    fact[0] = 1;
    for (int i = 1; i <= D; ++i) fact[i] = fact[i - 1] * i;
    __int128 num = 0;
    for (int i = 0; i < kDeg; ++i)
        for (int j = 0; j < kDeg && i + j + 2 <= D; ++j)
            if (a.c[i][j] != 0) num += (__int128)a.c[i][j] * fact[i] * fact[j] * (fact[D] / fact[i + j + 2]);
    return (double)num / (double)fact[D] * std::sqrt((double)scale);
}

int k_of(int k) { return k == 0 ? 1 : k == 1 ? 3 : k == 2 ? 6 : k == 3 ? 10 : 0; }

// Coefficients of the bathymetry, and the order of the reference and edge
// tables: max(k, 1), so that a linear h_b is exact at every order.
int kb_of(int k) { return k == 0 ? 3 : k_of(k); }

// Coefficients of a trace on an edge (degree max(k, 1) in the edge
// parameter): the length of the edge table's Legendre expansions.
int nb_of(int k) { return k == 0 ? 2 : k + 1; }

template <int K>
constexpr int kb_const() { return K == 1 ? 3 : K; }

template <int K>
constexpr int nt_const() { return K == 1 ? 1 : K == 3 ? 2 : K == 6 ? 3 : 4; }   // k + 1

template <int K>
constexpr int nb_const() { return K == 1 ? 2 : nt_const<K>(); }                // max(k, 1) + 1

// int_0^1 P_a P_b P_c ds for the shifted Legendre polynomials, a, b, c <= 3:
// the square of the Wigner 3j symbol (a b c; 0 0 0), zero unless a + b + c
// is even and a, b, c satisfy the triangle inequality, else
// [(2s-2a)! (2s-2b)! (2s-2c)! / (2s+1)!] [s! / ((s-a)! (s-b)! (s-c)!)]^2
// with 2s = a + b + c.  Exact in double (factorials up to 13!).
struct Legendre3 {
    double v[4][4][4];
};

constexpr double factorial(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

constexpr Legendre3 legendre3() {
    Legendre3 t{};
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                const int S = a + b + c;
                if (S % 2 || a > b + c || b > a + c || c > a + b) {
                    t.v[a][b][c] = 0.0;
                    continue;
                }
                const int s = S / 2;
                const double r = factorial(s) / (factorial(s - a) * factorial(s - b) * factorial(s - c));
                t.v[a][b][c] =
                    factorial(2 * s - 2 * a) * factorial(2 * s - 2 * b) * factorial(2 * s - 2 * c) / factorial(2 * s + 1) * r * r;
            }
    return t;
}

// ------------------------------------------------------------ edge tables
// Polynomials in the edge parameter s with integer coefficients.
constexpr int kDeg1 = 10;
struct Poly1 {
    long long c[kDeg1];
};

Poly1 mul1(const Poly1& a, const Poly1& b) {
    Poly1 q;
    std::memset(&q, 0, sizeof(q));
    for (int i = 0; i < kDeg1; ++i)
        for (int j = 0; i + j < kDeg1; ++j) q.c[i + j] += a.c[i] * b.c[j];
    return q;
}

// phi^_p (without its square-root factor) along local edge q of the
// reference triangle, x = x0 + xs s, y = y0 + ys s; `back`: s -> 1 - s.
Poly1 basis_on_edge(int p, int q, bool back) {
    static const int lin[3][4] = {{0, 1, 0, 0}, {1, -1, 0, 1}, {0, 0, 1, -1}};   // x0, xs, y0, ys
    int x0 = lin[q][0], xs = lin[q][1], y0 = lin[q][2], ys = lin[q][3];
    if (back) {
        x0 += xs;
        xs = -xs;
        y0 += ys;
        ys = -ys;
    }
    Poly1 X, Y, out;
    std::memset(&X, 0, sizeof(X));
    std::memset(&Y, 0, sizeof(Y));
    std::memset(&out, 0, sizeof(out));
    X.c[0] = x0;
    X.c[1] = xs;
    Y.c[0] = y0;
    Y.c[1] = ys;
    for (int t = 0; t < 10; ++t) {
        const long long co = (long long)kCoef[p][t];
        if (co == 0) continue;
        Poly1 term;
        std::memset(&term, 0, sizeof(term));
        term.c[0] = co;
        for (int a = 0; a < kMono[t][0]; ++a) term = mul1(term, X);
        for (int b = 0; b < kMono[t][1]; ++b) term = mul1(term, Y);
        for (int i = 0; i < kDeg1; ++i) out.c[i] += term.c[i];
    }
    return out;
}

// int_0^1 of the polynomial, exactly over the common denominator 2520 =
// lcm(1..10), then times the square root of the scale product.
double integrate1(const Poly1& a, long long scale) {
    long long num = 0;
    for (int i = 0; i < kDeg1; ++i) num += a.c[i] * (2520 / (i + 1));
    return (double)num / 2520.0 * std::sqrt((double)scale);
}

// Velocity projection: one thread per element assembles the lower triangle
// of the H-weighted mass matrix, factors it (Cholesky, in registers) and
// solves for both velocity components (project_element; k_dg_project
// stores them, and the volume pass of a Runge-Kutta step computes them in
// place of reading them).
template <int K>
__device__ __forceinline__ void project_element(long long ne, long long e, const double* __restrict__ c,
                                                const double* __restrict__ B, const double* __restrict__ hb,
                                                const double* __restrict__ T, double (&uo)[2][K]) {
#pragma clang fp contract(fast)   // fused multiply-adds, as in k_dg_volume
    const double b11 = B[e], b12 = B[ne + e], b21 = B[2 * ne + e], b22 = B[3 * ne + e];
    const double ad = std::fabs(b11 * b22 - b12 * b21);
    const double sd = 1.0 / std::sqrt(ad);
    constexpr int NL = K * (K + 1) / 2;
    double L[NL];                                           // row-major lower triangle
#pragma unroll
    for (int q = 0; q < NL; ++q) L[q] = 0.0;
    // one coefficient of H = xi + h_b at a time (a rolled loop keeps the
    // table's scalar operands of one step live, not all K^3 of them)
#pragma unroll 1
    for (int i = 0; i < K; ++i) {
        const double h = c[(long long)i * ne + e] + hb[(long long)i * ne + e];
        const double* Ti = T + i * K;
#pragma unroll
        for (int p = 0; p < K; ++p)
#pragma unroll
            for (int m = 0; m <= p; ++m) L[p * (p + 1) / 2 + m] += h * Ti[p * K * K + m];
    }
#pragma unroll
    for (int q = 0; q < NL; ++q) L[q] *= sd;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double d = L[j * (j + 1) / 2 + j];
#pragma unroll
        for (int q = 0; q < j; ++q) d -= L[j * (j + 1) / 2 + q] * L[j * (j + 1) / 2 + q];
        const double ljj = std::sqrt(d);
        L[j * (j + 1) / 2 + j] = ljj;
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
            double v = L[i * (i + 1) / 2 + j];
#pragma unroll
            for (int q = 0; q < j; ++q) v -= L[i * (i + 1) / 2 + q] * L[j * (j + 1) / 2 + q];
            L[i * (i + 1) / 2 + j] = v / ljj;
        }
    }
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {
        double y[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            double v = c[(long long)((1 + comp) * K + i) * ne + e];
#pragma unroll
            for (int q = 0; q < i; ++q) v -= L[i * (i + 1) / 2 + q] * y[q];
            y[i] = v / L[i * (i + 1) / 2 + i];
        }
#pragma unroll
        for (int i = K - 1; i >= 0; --i) {
            double v = y[i];
#pragma unroll
            for (int q = i + 1; q < K; ++q) v -= L[q * (q + 1) / 2 + i] * y[q];
            y[i] = v / L[i * (i + 1) / 2 + i];
        }
#pragma unroll
        for (int i = 0; i < K; ++i) uo[comp][i] = y[i];
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_dg_project(long long ne, const double* __restrict__ c,
                                                    const double* __restrict__ B, const double* __restrict__ hb,
                                                    const double* __restrict__ T, double* __restrict__ u) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    double uo[2][K];
    project_element<K>(ne, e, c, B, hb, T, uo);
#pragma unroll
    for (int comp = 0; comp < 2; ++comp)
#pragma unroll
        for (int i = 0; i < K; ++i) u[(long long)(comp * K + i) * ne + e] = uo[comp][i];
}

// One thread per element: for every test function p the mass flux and, per
// i, the sums over m of the three-function integrals, contracted with the
// coefficients of i.  The velocity enters the advective terms only through
// u d/dx1 + v d/dx2 = (1/det) [(B22 u - B12 v) d/dx^1 + (B11 v - B21 u) d/dx^2],
// so the element's map is folded into two combined velocity vectors first
// and each (p, i) costs four multiply-adds per m.  The pressure term
// g xi (H + h_b) / 2 = g xi (xi + 2 h_b) / 2 is one product of two P^k
// fields.  With RHS the source (g xi grad h_b, friction, Coriolis) and the
// body force are added: out = E + R + F.
template <int K, bool RHS, bool PROJ = false>
__global__ __launch_bounds__(256) void k_dg_volume(long long ne, const double* __restrict__ c,
                                                   const double* __restrict__ u, const double* __restrict__ B,
                                                   const double* __restrict__ hb, double g,
                                                   const double* __restrict__ ref, double* __restrict__ out,
                                                   double tau, double fc, const double* __restrict__ F,
                                                   const double* __restrict__ T, double* __restrict__ uout) {
    // The library is built with contraction off so that the multigrid
    // kernels round every multiply and add as written (bitwise parity with
    // the oracle); the DG terms are checked to a tolerance and cost FP64
    // issue, so here a * b + c is one fused multiply-add.
#pragma clang fp contract(fast)
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const double b11 = B[e], b12 = B[ne + e], b21 = B[2 * ne + e], b22 = B[3 * ne + e];
    constexpr int KT = kb_const<K>();                    // table order and bathymetry coefficients
    // PROJ: the element's velocity from its own state (the projection of a
    // Runge-Kutta stage), stored for the edge pass and used from registers
    double uo[2][K];
    if constexpr (PROJ) {
        project_element<K>(ne, e, c, B, hb, T, uo);
#pragma unroll
        for (int comp = 0; comp < 2; ++comp)
#pragma unroll
            for (int i = 0; i < K; ++i) uout[(long long)(comp * K + i) * ne + e] = uo[comp][i];
    }
    double xi[K], U[K], V[K], wa[K], wb[K], w[K], hv[KT];
#pragma unroll
    for (int i = 0; i < KT; ++i) hv[i] = hb[(long long)i * ne + e];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        xi[i] = c[(long long)i * ne + e];
        U[i] = c[(long long)(K + i) * ne + e];
        V[i] = c[(long long)(2 * K + i) * ne + e];
        const double uu = PROJ ? uo[0][i] : u[(long long)i * ne + e];
        const double vv = PROJ ? uo[1][i] : u[(long long)(K + i) * ne + e];
        wa[i] = b22 * uu - b12 * vv;
        wb[i] = b11 * vv - b21 * uu;
        w[i] = xi[i] + 2.0 * hv[i];
    }
    const double det = b11 * b22 - b12 * b21;
    const double s2 = 1.0 / det;                         // two-function integrals
    const double s3 = s2 / std::sqrt(std::fabs(det));    // three-function integrals
    // (for k = 0 the gradient of the one test function vanishes and only
    // the source remains; the h_b products there need the order-1 table)
    const double* G0 = ref;
    const double* G1 = ref + KT * KT;
    const double* H0 = ref + 2 * KT * KT;
    const double* H1 = H0 + KT * KT * KT;
    for (int p = 0; p < K; ++p) {
        double e1 = 0.0, e2 = 0.0, e3 = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const double gx = G0[p * KT + i], gy = G1[p * KT + i];
            const double d1 = b22 * gx - b21 * gy;       // x1-derivative direction
            const double d2 = b11 * gy - b12 * gx;       // x2-derivative direction
            e1 += U[i] * d1 + V[i] * d2;
            double t = 0.0, h0x = 0.0, h1x = 0.0;
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const double h0 = H0[(p * KT + i) * KT + m], h1 = H1[(p * KT + i) * KT + m];
                t += h0 * wa[m] + h1 * wb[m];
                h0x += h0 * w[m];
                h1x += h1 * w[m];
            }
            // sums over m of w_m dx1(.) and w_m dx2(.) (times det)
            const double px = b22 * h0x - b21 * h1x, py = b11 * h1x - b12 * h0x;
            e2 += U[i] * t + 0.5 * g * xi[i] * px;
            e3 += V[i] * t + 0.5 * g * xi[i] * py;
        }
        double o1 = e1 * s2, o2 = e2 * s3, o3 = e3 * s3;
        if constexpr (RHS) {
            // (g xi dh_b/dx_l, phi_p): the three-function integrals with the
            // derivative on h_b's function m
            double sx = 0.0, sy = 0.0;
#pragma unroll
            for (int m = 0; m < KT; ++m) {
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    a0 += xi[i] * H0[(m * KT + p) * KT + i];
                    a1 += xi[i] * H1[(m * KT + p) * KT + i];
                }
                sx += hv[m] * a0;
                sy += hv[m] * a1;
            }
            const double Up = c[(long long)(K + p) * ne + e], Vp = c[(long long)(2 * K + p) * ne + e];
            o2 += g * s3 * (b22 * sx - b21 * sy) + (fc * Vp - tau * Up);
            o3 += g * s3 * (b11 * sy - b12 * sx) - (fc * Up + tau * Vp);
            if (F) {
                o1 += F[(long long)p * ne + e];
                o2 += F[(long long)(K + p) * ne + e];
                o3 += F[(long long)(2 * K + p) * ne + e];
            }
        }
        out[(long long)p * ne + e] = o1;
        out[(long long)(K + p) * ne + e] = o2;
        out[(long long)(2 * K + p) * ne + e] = o3;
    }
}

// Block order of the edge pass.  The hardware deals consecutive blocks to
// the eight XCDs in turn, each with its own L2.  Here every XCD runs a
// contiguous range of a sequence that pairs block l with block l + H (H half
// the blocks, rounded up): on the split-quad numbering the second half of
// the elements holds the first half's edge neighbours, so an element's
// coefficients are still in its XCD's L2 when the neighbouring waves gather
// them.  Any other numbering only loses that benefit: the map is a
// bijection of the block indices.
__device__ __forceinline__ long long edge_block(long long b, long long nb) {
    const long long per = nb >> 3, rem = nb & 7;
    const long long x = b & 7, r = b >> 3;
    const long long lam = (x < rem) ? x * (per + 1) + r : rem * (per + 1) + (x - rem) * per + r;
    const long long H = (nb + 1) >> 1, pairs = nb - H;
    if (lam < 2 * pairs) return (lam & 1) ? H + (lam >> 1) : (lam >> 1);
    return lam - pairs;      // the unpaired middle block of an odd count
}

// Edge terms: one thread per element, edges in turn.  Every basis
// function restricted to an edge is a polynomial of degree max(k, 1) in the
// edge parameter s, so each field's trace is expanded in shifted Legendre
// polynomials P_a(s) on [0, 1] (coefficients C[q][i][a] of the table), the
// flux's products of two traces are integrated against P_a with the exact
// table L3[a][b][c] = int P_a P_b P_c, and the result is taken back to the
// test functions with C again: exact integrals as with full triple-product
// tables, at K (k + 1) instead of K^2 operations per field and edge side.
// A neighbour's edge runs the other way (s -> 1 - s), which flips the sign
// of its odd Legendre coefficients; a prescribed exterior state is a
// polynomial in the element's own basis on the same edge.  The neighbour's
// local edge index selects its rows of C, which every lane reads from a
// copy of the (small) table in LDS: serving the lanes of a wavefront one
// neighbour kind at a time, so as to read the table at wave-uniform
// addresses, held every value live across that loop and cost a quarter of
// the occupancy.  The result is written to out once (SUB: subtracted from
// it).
template <int K, bool SUB>
__global__ __launch_bounds__(256) void k_dg_edges(long long ne, const double* __restrict__ c,
                                                  const double* __restrict__ u, const double* __restrict__ B,
                                                  const double* __restrict__ hb, const int* __restrict__ nbr,
                                                  const int* __restrict__ nq, long long nb,
                                                  const double* __restrict__ cb, const double* __restrict__ ub,
                                                  double g, const double* __restrict__ tab,
                                                  double* __restrict__ out) {
#pragma clang fp contract(fast)   // fused multiply-adds, as in k_dg_volume
    constexpr int KT = kb_const<K>();    // bathymetry coefficients (and rows of C)
    constexpr int NT = nt_const<K>();    // Legendre coefficients of a state trace
    constexpr int NB = nb_const<K>();    // ... of the bathymetry's trace (table stride)
    // the coefficient gathers: unrolled at orders 0 and 1; at orders 2 and 3
    // rolled, or every load would be hoisted and the registers would spill
    constexpr int UR = K <= 3 ? KT : 1;
    const long long e0 = edge_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    const bool live = e0 < ne;
    const long long e = live ? e0 : 0;     // lanes past the end read element 0 and write nothing
    const double b11 = B[e], b12 = B[ne + e], b21 = B[2 * ne + e], b22 = B[3 * ne + e];
    const double adet = std::fabs(b11 * b22 - b12 * b21);
    const double a = 1.0 / std::sqrt(adet);
    const double v1 = std::sqrt(2.0 / adet);                       // value of phi_e1
    const double umx = u[e] * v1, umy = u[(long long)K * ne + e] * v1, Hm = (c[e] + hb[e]) * v1;
    // every edge's integrals against P_t (scaled), one private LDS column per
    // thread (structure of arrays: no bank conflicts, and no thread reads
    // another's column); the map to the test functions and the one write of
    // out come after the last edge
    __shared__ double sG[3 * 3 * NT][256];
    __shared__ double sC[3 * KT * NB];
    const int tid = threadIdx.x;
    for (int j = tid; j < 3 * KT * NB; j += 256) sC[j] = tab[j];
    __syncthreads();                     // every thread reaches it: no return above
    const double* Ctr = tab;
    constexpr Legendre3 L3 = legendre3();   // compile-time constants: the zeros fold away
#pragma unroll 1
    for (int q = 0; q < 3; ++q) {
        const double dx = q == 0 ? b11 : (q == 1 ? b12 - b11 : -b12);
        const double dy = q == 0 ? b21 : (q == 1 ? b22 - b21 : -b22);
        const double L = std::sqrt(dx * dx + dy * dy);
        const double n1 = dy / L, n2 = -dx / L;
        const double* Cq = Ctr + q * KT * NB;
        // the element's traces (physical values): xi, U, V, u . n, xi + 2 h_b
        double Xm[NT], Um[NT], Vm[NT], Nm[NT], Wm[NB];
#pragma unroll
        for (int t = 0; t < NT; ++t) Xm[t] = Um[t] = Vm[t] = Nm[t] = 0.0;
#pragma unroll
        for (int t = 0; t < NB; ++t) Wm[t] = 0.0;
#pragma unroll UR
        for (int i = 0; i < KT; ++i) {
            double w = 2.0 * hb[(long long)i * ne + e];
            if (i < K) {
                const double x = c[(long long)i * ne + e];
                const double U = c[(long long)(K + i) * ne + e], V = c[(long long)(2 * K + i) * ne + e];
                const double un = u[(long long)i * ne + e] * n1 + u[(long long)(K + i) * ne + e] * n2;
                w += x;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const double ct = Cq[i * NB + t];
                    Xm[t] += x * ct;
                    Um[t] += U * ct;
                    Vm[t] += V * ct;
                    Nm[t] += un * ct;
                }
            }
#pragma unroll
            for (int t = 0; t < NB; ++t) Wm[t] += w * Cq[i * NB + t];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            Xm[t] *= a;
            Um[t] *= a;
            Vm[t] *= a;
            Nm[t] *= a;
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) Wm[t] *= a;
        // kind 0..2: a neighbour, across its local edge kind; 3: a prescribed
        // state; anything out of range: no term
        const int fr = live ? nbr[(long long)q * ne + e] : -1;
        int kind = -1;
        long long f = 0;
        if (fr >= 0) {
            const int qr = nq[(long long)q * ne + e];
            if ((long long)fr < ne && qr >= 0 && qr <= 2) {
                kind = qr;
                f = fr;
            }
        } else if (fr <= -2 && cb && ub && (long long)(-2 - (long long)fr) < nb) {
            kind = 3;
            f = -2 - (long long)fr;
        }
#pragma unroll
        for (int t = 0; t < 3 * NT; ++t) sG[q * 3 * NT + t][tid] = 0.0;
        if (kind >= 0) {
            const int ks = kind;
            const bool ghost = ks == 3;
            const double* cs = ghost ? cb : c;
            const double* us = ghost ? ub : u;
            const long long st = ghost ? nb : ne;
            const long long fg = ghost ? e : f;          // geometry and bathymetry of the exterior side
            const double c11 = B[fg], c12 = B[ne + fg], c21 = B[2 * ne + fg], c22 = B[3 * ne + fg];
            const double fdet = std::fabs(c11 * c22 - c12 * c21);
            const double bsc = 1.0 / std::sqrt(fdet);
            const double w1 = std::sqrt(2.0 / fdet);
            const double* Cn = sC + (ghost ? q : ks) * KT * NB;
            double Xp[NT], Up[NT], Vp[NT], Np[NT], Wp[NB];
#pragma unroll
            for (int t = 0; t < NT; ++t) Xp[t] = Up[t] = Vp[t] = Np[t] = 0.0;
#pragma unroll
            for (int t = 0; t < NB; ++t) Wp[t] = 0.0;
#pragma unroll UR
            for (int i = 0; i < KT; ++i) {
                double w = 2.0 * hb[(long long)i * ne + fg];
                if (i < K) {
                    const double x = cs[(long long)i * st + f];
                    const double U = cs[(long long)(K + i) * st + f], V = cs[(long long)(2 * K + i) * st + f];
                    const double un = us[(long long)i * st + f] * n1 + us[(long long)(K + i) * st + f] * n2;
                    w += x;
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const double ct = Cn[i * NB + t];
                        Xp[t] += x * ct;
                        Up[t] += U * ct;
                        Vp[t] += V * ct;
                        Np[t] += un * ct;
                    }
                }
#pragma unroll
                for (int t = 0; t < NB; ++t) Wp[t] += w * Cn[i * NB + t];
            }
            // scale, and for a neighbour flip the odd coefficients (s -> 1 - s)
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                const double sc = (!ghost && (t & 1)) ? -bsc : bsc;
                if (t < NT) {
                    Xp[t] *= sc;
                    Up[t] *= sc;
                    Vp[t] *= sc;
                    Np[t] *= sc;
                }
                Wp[t] *= sc;
            }
            const double Hp = (cs[f] + hb[fg]) * w1;
            const double lam = fmax(std::fabs(umx * n1 + umy * n2) + std::sqrt(g * Hm),
                                    std::fabs((us[f] * n1 + us[(long long)K * st + f] * n2) * w1) + std::sqrt(g * Hp));
            // int P_t F ds for the three flux rows, t < NT: each product of two
            // traces is formed once and scattered into the t accumulators (the
            // zero integrals fold away), which keeps few values live
            double qun[NT], qvn[NT], qxw[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) qun[t] = qvn[t] = qxw[t] = 0.0;
#pragma unroll
            for (int b2 = 0; b2 < NT; ++b2) {
#pragma unroll
                for (int c2 = 0; c2 < NB; ++c2) {
                    const double px = Xm[b2] * Wm[c2] + Xp[b2] * Wp[c2];
                    double pu = 0.0, pv = 0.0;
                    if (c2 < NT) {
                        pu = Um[b2] * Nm[c2] + Up[b2] * Np[c2];
                        pv = Vm[b2] * Nm[c2] + Vp[b2] * Np[c2];
                    }
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const double l = L3.v[t][b2][c2];
                        if (l == 0.0) continue;
                        if (c2 < NT) {
                            qun[t] += l * pu;
                            qvn[t] += l * pv;
                        }
                        qxw[t] += l * px;
                    }
                }
            }
            double G1[NT], G2[NT], G3[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double inv = 1.0 / (2 * t + 1);    // int P_t^2
                G1[t] = inv * (0.5 * (n1 * (Um[t] + Up[t]) + n2 * (Vm[t] + Vp[t])) + 0.5 * lam * (Xm[t] - Xp[t]));
                G2[t] = 0.5 * qun[t] + 0.25 * g * n1 * qxw[t] + 0.5 * lam * inv * (Um[t] - Up[t]);
                G3[t] = 0.5 * qvn[t] + 0.25 * g * n2 * qxw[t] + 0.5 * lam * inv * (Vm[t] - Vp[t]);
            }
            const double fac = L * a;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                sG[(q * 3 + 0) * NT + t][tid] = fac * G1[t];
                sG[(q * 3 + 1) * NT + t][tid] = fac * G2[t];
                sG[(q * 3 + 2) * NT + t][tid] = fac * G3[t];
            }
        }
    }
    if (!live) return;
#pragma unroll 1
    for (int p = 0; p < K; ++p) {
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double ct = Ctr[(q * KT + p) * NB + t];
                s1 += ct * sG[(q * 3 + 0) * NT + t][tid];
                s2 += ct * sG[(q * 3 + 1) * NT + t][tid];
                s3 += ct * sG[(q * 3 + 2) * NT + t][tid];
            }
        double* o = out + (long long)p * ne + e;
        const long long kn = (long long)K * ne;
        if (SUB) {
            o[0] -= s1;
            o[kn] -= s2;
            o[2 * kn] -= s3;
        } else {
            o[0] = s1;
            o[kn] = s2;
            o[2 * kn] = s3;
        }
    }
}

// One stage of the Runge-Kutta combination: y = a x + b (y + dt r).
__global__ __launch_bounds__(256) void k_dg_stage(long long n, double a, const double* __restrict__ x, double b,
                                                  double* __restrict__ y, double dt, const double* __restrict__ r) {
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        y[i] = a * x[i] + b * (y[i] + dt * r[i]);
}

// One thread per element in blocks of 256: a launch holds at most 2^32 - 1
// work-items, so ne is capped at the largest multiple of 256 below 2^32.
bool dg_size_ok(long long ne) { return ne >= 0 && ne <= (1LL << 32) - 256; }

// The reason of the last MG_EDEVICE of this thread (dg_last_error).
thread_local char g_dg_error[160] = "";

int dg_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return MG_OK;
    snprintf(g_dg_error, sizeof g_dg_error, "%s: %s", what, hipGetErrorName(e));
    return MG_EDEVICE;
}

// A device entry point starts from a clear error status: hipGetLastError
// also reports what an earlier call of another library left pending, which
// must not be taken for a failure of this entry point's launches.
void dg_begin() {
    (void)hipGetLastError();
    g_dg_error[0] = 0;
}

// proj (with rhs): the velocity is computed from c with the product table T
// and stored to uout instead of read from u
int launch_volume(int K, bool rhs, long long ne, const double* c, const double* u, const double* B, const double* hb,
                  double g, const double* ref, double* out, double tau, double fc, const double* F, hipStream_t st,
                  bool proj = false, const double* T = nullptr, double* uout = nullptr) {
    const unsigned nbk = (unsigned)((ne + 255) / 256);
#define DG_VOL(KK)                                                                                         \
    if (proj)                                                                                              \
        k_dg_volume<KK, true, true><<<nbk, 256, 0, st>>>(ne, c, u, B, hb, g, ref, out, tau, fc, F, T, uout); \
    else if (rhs)                                                                                          \
        k_dg_volume<KK, true><<<nbk, 256, 0, st>>>(ne, c, u, B, hb, g, ref, out, tau, fc, F, T, uout);    \
    else                                                                                                   \
        k_dg_volume<KK, false><<<nbk, 256, 0, st>>>(ne, c, u, B, hb, g, ref, out, tau, fc, F, T, uout);
    switch (K) {
        case 1: DG_VOL(1) break;
        case 3: DG_VOL(3) break;
        case 6: DG_VOL(6) break;
        default: DG_VOL(10) break;
    }
#undef DG_VOL
    return dg_status(hipGetLastError(), "volume kernel launch");
}

int launch_edges(int K, bool sub, long long ne, const double* c, const double* u, const double* B, const double* hb,
                 const int* nbr, const int* nq, long long nb, const double* cb, const double* ub, double g,
                 const double* table, double* out, hipStream_t st) {
    const unsigned nbk = (unsigned)((ne + 255) / 256);
#define DG_EDGE(KK)                                                                                          \
    if (sub)                                                                                                 \
        k_dg_edges<KK, true><<<nbk, 256, 0, st>>>(ne, c, u, B, hb, nbr, nq, nb, cb, ub, g, table, out);    \
    else                                                                                                     \
        k_dg_edges<KK, false><<<nbk, 256, 0, st>>>(ne, c, u, B, hb, nbr, nq, nb, cb, ub, g, table, out);
    switch (K) {
        case 1: DG_EDGE(1) break;
        case 3: DG_EDGE(3) break;
        case 6: DG_EDGE(6) break;
        default: DG_EDGE(10) break;
    }
#undef DG_EDGE
    return dg_status(hipGetLastError(), "edge kernel launch");
}

int launch_project(int K, long long ne, const double* c, const double* B, const double* hb, const double* T,
                   double* u, hipStream_t st) {
    const unsigned nbk = (unsigned)((ne + 255) / 256);
    switch (K) {
        case 1: k_dg_project<1><<<nbk, 256, 0, st>>>(ne, c, B, hb, T, u); break;
        case 3: k_dg_project<3><<<nbk, 256, 0, st>>>(ne, c, B, hb, T, u); break;
        case 6: k_dg_project<6><<<nbk, 256, 0, st>>>(ne, c, B, hb, T, u); break;
        default: k_dg_project<10><<<nbk, 256, 0, st>>>(ne, c, B, hb, T, u); break;
    }
    return dg_status(hipGetLastError(), "projection kernel launch");
}

int launch_stage(long long n, double a, const double* x, double b, double* y, double dt, const double* r,
                 hipStream_t st) {
    const long long want = (n + 255) / 256;
    const unsigned nbk = (unsigned)(want < 65536 ? want : 65536);
    k_dg_stage<<<nbk, 256, 0, st>>>(n, a, x, b, y, dt, r);
    return dg_status(hipGetLastError(), "stage kernel launch");
}

// the edge arguments: a prescribed-state count needs both state arrays
bool ghosts_ok(long long nb, const double* cb, const double* ub) {
    return nb >= 0 && nb <= 0x7fffffffLL && (nb == 0 || (cb && ub));
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call on that device (with it current) and kept.
int scratch_address(double** out) {
    int dev = -1;
    if (int rc = dg_status(hipGetDevice(&dev), "current device")) return rc;
    if (dev < 0 || dev >= kMaxDevices) {
        snprintf(g_dg_error, sizeof g_dg_error, "device %d beyond the scratch table", dev);
        return MG_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (int rc = dg_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address")) return rc;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MG_OK;
}

// One SSP-RK3 step with the saved state and the right-hand side in work
// (6 K ne doubles): the body of both RK entry points.
int rk3_step(int k, long long ne, double* c, double* u, double* work, const double* B, const double* hb,
             const int* nbr, const int* nq, long long nb, const double* cb3, const double* ub3, double g, double tau,
             double fc, const double* F3, const double* ref, const double* T, const double* table, double dt,
             void* stream) {
    const int K = k_of(k);
    if (!K || !dg_size_ok(ne) || !ghosts_ok(nb, cb3, ub3) || !std::isfinite(dt)) return MG_EINVAL;
    if (ne == 0) return MG_OK;
    if (!c || !u || !work || !B || !hb || !nbr || !nq || !ref || !T || !table) return MG_EINVAL;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const long long n = 3LL * K * ne;
    double* c0 = work;
    double* r = work + n;
    dg_begin();
    const int cp = dg_status(hipMemcpyAsync(c0, c, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, st),
                             "copy of the state");
    if (cp != MG_OK) return cp;
    const double wa[3] = {0.0, 0.75, 1.0 / 3.0}, wb[3] = {1.0, 0.25, 2.0 / 3.0};
    for (int s = 0; s < 3; ++s) {
        // the stage's velocity: projected inside the volume pass up to order
        // 2; at order 3 the projection's serial Cholesky chain runs faster
        // on its own (three wavefronts per SIMD against two in the fused
        // pass) than the saved traffic is worth
        const bool fuse = K <= 6;
        int rc = fuse ? MG_OK : launch_project(K, ne, c, B, hb, T, u, st);
        if (rc == MG_OK)
            rc = launch_volume(K, true, ne, c, u, B, hb, g, ref, r, tau, fc, F3 ? F3 + s * n : nullptr, st, fuse,
                               T, u);
        if (rc == MG_OK)
            rc = launch_edges(K, true, ne, c, u, B, hb, nbr, nq, nb, nb ? cb3 + s * 3LL * K * nb : nullptr,
                              nb ? ub3 + s * 2LL * K * nb : nullptr, g, table, r, st);
        if (rc == MG_OK) rc = launch_stage(n, wa[s], c0, wb[s], c, dt, r, st);
        if (rc != MG_OK) return rc;
    }
    return MG_OK;
}


}  // namespace

extern "C" {

const char* dg_last_error(void) { return g_dg_error; }

int dg_basis_values(int k, long long npts, const double* x, const double* y, double* out) {
    const int K = k_of(k);
    if (!K || npts < 0 || (npts > 0 && (!x || !y || !out))) return MG_EINVAL;
    for (int p = 0; p < K; ++p) {
        const double sc = std::sqrt((double)kScale[p]);
        for (long long q = 0; q < npts; ++q) {
            double v = 0.0;
            for (int t = 0; t < 10; ++t) {
                if (kCoef[p][t] == 0.0) continue;
                v += kCoef[p][t] * std::pow(x[q], kMono[t][0]) * std::pow(y[q], kMono[t][1]);
            }
            out[(long long)p * npts + q] = sc * v;
        }
    }
    return MG_OK;
}

long long dg_reference_size(int k) {
    const long long K = k_of(k) ? kb_of(k) : 0;
    return K ? 2 * K * K + 2 * K * K * K : 0;
}

int dg_reference_integrals(int k, double* ref) {
    const int K = k_of(k) ? kb_of(k) : 0;
    if (!K || !ref) return MG_EINVAL;
    Poly phi[kMaxK], dphi[2][kMaxK];
    for (int p = 0; p < K; ++p) {
        phi[p] = basis_poly(p);
        dphi[0][p] = deriv(phi[p], 0);
        dphi[1][p] = deriv(phi[p], 1);
    }
    const long long* sc = kScale;
    for (int l = 0; l < 2; ++l)
        for (int p = 0; p < K; ++p)
            for (int i = 0; i < K; ++i) {
                const Poly dp_i = mul(dphi[l][p], phi[i]);
                ref[(l * K + p) * K + i] = integrate(dp_i, sc[p] * sc[i]);
                for (int m = 0; m < K; ++m)
                    ref[2 * K * K + ((l * K + p) * K + i) * K + m] =
                        integrate(mul(dp_i, phi[m]), sc[p] * sc[i] * sc[m]);
            }
    return MG_OK;
}

long long dg_product_size(int k) {
    const long long K = k_of(k);
    return K * K * K;
}

int dg_product_integrals(int k, double* T) {
    const int K = k_of(k);
    if (!K || !T) return MG_EINVAL;
    Poly phi[kMaxK];
    for (int p = 0; p < K; ++p) phi[p] = basis_poly(p);
    for (int p = 0; p < K; ++p)
        for (int i = 0; i < K; ++i) {
            const Poly pi = mul(phi[p], phi[i]);
            for (int m = 0; m < K; ++m)
                T[(p * K + i) * K + m] = integrate(mul(pi, phi[m]), kScale[p] * kScale[i] * kScale[m]);
        }
    return MG_OK;
}

int dg_velocity_projection(int k, long long ne, const double* c, const double* B, const double* hb,
                           const double* T, double* u, void* stream) {
    const int K = k_of(k);
    if (!K || !dg_size_ok(ne)) return MG_EINVAL;
    if (ne == 0) return MG_OK;
    if (!c || !B || !hb || !T || !u) return MG_EINVAL;
    dg_begin();
    return launch_project(K, ne, c, B, hb, T, u, static_cast<hipStream_t>(stream));
}

long long dg_edge_table_size(int k) {
    if (!k_of(k)) return 0;
    return 3LL * kb_of(k) * nb_of(k);
}

int dg_edge_integrals(int k, double* table) {
    if (!k_of(k) || !table) return MG_EINVAL;
    const int KT = kb_of(k), NB = nb_of(k);
    // shifted Legendre polynomials on [0, 1]: 1, 2s - 1, 6s^2 - 6s + 1,
    // 20s^3 - 30s^2 + 12s - 1
    static const long long leg[4][4] = {{1, 0, 0, 0}, {-1, 2, 0, 0}, {1, -6, 6, 0}, {-1, 12, -30, 20}};
    for (int q = 0; q < 3; ++q)
        for (int i = 0; i < KT; ++i) {
            const Poly1 tr = basis_on_edge(i, q, false);
            for (int a = 0; a < NB; ++a) {
                Poly1 P;
                std::memset(&P, 0, sizeof(P));
                for (int j = 0; j < 4; ++j) P.c[j] = leg[a][j] * (2 * a + 1);   // exact before the one division
                table[(q * KT + i) * NB + a] = integrate1(mul1(tr, P), kScale[i]);
            }
        }
    return MG_OK;
}

int dg_edge_terms(int k, long long ne, const double* c, const double* u, const double* B, const double* hb,
                  const int* nbr, const int* nq, long long nb, const double* cb, const double* ub, double g,
                  const double* table, double* out, void* stream) {
    const int K = k_of(k);
    if (!K || !dg_size_ok(ne) || !ghosts_ok(nb, cb, ub)) return MG_EINVAL;
    if (ne == 0) return MG_OK;
    if (!c || !u || !B || !hb || !nbr || !nq || !table || !out) return MG_EINVAL;
    dg_begin();
    return launch_edges(K, false, ne, c, u, B, hb, nbr, nq, nb, cb, ub, g, table, out,
                        static_cast<hipStream_t>(stream));
}

int dg_volume_integrals(int k, long long ne, const double* c, const double* u, const double* B, const double* hb,
                        double g, const double* ref, double* out, void* stream) {
    const int K = k_of(k);
    if (!K || !dg_size_ok(ne)) return MG_EINVAL;
    if (ne == 0) return MG_OK;
    if (!c || !u || !B || !hb || !ref || !out) return MG_EINVAL;
    dg_begin();
    return launch_volume(K, false, ne, c, u, B, hb, g, ref, out, 0.0, 0.0, nullptr,
                         static_cast<hipStream_t>(stream));
}

int dg_rhs(int k, long long ne, const double* c, const double* u, const double* B, const double* hb,
           const int* nbr, const int* nq, long long nb, const double* cb, const double* ub, double g, double tau,
           double fc, const double* F, const double* ref, const double* table, double* out, void* stream) {
    const int K = k_of(k);
    if (!K || !dg_size_ok(ne) || !ghosts_ok(nb, cb, ub)) return MG_EINVAL;
    if (ne == 0) return MG_OK;
    if (!c || !u || !B || !hb || !nbr || !nq || !ref || !table || !out) return MG_EINVAL;
    dg_begin();
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const int rc = launch_volume(K, true, ne, c, u, B, hb, g, ref, out, tau, fc, F, st);
    if (rc != MG_OK) return rc;
    return launch_edges(K, true, ne, c, u, B, hb, nbr, nq, nb, cb, ub, g, table, out, st);
}

int dg_ssp_rk3_step(int k, long long ne, double* c, double* u, double* work, const double* B, const double* hb,
                    const int* nbr, const int* nq, long long nb, const double* cb3, const double* ub3, double g,
                    double tau, double fc, const double* F3, const double* ref, const double* T,
                    const double* table, double dt, void* stream) {
    if (ne > 0 && !work) return MG_EINVAL;
    return rk3_step(k, ne, c, u, work, B, hb, nbr, nq, nb, cb3, ub3, g, tau, fc, F3, ref, T, table, dt, stream);
}

int dg_ssp_rk3_step_noalloc(int k, long long ne, double* c, double* u, const double* B, const double* hb,
                            const int* nbr, const int* nq, long long nb, const double* cb3, const double* ub3,
                            double g, double tau, double fc, const double* F3, const double* ref, const double* T,
                            const double* table, double dt, void* stream) {
    g_dg_error[0] = 0;
    const int K = k_of(k);
    if (!K || ne < 0) return MG_EINVAL;
    if (6LL * K * ne > kDgScratchDoubles) {
        snprintf(g_dg_error, sizeof g_dg_error, "6 K ne = %lld doubles exceed the fixed scratch of %lld", 6LL * K * ne,
                 kDgScratchDoubles);
        return MG_EINVAL;
    }
    if (ne == 0) return rk3_step(k, ne, c, u, nullptr, B, hb, nbr, nq, nb, cb3, ub3, g, tau, fc, F3, ref, T, table, dt,
                                 stream);
    if (!c || !u || !B || !hb || !nbr || !nq || !ref || !T || !table) return MG_EINVAL;
    dg_begin();
    double* w = nullptr;
    if (int rc = scratch_address(&w)) return rc;
    return rk3_step(k, ne, c, u, w, B, hb, nbr, nq, nb, cb3, ub3, g, tau, fc, F3, ref, T, table, dt, stream);
}

}  // extern "C"
