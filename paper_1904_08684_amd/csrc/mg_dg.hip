// Volume terms of the quadrature-free DG shallow-water scheme (see dg.h):
// exact reference integrals on the host, one GPU thread per element.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "dg.h"
#include "mg.h"

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

// One thread per element: for every test function p the two-function terms
// (mass flux and bathymetry) and, per i, the sums over m of the
// three-function integrals, contracted with the coefficients of i.  The
// velocity enters the advective terms only through
// u d/dx1 + v d/dx2 = (1/det) [(B22 u - B12 v) d/dx^1 + (B11 v - B21 u) d/dx^2],
// so the element's map is folded into two combined velocity vectors first
// and each (p, i) costs four multiply-adds per m.
template <int K>
__global__ __launch_bounds__(256) void k_dg_volume(long long ne, const double* __restrict__ c,
                                                   const double* __restrict__ u, const double* __restrict__ B,
                                                   const double* __restrict__ hb, double g,
                                                   const double* __restrict__ ref, double* __restrict__ out) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const double b11 = B[e], b12 = B[ne + e], b21 = B[2 * ne + e], b22 = B[3 * ne + e];
    double xi[K], U[K], V[K], wa[K], wb[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        xi[i] = c[(long long)i * ne + e];
        U[i] = c[(long long)(K + i) * ne + e];
        V[i] = c[(long long)(2 * K + i) * ne + e];
        const double uu = u[(long long)i * ne + e], vv = u[(long long)(K + i) * ne + e];
        wa[i] = b22 * uu - b12 * vv;
        wb[i] = b11 * vv - b21 * uu;
    }
    const double det = b11 * b22 - b12 * b21;
    const double s2 = 1.0 / det;                         // two-function integrals
    const double s3 = s2 / std::sqrt(std::fabs(det));    // three-function integrals
    const double gh = g * hb[e];
    const double* G0 = ref;
    const double* G1 = ref + K * K;
    const double* H0 = ref + 2 * K * K;
    const double* H1 = H0 + K * K * K;
    for (int p = 0; p < K; ++p) {
        double e1 = 0.0, l2 = 0.0, l3 = 0.0, e2 = 0.0, e3 = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const double gx = G0[p * K + i], gy = G1[p * K + i];
            const double d1 = b22 * gx - b21 * gy;       // x1-derivative direction
            const double d2 = b11 * gy - b12 * gx;       // x2-derivative direction
            e1 += U[i] * d1 + V[i] * d2;
            l2 += xi[i] * d1;
            l3 += xi[i] * d2;
            double t = 0.0, h0x = 0.0, h1x = 0.0;
#pragma unroll
            for (int m = 0; m < K; ++m) {
                const double h0 = H0[(p * K + i) * K + m], h1 = H1[(p * K + i) * K + m];
                t += h0 * wa[m] + h1 * wb[m];
                h0x += h0 * xi[m];
                h1x += h1 * xi[m];
            }
            // sums over m of xi_m dx1(.) and xi_m dx2(.) (times det)
            const double px = b22 * h0x - b21 * h1x, py = b11 * h1x - b12 * h0x;
            e2 += U[i] * t + 0.5 * g * xi[i] * px;
            e3 += V[i] * t + 0.5 * g * xi[i] * py;
        }
        out[(long long)p * ne + e] = e1 * s2;
        out[(long long)(K + p) * ne + e] = e2 * s3 + gh * l2 * s2;
        out[(long long)(2 * K + p) * ne + e] = e3 * s3 + gh * l3 * s2;
    }
}

// Velocity projection: one thread per element assembles the lower triangle
// of the H-weighted mass matrix, factors it (Cholesky, in registers) and
// solves for both velocity components.
template <int K>
__global__ __launch_bounds__(256) void k_dg_project(long long ne, const double* __restrict__ c,
                                                    const double* __restrict__ B, const double* __restrict__ hb,
                                                    const double* __restrict__ T, double* __restrict__ u) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= ne) return;
    const double b11 = B[e], b12 = B[ne + e], b21 = B[2 * ne + e], b22 = B[3 * ne + e];
    const double ad = std::fabs(b11 * b22 - b12 * b21);
    const double sd = 1.0 / std::sqrt(ad);
    constexpr int NL = K * (K + 1) / 2;
    double L[NL];                                           // row-major lower triangle
#pragma unroll
    for (int q = 0; q < NL; ++q) L[q] = 0.0;
    // one coefficient of H at a time (a rolled loop keeps the table's scalar
    // operands of one step live, not all K^3 of them)
#pragma unroll 1
    for (int i = 0; i < K; ++i) {
        double h = c[(long long)i * ne + e];
        if (i == 0) h += hb[e] * std::sqrt(ad) * 0.70710678118654752440;   // h_b = (h_b sqrt|det| / sqrt 2) phi_e1
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
        for (int i = 0; i < K; ++i) u[(long long)(comp * K + i) * ne + e] = y[i];
    }
}

// Interior-edge terms: one thread per element, edges in turn; for each edge
// the neighbour's coefficients are gathered and both sides' contributions to
// every test function p are added to out.  The table offsets depend on the
// neighbour's local edge index q'; lanes of a wavefront are served one q'
// value at a time so that the table is always read at a wave-uniform address.
template <int K>
__global__ __launch_bounds__(256) void k_dg_edges(long long ne, const double* __restrict__ c,
                                                  const double* __restrict__ u, const double* __restrict__ B,
                                                  const double* __restrict__ hb, const int* __restrict__ nbr,
                                                  const int* __restrict__ nq, double g,
                                                  const double* __restrict__ tab, double* __restrict__ out) {
    const long long e0 = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool live = e0 < ne;
    const long long e = live ? e0 : 0;     // lanes past the end compute nothing but join the ballots
    const double b11 = B[e], b12 = B[ne + e], b21 = B[2 * ne + e], b22 = B[3 * ne + e];
    const double adet = std::fabs(b11 * b22 - b12 * b21);
    const double a = 1.0 / std::sqrt(adet);
    const double hm = hb[e];
    double xi[K], U[K], V[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        xi[i] = c[(long long)i * ne + e];
        U[i] = c[(long long)(K + i) * ne + e];
        V[i] = c[(long long)(2 * K + i) * ne + e];
    }
    const double v1 = std::sqrt(2.0 / adet);                       // value of phi_e1
    const double umx = u[e] * v1, umy = u[(long long)K * ne + e] * v1, Hm = xi[0] * v1 + hm;
    if (live)
        for (int t = 0; t < 3 * K; ++t) out[(long long)t * ne + e] = 0.0;
    const double* O2 = tab;
    const double* O3 = tab + 3 * K * K;
    const double* N2 = tab + 3 * K * K + 3 * K * K * K;
    const double* N3 = tab + 12 * K * K + 3 * K * K * K;
    for (int q = 0; q < 3; ++q) {
        const double dx = q == 0 ? b11 : (q == 1 ? b12 - b11 : -b12);
        const double dy = q == 0 ? b21 : (q == 1 ? b22 - b21 : -b22);
        const double L = std::sqrt(dx * dx + dy * dy);
        const double n1 = dy / L, n2 = -dx / L;
        // an index outside [0, ne) or a local edge outside 0..2 counts as boundary
        const int fr = live ? nbr[(long long)q * ne + e] : -1;
        const int qr = fr >= 0 ? nq[(long long)q * ne + e] : -1;
        const bool ok = fr >= 0 && (long long)fr < ne && qr >= 0 && qr <= 2;
        const int f = ok ? fr : 0, qp = ok ? qr : -1;
        bool todo = ok;
        for (;;) {
            const unsigned long long mask = __ballot(todo);
            if (mask == 0) break;
            const int qs = __builtin_amdgcn_readfirstlane(__shfl(qp, __ffsll((long long)mask) - 1));
            if (!(todo && qp == qs)) continue;
            todo = false;
            // the neighbour
            const double c11 = B[f], c12 = B[ne + f], c21 = B[2 * ne + f], c22 = B[3 * ne + f];
            const double fdet = std::fabs(c11 * c22 - c12 * c21);
            const double bsc = 1.0 / std::sqrt(fdet);
            const double w1 = std::sqrt(2.0 / fdet);
            double xo[K], Uo[K], Vo[K], wn[K], wo[K];
#pragma unroll
            for (int i = 0; i < K; ++i) {
                xo[i] = c[(long long)i * ne + f];
                Uo[i] = c[(long long)(K + i) * ne + f];
                Vo[i] = c[(long long)(2 * K + i) * ne + f];
                wo[i] = u[(long long)i * ne + f] * n1 + u[(long long)(K + i) * ne + f] * n2;
                wn[i] = u[(long long)i * ne + e] * n1 + u[(long long)(K + i) * ne + e] * n2;
            }
            const double hp = hb[f];
            const double Hp = xo[0] * w1 + hp;
            const double lam = fmax(std::fabs(umx * n1 + umy * n2) + std::sqrt(g * Hm),
                                    std::fabs((u[f] * n1 + u[(long long)K * ne + f] * n2) * w1) + std::sqrt(g * Hp));
            const double* o2 = O2 + q * K * K;
            const double* o3 = O3 + q * K * K * K;
            const double* m2 = N2 + (q * 3 + qs) * K * K;
            const double* m3 = N3 + (q * 3 + qs) * K * K * K;
            const double aa = a * a, aaa = aa * a, ab = a * bsc, abb = ab * bsc;
            for (int p = 0; p < K; ++p) {
                double jX = 0.0, jU = 0.0, jV = 0.0, kX = 0.0, kU = 0.0, kV = 0.0;
                double r2o = 0.0, r3o = 0.0, r2n = 0.0, r3n = 0.0;
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const double t2 = o2[p * K + i], s2 = m2[p * K + i];
                    jX += xi[i] * t2;
                    jU += U[i] * t2;
                    jV += V[i] * t2;
                    kX += xo[i] * s2;
                    kU += Uo[i] * s2;
                    kV += Vo[i] * s2;
                    double sw = 0.0, sx = 0.0, tw = 0.0, tx = 0.0;
#pragma unroll
                    for (int m = 0; m < K; ++m) {
                        const double t3 = o3[(p * K + i) * K + m], s3 = m3[(p * K + i) * K + m];
                        sw += t3 * wn[m];
                        sx += t3 * xi[m];
                        tw += s3 * wo[m];
                        tx += s3 * xo[m];
                    }
                    r2o += U[i] * sw + 0.5 * g * n1 * xi[i] * sx;
                    r3o += V[i] * sw + 0.5 * g * n2 * xi[i] * sx;
                    r2n += Uo[i] * tw + 0.5 * g * n1 * xo[i] * tx;
                    r3n += Vo[i] * tw + 0.5 * g * n2 * xo[i] * tx;
                }
                const double own1 = aa * (n1 * jU + n2 * jV);
                const double own2 = aaa * r2o + aa * g * hm * n1 * jX;
                const double own3 = aaa * r3o + aa * g * hm * n2 * jX;
                const double nb1 = ab * (n1 * kU + n2 * kV);
                const double nb2 = abb * r2n + ab * g * hp * n1 * kX;
                const double nb3 = abb * r3n + ab * g * hp * n2 * kX;
                const double s1v = L * (0.5 * (own1 + nb1) + 0.5 * lam * (aa * jX - ab * kX));
                const double s2v = L * (0.5 * (own2 + nb2) + 0.5 * lam * (aa * jU - ab * kU));
                const double s3v = L * (0.5 * (own3 + nb3) + 0.5 * lam * (aa * jV - ab * kV));
                out[(long long)p * ne + e] += s1v;
                out[(long long)(K + p) * ne + e] += s2v;
                out[(long long)(2 * K + p) * ne + e] += s3v;
            }
        }
    }
}

}  // namespace

extern "C" {

long long dg_reference_size(int k) {
    const long long K = k_of(k);
    return K ? 2 * K * K + 2 * K * K * K : 0;
}

int dg_reference_integrals(int k, double* ref) {
    const int K = k_of(k);
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
    if (!K || ne < 0 || ne > 256LL * 0x7fffffffLL) return MG_EINVAL;
    if (ne == 0) return MG_OK;
    if (!c || !B || !hb || !T || !u) return MG_EINVAL;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned nb = (unsigned)((ne + 255) / 256);
    switch (K) {
        case 1: k_dg_project<1><<<nb, 256, 0, st>>>(ne, c, B, hb, T, u); break;
        case 3: k_dg_project<3><<<nb, 256, 0, st>>>(ne, c, B, hb, T, u); break;
        case 6: k_dg_project<6><<<nb, 256, 0, st>>>(ne, c, B, hb, T, u); break;
        default: k_dg_project<10><<<nb, 256, 0, st>>>(ne, c, B, hb, T, u); break;
    }
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EDEVICE;
}

long long dg_edge_table_size(int k) {
    const long long K = k_of(k);
    return 12 * K * K + 12 * K * K * K;
}

int dg_edge_integrals(int k, double* table) {
    const int K = k_of(k);
    if (!K || !table) return MG_EINVAL;
    Poly1 own[3][kMaxK], back[3][kMaxK];
    for (int q = 0; q < 3; ++q)
        for (int p = 0; p < K; ++p) {
            own[q][p] = basis_on_edge(p, q, false);
            back[q][p] = basis_on_edge(p, q, true);
        }
    double* O2 = table;
    double* O3 = O2 + 3 * K * K;
    double* N2 = O3 + 3 * K * K * K;
    double* N3 = N2 + 9 * K * K;
    for (int q = 0; q < 3; ++q)
        for (int p = 0; p < K; ++p)
            for (int i = 0; i < K; ++i) {
                const Poly1 pi = mul1(own[q][p], own[q][i]);
                O2[(q * K + p) * K + i] = integrate1(pi, kScale[p] * kScale[i]);
                for (int m = 0; m < K; ++m)
                    O3[((q * K + p) * K + i) * K + m] =
                        integrate1(mul1(pi, own[q][m]), kScale[p] * kScale[i] * kScale[m]);
            }
    for (int q = 0; q < 3; ++q)
        for (int r = 0; r < 3; ++r)
            for (int p = 0; p < K; ++p)
                for (int i = 0; i < K; ++i) {
                    const Poly1 pi = mul1(own[q][p], back[r][i]);
                    N2[((q * 3 + r) * K + p) * K + i] = integrate1(pi, kScale[p] * kScale[i]);
                    for (int m = 0; m < K; ++m)
                        N3[(((q * 3 + r) * K + p) * K + i) * K + m] =
                            integrate1(mul1(pi, back[r][m]), kScale[p] * kScale[i] * kScale[m]);
                }
    return MG_OK;
}

int dg_edge_terms(int k, long long ne, const double* c, const double* u, const double* B, const double* hb,
                  const int* nbr, const int* nq, double g, const double* table, double* out, void* stream) {
    const int K = k_of(k);
    if (!K || ne < 0 || ne > 256LL * 0x7fffffffLL) return MG_EINVAL;
    if (ne == 0) return MG_OK;
    if (!c || !u || !B || !hb || !nbr || !nq || !table || !out) return MG_EINVAL;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned nb = (unsigned)((ne + 255) / 256);
    switch (K) {
        case 1: k_dg_edges<1><<<nb, 256, 0, st>>>(ne, c, u, B, hb, nbr, nq, g, table, out); break;
        case 3: k_dg_edges<3><<<nb, 256, 0, st>>>(ne, c, u, B, hb, nbr, nq, g, table, out); break;
        case 6: k_dg_edges<6><<<nb, 256, 0, st>>>(ne, c, u, B, hb, nbr, nq, g, table, out); break;
        default: k_dg_edges<10><<<nb, 256, 0, st>>>(ne, c, u, B, hb, nbr, nq, g, table, out); break;
    }
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EDEVICE;
}

int dg_volume_integrals(int k, long long ne, const double* c, const double* u, const double* B, const double* hb,
                        double g, const double* ref, double* out, void* stream) {
    const int K = k_of(k);
    if (!K || ne < 0 || ne > 256LL * 0x7fffffffLL) return MG_EINVAL;
    if (ne == 0) return MG_OK;
    if (!c || !u || !B || !hb || !ref || !out) return MG_EINVAL;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned nb = (unsigned)((ne + 255) / 256);
    switch (K) {
        case 1: k_dg_volume<1><<<nb, 256, 0, st>>>(ne, c, u, B, hb, g, ref, out); break;
        case 3: k_dg_volume<3><<<nb, 256, 0, st>>>(ne, c, u, B, hb, g, ref, out); break;
        case 6: k_dg_volume<6><<<nb, 256, 0, st>>>(ne, c, u, B, hb, g, ref, out); break;
        default: k_dg_volume<10><<<nb, 256, 0, st>>>(ne, c, u, B, hb, g, ref, out); break;
    }
    return hipGetLastError() == hipSuccess ? MG_OK : MG_EDEVICE;
}

}  // extern "C"
