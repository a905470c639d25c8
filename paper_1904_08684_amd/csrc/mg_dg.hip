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
