/* Volume terms of the quadrature-free discontinuous Galerkin discretisation
 * of the shallow water equations on triangles (the paper's Sec. 2.2,
 * equations mass_basis and momentum_basis_u): for every
 * element e and test function p,
 *
 *   E[j][p][e] = (A~(c, u), grad(phi_ep e_j))_{Omega_e},  j = 0, 1, 2,
 *
 * with the flux tensor rows (U, V), (U u + g xi (H + h_b) / 2, U v),
 * (V u, V v + g xi (H + h_b) / 2), H = xi + h_b, evaluated algebraically:
 * products of element coefficients with integrals of products of the
 * reference basis and its gradients, scaled by the element's affine map.
 *
 * Reference triangle (0,0), (1,0), (0,1); F_e(x^) = B_e x^ + a_e1 with
 * B_e = [a_e2 - a_e1, a_e3 - a_e1]; the element basis is
 * phi_ep = |det B_e|^(-1/2) phi^_p o F_e^-1 with the paper's ten orthonormal
 * polynomials phi^_1 .. phi^_10 (K(k) = 1, 3, 6, 10 of them for order
 * k = 0..3), so that the paper's factors 1/|det B_e| and 1/|det B_e|^(3/2)
 * appear (written with det B_e itself, which keeps the sign right for
 * elements of either orientation).  h_b is constant on each element.
 *
 * Status codes are those of mg.h. */
#ifndef DG_H
#define DG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Doubles in the reference table of order k: 2 K^2 + 2 K^3, or 0 for k
 * outside 0..3. */
long long dg_reference_size(int k);

/* Host: the exact reference integrals of order k into ref (caller-owned,
 * dg_reference_size(k) doubles): G[l][p][i] = int d_l phi^_p phi^_i, then
 * H[l][p][i][m] = int d_l phi^_p phi^_i phi^_m over the reference triangle,
 * l = 0, 1 (d/dx^1, d/dx^2), row-major.  Computed from the monomial
 * integrals a! b! / (a + b + 2)!.  MG_EINVAL for a bad k or NULL ref. */
int dg_reference_integrals(int k, double* ref);

/* Device: the volume terms of ne elements of order k, all arrays in device
 * memory, element index fastest (structure of arrays):
 *   c[(j K + i) ne + e]    coefficients of xi, U, V (j = 0, 1, 2)
 *   u[(j K + i) ne + e]    coefficients of u, v (j = 0, 1)
 *   B[q ne + e]            B_e entries B11, B12, B21, B22 (q = 0..3)
 *   hb[e]                  bathymetry on the element
 *   ref                    the table of dg_reference_integrals, on the device
 *   out[(j K + p) ne + e]  E[j][p][e]
 * Enqueued on `stream` (a hipStream_t, NULL = the default stream); returns
 * once launched.  MG_EINVAL for a bad k, ne < 0, ne above 256 (2^31 - 1) or
 * a NULL array (ne = 0 is a no-op), MG_EDEVICE for a launch failure.
 * Elements with det B_e = 0 give non-finite values. */
int dg_volume_integrals(int k, long long ne, const double* c, const double* u, const double* B,
                        const double* hb, double g, const double* ref, double* out, void* stream);

/* Doubles in the product table of order k: K^3, or 0 for k outside 0..3. */
long long dg_product_size(int k);

/* Host: T[p][i][m] = int phi^_p phi^_i phi^_m over the reference triangle,
 * row-major, exact like dg_reference_integrals.  MG_EINVAL for a bad k or
 * NULL T. */
int dg_product_integrals(int k, double* T);

/* Device: the velocity of every element from the paper's second discrete
 * equation (variational_disc_2), (u H, psi) = (q, psi) for all psi in P^k
 * of the element, H = xi + h_b, q = (U, V): per element the H-weighted mass
 * matrix M[p][m] = |det B_e|^(-1/2) sum_i H_i T[p][i][m] (the constant h_b
 * enters the coefficient of phi_e1), a Cholesky factorisation and two
 * solves.  Arrays as for dg_volume_integrals: c (3K x ne), B (4 x ne),
 * hb (ne), T the table of dg_product_integrals on the device, u (2K x ne)
 * the result.  MG_EINVAL / MG_EDEVICE as dg_volume_integrals; a depth that
 * is not positive on the element leaves non-finite values there. */
int dg_velocity_projection(int k, long long ne, const double* c, const double* B, const double* hb,
                           const double* T, double* u, void* stream);

/* Doubles in the edge table of order k: 12 K^2 + 12 K^3, or 0 for a bad k. */
long long dg_edge_table_size(int k);

/* Host: the exact edge integrals of order k, with the local edges of the
 * reference triangle q0 (0,0)->(1,0), q1 (1,0)->(0,1), q2 (0,1)->(0,0)
 * parametrised by s in [0, 1], and a neighbour's edge q' traversed backwards
 * (its parameter 1 - s), row-major in this order:
 *   O2[q][p][i]      = int phi^_p phi^_i            along q
 *   O3[q][p][i][m]   = int phi^_p phi^_i phi^_m     along q
 *   N2[q][q'][p][i]  = int phi^_p(q, s) phi^_i(q', 1 - s)
 *   N3[q][q'][p][i][m] = int phi^_p(q, s) phi^_i(q', 1 - s) phi^_m(q', 1 - s)
 * MG_EINVAL for a bad k or NULL table. */
int dg_edge_integrals(int k, double* table);

/* Device: the interior-edge terms of every element,
 *   S[j][p][e] = sum over the local edges q of e that have a neighbour of
 *                int_E F_j phi_ep ds,
 * with the Lax-Friedrichs flux F = (A(c-, u-) n + A(c+, u+) n) / 2
 * + lambda_E (c- - c+) / 2 (the paper cites Lax-Friedrichs without fixing
 * the wave speed; here lambda_E = max over both sides of |u_mean . n| +
 * sqrt(g H_mean), element means, constant on the edge), n the unit outward
 * normal, the flux tensor and basis of dg_volume_integrals, evaluated
 * algebraically with the table of dg_edge_integrals (on the device).
 * nbr[q ne + e] is the element across local edge q (-1: domain boundary,
 * skipped), nq[q ne + e] its local index of that edge; both int32 device
 * arrays (an index outside [0, ne) or 0..2 is taken as boundary).  Other arrays as dg_volume_integrals; out (3K x ne).  Elements must
 * be counter-clockwise (det B_e > 0) and the mesh conforming.  Status codes
 * as dg_volume_integrals. */
int dg_edge_terms(int k, long long ne, const double* c, const double* u, const double* B, const double* hb,
                  const int* nbr, const int* nq, double g, const double* table, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif
