/* The quadrature-free discontinuous Galerkin discretisation of the shallow
 * water equations on triangles (the paper's Sec. 2.2): volume terms,
 * velocity projection, Lax-Friedrichs edge terms, the source, the whole
 * right-hand side of the semi-discrete system and one SSP-RK3 time step.
 * The volume terms (equations mass_basis and momentum_basis_u) are, for
 * every element e and test function p,
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
 * elements of either orientation).  The bathymetry h_b is a field of order
 * max(k, 1), KB = 3, 3, 6, 10 coefficients per element for k = 0..3; the
 * paper's algebraic form, with h_b outside the integral, is the case of a
 * field with only the constant mode (coefficient h_b sqrt(|det B_e| / 2)),
 * and a linear h_b (the convergence test of Sec. 3.1) is exact at every
 * order.  (At k = 0 a piecewise-constant h_b would make the scheme
 * inconsistent where xi != 0: the pressure flux jumps with h_b across the
 * edges while g xi grad h_b vanishes inside the elements.)  The reference
 * and edge tables therefore cover the first KB basis functions.  The element
 * basis is orthonormal, so the mass matrix of the semi-discrete system is the
 * identity.
 *
 * Status codes are those of mg.h. */
#ifndef DG_H
#define DG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Host: the reason of this thread's last MG_EDEVICE from a dg_ entry point
 * (the step and the HIP error name; also the size limit behind an MG_EINVAL
 * of dg_ssp_rk3_step_noalloc), or "" (library-owned string, valid
 * until the thread's next dg_ call). */
const char* dg_last_error(void);

/* Host: the values of the K(k) reference basis polynomials at npts points
 * (x[q], y[q]) of the reference plane: out[p npts + q] = phi^_(p+1)(x_q, y_q)
 * (caller-owned arrays).  MG_EINVAL for a bad k, npts < 0 or a NULL array. */
int dg_basis_values(int k, long long npts, const double* x, const double* y, double* out);

/* Doubles in the reference table for order k: 2 KB^2 + 2 KB^3, or 0 for k
 * outside 0..3. */
long long dg_reference_size(int k);

/* Host: the exact reference integrals for order k into ref (caller-owned,
 * dg_reference_size(k) doubles): G[l][p][i] = int d_l phi^_p phi^_i, then
 * H[l][p][i][m] = int d_l phi^_p phi^_i phi^_m over the reference triangle,
 * l = 0, 1 (d/dx^1, d/dx^2), all indices below KB, row-major.  Computed
 * from the monomial integrals a! b! / (a + b + 2)!.  MG_EINVAL for a bad k
 * or NULL ref. */
int dg_reference_integrals(int k, double* ref);

/* Device: the volume terms of ne elements of order k, all arrays in device
 * memory, element index fastest (structure of arrays):
 *   c[(j K + i) ne + e]    coefficients of xi, U, V (j = 0, 1, 2)
 *   u[(j K + i) ne + e]    coefficients of u, v (j = 0, 1)
 *   B[q ne + e]            B_e entries B11, B12, B21, B22 (q = 0..3)
 *   hb[i ne + e]           coefficients of the bathymetry (i < KB)
 *   ref                    the table of dg_reference_integrals, on the device
 *   out[(j K + p) ne + e]  E[j][p][e]
 * Enqueued on `stream` (a hipStream_t, NULL = the default stream); returns
 * once launched.  MG_EINVAL for a bad k, ne < 0, ne above 2^32 - 256 (one
 * thread per element, at most 2^32 - 1 work-items per launch) or
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
 * matrix M[p][m] = |det B_e|^(-1/2) sum_i H_i T[p][i][m], a Cholesky
 * factorisation and two solves.  Arrays as for dg_volume_integrals: c
 * (3K x ne), B (4 x ne), hb (KB x ne; its modes from K on are orthogonal to
 * every product of two test functions and do not enter), T the table of
 * dg_product_integrals on the device, u (2K x ne) the result.  MG_EINVAL /
 * MG_EDEVICE as dg_volume_integrals; a depth that is not positive on the
 * element leaves non-finite values there. */
int dg_velocity_projection(int k, long long ne, const double* c, const double* B, const double* hb,
                           const double* T, double* u, void* stream);

/* Doubles in the edge table for order k: 3 KB NB with NB = max(k, 1) + 1
 * (2, 2, 3, 4), or 0 for a bad k. */
long long dg_edge_table_size(int k);

/* Host: the exact edge-trace table for order k: with the local edges of the
 * reference triangle q0 (0,0)->(1,0), q1 (1,0)->(0,1), q2 (0,1)->(0,0)
 * parametrised by s in [0, 1], every basis function restricted to an edge
 * is a polynomial of degree max(k, 1) in s, expanded here in the shifted
 * Legendre polynomials P_0 = 1, P_1 = 2s - 1, P_2, P_3 on [0, 1]:
 *   C[q][i][a] = (2a + 1) int_0^1 phi^_i(edge q at s) P_a(s) ds,
 * i < KB, a < NB, row-major.  A neighbour traverses the shared edge the
 * other way (s -> 1 - s), which negates its odd coefficients.  The edge
 * kernel multiplies traces with the exact integrals int P_a P_b P_c (built
 * into the kernel), so the products of three basis functions along an edge
 * never need a table of their own.  MG_EINVAL for a bad k or NULL table. */
int dg_edge_integrals(int k, double* table);

/* Device: the edge terms of every element,
 *   S[j][p][e] = sum over the local edges q of e that have an exterior
 *                state of int_E F_j phi_ep ds,
 * with the Lax-Friedrichs flux F = (A(c-, u-) n + A(c+, u+) n) / 2
 * + lambda_E (c- - c+) / 2 (the paper cites Lax-Friedrichs without fixing
 * the wave speed; here lambda_E = max over both sides of |u_mean . n| +
 * sqrt(g H_mean), element means, constant on the edge), n the unit outward
 * normal, the flux tensor and basis of dg_volume_integrals, evaluated
 * algebraically with the trace table of dg_edge_integrals (on the device).
 * nbr[q ne + e] names the exterior side of local edge q (int32, device):
 *   f in [0, ne)   the element across the edge, nq[q ne + e] its local
 *                  index of that edge (0..2);
 *   -2 - b         a prescribed (Dirichlet) state, b in [0, nb): the
 *                  polynomials cb[(j K + i) nb + b] (xi, U, V) and
 *                  ub[(j K + i) nb + b] (u, v) in the basis of element e,
 *                  whose traces on the edge are the exterior values; the
 *                  exterior bathymetry is e's own;
 *   anything else  no term (e.g. -1 on a boundary left open).
 * Other arrays as dg_volume_integrals; out (3K x ne).  nb = 0 allows NULL
 * cb and ub.  Elements must be counter-clockwise (det B_e > 0) and the mesh
 * conforming.  Status codes as dg_volume_integrals (MG_EINVAL also for
 * nb < 0, nb above 2^31 - 1, or nb > 0 with a NULL cb or ub). */
int dg_edge_terms(int k, long long ne, const double* c, const double* u, const double* B, const double* hb,
                  const int* nbr, const int* nq, long long nb, const double* cb, const double* ub, double g,
                  const double* table, double* out, void* stream);

/* Device: the right-hand side of the semi-discrete system (the paper's
 * variational_disc_1 with the source r(c) of eq:def_r and a body force;
 * with the orthonormal basis the mass matrix is the identity):
 *   out = dc/dt = E - S + R + F,
 * E as dg_volume_integrals, S as dg_edge_terms (same nbr, nq, nb, cb, ub),
 * R[j][p][e] = (r(c), phi_ep e_j) with r = (0, -tau U + fc V + g xi dh_b/dx1,
 * -tau V - fc U + g xi dh_b/dx2) (tau_bf and f_c constants), and F
 * (3K x ne, the coefficients of the body force's L2 projection; NULL for
 * none).  ref is the table of dg_reference_integrals (its three-function
 * part also gives the bathymetry source), table that of dg_edge_integrals,
 * both on the device.  out must not alias an input.  Status codes as
 * dg_edge_terms. */
int dg_rhs(int k, long long ne, const double* c, const double* u, const double* B, const double* hb,
           const int* nbr, const int* nq, long long nb, const double* cb, const double* ub, double g, double tau,
           double fc, const double* F, const double* ref, const double* table, double* out, void* stream);

/* Device: one step of length dt of the three-stage strong-stability-
 * preserving Runge-Kutta method of Shu and Osher (the paper names no
 * integrator):
 *   c1 = c + dt L(c),  c2 = 3/4 c + 1/4 (c1 + dt L(c1)),
 *   c3 = 1/3 c + 2/3 (c2 + dt L(c2)),
 * L the right-hand side of dg_rhs, the velocity u first projected from each
 * stage state (dg_velocity_projection).  Stage s = 0, 1, 2 is at time
 * t + (0, 1, 1/2)[s] dt; its body force is F3 + s 3K ne (F3 NULL: none) and
 * its prescribed states cb3 + s 3K nb and ub3 + s 2K nb.  c (3K x ne) is
 * advanced in place; u (2K x ne) is left holding the velocity of the last
 * stage's state; work is caller-owned device scratch of 6K ne doubles.
 * Needs the tables of dg_reference_integrals (ref), dg_product_integrals
 * (T) and dg_edge_integrals (table) on the device.  Enqueued on stream;
 * status codes as dg_rhs (MG_EINVAL also for a non-finite dt). */
int dg_ssp_rk3_step(int k, long long ne, double* c, double* u, double* work, const double* B, const double* hb,
                    const int* nbr, const int* nq, long long nb, const double* cb3, const double* ub3, double g,
                    double tau, double fc, const double* F3, const double* ref, const double* T,
                    const double* table, double dt, void* stream);

/* Device, for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): dg_ssp_rk3_step without
 * the work argument.  The saved state and the right-hand side live in a
 * fixed 64 MiB device array of the library (2^23 doubles, held on every
 * device the library runs on until the process ends), so 6 K ne must not
 * exceed 2^23 (e.g. ne <= 139810 at k = 3, 466033 at k = 1); larger meshes
 * get MG_EINVAL with the reason in dg_last_error.  The call allocates
 * nothing.  Every call on a device shares that device's array, so calls
 * that overlap on one device (two streams, two threads) race and must be
 * ordered by the caller.  Other arguments, results and status codes as
 * dg_ssp_rk3_step. */
int dg_ssp_rk3_step_noalloc(int k, long long ne, double* c, double* u, const double* B, const double* hb,
                            const int* nbr, const int* nq, long long nb, const double* cb3, const double* ub3,
                            double g, double tau, double fc, const double* F3, const double* ref, const double* T,
                            const double* table, double dt, void* stream);

#ifdef __cplusplus
}
#endif

#endif
