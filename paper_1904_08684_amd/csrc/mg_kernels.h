// Host-side launchers of the HIP kernels.  Each returns hipSuccess or the
// error of the launch.  `prec` is 0 for FP64 fields, 1 for FP32 fields.
#pragma once

#include <hip/hip_runtime.h>

#include "mg_internal.h"

namespace mg {

// Faces of a cell level: x-, y- and z-face coefficient arrays (null for node grids).
struct Faces {
    const void* b[3];
    // FP64 cell values k in colour-split layout (finest 3-D cell level, or
    // null): column-marching kernels form the faces from them
    const void* k = nullptr;
};

// One Gauss-Seidel half-sweep over colour `colour` (0 red, 1 black):
// u_i <- (f_i / s + sum of neighbours) / (2d) on a node grid,
// u_i <- (f_i / s + off_i) / diag_i on a cell grid.
// zero: every neighbour is known to be zero (first sweep from a zero guess).
hipError_t launch_gs(const Geom& g, int prec, int colour, bool zero, void* u, const void* f,
                     const Faces& fc, double s, hipStream_t st);
// 1 to 3 fused red-black sweeps (2 sweeps half-sweeps, colours first_colour,
// 1 - first_colour, ...) on a level where use_tb holds, from u (zero: from a
// zero iterate, u not read) into out; out's boundary and padding must be zero.
hipError_t launch_gs_tb(const Geom& g, int prec, int sweeps, int first_colour, bool zero, const void* u,
                        const void* f, void* out, double s, hipStream_t st);

// Damped Jacobi: out = u + (omega r) / (diag s), out of place.
hipError_t launch_jacobi(const Geom& g, int prec, bool zero, const void* u, const void* f, void* out,
                         const Faces& fc, double s, double omega, hipStream_t st);

// r = f - A u on the unknowns; with `norm`, per-block (sum r^2, max |r|)
// pairs are written to partials[2 * block] and *nblocks is set.
hipError_t launch_residual(const Geom& g, int prec, const void* u, const void* f, void* r,
                           const Faces& fc, double s, bool norm, bool store, double* partials,
                           long long* nblocks, hipStream_t st);

// Upper bound of the partials pairs launch_residual may produce on level g.
long long residual_blocks(const Geom& g);

// f_coarse = R r_fine (full weighting on node grids, 2^d mean on cell grids).
hipError_t launch_restrict(const Geom& gf, const Geom& gc, int prec, const void* r, void* fcoarse,
                           hipStream_t st);

// Residual and restriction in one pass (3-D node levels with fused_transfers):
// f_coarse = R (f - A u) without writing the fine residual.
bool fused_transfers(const Geom& gf);
hipError_t launch_residual_restrict(const Geom& gf, const Geom& gc, int prec, const void* u, const void* f,
                                    void* fcoarse, double s, hipStream_t st);

// u_fine += P e_coarse on the colours in `colour_mask` (bit 0 red, bit 1 black).
hipError_t launch_prolong(const Geom& gf, const Geom& gc, int prec, void* u, const void* ec,
                          int colour_mask, hipStream_t st);
// 2-D node levels running point kernels (fused_point_transfers): residual +
// full weighting into the coarse f in one launch, and interpolation +
// correction + the first damped-Jacobi sweep (u, coarse e -> out, out of
// place) in one launch; both bitwise equal to the separate operations.
bool fused_point_transfers(const Geom& gf);
hipError_t launch_residual_restrict_pt(const Geom& gf, const Geom& gc, int prec, const void* u, const void* f,
                                       void* fcoarse, double s, hipStream_t st);
hipError_t launch_prolong_jacobi(const Geom& gf, const Geom& gc, int prec, const void* u, const void* ec,
                                 const void* f, void* out, double s, double omega, hipStream_t st);
// Two damped-Jacobi sweeps of a 2-D point level in one launch (u -> out, out
// of place; zero: from a zero iterate; ec non-null: the iterate is first
// corrected by the interpolation of the coarse error ec of level gc; fco
// non-null: the residual after the sweeps is also restricted into level
// gc's right-hand side fco), bitwise equal to the separate operations.
hipError_t launch_jacobi2(const Geom& g, const Geom* gc, int prec, bool zero, const void* u, const void* ec,
                          const void* f, void* out, void* fco, double s, double omega, hipStream_t st);
// The finest 3-D cell level (FP64, faces from k): residual and the mean of
// the eight children into the coarse f in one pass, bitwise equal to the
// residual then the restriction.
// Cell levels with stored face coefficients (fc.b): residual and the 2^d
// mean into the coarse f in one launch over the coarse cells, bitwise equal
// to the two operations.
hipError_t launch_cell_res_restrict_pt(const Geom& gf, const Geom& gc, int prec, const void* u, const void* f,
                                       const Faces& fc, void* fco, double s, hipStream_t st);
bool cell_res_restrict_fused(const Geom& gf);
hipError_t launch_cell_res_restrict(const Geom& gf, const Geom& gc, const void* u, const void* f, const void* k,
                                    void* fco, double s, hipStream_t st);

// Coarsest solve u = A^-1 f with the FP64 lower Cholesky factor L (m x m, row major).
hipError_t launch_coarse(const Geom& g, int prec, const void* f, void* u, const double* L, int m,
                         hipStream_t st);

// One V-cycle from the top level of P (right-hand side f, iterate u in
// device memory; u read unless P.from_zero) down to the coarsest and back,
// in one workgroup with every level's fields in LDS; u receives the result.
hipError_t launch_tail(const TailPlan& P, int prec, const void* f, void* u, hipStream_t st);

// Deterministic reduction of `count` (sum, max) pairs to out[0..1];
// scratch holds at least 2 * ceil(count / 4096) doubles.
// Constant 3^d-point node stencil (a Galerkin coarse operator R A P):
// weights by offset, z offset slowest and x fastest (2-D: the first 9).
struct Stencil27 {
    double w[27];
};

// FP64 node grids with a 3^d-point stencil W: damped Jacobi out of place
// (out = u + (omega r) / W_centre; zero: u is zero) and r = f - A u (with
// `norm`, per-block (sum r^2, max |r|) pairs as launch_residual).
hipError_t launch_jacobi27(const Geom& g, bool zero, const void* u, const void* f, void* out, const Stencil27& W,
                           double omega, hipStream_t st);
hipError_t launch_residual27(const Geom& g, const void* u, const void* f, void* r, const Stencil27& W, bool norm,
                             bool store, double* partials, long long* nblocks, hipStream_t st);

// Cell grids: a -= (sum of a over all cells) / (number of cells), the sum
// through per-block partials and launch_reduce into out[0].
hipError_t launch_project(const Geom& g, double* a, double* partials, double* scratch, double* out,
                          hipStream_t st);

// Fixed-order reduction of (sum, max) partial pairs into out[0..1]; with
// mx_copy the maximum is also stored there.
hipError_t launch_reduce(const double* partials, long long count, double* scratch, double* out,
                         hipStream_t st, double* mx_copy = nullptr, const double* move_src = nullptr,
                         double* move_dst = nullptr);
long long reduce_scratch_pairs(long long count);

// natural FP64 array <-> colour-split level field (node grids: interior only).
hipError_t launch_pack(const Geom& g, int prec, const double* nat, void* split, hipStream_t st);
hipError_t launch_unpack(const Geom& g, int prec, const void* split, double* nat, hipStream_t st);

// Mixed precision: sigma = 2^floor(log2 *basis) (basis: the largest |r| of
// the refinement's previous residual), stored to *sigma; f32 = fl32(r64 /
// sigma).  And u64 += sigma * c32.
hipError_t launch_cast(const Geom& g, const double* r64, float* f32, const double* basis, double* sigma,
                       hipStream_t st);
// r = f - A u on a 3-D node level where use_zmarch holds (FP64), written as
// f32 = fl32(r / sigma) with sigma = 2^floor(log2 *basis) stored to *sigma,
// and per-block (sum r^2, max |r|) partials: the residual and the cast of a
// refinement step in one pass.  *nblocks is set as by launch_residual.
hipError_t launch_residual_cast(const Geom& g, const void* u, const void* f, float* f32, double s,
                                const double* basis, double* sigma, double* partials, long long* nblocks,
                                hipStream_t st);
hipError_t launch_update(const Geom& g, double* u64, const float* c32, const double* sigma,
                         hipStream_t st);
// u' = u + red[2] fl64(c32) written to uo, and the residual of u' cast to f32
// with 2^floor(log2 red[3]) (stored to red[5]) plus norm partials, in one
// pass (3-D node levels that march columns).
hipError_t launch_update_residual_cast(const Geom& g, const double* u, const float* c32, const double* f, double* uo,
                                       float* f32, double s, double* red, double* partials, long long* nblocks,
                                       hipStream_t st);
// Groups of four elements in one level field (both colours, padding included).
long long field_quads(const Geom& g);

// Zero `bytes` bytes (a kernel, not a memset, so the call is graph-capturable).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);

// Preconditioned-CG vector operations over whole FP64 level fields (bytes a
// multiple of 16).  launch_dot writes dot_blocks(bytes) partial pairs (sum, 0)
// for launch_reduce; sc points to device scalars: sc[0] = rho, sc[2] = p . q,
// sc[4] = rho_new.
long long dot_blocks(size_t bytes);
hipError_t launch_dot(const double* a, const double* b, size_t bytes, double* partials, hipStream_t st);
hipError_t launch_pcg_step(double* x, const double* p, double* r, const double* q, const double* sc, size_t bytes,
                           hipStream_t st);
hipError_t launch_pcg_dir(double* p, const double* z, const double* sc, size_t bytes, hipStream_t st);
hipError_t launch_scalar_copy(double* dst, const double* src, hipStream_t st);

// Iteration space of the point-per-thread kernels over one or both colours.
Space level_space(const Geom& g, int ncol, int col0);

// ------------------------------------------------------------ batched ops
// One level operation of one request, resident in device memory, executed
// tile by tile by the batched kernel with the same device code as the
// stand-alone launches.  Serving runs node grids with FP64 outer and FP32
// inner arithmetic, so each op has a fixed precision.
enum BOp : int {
    BOP_PACK = 0,      // f64 (split) <- natural FP64 array at *io[0]
    BOP_ZERO,          // n 16-byte words at a
    BOP_RES64,         // r64 = f64 - A u64, per-tile (sum r^2, max |r|) to part
    BOP_REDUCE,        // part[0..n) -> red[0..1] and res[0..1]
    BOP_CAST,          // f32 = fl32(r64 / sigma), sigma = 2^floor(log2 red[3]) -> red[2]
    BOP_GS,            // FP32 GS half-sweep (colour-offset pointers)
    BOP_GS_ZERO,       // FP32 GS half-sweep from a zero iterate
    BOP_JAC,           // FP32 damped Jacobi, out of place
    BOP_JAC_ZERO,      // FP32 damped Jacobi from a zero iterate
    BOP_RES32,         // FP32 residual
    BOP_RESTRICT,      // FP32 full weighting
    BOP_PROLONG,       // FP32 interpolation + correction
    BOP_COARSE,        // FP32 in, FP64 Cholesky solve, FP32 out
    BOP_UPDATE,        // u64 += sigma * u32
    BOP_UNPACK,        // natural FP64 array at *io[1] <- u64 (split)
    BOP_GS_M,          // FP32 GS half-sweep, 3-D column marching (zs)
    BOP_JAC_M,         // FP32 damped Jacobi, 2-D row marching (ys)
    BOP_JAC_ZERO_M,    // the same from a zero iterate
    BOP_RES32_M,       // FP32 residual, marching (3-D: zs, 2-D: ys)
    BOP_RES64_M,       // FP64 residual with per-tile partials, marching
    BOP_COUNT
};

struct BItem {
    int op, dim;
    Geom g, gc;
    Space sp;
    ZSpace zs;             // tiling of the marching forms
    YSpace ys;
    long long tiles;       // blocks of 256 threads the op needs
    int w;                 // work units per tile (a unit ~ 256 points) for batched scheduling
    long long n;           // elements (pack/unpack), 16-byte words (zero), pairs (reduce)
    void* a;
    void* b;
    void* c;
    const double* L;
    int m;
    double* part;
    double* red;
    double* res;
    void* const* io;
    double s, omega;
};

// A batched launch: entries sorted by `prefix`, the first global work unit of
// each; an entry spans tiles x w units.
struct BEntry {
    const BItem* item;
    long long prefix;
};

// Persistent batched kernel over n entries with `total` work units in all.
hipError_t launch_batch(const BEntry* d_entries, int n, long long total, hipStream_t st);

}  // namespace mg
