// HIP kernels of the V-cycle for gfx950 (MI355X).
//
// Every level operation is a streaming stencil sweep over colour-split
// storage (see mg_internal.h).  The operations are HBM-bandwidth bound
// (~0.4 flop/byte against a machine balance near 10), so the kernels are
// written for coalesced 64-lane row accesses, neighbour reuse in L1/L2,
// and XCD-aware block ordering; none of them is a dense contraction, so
// none uses MFMA.
//
// Floating-point evaluation order follows the textbook formulas term by
// term (neighbours x-, x+, y-, y+, z-, z+; transfer terms in tensor-product
// order) and the library is compiled with -ffp-contract=off, so each
// operation rounds exactly as the written formula does.

#include <cmath>
#include <type_traits>
#include <utility>

#include <hip/hip_runtime.h>

#include "mg_kernels.h"

namespace mg {
namespace {

constexpr int kReduceChunk = 4096;

// Workgroups are dispatched round-robin over the 8 XCDs (block b to XCD
// b % 8).  Renumber so that each XCD walks a contiguous run of logical
// tiles: consecutive rows and planes then meet in the same XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int x = b & 7, k = b >> 3;
    return (x < rem) ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

struct Pt {
    int xs, y, z, c;
};

// Logical block id, thread id and thread count of the block running an
// operation: a plain launch (block ids XCD-renumbered) or one tile of a
// batched launch.
struct Ex {
    int b, t, nt;
};

__device__ __forceinline__ Ex solo_ex() {
    Ex e;
    e.b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    e.t = (int)(threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z));
    e.nt = (int)(blockDim.x * blockDim.y * blockDim.z);
    return e;
}

__device__ __forceinline__ bool map_point(const Ex& ex, const Space& sp, Pt& p) {
    if (ex.t >= (1 << (sp.lx + sp.ly + sp.lz))) return false;
    int b = ex.b;
    int t = ex.t;
    const int lx = t & ((1 << sp.lx) - 1);
    t >>= sp.lx;
    const int ly = t & ((1 << sp.ly) - 1);
    t >>= sp.ly;
    const int lz = t;
    const int tx = b % sp.ntx;
    b /= sp.ntx;
    const int tc = b % sp.ncol;
    b /= sp.ncol;
    const int ty = b % sp.nty;
    const int tz = b / sp.nty;
    p.xs = (tx << sp.lx) + lx;
    p.y = sp.y0 + (ty << sp.ly) + ly;
    p.z = sp.z0 + (tz << sp.lz) + lz;
    p.c = sp.col0 + tc;
    return p.xs < sp.xr && p.y < sp.y0 + sp.yr && p.z < sp.z0 + sp.zr;
}

__device__ __forceinline__ long long row_off(const Geom& g, int y, int z) {
    return (long long)z * g.plane + (long long)y * g.pitch;
}

// Fixed-order block reduction of (sum, max) over all threads of the block
// (a power of two, at most 1024): a shuffle tree inside each wavefront, then
// thread 0 adds the wavefront results in order.  Deterministic.
__device__ void block_sum_max(double sq, double mx, double* out2, double* mx_copy = nullptr) {
    __shared__ double s_sq[16];
    __shared__ double s_mx[16];
    const int nt = (int)(blockDim.x * blockDim.y * blockDim.z);
    const int t = (int)(threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z));
    const int w = nt < 64 ? nt : 64;
    for (int o = w >> 1; o > 0; o >>= 1) {
        sq = sq + __shfl_down(sq, o, w);
        mx = fmax(mx, __shfl_down(mx, o, w));
    }
    if ((t & 63) == 0) {
        s_sq[t >> 6] = sq;
        s_mx[t >> 6] = mx;
    }
    __syncthreads();
    if (t == 0) {
        double a = s_sq[0], b = s_mx[0];
        for (int i = 1; i < (nt + 63) / 64; ++i) {
            a = a + s_sq[i];
            b = fmax(b, s_mx[i]);
        }
        out2[0] = a;
        out2[1] = b;
        if (mx_copy) *mx_copy = b;
    }
}

// ------------------------------------------------------------ node grids
// Sum of the 2d neighbours of the point at row offset ro (+ xs) in the
// other colour plane o; par = x & 1.
template <typename T, int D>
__device__ __forceinline__ T node_nb(const T* __restrict__ o, long long ro, int par, const Geom& g) {
    T nb = o[ro - 1 + par];
    nb = nb + o[ro + par];
    nb = nb + o[ro - g.pitch];
    nb = nb + o[ro + g.pitch];
    if (D == 3) {
        nb = nb + o[ro - g.plane];
        nb = nb + o[ro + g.plane];
    }
    return nb;
}

// a / 6 correctly rounded with one multiply and two FMAs (Markstein's
// correction step): q0 = a y with y = RN(1/6) is faithful, r = a - 6 q0 is
// exact, and RN(q0 + r y) is then the correctly rounded quotient.  Equal to
// a / 6 for every finite a away from the subnormal range (checked over 4e8
// random doubles and every float mantissa of one binade), except that -0
// gives +0.
__device__ __forceinline__ double div6(double a) {
    constexpr double y = 1.0 / 6.0;
    const double q0 = a * y;
    return __builtin_fma(__builtin_fma(-q0, 6.0, a), y, q0);
}
__device__ __forceinline__ float div6(float a) {
    constexpr float y = 1.0f / 6.0f;
    const float q0 = a * y;
    return __builtin_fmaf(__builtin_fmaf(-q0, 6.0f, a), y, q0);
}

// (f / s + nb) / (2 D), the Gauss-Seidel update.  P2: s is a power of two
// and rs = 1 / s, so f / s = f rs exactly and the division by 2D is a
// multiplication by 1/4 (2-D) or Markstein's division by 6 (3-D): the same
// rounding without the division sequences (away from the subnormal range).
template <typename T, int D, bool P2>
__device__ __forceinline__ T gs_value(T fv, T nb, T s, T rs) {
    if constexpr (P2 && D == 2) return (fv * rs + nb) * T(0.25);
    else if constexpr (P2 && D == 3) return div6(fv * rs + nb);
    else return (fv / s + nb) / T(2 * D);
}

template <typename T, int D, bool ZERO, bool P2 = false>
__device__ __forceinline__ void pt_node_gs(const Pt& p, Geom g, Space sp, T* __restrict__ me,
                                                 const T* __restrict__ other, const T* __restrict__ f,
                                                 T s, T rs = T(0)) {
    const int par = (p.y + p.z + p.c) & 1;
    const int x = 2 * p.xs + par;
    if (x < 1 || x > g.n - 2) return;
    const long long ro = row_off(g, p.y, p.z) + p.xs;
    const T nb = ZERO ? T(0) : node_nb<T, D>(other, ro, par, g);
    me[ro] = gs_value<T, D, P2>(f[ro], nb, s, rs);
}

template <typename T, int D, bool ZERO, bool P2 = false>
__device__ __forceinline__ void d_node_gs(const Ex& ex, Geom g, Space sp, T* __restrict__ me,
                                                 const T* __restrict__ other, const T* __restrict__ f,
                                                 T s, T rs = T(0)) {
    Pt p;
    if (!map_point(ex, sp, p)) return;
    pt_node_gs<T, D, ZERO, P2>(p, g, sp, me, other, f, s, rs);
}

template <typename T, int D, bool ZERO, bool P2>
__global__ __launch_bounds__(256) void k_node_gs(Geom g, Space sp, T* __restrict__ me,
                                                 const T* __restrict__ other, const T* __restrict__ f,
                                                 T s, T rs) {
    d_node_gs<T, D, ZERO, P2>(solo_ex(), g, sp, me, other, f, s, rs);
}

// (omega r) / (2 D s).  P2: s is a power of two and rs = 1 / s (exact), so
// the quotient is the product with the exact reciprocal 2^-2 rs (D = 2) or
// the correctly rounded division by 6 of (omega r) rs (D = 3): the same
// rounding as the division, without its instruction sequence (away from
// the subnormal range).
template <typename T, int D, bool P2>
__device__ __forceinline__ T jacobi_step(T w, T s, T rs) {
    if constexpr (P2 && D == 2) return w * (rs * T(0.25));
    else if constexpr (P2 && D == 3) return div6(w * rs);
    else return w / (T(2 * D) * s);
}

template <typename T, int D, bool ZERO, bool P2 = false>
__device__ __forceinline__ void pt_node_jacobi(const Pt& p, Geom g, Space sp, const T* __restrict__ u,
                                                     const T* __restrict__ f, T* __restrict__ out,
                                                     T s, T omega, T rs = T(0)) {
    const int par = (p.y + p.z + p.c) & 1;
    const int x = 2 * p.xs + par;
    if (x < 1 || x > g.n - 2) return;
    const long long ro = row_off(g, p.y, p.z) + p.xs;
    const long long me = (long long)p.c * g.cs + ro;
    const T uc = ZERO ? T(0) : u[me];
    const T nb = ZERO ? T(0) : node_nb<T, D>(u + (long long)(1 - p.c) * g.cs, ro, par, g);
    const T r = f[me] - (T(2 * D) * uc - nb) * s;
    out[me] = uc + jacobi_step<T, D, P2>(omega * r, s, rs);
}

template <typename T, int D, bool ZERO, bool P2>
__device__ __forceinline__ void d_node_jacobi(const Ex& ex, Geom g, Space sp, const T* __restrict__ u,
                                                     const T* __restrict__ f, T* __restrict__ out,
                                                     T s, T omega, T rs) {
    Pt p;
    if (!map_point(ex, sp, p)) return;
    pt_node_jacobi<T, D, ZERO, P2>(p, g, sp, u, f, out, s, omega, rs);
}

template <typename T, int D, bool ZERO, bool P2>
__global__ __launch_bounds__(256) void k_node_jacobi(Geom g, Space sp, const T* __restrict__ u,
                                                     const T* __restrict__ f, T* __restrict__ out,
                                                     T s, T omega, T rs) {
    d_node_jacobi<T, D, ZERO, P2>(solo_ex(), g, sp, u, f, out, s, omega, rs);
}

// Residual at point p (false outside the unknowns): its index and value.
template <typename T, int D>
__device__ __forceinline__ bool pt_node_residual(const Pt& p, const Geom& g, const T* __restrict__ u,
                                                 const T* __restrict__ f, T s, long long& me, T& rv) {
    const int par = (p.y + p.z + p.c) & 1;
    const int x = 2 * p.xs + par;
    if (x < 1 || x > g.n - 2) return false;
    const long long ro = row_off(g, p.y, p.z) + p.xs;
    me = (long long)p.c * g.cs + ro;
    const T nb = node_nb<T, D>(u + (long long)(1 - p.c) * g.cs, ro, par, g);
    rv = f[me] - (T(2 * D) * u[me] - nb) * s;
    return true;
}

template <typename T, int D, bool NORM, bool STORE>
__device__ __forceinline__ void d_node_residual(const Ex& ex, Geom g, Space sp, const T* __restrict__ u,
                                                       const T* __restrict__ f, T* __restrict__ r,
                                                       T s, double* __restrict__ part) {
    double sq = 0.0, mx = 0.0;
    Pt p;
    long long me;
    T rv;
    if (map_point(ex, sp, p) && pt_node_residual<T, D>(p, g, u, f, s, me, rv)) {
        if (STORE) r[me] = rv;
        const double dv = (double)rv;
        sq = dv * dv;
        mx = fabs(dv);
    }
    if (NORM) block_sum_max(sq, mx, part + 2 * (long long)ex.b);
}

template <typename T, int D, bool NORM, bool STORE>
__global__ __launch_bounds__(256) void k_node_residual(Geom g, Space sp, const T* __restrict__ u,
                                                       const T* __restrict__ f, T* __restrict__ r,
                                                       T s, double* __restrict__ part) {
    d_node_residual<T, D, NORM, STORE>(solo_ex(), g, sp, u, f, r, s, part);
}

// ---------------------------------------------- 3-D node grids, column marching
__device__ __forceinline__ void zm_tile(const ZSpace& zs, int b, int& tx, int& ty, int& tz) {
    tx = b % zs.ntx;
    b /= zs.ntx;
    ty = b % zs.nty;
    tz = b / zs.nty;
}

template <bool NT, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Half-sweep of one colour; the thread's column of the other colour at
// z-1, z, z+1 stays in registers while it walks its planes, U planes at a
// time so that U planes of loads are in flight per thread.  f and the
// updated colour are pure streams (NT: non-temporal).
template <typename T, int U, bool NT, bool P2 = false>
__device__ __forceinline__ void d_node_gs_zm(const Ex& ex, Geom g, ZSpace zs, T* __restrict__ me,
                                                     const T* __restrict__ other,
                                                     const T* __restrict__ f, T s, int colour, T rs = T(0)) {
    int tx, ty, tz;
    zm_tile(zs, ex.b, tx, ty, tz);
    const int xs = tx * 64 + (ex.t & 63);
    const int y = 1 + ty * zs.rows + (ex.t >> 6);
    if (xs >= zs.xr || y > g.n - 2) return;
    const int z0 = 1 + tz * zs.zc;
    const int z1 = min(z0 + zs.zc, g.n - 1);
    const long long pl = g.plane;
    long long ro = row_off(g, y, z0) + xs;
    const long long xl = xs > 0 ? -1 : 0;     // offset of x >> 1 - 1, clamped at the row start
    T zv[U + 2];
    zv[U] = other[ro - pl];
    zv[U + 1] = other[ro];
    int z = z0;
    for (; z + U <= z1; z += U, ro += U * pl) {
        zv[0] = zv[U];
        zv[1] = zv[U + 1];
        T xo[U], ym[U], yp[U], fv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const long long rk = ro + k * pl;
            const int par = (y + z + k + colour) & 1;
            zv[k + 2] = other[rk + pl];
            xo[k] = other[rk + (par ? 1 : xl)];
            ym[k] = other[rk - g.pitch];
            yp[k] = other[rk + g.pitch];
            fv[k] = ld_stream<NT>(f + rk);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int par = (y + z + k + colour) & 1;
            if (par | xs) {   // x = 2 xs + par >= 1
                T nb = par ? zv[k + 1] : xo[k];
                nb = nb + (par ? xo[k] : zv[k + 1]);
                nb = nb + ym[k];
                nb = nb + yp[k];
                nb = nb + zv[k];
                nb = nb + zv[k + 2];
                st_stream<NT>(me + ro + k * pl, gs_value<T, 3, P2>(fv[k], nb, s, rs));
            }
        }
    }
    T om = zv[U], oc = zv[U + 1];
    for (; z < z1; ++z, ro += pl) {
        const T op = other[ro + pl];
        const int par = (y + z + colour) & 1;
        const T xo = other[ro + (par ? 1 : xl)];
        const T ym = other[ro - g.pitch];
        const T yp = other[ro + g.pitch];
        if (par | xs) {
            T nb = par ? oc : xo;
            nb = nb + (par ? xo : oc);
            nb = nb + ym;
            nb = nb + yp;
            nb = nb + om;
            nb = nb + op;
            st_stream<NT>(me + ro, gs_value<T, 3, P2>(ld_stream<NT>(f + ro), nb, s, rs));
        }
        om = oc;
        oc = op;
    }
}

template <typename T, int U, bool NT, bool P2>
__global__ __launch_bounds__(1024) void k_node_gs_zm(Geom g, ZSpace zs, T* __restrict__ me,
                                                     const T* __restrict__ other,
                                                     const T* __restrict__ f, T s, int colour, T rs) {
    d_node_gs_zm<T, U, NT, P2>(solo_ex(), g, zs, me, other, f, s, colour, rs);
}

// r = f - A u at both colours of the thread's column; both colours' z-1, z,
// z+1 values stay in registers, U planes per step.
// CAST (FP64): the residual is stored as r32 = fl32(r / sigma) instead of r.
// JAC (1, or 2 with s a power of two and rs = 1 / s): a damped-Jacobi sweep,
// r receiving u + (omega res) / (6 s) as pt_node_jacobi forms it.
template <typename T, int U, bool NT, bool NORM, bool STORE, bool CAST = false, int JAC = 0>
__device__ __forceinline__ void d_node_res_zm(const Ex& ex, Geom g, ZSpace zs, const T* __restrict__ u,
                                                      const T* __restrict__ f, T* __restrict__ r, T s,
                                                      double* __restrict__ part, float* __restrict__ r32 = nullptr,
                                                      double sigma = 1.0, T omega = T(0), T rs = T(0)) {
    double sq = 0.0, mx = 0.0;
    int tx, ty, tz;
    zm_tile(zs, ex.b, tx, ty, tz);
    const int xs = tx * 64 + (ex.t & 63);
    const int y = 1 + ty * zs.rows + (ex.t >> 6);
    if (xs < zs.xr && y <= g.n - 2) {
        const T* __restrict__ R = u;           // red plane
        const T* __restrict__ B = u + g.cs;    // black plane
        const long long pl = g.plane, cs = g.cs;
        const int z0 = 1 + tz * zs.zc;
        const int z1 = min(z0 + zs.zc, g.n - 1);
        const long long xl = xs > 0 ? -1 : 0;
        long long ro = row_off(g, y, z0) + xs;
        T rv[U + 2], bv[U + 2];
        rv[U] = R[ro - pl];
        rv[U + 1] = R[ro];
        bv[U] = B[ro - pl];
        bv[U + 1] = B[ro];
        auto point = [&](T xm, T xp, T ym, T yp, T zm, T zp, T uc, T fv, long long at) {
            T nb = xm;
            nb = nb + xp;
            nb = nb + ym;
            nb = nb + yp;
            nb = nb + zm;
            nb = nb + zp;
            const T v = fv - (T(6) * uc - nb) * s;
            if constexpr (JAC > 0) st_stream<NT>(r + at, uc + jacobi_step<T, 3, JAC == 2>(omega * v, s, rs));
            else if constexpr (CAST) st_stream<NT>(r32 + at, (float)((double)v / sigma));
            else if (STORE) st_stream<NT>(r + at, v);
            const double dv = (double)v;
            sq = sq + dv * dv;
            mx = fmax(mx, fabs(dv));
        };
        int z = z0;
        for (; z + U <= z1; z += U, ro += U * pl) {
            rv[0] = rv[U];
            rv[1] = rv[U + 1];
            bv[0] = bv[U];
            bv[1] = bv[U + 1];
            T bx[U], rx[U], bym[U], byp[U], rym[U], ryp[U], fr[U], fb[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const long long rk = ro + k * pl;
                const int pr = (y + z + k) & 1;   // x parity of the red point; the black one has 1 - pr
                rv[k + 2] = R[rk + pl];
                bv[k + 2] = B[rk + pl];
                bx[k] = B[rk + (pr ? 1 : xl)];
                rx[k] = R[rk + (pr ? xl : 1)];
                bym[k] = B[rk - g.pitch];
                byp[k] = B[rk + g.pitch];
                rym[k] = R[rk - g.pitch];
                ryp[k] = R[rk + g.pitch];
                fr[k] = ld_stream<NT>(f + rk);
                fb[k] = ld_stream<NT>(f + cs + rk);
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const long long rk = ro + k * pl;
                const int pr = (y + z + k) & 1;
                if (pr | xs)
                    point(pr ? bv[k + 1] : bx[k], pr ? bx[k] : bv[k + 1], bym[k], byp[k], bv[k], bv[k + 2],
                          rv[k + 1], fr[k], rk);
                if ((1 - pr) | xs)
                    point(pr ? rx[k] : rv[k + 1], pr ? rv[k + 1] : rx[k], rym[k], ryp[k], rv[k], rv[k + 2],
                          bv[k + 1], fb[k], cs + rk);
            }
        }
        T rm = rv[U], rc = rv[U + 1], bm = bv[U], bc = bv[U + 1];
        for (; z < z1; ++z, ro += pl) {
            const T rp = R[ro + pl];
            const T bp = B[ro + pl];
            const int pr = (y + z) & 1;
            const T bx = B[ro + (pr ? 1 : xl)];
            const T rx = R[ro + (pr ? xl : 1)];
            if (pr | xs)
                point(pr ? bc : bx, pr ? bx : bc, B[ro - g.pitch], B[ro + g.pitch], bm, bp, rc,
                      ld_stream<NT>(f + ro), ro);
            if ((1 - pr) | xs)
                point(pr ? rx : rc, pr ? rc : rx, R[ro - g.pitch], R[ro + g.pitch], rm, rp, bc,
                      ld_stream<NT>(f + cs + ro), cs + ro);
            rm = rc;
            rc = rp;
            bm = bc;
            bc = bp;
        }
    }
    if (NORM) block_sum_max(sq, mx, part + 2 * (long long)ex.b);
}

// Damped-Jacobi sweep of a 3-D node level along columns (u -> out).
template <typename T, int U, bool NT, bool P2>
__global__ __launch_bounds__(1024) void k_node_jac_zm(Geom g, ZSpace zs, const T* __restrict__ u,
                                                      const T* __restrict__ f, T* __restrict__ out, T s, T omega,
                                                      T rs) {
    d_node_res_zm<T, U, NT, false, false, false, P2 ? 2 : 1>(solo_ex(), g, zs, u, f, out, s, nullptr, nullptr, 1.0,
                                                             omega, rs);
}

template <typename T, int U, bool NT, bool NORM, bool STORE>
__global__ __launch_bounds__(1024) void k_node_res_zm(Geom g, ZSpace zs, const T* __restrict__ u,
                                                      const T* __restrict__ f, T* __restrict__ r, T s,
                                                      double* __restrict__ part) {
    d_node_res_zm<T, U, NT, NORM, STORE>(solo_ex(), g, zs, u, f, r, s, part);
}

// ------------------------------------------------ 2-D node grids, row marching
// Damped Jacobi (both colours, out of place) and residual walking rows: lane
// x >> 1 keeps rows y-1, y, y+1 of both colours in registers, so a row of
// each colour is loaded once instead of three times.  Same formulas and
// evaluation order as the point kernels (x-, x+, y-, y+).
template <typename T, bool ZERO>
__device__ __forceinline__ void d_node_jac_ym(const Ex& ex, Geom g, YSpace ys, const T* __restrict__ u,
                                              const T* __restrict__ f, T* __restrict__ out, T s, T omega) {
    const int tx = ex.b % ys.ntx, ty = ex.b / ys.ntx;
    const int xs = tx * 64 + (ex.t & 63);
    const int y0 = 1 + (ty * ys.rows + (ex.t >> 6)) * ys.yc, y1 = min(y0 + ys.yc, g.n - 1);
    if (xs >= ys.xr || y0 >= y1) return;
    const T* __restrict__ R = u;
    const T* __restrict__ B = u + g.cs;
    const long long cs = g.cs, pt = g.pitch;
    const long long xl = xs > 0 ? -1 : 0;
    const T D = T(4) * s;
    long long ro = (long long)y0 * pt + xs;
    T rm = T(0), rc = T(0), bm = T(0), bc = T(0);
    if (!ZERO) {
        rm = R[ro - pt];
        rc = R[ro];
        bm = B[ro - pt];
        bc = B[ro];
    }
    for (int y = y0; y < y1; ++y, ro += pt) {
        const int pr = y & 1;   // x parity of the red point; the black one has 1 - pr
        T rp = T(0), bp = T(0), bx = T(0), rx = T(0);
        if (!ZERO) {
            rp = R[ro + pt];
            bp = B[ro + pt];
            bx = B[ro + (pr ? 1 : xl)];
            rx = R[ro + (pr ? xl : 1)];
        }
        const T fr = f[ro], fb = f[cs + ro];
        if (pr | xs) {
            T nb = T(0);
            if (!ZERO) {
                nb = pr ? bc : bx;
                nb = nb + (pr ? bx : bc);
                nb = nb + bm;
                nb = nb + bp;
            }
            const T r = fr - (T(4) * rc - nb) * s;
            out[ro] = rc + (omega * r) / D;
        }
        if ((1 - pr) | xs) {
            T nb = T(0);
            if (!ZERO) {
                nb = pr ? rx : rc;
                nb = nb + (pr ? rc : rx);
                nb = nb + rm;
                nb = nb + rp;
            }
            const T r = fb - (T(4) * bc - nb) * s;
            out[cs + ro] = bc + (omega * r) / D;
        }
        rm = rc;
        rc = rp;
        bm = bc;
        bc = bp;
    }
}

template <typename T, bool ZERO>
__global__ __launch_bounds__(256) void k_node_jac_ym(Geom g, YSpace ys, const T* __restrict__ u,
                                                     const T* __restrict__ f, T* __restrict__ out, T s, T omega) {
    d_node_jac_ym<T, ZERO>(solo_ex(), g, ys, u, f, out, s, omega);
}

template <typename T, bool NORM, bool STORE>
__device__ __forceinline__ void d_node_res_ym(const Ex& ex, Geom g, YSpace ys, const T* __restrict__ u,
                                              const T* __restrict__ f, T* __restrict__ r, T s,
                                              double* __restrict__ part) {
    double sq = 0.0, mx = 0.0;
    const int tx = ex.b % ys.ntx, ty = ex.b / ys.ntx;
    const int xs = tx * 64 + (ex.t & 63);
    const int y0 = 1 + (ty * ys.rows + (ex.t >> 6)) * ys.yc, y1 = min(y0 + ys.yc, g.n - 1);
    if (xs < ys.xr && y0 < y1) {
        const T* __restrict__ R = u;
        const T* __restrict__ B = u + g.cs;
        const long long cs = g.cs, pt = g.pitch;
        const long long xl = xs > 0 ? -1 : 0;
        long long ro = (long long)y0 * pt + xs;
        T rm = R[ro - pt], rc = R[ro], bm = B[ro - pt], bc = B[ro];
        for (int y = y0; y < y1; ++y, ro += pt) {
            const int pr = y & 1;
            const T rp = R[ro + pt], bp = B[ro + pt];
            const T bx = B[ro + (pr ? 1 : xl)];
            const T rx = R[ro + (pr ? xl : 1)];
            const T fr = f[ro], fb = f[cs + ro];
            if (pr | xs) {
                T nb = pr ? bc : bx;
                nb = nb + (pr ? bx : bc);
                nb = nb + bm;
                nb = nb + bp;
                const T v = fr - (T(4) * rc - nb) * s;
                if (STORE) r[ro] = v;
                const double dv = (double)v;
                sq = sq + dv * dv;
                mx = fmax(mx, fabs(dv));
            }
            if ((1 - pr) | xs) {
                T nb = pr ? rx : rc;
                nb = nb + (pr ? rc : rx);
                nb = nb + rm;
                nb = nb + rp;
                const T v = fb - (T(4) * bc - nb) * s;
                if (STORE) r[cs + ro] = v;
                const double dv = (double)v;
                sq = sq + dv * dv;
                mx = fmax(mx, fabs(dv));
            }
            rm = rc;
            rc = rp;
            bm = bc;
            bc = bp;
        }
    }
    if (NORM) block_sum_max(sq, mx, part + 2 * (long long)ex.b);
}

template <typename T, bool NORM, bool STORE>
__global__ __launch_bounds__(256) void k_node_res_ym(Geom g, YSpace ys, const T* __restrict__ u,
                                                     const T* __restrict__ f, T* __restrict__ r, T s,
                                                     double* __restrict__ part) {
    d_node_res_ym<T, NORM, STORE>(solo_ex(), g, ys, u, f, r, s, part);
}

// ------------------------------------------ 3-D node grids, temporal blocking
// S red-black half-sweeps (colours c1, 1 - c1, c1, ...) fused into one pass.
// Half-sweep k updates its colour from half-sweep k - 1's values of the other
// colour (k = 0: the iterate), so the pass runs as a wavefront in z: at step
// t, stage 0 loads plane t of the other colour and stage k updates plane t - k.
// Each block owns a region of 64 positions (x >> 1) by 16 R rows; stage k's
// current plane sits in LDS for the x and y neighbours of stage k + 1, the
// z neighbours stay in registers (planes p - 1, p, p + 1 of each stage at the
// thread's own position).  Values near the region edge go stale one point
// per stage, so only positions at least ceil(S/2) columns and S rows inside
// are written; neighbouring regions overlap by that halo.  Every point takes
// the same operands in the same order as the one-colour kernels, so the
// result is bitwise that of S separate half-sweeps.  The output goes to a
// second buffer (a neighbouring block may still read the iterate); both
// colours of every interior node are written, boundary nodes stay zero.
// Workgroup barrier that orders LDS accesses only: global loads issued
// before it stay in flight (a full __syncthreads waits for every
// outstanding load, which would expose the latency the one-step-ahead loads
// are meant to hide).  Only LDS carries data between the block's waves here.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t rsc, unsigned voff, int soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rsc, voff, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rsc, voff, soff, 0));
}

template <typename T, int S, int R, int NW, int PF, bool P2, bool BUF>
__global__ __launch_bounds__(64 * NW) void k_node_gs_tb(Geom g, TbSpace ts, const T* __restrict__ uin,
                                                        const T* __restrict__ f, T* __restrict__ uout, T s, T rs,
                                                        int c1, int zero) {
    constexpr int W = kTbLanes, RY = NW * R, LP = W + 2, LR = RY + 2, H = (S + 1) / 2;
    __shared__ T lds[S][LR][LP];
    {
        T* lf = &lds[0][0][0];
        for (int i = (int)threadIdx.x; i < S * LR * LP; i += (int)blockDim.x) lf[i] = T(0);
    }
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int tx = b % ts.ntx, ty = (b / ts.ntx) % ts.nty, tz = b / (ts.ntx * ts.nty);
    const int lane = (int)threadIdx.x & 63;
    // rows belong to whole wavefronts: everything that depends on y or z only
    // is wavefront-uniform and lives in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int n = g.n;
    const int xg = tx * (W - 2 * H) - H + lane;
    const int Z0 = 1 + tz * ts.zc, Z1 = min(Z0 + ts.zc, n - 1);
    const int c0 = 1 - c1;
    const long long cs = g.cs, pl = g.plane;
    // lane offset of every access: x >> 1 clamped into the row (values of
    // positions outside the grid are masked, never their addresses)
    const unsigned xo = (unsigned)min(max(xg, 0), g.half - 1);
    const bool xreg = xg >= 0 && xg < g.half;
    const bool xin0 = xreg && xg >= 1 && 2 * xg <= n - 2;   // x = 2 (x >> 1) is an unknown column
    const bool xin1 = xreg && 2 * xg + 1 <= n - 2;           // x = 2 (x >> 1) + 1 is
    const bool xout = xreg && lane >= H && lane < W - H;
    int yg[R];
    long long yo[R];   // offset of the (clamped) row
#pragma unroll
    for (int r = 0; r < R; ++r) {
        yg[r] = ty * (RY - 2 * S) - S + wv * R + r;
        yo[r] = (long long)min(max(yg[r], 0), n - 1) * g.pitch;
    }
    auto yin = [&](int r) { return yg[r] >= 1 && yg[r] <= n - 2; };
    auto yout = [&](int r) { return wv * R + r >= S && wv * R + r < RY - S && yg[r] <= n - 2; };
    auto pin = [&](int p) { return p >= 1 && p <= n - 2; };
    auto pcl = [&](int p) -> long long { return (long long)min(max(p, 0), n - 1) * pl; };
    // (unused without BUF; the byte count is only meaningful below 2 GiB)
    const int fbytes = BUF ? (int)(2 * cs * (long long)sizeof(T)) : 0;
    const __amdgpu_buffer_rsrc_t ru = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(uin), 0, fbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rf = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(f), 0, fbytes, 0x00020000);
    const unsigned xb = xo * (unsigned)sizeof(T);
    // element (colour c, plane p clamped, row r) at the thread's lane
    auto ld = [&](const T* base, __amdgpu_buffer_rsrc_t rsc, int c, int p, int r) -> T {
        const long long e = c * cs + pcl(p) + yo[r];
        if constexpr (BUF) return buf_load<T>(rsc, xb, (int)(e * (long long)sizeof(T)));
        else return base[e + xo];
    };
    // is the colour-c point of row r on plane p an unknown? (par: its x parity)
    auto inside = [&](int r, int p, int par) { return yin(r) && pin(p) && (par ? xin1 : xin0); };
    // Operands that come from HBM are loaded one step ahead: qu = iterate on
    // plane t (stage 0), qf[k - 1] = right-hand side of stage k <= PF on plane
    // t - k (stages 1 and 2 touch a plane of f first; later stages re-read
    // it from L2 where it is used).
    T qu[R], qf[PF][R];
    T old[S][R], cur[S][R];
    const int t0 = Z0 - S;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        qu[r] = zero ? T(0) : ld(uin, ru, c0, t0, r);
#pragma unroll
        for (int k = 1; k <= PF; ++k) qf[k - 1][r] = ld(f, rf, (c1 + k - 1) & 1, t0 - k, r);
#pragma unroll
        for (int k = 0; k < S; ++k) {
            old[k][r] = T(0);
            cur[k][r] = T(0);
        }
    }
    __syncthreads();
    for (int t = t0; t < Z1 + S; ++t) {
        // stage k's plane t - 1 - k becomes visible to stage k + 1
#pragma unroll
        for (int k = 0; k < S; ++k)
#pragma unroll
            for (int r = 0; r < R; ++r) lds[k][1 + wv * R + r][1 + lane] = cur[k][r];
        __syncthreads();
        T nw[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            nw[r] = inside(r, t, (yg[r] + t + c0) & 1) ? qu[r] : T(0);
            if (!zero) qu[r] = ld(uin, ru, c0, t + 1, r);
        }
#pragma unroll
        for (int k = 1; k <= S; ++k) {
            const int p = t - k, ck = (c1 + k - 1) & 1;
            const bool zout = k >= S - 1 && p >= Z0 && p < Z1;
            T nk[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int ly = wv * R + r;
                const int par = (yg[r] + p + ck) & 1;
                const T* lrow = &lds[k - 1][1 + ly][1 + lane];
                const T own = cur[k - 1][r];
                T nb;
                if (par) {
                    nb = own;
                    nb = nb + lrow[1];
                } else {
                    nb = lrow[-1];
                    nb = nb + own;
                }
                nb = nb + lrow[-LP];
                nb = nb + lrow[LP];
                nb = nb + old[k - 1][r];
                nb = nb + nw[r];
                T fv;
                if (k <= PF) {
                    fv = qf[k - 1][r];
                    qf[k - 1][r] = ld(f, rf, ck, p + 1, r);
                } else {
                    fv = ld(f, rf, ck, p, r);
                }
                // s is a power of two when P2: f * (1 / s) rounds exactly as f / s
                T v = div6((P2 ? fv * rs : fv / s) + nb);
                const bool in = inside(r, p, par);
                v = in ? v : T(0);
                if (zout && yout(r) && xout && in) {
                    // FP64 output streams past the L2 (less eviction of the halo
                    // and right-hand-side planes later stages re-read)
                    T* dst = uout + (ck * cs + p * pl + yo[r] + xo);
                    if (sizeof(T) == 8) __builtin_nontemporal_store(v, dst);
                    else *dst = v;
                }
                nk[r] = v;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                old[k - 1][r] = cur[k - 1][r];
                cur[k - 1][r] = nw[r];
                nw[r] = nk[r];
            }
        }
        __syncthreads();
    }
}

// Calls f(integral_constant<int, I>) for I = B .. E - 1 (compile-time indices
// for register arrays in unrolled bodies).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <int X>
constexpr int md2() { return ((X % 2) + 2) % 2; }

// The same fused pass as k_node_gs_tb (same regions, halos, chunks, operand
// order and output), written for fewer instructions per point update.
// BUF: fields below 2 GiB are read through buffer resources, the lane's byte
// offset in a vector register and the plane's in a scalar one (no per-load
// 64-bit address arithmetic).  Offsets stay inside the field (planes are
// clamped at the ends of the grid), so the range check never clips a value
// that is used.  Barriers order LDS only (lds_barrier), so the loads issued
// one step ahead stay in flight across them.
//
// Instruction economy.  The x parity of the point a thread updates is the
// same for every stage of a step and alternates with the row and the step,
// and stage k keeps its planes p - 1 and p in two register slots chosen by
// the plane's parity: the march is unrolled two steps at a time (relative to
// the chunk's first step) so that every slot index, x-neighbour offset and
// lane mask is fixed at compile time.  Pairs of steps whose planes all lie
// inside the grid and whose final stages all store run without clamps or
// plane tests; the lead-in and lead-out pairs test each step.
template <typename T, int S, int R, int NW, int PF, bool P2, bool BUF>
__global__ __launch_bounds__(64 * NW) void k_node_gs_tbu(Geom g, TbSpace ts, const T* __restrict__ uin,
                                                        const T* __restrict__ f, T* __restrict__ uout, T s, T rs,
                                                        int c1, int zero) {
    constexpr int W = kTbLanes, RY = NW * R, LP = W + 2, LR = RY + 2, H = (S + 1) / 2;
    __shared__ T lds[S][LR][LP];
    {
        T* lf = &lds[0][0][0];
        for (int i = (int)threadIdx.x; i < S * LR * LP; i += (int)blockDim.x) lf[i] = T(0);
    }
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int tx = b % ts.ntx, ty = (b / ts.ntx) % ts.nty, tz = b / (ts.ntx * ts.nty);
    const int lane = (int)threadIdx.x & 63;
    // rows belong to whole wavefronts: everything that depends on y or z only
    // is wavefront-uniform and lives in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int n = g.n;
    const int xg = tx * (W - 2 * H) - H + lane;
    const int Z0 = 1 + tz * ts.zc, Z1 = min(Z0 + ts.zc, n - 1);
    const int c0 = 1 - c1;
    const long long cs = g.cs, pl = g.plane;
    // lane offset of every access: x >> 1 clamped into the row (values of
    // positions outside the grid are masked, never their addresses)
    const int xo = min(max(xg, 0), g.half - 1);
    const bool xreg = xg >= 0 && xg < g.half;
    const bool xin0 = xreg && xg >= 1 && 2 * xg <= n - 2;   // x = 2 (x >> 1) is an unknown column
    const bool xin1 = xreg && 2 * xg + 1 <= n - 2;           // x = 2 (x >> 1) + 1 is
    const bool xout = xreg && lane >= H && lane < W - H;
    const int ly0 = 1 + wv * R;                               // the wavefront's first LDS row
    const int t0 = Z0 - S;
    // The point of row r updated at step t has x parity (y + t + c1 + 1) & 1
    // in every stage; rows being consecutive, that is pw ^ ((r + rel) & 1)
    // with rel = t - t0.  Per parity class q: the x-neighbour's LDS offset,
    // the unknown mask and the store mask.
    const int yw = ty * (RY - 2 * S) - S + wv * R;             // the wavefront's first row
    const int pw = (yw + t0 + c1 + 1) & 1;
    int dx[2];
    bool m[2][R], sm[2][R];
    unsigned vo[R];                                            // byte offset of the lane in row r
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const bool odd = (pw ^ q) != 0;
        dx[q] = odd ? 1 : -1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = yw + r;
            const bool yin = y >= 1 && y <= n - 2;
            const bool yout = wv * R + r >= S && wv * R + r < RY - S && y <= n - 2;
            m[q][r] = yin && (odd ? xin1 : xin0);
            sm[q][r] = yout && xout && (odd ? xin1 : xin0);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        vo[r] = (unsigned)(((long long)min(max(yw + r, 0), n - 1) * g.pitch + xo) * (long long)sizeof(T));
    // (unused without BUF; the byte count is only meaningful below 2 GiB)
    const int fbytes = BUF ? (int)(2 * cs * (long long)sizeof(T)) : 0;
    const __amdgpu_buffer_rsrc_t ru = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(uin), 0, fbytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rf = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(f), 0, fbytes, 0x00020000);
    // element offset of (colour c, plane p), p clamped into the grid where
    // it may leave it
    auto poff = [&](auto gc, int c, int p) -> long long {
        if constexpr (decltype(gc)::value) p = min(max(p, 0), n - 1);
        return c * cs + (long long)p * pl;
    };
    auto ld = [&](const T* base, __amdgpu_buffer_rsrc_t rsc, long long e, int r) -> T {
        if constexpr (BUF) return buf_load<T>(rsc, vo[r], (int)(e * (long long)sizeof(T)));
        else return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base + e) + vo[r]);
    };
    auto pin = [&](int p) { return p >= 1 && p <= n - 2; };
    // A[k][i][r]: stage k's value in row r on the plane p with p - t0 = i
    // mod 2 (stage 0 is the iterate), the two planes behind stage k's
    // newest; nw[r]: the newest value of the stage just computed.
    // Right-hand-side and iterate loads run one step ahead: qu = iterate on
    // plane t, qf[k - 1] = right-hand side of stage k <= PF on plane t - k
    // (later stages re-read it from L2).
    T A[S][2][R], nw[R], qu[R], qf[PF > 0 ? PF : 1][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        qu[r] = zero ? T(0) : ld(uin, ru, poff(std::true_type{}, c0, t0), r);
#pragma unroll
        for (int k = 1; k <= PF; ++k) qf[k - 1][r] = ld(f, rf, poff(std::true_type{}, (c1 + k - 1) & 1, t0 - k), r);
        nw[r] = T(0);
#pragma unroll
        for (int k = 0; k < S; ++k) A[k][0][r] = A[k][1][r] = T(0);
    }
    __syncthreads();
    // one step of the march: J = (t - t0) mod 2; GEN: planes and stores tested
    auto step = [&](auto jc, auto gc, const int t) {
        constexpr int J = decltype(jc)::value;
        constexpr bool GEN = decltype(gc)::value;
        // stage k's plane t - 1 - k becomes visible to stage k + 1
        static_for<0, S>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[k][ly0 + r][1 + lane] = A[k][md2<J - 1 - k>()][r];
        });
        lds_barrier();
        {
            const bool p0 = !GEN || pin(t);
            const long long e = poff(gc, c0, t + 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                nw[r] = (p0 && m[(r + J) & 1][r]) ? qu[r] : T(0);
                if (!zero) qu[r] = ld(uin, ru, e, r);
            }
        }
        static_for<1, S + 1>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            // keep each stage's LDS reads and loads in its own stretch of code
            // (hoisting them all to the top of the step runs out of registers)
            __builtin_amdgcn_sched_barrier(0);
            const int p = t - k, ck = (c1 + k - 1) & 1;
            const bool pk = !GEN || pin(p);
            const bool st = k >= S - 1 && (!GEN || (p >= Z0 && p < Z1));
            const long long ef = poff(gc, ck, k <= PF ? p + 1 : p);
            T* const dstp = uout + (ck * cs + (long long)p * pl);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r > 0) __builtin_amdgcn_sched_barrier(0);
                const int q = (r + J) & 1;
                const T* lrow = &lds[k - 1][ly0 + r][1 + lane];
                // x neighbours (own position and the lane beside it), y - 1,
                // y + 1, z - 1, z + 1: the half-sweep's order
                T nb = A[k - 1][md2<J - k>()][r];
                nb = nb + lrow[dx[q]];
                nb = nb + lrow[-LP];
                nb = nb + lrow[LP];
                nb = nb + A[k - 1][md2<J - k - 1>()][r];
                nb = nb + nw[r];
                T fv;
                if constexpr (k <= PF) {
                    fv = qf[k - 1][r];
                    qf[k - 1][r] = ld(f, rf, ef, r);
                } else {
                    fv = ld(f, rf, ef, r);
                }
                // s is a power of two when P2: f * (1 / s) rounds exactly as f / s
                T v = div6((P2 ? fv * rs : fv / s) + nb);
                v = (pk && m[q][r]) ? v : T(0);
                if (st && pk && sm[q][r]) {
                    // FP64 output streams past the L2 (less eviction of the halo
                    // and right-hand-side planes later stages re-read)
                    T* dst = reinterpret_cast<T*>(reinterpret_cast<char*>(dstp) + vo[r]);
                    if constexpr (sizeof(T) == 8) __builtin_nontemporal_store(v, dst);
                    else *dst = v;
                }
                // stage k - 1's plane p + 1 takes the slot of its plane p - 1
                A[k - 1][md2<J - k - 1>()][r] = nw[r];
                nw[r] = v;
            }
        });
        lds_barrier();
    };
    // Steps t0 .. Z1 + S - 1 in pairs: lead-in pairs, the pairs whose planes
    // all lie inside the grid (t >= Z0 + S) and whose final stages all store
    // (t + 2 - S < Z1, t + 2 <= n - 2), then the rest.  Three separate loops:
    // one loop with both bodies behind a branch makes the register allocator
    // spill.
    const int N = Z1 - Z0 + 2 * S;
    auto gen = [&](int rel) {
        static_for<0, 2>([&](auto jc) {
            if (rel + decltype(jc)::value < N) step(jc, std::true_type{}, t0 + rel + decltype(jc)::value);
        });
    };
    int rel = 0;
    for (; rel < 2 * S && rel < N; rel += 2) gen(rel);
    for (; rel + 2 < N && t0 + rel + 2 <= n - 2; rel += 2)
        static_for<0, 2>([&](auto jc) { step(jc, std::false_type{}, t0 + rel + decltype(jc)::value); });
    for (; rel < N; rel += 2) gen(rel);
}

// ------------------------------------ 3-D node grids, fused transfer kernels
// Residual and full weighting in one pass, marching fine planes.  A block of
// NW wavefronts owns 64 positions of x >> 1 (fine x 126 tx .. 126 tx + 127)
// by 32 fine rows and the coarse points I0 .. I0 + 62, J0 .. J0 + 14 whose
// 3 x 3 fine footprints lie inside.  Each thread owns an (x >> 1, y) column of
// both colours for R rows and keeps the iterate on planes z - 1, z, z + 1 in
// registers; the fine residual of plane z goes to one LDS plane, from which
// every coarse point adds its nine terms of that plane: planes arrive in the
// order z offset -1, 0, +1, so the 27 terms are accumulated in the same order
// as by the separate kernels and only one residual plane is ever held.  The
// fine residual is never written: the pass reads u and f and writes
// f_coarse, 16 + 8 / 8 B per fine point.
constexpr int kRrCX = 63;                  // coarse points per region in x
template <typename T, int R, int NW>
__global__ __launch_bounds__(64 * NW, 4) void k_node_res_restrict_zm(Geom gf, Geom gc, int ntx, int nty, int kc,
                                                                  const T* __restrict__ u, const T* __restrict__ f,
                                                                  T* __restrict__ fcoarse, T s) {
    constexpr int RY = NW * R, CY = (RY - 1) / 2, NQ = kRrCX * CY;
    constexpr int NT = 64 * NW, QP = (NQ + NT - 1) / NT;
    // two residual planes: plane z is restricted from one while plane z + 1
    // is written to the other, so one barrier per plane suffices
    __shared__ T rpl[2][RY][2 * 64 + 2];
    const int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    const int tx = b % ntx, ty = (b / ntx) % nty, tz = b / (ntx * nty);
    const int lane = (int)threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int n = gf.n;
    const int xs = kRrCX * tx + lane;
    const int yb = 2 * CY * ty + 1;
    const int K0 = 1 + tz * kc, K1 = min(K0 + kc, gc.n - 1);
    const int I0 = 1 + kRrCX * tx, J0 = 1 + CY * ty;
    const T* __restrict__ RD = u;            // red (even x + y + z) points
    const T* __restrict__ BK = u + gf.cs;    // black points
    const bool xreg = xs < gf.half;
    int yg[R];
    bool rowin[R];
    long long ro[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        yg[r] = yb + wv * R + r;
        rowin[r] = xreg && yg[r] <= n - 1;
        ro[r] = rowin[r] ? (long long)yg[r] * gf.pitch + xs : 0;
    }
    // iterate of both colours on planes z - 1, z, z + 1 of the thread's rows,
    // and the right-hand side of plane z, loaded one plane ahead
    T rm[R], rc[R], rn[R], bm[R], bc[R], bn[R], fr[R], fb[R];
    const int zf0 = 2 * K0 - 1, zf1 = 2 * K1 - 1;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const long long a = ro[r] + (long long)(zf0 - 1) * gf.plane, c = a + gf.plane;
        rm[r] = rowin[r] ? RD[a] : T(0);
        bm[r] = rowin[r] ? BK[a] : T(0);
        rc[r] = rowin[r] ? RD[c] : T(0);
        bc[r] = rowin[r] ? BK[c] : T(0);
        fr[r] = rowin[r] ? f[c] : T(0);
        fb[r] = rowin[r] ? f[gf.cs + c] : T(0);
    }
    // coarse points of this thread and their open accumulations
    T acc[QP];
#pragma unroll
    for (int q = 0; q < QP; ++q) acc[q] = T(0);
    for (int z = zf0; z <= zf1; ++z) {
        T(*rp)[2 * 64 + 2] = rpl[z & 1];
        const bool zin = z >= 1 && z <= n - 2;
        const long long zo = (long long)z * gf.plane;
        T frn[R], fbn[R];
        if constexpr (sizeof(T) == 4) {
            // FP32: this plane's x neighbours and the y neighbours beyond the
            // thread's rows first, then the next plane's loads, which stay in
            // flight across the LDS-only barrier (FP64 measured faster with
            // the loads in the order below: the hoisted values cost registers)
            bool rin[R], bin[R];
            T bx[R], rx[R], byl = T(0), ryl = T(0), byh = T(0), ryh = T(0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int y = yg[r];
                const int pr = (y + z) & 1;   // x parity of the red point
                const bool yin = rowin[r] && y >= 1 && y <= n - 2 && zin;
                const int xr = 2 * xs + pr, xb = 2 * xs + 1 - pr;
                rin[r] = yin && xr >= 1 && xr <= n - 2;
                bin[r] = yin && xb >= 1 && xb <= n - 2;
                const long long a = ro[r] + zo;
                // black neighbours of the red point: x - 1, x + 1 at x >> 1 - 1 + pr, x >> 1 + pr
                bx[r] = rin[r] ? BK[a + (pr ? 1 : -1)] : T(0);
                rx[r] = bin[r] ? RD[a + (pr ? -1 : 1)] : T(0);
                if (r == 0) {
                    byl = rin[r] ? BK[a - gf.pitch] : T(0);
                    ryl = bin[r] ? RD[a - gf.pitch] : T(0);
                }
                if (r == R - 1) {
                    byh = rin[r] ? BK[a + gf.pitch] : T(0);
                    ryh = bin[r] ? RD[a + gf.pitch] : T(0);
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const long long a = ro[r] + zo + gf.plane;
                const bool ld = rowin[r] && z + 1 <= n - 1;
                rn[r] = ld ? RD[a] : T(0);
                bn[r] = ld ? BK[a] : T(0);
                frn[r] = ld ? f[a] : T(0);
                fbn[r] = ld ? f[gf.cs + a] : T(0);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int pr = (yg[r] + z) & 1;
                T vr = T(0), vb = T(0);
                if (rin[r]) {
                    T nb = pr ? bc[r] : bx[r];
                    nb = nb + (pr ? bx[r] : bc[r]);
                    nb = nb + (r > 0 ? bc[r - 1] : byl);
                    nb = nb + (r < R - 1 ? bc[r + 1] : byh);
                    nb = nb + bm[r];
                    nb = nb + bn[r];
                    vr = fr[r] - (T(6) * rc[r] - nb) * s;
                }
                if (bin[r]) {
                    T nb = pr ? rx[r] : rc[r];
                    nb = nb + (pr ? rc[r] : rx[r]);
                    nb = nb + (r > 0 ? rc[r - 1] : ryl);
                    nb = nb + (r < R - 1 ? rc[r + 1] : ryh);
                    nb = nb + rm[r];
                    nb = nb + rn[r];
                    vb = fb[r] - (T(6) * bc[r] - nb) * s;
                }
                rp[wv * R + r][2 * lane + pr] = vr;
                rp[wv * R + r][2 * lane + 1 - pr] = vb;
            }
            lds_barrier();
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const long long a = ro[r] + zo + gf.plane;
                const bool ld = rowin[r] && z + 1 <= n - 1;
                rn[r] = ld ? RD[a] : T(0);
                bn[r] = ld ? BK[a] : T(0);
                frn[r] = ld ? f[a] : T(0);
                fbn[r] = ld ? f[gf.cs + a] : T(0);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int y = yg[r];
                const int pr = (y + z) & 1;   // x parity of the red point
                const bool yin = rowin[r] && y >= 1 && y <= n - 2 && zin;
                const int xr = 2 * xs + pr, xb = 2 * xs + 1 - pr;
                const bool rin = yin && xr >= 1 && xr <= n - 2, bin = yin && xb >= 1 && xb <= n - 2;
                const long long a = ro[r] + zo;
                T vr = T(0), vb = T(0);
                if (rin) {
                    // black neighbours of the red point: x - 1, x + 1 at x >> 1 - 1 + pr, x >> 1 + pr
                    const T bx = BK[a + (pr ? 1 : -1)];
                    T nb = pr ? bc[r] : bx;
                    nb = nb + (pr ? bx : bc[r]);
                    nb = nb + (r > 0 ? bc[r - 1] : BK[a - gf.pitch]);
                    nb = nb + (r < R - 1 ? bc[r + 1] : BK[a + gf.pitch]);
                    nb = nb + bm[r];
                    nb = nb + bn[r];
                    vr = fr[r] - (T(6) * rc[r] - nb) * s;
                }
                if (bin) {
                    const T rx = RD[a + (pr ? -1 : 1)];
                    T nb = pr ? rx : rc[r];
                    nb = nb + (pr ? rc[r] : rx);
                    nb = nb + (r > 0 ? rc[r - 1] : RD[a - gf.pitch]);
                    nb = nb + (r < R - 1 ? rc[r + 1] : RD[a + gf.pitch]);
                    nb = nb + rm[r];
                    nb = nb + rn[r];
                    vb = fb[r] - (T(6) * bc[r] - nb) * s;
                }
                rp[wv * R + r][2 * lane + pr] = vr;
                rp[wv * R + r][2 * lane + 1 - pr] = vb;
            }
            __syncthreads();
        }
        // fine plane z is offset -1 of coarse plane (z + 1) / 2 and +1 of
        // (z - 1) / 2 when odd, offset 0 of z / 2 when even
        const bool odd = z & 1;
#pragma unroll
        for (int q = 0; q < QP; ++q) {
            const int qi = (int)threadIdx.x + NT * q;
            if (qi < NQ) {
                const int ci = qi % kRrCX, cj = qi / kRrCX;
                const int I = I0 + ci, J = J0 + cj;
                if (I <= gc.n - 2 && J <= gc.n - 2) {
                    const int lx = 2 * ci + 2, ly = 2 * cj + 1;
                    auto plane_terms = [&](int wz, bool first, T a0) -> T {
                        T a = a0;
                        bool fst = first;
#pragma unroll
                        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                            for (int ox = -1; ox <= 1; ++ox) {
                                const int wgt = (2 - (ox < 0 ? -ox : ox)) * (2 - (oy < 0 ? -oy : oy)) * wz;
                                const T term = (T(wgt) / T(64)) * rp[ly + oy][lx + ox];
                                a = fst ? term : a + term;
                                fst = false;
                            }
                        return a;
                    };
                    if (odd) {
                        const int Ke = (z - 1) >> 1, Ks = (z + 1) >> 1;
                        if (Ke >= K0) {
                            const T done = plane_terms(1, false, acc[q]);
                            fcoarse[(long long)((I + J + Ke) & 1) * gc.cs + row_off(gc, J, Ke) + (I >> 1)] = done;
                        }
                        if (Ks < K1) acc[q] = plane_terms(1, true, T(0));
                    } else {
                        acc[q] = plane_terms(2, false, acc[q]);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            rm[r] = rc[r];
            rc[r] = rn[r];
            bm[r] = bc[r];
            bc[r] = bn[r];
            fr[r] = frn[r];
            fb[r] = fbn[r];
        }
    }
}

// Interpolation + correction walking fine columns.  A thread owns one
// (x >> 1, y) column of one colour; for every coarse plane Z it forms once
// the y-interpolated values for an even and an odd fine x (the column's x
// parity flips with z) and reuses them for the fine planes 2Z - 1 .. 2Z + 1.
// Same evaluation order as the point kernel: x, then y, then z.
template <typename T>
__global__ __launch_bounds__(256) void k_node_prolong_zm(Geom gf, Geom gc, ZSpace zs, int colour,
                                                         T* __restrict__ u, const T* __restrict__ ec) {
    int tx, ty, tz;
    {
        int b = xcd_remap((int)blockIdx.x, (int)gridDim.x);
        tx = b % zs.ntx;
        b /= zs.ntx;
        ty = b % zs.nty;
        tz = b / zs.nty;
    }
    const int xs = tx * 64 + (int)threadIdx.x;
    const int y = 1 + ty * zs.rows + (int)threadIdx.y;
    if (xs >= zs.xr || y > gf.n - 2) return;
    const int z0 = 1 + tz * zs.zc;
    const int z1 = min(z0 + zs.zc, gf.n - 1);
    const T half = T(0.5);
    const int Y0 = y >> 1, Y1 = (y + 1) >> 1;
    const bool yodd = y & 1;
    // coarse value at (X, Yc, Z), X in {xs, xs + 1}
    auto E = [&](int X, int Yc, int Z) -> T {
        return ec[(long long)((X + Yc + Z) & 1) * gc.cs + row_off(gc, Yc, Z) + (X >> 1)];
    };
    // y-interpolated values of plane Z for an even fine x (X = xs) and an odd one (X = xs, xs + 1)
    auto plane = [&](int Z, T& ev, T& od) {
        const T a0 = E(xs, Y0, Z), b0 = E(xs + 1, Y0, Z);
        const T ix_e0 = a0, ix_o0 = half * (a0 + b0);
        if (yodd) {
            const T a1 = E(xs, Y1, Z), b1 = E(xs + 1, Y1, Z);
            ev = half * (ix_e0 + a1);
            od = half * (ix_o0 + half * (a1 + b1));
        } else {
            ev = ix_e0;
            od = ix_o0;
        }
    };
    int Zlo = z0 >> 1;
    T lo_e, lo_o, hi_e, hi_o;
    const long long ro0 = row_off(gf, y, z0) + xs + (long long)colour * gf.cs;
    // the column's iterate for the whole chunk, loaded before any store
    // (the loads of later planes would otherwise wait behind earlier stores)
    T uv[kZChunk];
#pragma unroll
    for (int k = 0; k < kZChunk; ++k) uv[k] = z0 + k < z1 ? u[ro0 + k * gf.plane] : T(0);
    plane(Zlo, lo_e, lo_o);
    plane(Zlo + 1, hi_e, hi_o);
#pragma unroll
    for (int k = 0; k < kZChunk; ++k) {
        const int z = z0 + k;
        if (z >= z1) break;
        const int Zc = z >> 1;
        if (Zc != Zlo) {   // advance the two-plane window by one coarse plane
            lo_e = hi_e;
            lo_o = hi_o;
            Zlo = Zc;
            plane(Zlo + 1, hi_e, hi_o);
        }
        const int par = (y + z + colour) & 1;
        if (par | xs) {
            const T v0 = par ? lo_o : lo_e;
            const T e = (z & 1) ? half * (v0 + (par ? hi_o : hi_e)) : v0;
            u[ro0 + k * gf.plane] = uv[k] + e;
        }
    }
}

// Full weighting: f_c[X] = sum_{o in {-1,0,1}^d} prod_a (2 - |o_a|) / 4^d r[2X + o],
// summed with the z offset slowest and the x offset fastest, at coarse point
// p of the fine values rf(colour, x >> 1, y, z) (a stored residual, or one
// formed on the fly); false outside the unknowns.
template <typename T, int D, typename RF>
__device__ __forceinline__ bool pt_node_restrict_by(const Pt& p, const Geom& gc, RF&& rf, T* __restrict__ fcoarse) {
    const int par = (p.y + p.z + p.c) & 1;
    const int X = 2 * p.xs + par;
    if (X < 1 || X > gc.n - 2) return false;
    const int Y = p.y, Z = p.z;
    T acc = T(0);
    bool first = true;
#pragma unroll
    for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); ++oz) {
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                const int fx = 2 * X + ox, fy = 2 * Y + oy, fz = (D == 3) ? 2 * Z + oz : 0;
                const int wgt = (2 - (ox < 0 ? -ox : ox)) * (2 - (oy < 0 ? -oy : oy)) *
                                (D == 3 ? (2 - (oz < 0 ? -oz : oz)) : 1);
                const T w = T(wgt) / T(D == 3 ? 64 : 16);
                const T term = w * rf((fx + fy + fz) & 1, fx >> 1, fy, fz);
                acc = first ? term : acc + term;
                first = false;
            }
        }
    }
    fcoarse[(long long)p.c * gc.cs + row_off(gc, Y, Z) + p.xs] = acc;
    return true;
}

template <typename T, int D>
__device__ __forceinline__ void pt_node_restrict(const Pt& p, Geom gf, Geom gc, Space sp,
                                                       const T* __restrict__ r,
                                                       T* __restrict__ fcoarse) {
    pt_node_restrict_by<T, D>(p, gc, [&](int c, int xs, int y, int z) -> T {
        return r[(long long)c * gf.cs + row_off(gf, y, z) + xs];
    }, fcoarse);
}

// Residual and full weighting in one launch over the coarse points of a
// level that runs point kernels: each coarse point forms the residuals of
// its 3^d fine footprint as it sums them (nothing stored), each with the
// residual kernel's operands and order, so f_coarse is bitwise that of the
// residual then the restriction.
template <typename T, int D>
__global__ __launch_bounds__(256) void k_node_res_restrict_pt(Geom gf, Geom gc, Space sp, const T* __restrict__ u,
                                                              const T* __restrict__ f, T* __restrict__ fcoarse,
                                                              T s) {
    Pt p;
    if (!map_point(solo_ex(), sp, p)) return;
    pt_node_restrict_by<T, D>(p, gc, [&](int c, int xs, int y, int z) -> T {
        Pt q;
        q.xs = xs;
        q.y = y;
        q.z = z;
        q.c = c;
        long long me;
        T rv = T(0);
        pt_node_residual<T, D>(q, gf, u, f, s, me, rv);
        return rv;
    }, fcoarse);
}

template <typename T, int D>
__device__ __forceinline__ void d_node_restrict(const Ex& ex, Geom gf, Geom gc, Space sp,
                                                       const T* __restrict__ r,
                                                       T* __restrict__ fcoarse) {
    Pt p;
    if (!map_point(ex, sp, p)) return;
    pt_node_restrict<T, D>(p, gf, gc, sp, r, fcoarse);
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_node_restrict(Geom gf, Geom gc, Space sp,
                                                       const T* __restrict__ r,
                                                       T* __restrict__ fcoarse) {
    d_node_restrict<T, D>(solo_ex(), gf, gc, sp, r, fcoarse);
}

// Linear interpolation as the tensor product of the 1-D rule (even fine
// node: coarse value; odd: half the sum of the two coarse neighbours),
// along x first, then y, then z; then u += P e.
template <typename T, int D>
__device__ __forceinline__ void pt_node_prolong(const Pt& p, Geom gf, Geom gc, Space sp, T* __restrict__ u,
                                                      const T* __restrict__ ec) {
    const int par = (p.y + p.z + p.c) & 1;
    const int x = 2 * p.xs + par;
    if (x < 1 || x > gf.n - 2) return;
    const int y = p.y, z = p.z;
    const T half = T(0.5);
    const int X0 = x >> 1, X1 = (x + 1) >> 1, Y0 = y >> 1, Y1 = (y + 1) >> 1;
    const int Z0 = z >> 1, Z1 = (z + 1) >> 1;
    auto E = [&](int X, int Y, int Z) -> T {
        return ec[(long long)((X + Y + Z) & 1) * gc.cs + row_off(gc, Y, Z) + (X >> 1)];
    };
    auto ix = [&](int Y, int Z) -> T {
        return (x & 1) ? half * (E(X0, Y, Z) + E(X1, Y, Z)) : E(X0, Y, Z);
    };
    auto iy = [&](int Z) -> T { return (y & 1) ? half * (ix(Y0, Z) + ix(Y1, Z)) : ix(Y0, Z); };
    T e;
    if (D == 3)
        e = (z & 1) ? half * (iy(Z0) + iy(Z1)) : iy(Z0);
    else
        e = iy(0);
    const long long me = (long long)p.c * gf.cs + row_off(gf, y, z) + p.xs;
    u[me] = u[me] + e;
}

template <typename T, int D>
__device__ __forceinline__ void d_node_prolong(const Ex& ex, Geom gf, Geom gc, Space sp, T* __restrict__ u,
                                                      const T* __restrict__ ec) {
    Pt p;
    if (!map_point(ex, sp, p)) return;
    pt_node_prolong<T, D>(p, gf, gc, sp, u, ec);
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_node_prolong(Geom gf, Geom gc, Space sp, T* __restrict__ u,
                                                      const T* __restrict__ ec) {
    d_node_prolong<T, D>(solo_ex(), gf, gc, sp, u, ec);
}

// Iterate after interpolation + correction at fine node (x, y, z): u + P e
// formed as pt_node_prolong forms it (boundary nodes: u, uncorrected).
template <typename T, int D>
__device__ __forceinline__ T node_corrected(const Geom& gf, const Geom& gc, const T* __restrict__ u,
                                            const T* __restrict__ ec, int x, int y, int z) {
    const T uv = u[(long long)((x + y + z) & 1) * gf.cs + row_off(gf, y, z) + (x >> 1)];
    if (x < 1 || x > gf.n - 2 || y < 1 || y > gf.n - 2 || (D == 3 && (z < 1 || z > gf.n - 2))) return uv;
    const T half = T(0.5);
    const int X0 = x >> 1, X1 = (x + 1) >> 1, Y0 = y >> 1, Y1 = (y + 1) >> 1;
    const int Z0 = z >> 1, Z1 = (z + 1) >> 1;
    auto E = [&](int X, int Y, int Z) -> T {
        return ec[(long long)((X + Y + Z) & 1) * gc.cs + row_off(gc, Y, Z) + (X >> 1)];
    };
    auto ix = [&](int Y, int Z) -> T {
        return (x & 1) ? half * (E(X0, Y, Z) + E(X1, Y, Z)) : E(X0, Y, Z);
    };
    auto iy = [&](int Z) -> T { return (y & 1) ? half * (ix(Y0, Z) + ix(Y1, Z)) : ix(Y0, Z); };
    T e;
    if (D == 3)
        e = (z & 1) ? half * (iy(Z0) + iy(Z1)) : iy(Z0);
    else
        e = iy(0);
    return uv + e;
}

// Interpolation + correction fused with the first damped-Jacobi sweep that
// follows it: out = J(u + P e) at every unknown, with the corrected values
// of the point and its neighbours formed on the fly (never stored) and the
// operands in the order of the separate kernels, so out is bitwise what
// prolongation then a sweep give.
template <typename T, int D, bool P2>
__global__ __launch_bounds__(256) void k_node_prolong_jacobi(Geom gf, Geom gc, Space sp, const T* __restrict__ u,
                                                             const T* __restrict__ ec, const T* __restrict__ f,
                                                             T* __restrict__ out, T s, T omega, T rs) {
    Pt p;
    if (!map_point(solo_ex(), sp, p)) return;
    const int par = (p.y + p.z + p.c) & 1;
    const int x = 2 * p.xs + par, y = p.y, z = p.z;
    if (x < 1 || x > gf.n - 2) return;
    const long long me = (long long)p.c * gf.cs + row_off(gf, y, z) + p.xs;
    const T uc = node_corrected<T, D>(gf, gc, u, ec, x, y, z);
    T nb = node_corrected<T, D>(gf, gc, u, ec, x - 1, y, z);
    nb = nb + node_corrected<T, D>(gf, gc, u, ec, x + 1, y, z);
    nb = nb + node_corrected<T, D>(gf, gc, u, ec, x, y - 1, z);
    nb = nb + node_corrected<T, D>(gf, gc, u, ec, x, y + 1, z);
    if (D == 3) {
        nb = nb + node_corrected<T, D>(gf, gc, u, ec, x, y, z - 1);
        nb = nb + node_corrected<T, D>(gf, gc, u, ec, x, y, z + 1);
    }
    const T r = f[me] - (T(2 * D) * uc - nb) * s;
    out[me] = uc + jacobi_step<T, D, P2>(omega * r, s, rs);
}

// Two damped-Jacobi sweeps of a 2-D node level in one launch.  A block owns
// a tile of kJ2 x kJ2 nodes: it loads the iterate (natural layout, from
// zero when ZERO; with PRO the iterate corrected by the interpolated coarse
// error, formed as the prolongation forms it) and f on the tile with a halo
// of two into LDS, runs the first sweep on the tile and one ring of halo and
// the second on the tile, and writes the tile to out.  RR (a halo of four):
// the sweeps cover three and two rings, the residual is formed on the tile
// and one ring, and the block's coarse points (the even nodes of its tile)
// restrict it into fco with the full weighting's order.  Every point takes
// the point kernels' operands in their order, so out (and fco) are bitwise
// what the separate launches give; boundary nodes are neither updated nor
// written.
constexpr int kJ2 = 16;

template <typename T, bool P2, bool ZERO, bool PRO, bool RR>
__global__ __launch_bounds__(256) void k_node_jacobi2(Geom g, Geom gc, int ntx, const T* __restrict__ u,
                                                      const T* __restrict__ ec, const T* __restrict__ f,
                                                      T* __restrict__ out, T* __restrict__ fco, T s, T omega,
                                                      T rs) {
    // RR: the restriction reads residuals on one ring around the tile, which
    // read the second sweep on two rings, which reads the first on three
    constexpr int H = RR ? 4 : 2, L = kJ2 + 2 * H;
    __shared__ T a[L][L + 1], b[L][L + 1], ff[L][L + 1];
    __shared__ T rr[RR ? L : 1][RR ? L + 1 : 1];
    const int blk = (int)blockIdx.x;
    const int tx0 = (blk % ntx) * kJ2, ty0 = (blk / ntx) * kJ2;
    const int x0 = tx0 - H, y0 = ty0 - H;
    const int n = g.n;
    auto at = [&](int x, int y) -> long long {
        return (long long)((x + y) & 1) * g.cs + row_off(g, y, 0) + (x >> 1);
    };
    auto interior = [&](int x, int y) { return x >= 1 && x <= n - 2 && y >= 1 && y <= n - 2; };
    for (int i = (int)threadIdx.x; i < L * L; i += 256) {
        const int ly = i / L, lx = i % L, x = x0 + lx, y = y0 + ly;
        T uv = T(0), fv = T(0);
        if (x >= 0 && x < n && y >= 0 && y < n) {
            if (PRO) uv = node_corrected<T, 2>(g, gc, u, ec, x, y, 0);
            else if (!ZERO) uv = u[at(x, y)];
            fv = f[at(x, y)];
        }
        a[ly][lx] = uv;
        ff[ly][lx] = fv;
    }
    __syncthreads();
    // the residual at a node from src (x - 1, x + 1, y - 1, y + 1: the order
    // of the point kernels), and the sweep's value from it
    auto resid = [&](T (*src)[L + 1], int ly, int lx) -> T {
        T nb = src[ly][lx - 1];
        nb = nb + src[ly][lx + 1];
        nb = nb + src[ly - 1][lx];
        nb = nb + src[ly + 1][lx];
        return ff[ly][lx] - (T(4) * src[ly][lx] - nb) * s;
    };
    auto sweep = [&](T (*src)[L + 1], int ly, int lx) -> T {
        return src[ly][lx] + jacobi_step<T, 2, P2>(omega * resid(src, ly, lx), s, rs);
    };
    // first sweep on the tile and H - 1 rings (off the unknowns its output
    // holds zero, as the second buffer of the separate sweeps does)
    for (int i = (int)threadIdx.x; i < (L - 2) * (L - 2); i += 256) {
        const int ly = 1 + i / (L - 2), lx = 1 + i % (L - 2);
        b[ly][lx] = interior(x0 + lx, y0 + ly) ? sweep(a, ly, lx) : T(0);
    }
    __syncthreads();
    if constexpr (!RR) {
        for (int i = (int)threadIdx.x; i < kJ2 * kJ2; i += 256) {
            const int ly = H + i / kJ2, lx = H + i % kJ2, x = x0 + lx, y = y0 + ly;
            if (interior(x, y)) out[at(x, y)] = sweep(b, ly, lx);
        }
    } else {
        // second sweep on the tile and two rings (into a, which is no longer
        // read), writing the tile
        for (int i = (int)threadIdx.x; i < (L - 4) * (L - 4); i += 256) {
            const int ly = 2 + i / (L - 4), lx = 2 + i % (L - 4), x = x0 + lx, y = y0 + ly;
            const bool in = interior(x, y);
            const T v = in ? sweep(b, ly, lx) : T(0);
            a[ly][lx] = v;
            if (in && ly >= H && ly < H + kJ2 && lx >= H && lx < H + kJ2) out[at(x, y)] = v;
        }
        __syncthreads();
        for (int i = (int)threadIdx.x; i < (L - 6) * (L - 6); i += 256) {
            const int ly = 3 + i / (L - 6), lx = 3 + i % (L - 6);
            rr[ly][lx] = interior(x0 + lx, y0 + ly) ? resid(a, ly, lx) : T(0);
        }
        __syncthreads();
        // coarse points X, Y with 2X, 2Y on the tile
        const int t = (int)threadIdx.x;
        if (t < (kJ2 / 2) * (kJ2 / 2)) {
            const int X = tx0 / 2 + t % (kJ2 / 2), Y = ty0 / 2 + t / (kJ2 / 2);
            Pt p;
            p.y = Y;
            p.z = 0;
            p.c = (X + Y) & 1;
            p.xs = X >> 1;
            if (Y >= 1 && Y <= gc.n - 2)
                pt_node_restrict_by<T, 2>(p, gc, [&](int c, int xs, int y, int z) -> T {
                    const int x = 2 * xs + ((y + z + c) & 1);
                    return rr[y - y0][x - x0];
                }, fco);
        }
    }
}

// ------------------------------------------------------------ cell grids
// Face-coefficient sums of one cell: diag = sum of w_f beta_f (w_f = 2 on
// walls) and, unless ZERO, off = sum of beta_f u_neighbour over interior
// faces, both in the order x-, x+, y-, y+, z-, z+.
template <typename T, int D, bool ZERO>
__device__ __forceinline__ void cell_sums(const Geom& g, const T* __restrict__ o, long long ro,
                                          int par, int x, int y, int z,
                                          const T* __restrict__ bx, const T* __restrict__ by,
                                          const T* __restrict__ bz, T& dg, T& off) {
    const int N = g.n;
    const long long fb = (long long)z * g.fplane + (long long)y * g.fpitch + x;
    const T bxm = bx[fb], bxp = bx[fb + 1], bym = by[fb], byp = by[fb + g.fpitch];
    const bool wxm = x == 0, wxp = x == N - 1, wym = y == 0, wyp = y == N - 1;
    // wall faces weigh 2 (Dirichlet, odd ghost) or 0 (Neumann, no flux)
    const T ww = g.neu ? T(0) : T(2);
    dg = wxm ? ww * bxm : bxm;
    dg = dg + (wxp ? ww * bxp : bxp);
    dg = dg + (wym ? ww * bym : bym);
    dg = dg + (wyp ? ww * byp : byp);
    T bzm = T(0), bzp = T(0);
    bool wzm = true, wzp = true;
    if (D == 3) {
        bzm = bz[fb];
        bzp = bz[fb + g.fplane];
        wzm = z == 0;
        wzp = z == N - 1;
        dg = dg + (wzm ? ww * bzm : bzm);
        dg = dg + (wzp ? ww * bzp : bzp);
    }
    if (ZERO) {
        off = T(0);
        return;
    }
    // neighbour indices are clamped to the cell itself where the face is a wall
    const T vxm = o[wxm ? ro : ro - 1 + par];
    const T vxp = o[wxp ? ro : ro + par];
    const T vym = o[wym ? ro : ro - g.pitch];
    const T vyp = o[wyp ? ro : ro + g.pitch];
    off = wxm ? T(0) : bxm * vxm;
    off = off + (wxp ? T(0) : bxp * vxp);
    off = off + (wym ? T(0) : bym * vym);
    off = off + (wyp ? T(0) : byp * vyp);
    if (D == 3) {
        const T vzm = o[wzm ? ro : ro - g.plane];
        const T vzp = o[wzp ? ro : ro + g.plane];
        off = off + (wzm ? T(0) : bzm * vzm);
        off = off + (wzp ? T(0) : bzp * vzp);
    }
}

template <typename T, int D, bool ZERO>
__device__ __forceinline__ void pt_cell_gs(const Pt& p, Geom g, Space sp, T* __restrict__ me,
                                                 const T* __restrict__ other, const T* __restrict__ f,
                                                 const T* __restrict__ bx, const T* __restrict__ by,
                                                 const T* __restrict__ bz, T s) {
    const int par = (p.y + p.z + p.c) & 1;
    const int x = 2 * p.xs + par;
    const long long ro = row_off(g, p.y, p.z) + p.xs;
    T dg, off;
    cell_sums<T, D, ZERO>(g, other, ro, par, x, p.y, p.z, bx, by, bz, dg, off);
    me[ro] = (f[ro] / s + off) / dg;
}

template <typename T, int D, bool ZERO>
__device__ __forceinline__ void d_cell_gs(const Ex& ex, Geom g, Space sp, T* __restrict__ me,
                                                 const T* __restrict__ other, const T* __restrict__ f,
                                                 const T* __restrict__ bx, const T* __restrict__ by,
                                                 const T* __restrict__ bz, T s) {
    Pt p;
    if (!map_point(ex, sp, p)) return;
    pt_cell_gs<T, D, ZERO>(p, g, sp, me, other, f, bx, by, bz, s);
}

template <typename T, int D, bool ZERO>
__global__ __launch_bounds__(256) void k_cell_gs(Geom g, Space sp, T* __restrict__ me,
                                                 const T* __restrict__ other, const T* __restrict__ f,
                                                 const T* __restrict__ bx, const T* __restrict__ by,
                                                 const T* __restrict__ bz, T s) {
    d_cell_gs<T, D, ZERO>(solo_ex(), g, sp, me, other, f, bx, by, bz, s);
}

template <typename T, int D, bool ZERO>
__device__ __forceinline__ void pt_cell_jacobi(const Pt& p, Geom g, Space sp, const T* __restrict__ u,
                                                     const T* __restrict__ f, T* __restrict__ out,
                                                     const T* __restrict__ bx, const T* __restrict__ by,
                                                     const T* __restrict__ bz, T s, T omega) {
    const int par = (p.y + p.z + p.c) & 1;
    const int x = 2 * p.xs + par;
    const long long ro = row_off(g, p.y, p.z) + p.xs;
    const long long me = (long long)p.c * g.cs + ro;
    T dg, off;
    cell_sums<T, D, ZERO>(g, u + (long long)(1 - p.c) * g.cs, ro, par, x, p.y, p.z, bx, by, bz, dg, off);
    const T uc = ZERO ? T(0) : u[me];
    const T r = f[me] - (dg * uc - off) * s;
    out[me] = uc + (omega * r) / (dg * s);
}

template <typename T, int D, bool ZERO>
__device__ __forceinline__ void d_cell_jacobi(const Ex& ex, Geom g, Space sp, const T* __restrict__ u,
                                                     const T* __restrict__ f, T* __restrict__ out,
                                                     const T* __restrict__ bx, const T* __restrict__ by,
                                                     const T* __restrict__ bz, T s, T omega) {
    Pt p;
    if (!map_point(ex, sp, p)) return;
    pt_cell_jacobi<T, D, ZERO>(p, g, sp, u, f, out, bx, by, bz, s, omega);
}

template <typename T, int D, bool ZERO>
__global__ __launch_bounds__(256) void k_cell_jacobi(Geom g, Space sp, const T* __restrict__ u,
                                                     const T* __restrict__ f, T* __restrict__ out,
                                                     const T* __restrict__ bx, const T* __restrict__ by,
                                                     const T* __restrict__ bz, T s, T omega) {
    d_cell_jacobi<T, D, ZERO>(solo_ex(), g, sp, u, f, out, bx, by, bz, s, omega);
}

template <typename T, int D>
__device__ __forceinline__ T pt_cell_residual(const Pt& p, const Geom& g, const T* __restrict__ u,
                                              const T* __restrict__ f, const T* __restrict__ bx,
                                              const T* __restrict__ by, const T* __restrict__ bz, T s,
                                              long long& me) {
    const int par = (p.y + p.z + p.c) & 1;
    const int x = 2 * p.xs + par;
    const long long ro = row_off(g, p.y, p.z) + p.xs;
    me = (long long)p.c * g.cs + ro;
    T dg, off;
    cell_sums<T, D, false>(g, u + (long long)(1 - p.c) * g.cs, ro, par, x, p.y, p.z, bx, by, bz, dg, off);
    return f[me] - (dg * u[me] - off) * s;
}

template <typename T, int D, bool NORM, bool STORE>
__device__ __forceinline__ void d_cell_residual(const Ex& ex, Geom g, Space sp, const T* __restrict__ u,
                                                       const T* __restrict__ f, T* __restrict__ r,
                                                       const T* __restrict__ bx, const T* __restrict__ by,
                                                       const T* __restrict__ bz, T s,
                                                       double* __restrict__ part) {
    double sq = 0.0, mx = 0.0;
    Pt p;
    if (map_point(ex, sp, p)) {
        long long me;
        const T rv = pt_cell_residual<T, D>(p, g, u, f, bx, by, bz, s, me);
        if (STORE) r[me] = rv;
        const double dv = (double)rv;
        sq = dv * dv;
        mx = fabs(dv);
    }
    if (NORM) block_sum_max(sq, mx, part + 2 * (long long)ex.b);
}

template <typename T, int D, bool NORM, bool STORE>
__global__ __launch_bounds__(256) void k_cell_residual(Geom g, Space sp, const T* __restrict__ u,
                                                       const T* __restrict__ f, T* __restrict__ r,
                                                       const T* __restrict__ bx, const T* __restrict__ by,
                                                       const T* __restrict__ bz, T s,
                                                       double* __restrict__ part) {
    d_cell_residual<T, D, NORM, STORE>(solo_ex(), g, sp, u, f, r, bx, by, bz, s, part);
}

// ------------------------------- 3-D cell grids, coefficients from k on the fly
// On the finest cell level of a variable-coefficient problem every face
// coefficient is the harmonic mean of the two cells' k, ((2 ka) kb) / (ka + kb)
// with ka the lower-index cell (a wall face: the inner cell's k), the very
// operations that form the face arrays on the host, so a face formed here is
// bitwise the stored one.  Reading k of both colours (16 B per updated cell)
// replaces three face arrays read at stride two.  Threads march (x >> 1, y)
// columns of the updated colour over a chunk of planes and keep the other
// colour's u and k on planes z - 1, z, z + 1 in registers; x and y neighbours
// come from the L1 / L2.  The diagonal and off-diagonal sums take the faces
// in the order x-, x+, y-, y+, z-, z+, as cell_sums does.
__device__ __forceinline__ double harm(double ka, double kb) { return ((2.0 * ka) * kb) / (ka + kb); }

// dg, off of the cell with own k `kc` and u/k of its six neighbours (values
// at walls unused); ww: weight of a wall face (2 Dirichlet, 0 Neumann).
template <bool ZERO>
__device__ __forceinline__ void cell_sums_k(double kc, const double (&kn)[6], const double (&un)[6],
                                            const bool (&wall)[6], double ww, double& dg, double& off) {
    double b[6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
        b[i] = wall[i] ? kc : ((i & 1) ? harm(kc, kn[i]) : harm(kn[i], kc));   // odd i: the + face
    dg = wall[0] ? ww * b[0] : b[0];
#pragma unroll
    for (int i = 1; i < 6; ++i) dg = dg + (wall[i] ? ww * b[i] : b[i]);
    if (ZERO) {
        off = 0.0;
        return;
    }
    off = wall[0] ? 0.0 : b[0] * un[0];
#pragma unroll
    for (int i = 1; i < 6; ++i) off = off + (wall[i] ? 0.0 : b[i] * un[i]);
}

// Red-black half-sweep of colour `colour` (me/other: the two colour planes of
// u; km/ko: of k).
template <bool NT, bool ZERO>
__global__ __launch_bounds__(256) void k_cell_gs_zmk(Geom g, ZSpace zs, double* __restrict__ me,
                                                     const double* __restrict__ other,
                                                     const double* __restrict__ f,
                                                     const double* __restrict__ km,
                                                     const double* __restrict__ ko, double s, int colour) {
    const Ex ex = solo_ex();
    int tx, ty, tz;
    zm_tile(zs, ex.b, tx, ty, tz);
    const int xs = tx * 64 + (ex.t & 63);
    const int y = ty * zs.rows + (ex.t >> 6);
    const int N = g.n;
    if (xs >= zs.xr || y >= N) return;
    const int z0 = tz * zs.zc, z1 = min(z0 + zs.zc, N);
    const long long pl = g.plane, pt = g.pitch;
    const double ww = g.neu ? 0.0 : 2.0;
    const bool wym = y == 0, wyp = y == N - 1;
    // neighbour offsets clamped to the cell itself at walls (values unused)
    const long long oym = wym ? 0 : -pt, oyp = wyp ? 0 : pt;
    long long ro = row_off(g, y, z0) + xs;
    // z ring of the other colour: planes z - 1, z, z + 1 at the own position
    double um = 0.0, uc = 0.0, kmz = 0.0, kcz = 0.0;
    if (!ZERO) uc = other[ro];
    kcz = ko[ro];
    if (z0 > 0) {
        if (!ZERO) um = other[ro - pl];
        kmz = ko[ro - pl];
    }
    for (int z = z0; z < z1; ++z, ro += pl) {
        const bool wzm = z == 0, wzp = z == N - 1;
        const long long ozp = wzp ? 0 : pl;
        const double up = ZERO ? 0.0 : other[ro + ozp];
        const double kp = ko[ro + ozp];
        const int par = (y + z + colour) & 1;          // x = 2 xs + par
        const bool wxm = !par && xs == 0, wxp = par && xs == zs.xr - 1;
        // the x neighbour that is not at the own position: x >> 1 - 1 (par 0) or + 1 (par 1)
        const long long ox = par ? (wxp ? 0 : 1) : (wxm ? 0 : -1);
        double kn[6], un[6];
        const double kx = ko[ro + ox];
        kn[0] = par ? kcz : kx;
        kn[1] = par ? kx : kcz;
        kn[2] = ko[ro + oym];
        kn[3] = ko[ro + oyp];
        kn[4] = kmz;
        kn[5] = kp;
        if (!ZERO) {
            const double ux = other[ro + ox];
            un[0] = par ? uc : ux;
            un[1] = par ? ux : uc;
            un[2] = other[ro + oym];
            un[3] = other[ro + oyp];
            un[4] = um;
            un[5] = up;
        } else {
#pragma unroll
            for (int i = 0; i < 6; ++i) un[i] = 0.0;
        }
        const bool wall[6] = {wxm, wxp, wym, wyp, wzm, wzp};
        double dg, off;
        cell_sums_k<ZERO>(km[ro], kn, un, wall, ww, dg, off);
        st_stream<NT>(me + ro, (ld_stream<NT>(f + ro) / s + off) / dg);
        um = uc;
        uc = up;
        kmz = kcz;
        kcz = kp;
    }
}

// r = f - (dg u - off) s at both colours of the thread's column (u, k and f
// in colour-split layout, both colours); NORM: per-block (sum r^2, max |r|).
template <bool NT, bool NORM, bool STORE>
__global__ __launch_bounds__(256) void k_cell_res_zmk(Geom g, ZSpace zs, const double* __restrict__ u,
                                                      const double* __restrict__ f, double* __restrict__ r,
                                                      const double* __restrict__ k, double s,
                                                      double* __restrict__ part) {
    const Ex ex = solo_ex();
    double sq = 0.0, mx = 0.0;
    int tx, ty, tz;
    zm_tile(zs, ex.b, tx, ty, tz);
    const int xs = tx * 64 + (ex.t & 63);
    const int y = ty * zs.rows + (ex.t >> 6);
    const int N = g.n;
    if (xs < zs.xr && y < N) {
        const int z0 = tz * zs.zc, z1 = min(z0 + zs.zc, N);
        const long long pl = g.plane, pt = g.pitch, cs = g.cs;
        const double ww = g.neu ? 0.0 : 2.0;
        const bool wym = y == 0, wyp = y == N - 1;
        const long long oym = wym ? 0 : -pt, oyp = wyp ? 0 : pt;
        long long ro = row_off(g, y, z0) + xs;
        // z rings of both colours (c = 0, 1): u and k on planes z - 1, z
        double um[2], uc[2], kmz[2], kcz[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            uc[c] = u[c * cs + ro];
            kcz[c] = k[c * cs + ro];
            um[c] = z0 > 0 ? u[c * cs + ro - pl] : 0.0;
            kmz[c] = z0 > 0 ? k[c * cs + ro - pl] : 0.0;
        }
        for (int z = z0; z < z1; ++z, ro += pl) {
            const bool wzm = z == 0, wzp = z == N - 1;
            const long long ozp = wzp ? 0 : pl;
            double up[2], kp[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                up[c] = u[c * cs + ro + ozp];
                kp[c] = k[c * cs + ro + ozp];
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {       // the cell of colour c; its neighbours are colour 1 - c
                const int o = 1 - c;
                const long long oc = o * cs + ro;
                const int par = (y + z + c) & 1;
                const bool wxm = !par && xs == 0, wxp = par && xs == zs.xr - 1;
                const long long ox = par ? (wxp ? 0 : 1) : (wxm ? 0 : -1);
                double kn[6], un[6];
                const double kx = k[oc + ox], ux = u[oc + ox];
                kn[0] = par ? kcz[o] : kx;
                kn[1] = par ? kx : kcz[o];
                kn[2] = k[oc + oym];
                kn[3] = k[oc + oyp];
                kn[4] = kmz[o];
                kn[5] = kp[o];
                un[0] = par ? uc[o] : ux;
                un[1] = par ? ux : uc[o];
                un[2] = u[oc + oym];
                un[3] = u[oc + oyp];
                un[4] = um[o];
                un[5] = up[o];
                const bool wall[6] = {wxm, wxp, wym, wyp, wzm, wzp};
                double dg, off;
                cell_sums_k<false>(kcz[c], kn, un, wall, ww, dg, off);
                const double rv = ld_stream<NT>(f + c * cs + ro) - (dg * uc[c] - off) * s;
                if (STORE) st_stream<NT>(r + c * cs + ro, rv);
                sq = sq + rv * rv;
                mx = fmax(mx, fabs(rv));
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                um[c] = uc[c];
                uc[c] = up[c];
                kmz[c] = kcz[c];
                kcz[c] = kp[c];
            }
        }
    }
    if (NORM) block_sum_max(sq, mx, part + 2 * (long long)ex.b);
}

// Residual and the mean of the eight children in one pass on the finest
// 3-D cell level (faces formed from k as in k_cell_res_zmk): thread
// (x >> 1, Y) forms the residuals of fine rows 2Y and 2Y + 1, both colours,
// plane by plane, and adds them into coarse cell (x >> 1, Y, z >> 1) with
// the z offset slowest and the x offset fastest, as the restriction sums
// them.  Each residual takes k_cell_res_zmk's operands in its order, so the
// coarse right-hand side is bitwise that of the two kernels; the fine
// residual is never written.  Chunks hold an even number of planes.
template <bool NT>
__global__ __launch_bounds__(256) void k_cell_res_restrict_zmk(Geom g, Geom gc, ZSpace zs,
                                                               const double* __restrict__ u,
                                                               const double* __restrict__ f,
                                                               const double* __restrict__ k,
                                                               double* __restrict__ fco, double s) {
    const Ex ex = solo_ex();
    int tx, ty, tz;
    zm_tile(zs, ex.b, tx, ty, tz);
    const int xs = tx * 64 + (ex.t & 63);
    const int Y = ty * zs.rows + (ex.t >> 6);
    const int N = g.n;
    if (xs >= zs.xr || 2 * Y >= N) return;
    const int z0 = tz * zs.zc, z1 = min(z0 + zs.zc, N);
    const long long pl = g.plane, pt = g.pitch, cs = g.cs;
    const double ww = g.neu ? 0.0 : 2.0;
    // per fine row j (y = 2Y + j): wall flags, y offsets, row offset, and
    // the z rings of both colours (u and k on planes z - 1, z)
    bool wym[2], wyp[2];
    long long oym[2], oyp[2], ro[2];
    double um[2][2], uc[2][2], kmz[2][2], kcz[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int y = 2 * Y + j;
        wym[j] = y == 0;
        wyp[j] = y == N - 1;
        oym[j] = wym[j] ? 0 : -pt;
        oyp[j] = wyp[j] ? 0 : pt;
        ro[j] = row_off(g, y, z0) + xs;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            uc[j][c] = u[c * cs + ro[j]];
            kcz[j][c] = k[c * cs + ro[j]];
            um[j][c] = z0 > 0 ? u[c * cs + ro[j] - pl] : 0.0;
            kmz[j][c] = z0 > 0 ? k[c * cs + ro[j] - pl] : 0.0;
        }
    }
    double acc = 0.0;
    for (int z = z0; z < z1; ++z) {
        const bool wzm = z == 0, wzp = z == N - 1;
        const long long ozp = wzp ? 0 : pl;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int y = 2 * Y + j;
            double up[2], kp[2], rv[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                up[c] = u[c * cs + ro[j] + ozp];
                kp[c] = k[c * cs + ro[j] + ozp];
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int o = 1 - c;
                const long long oc = o * cs + ro[j];
                const int par = (y + z + c) & 1;
                const bool wxm = !par && xs == 0, wxp = par && xs == zs.xr - 1;
                const long long ox = par ? (wxp ? 0 : 1) : (wxm ? 0 : -1);
                double kn[6], un[6];
                const double kx = k[oc + ox], ux = u[oc + ox];
                kn[0] = par ? kcz[j][o] : kx;
                kn[1] = par ? kx : kcz[j][o];
                kn[2] = k[oc + oym[j]];
                kn[3] = k[oc + oyp[j]];
                kn[4] = kmz[j][o];
                kn[5] = kp[o];
                un[0] = par ? uc[j][o] : ux;
                un[1] = par ? ux : uc[j][o];
                un[2] = u[oc + oym[j]];
                un[3] = u[oc + oyp[j]];
                un[4] = um[j][o];
                un[5] = up[o];
                const bool wall[6] = {wxm, wxp, wym[j], wyp[j], wzm, wzp};
                double dg, off;
                cell_sums_k<false>(kcz[j][c], kn, un, wall, ww, dg, off);
                rv[c] = ld_stream<NT>(f + c * cs + ro[j]) - (dg * uc[j][c] - off) * s;
            }
            // x offset 0 is the colour with (y + z + c) even
            const int c0 = (y + z) & 1;
            acc = ((z & 1) == 0 && j == 0) ? rv[c0] : acc + rv[c0];
            acc = acc + rv[1 - c0];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                um[j][c] = uc[j][c];
                uc[j][c] = up[c];
                kmz[j][c] = kcz[j][c];
                kcz[j][c] = kp[c];
            }
            ro[j] += pl;
        }
        if (z & 1) {
            const int Z = z >> 1;
            fco[(long long)((xs + Y + Z) & 1) * gc.cs + row_off(gc, Y, Z) + (xs >> 1)] = acc * 0.125;
        }
    }
}

// Mean of the 2^d children, summed with the z offset slowest, then scaled, at
// coarse cell p of the fine values rf(colour, x >> 1, y, z).
template <typename T, int D, typename RF>
__device__ __forceinline__ bool pt_cell_restrict_by(const Pt& p, const Geom& gc, RF&& rf, T* __restrict__ fcoarse) {
    const int par = (p.y + p.z + p.c) & 1;
    const int X = 2 * p.xs + par, Y = p.y, Z = p.z;
    T acc = T(0);
    bool first = true;
#pragma unroll
    for (int oz = 0; oz <= (D == 3 ? 1 : 0); ++oz) {
#pragma unroll
        for (int oy = 0; oy <= 1; ++oy) {
#pragma unroll
            for (int ox = 0; ox <= 1; ++ox) {
                const int fx = 2 * X + ox, fy = 2 * Y + oy, fz = (D == 3) ? 2 * Z + oz : 0;
                const T v = rf((fx + fy + fz) & 1, fx >> 1, fy, fz);
                acc = first ? v : acc + v;
                first = false;
            }
        }
    }
    fcoarse[(long long)p.c * gc.cs + row_off(gc, Y, Z) + p.xs] = acc * T(D == 3 ? 0.125 : 0.25);
    return true;
}

template <typename T, int D>
__device__ __forceinline__ void pt_cell_restrict(const Pt& p, Geom gf, Geom gc, Space sp,
                                                       const T* __restrict__ r,
                                                       T* __restrict__ fcoarse) {
    pt_cell_restrict_by<T, D>(p, gc, [&](int c, int xs, int y, int z) -> T {
        return r[(long long)c * gf.cs + row_off(gf, y, z) + xs];
    }, fcoarse);
}

// Residual and the mean of the 2^d children in one launch over the coarse
// cells of a level with stored face coefficients: each coarse cell forms
// the residuals of its own children (each fine cell belongs to exactly one
// coarse cell: no residual is formed twice), with the residual kernel's
// operands and order, summed as the restriction sums them (bitwise equal to
// the two kernels; the fine residual is never written).
template <typename T, int D>
__global__ __launch_bounds__(256) void k_cell_res_restrict_pt(Geom gf, Geom gc, Space sp, const T* __restrict__ u,
                                                              const T* __restrict__ f, const T* __restrict__ bx,
                                                              const T* __restrict__ by, const T* __restrict__ bz,
                                                              T* __restrict__ fcoarse, T s) {
    Pt p;
    if (!map_point(solo_ex(), sp, p)) return;
    pt_cell_restrict_by<T, D>(p, gc, [&](int c, int xs, int y, int z) -> T {
        Pt q;
        q.xs = xs;
        q.y = y;
        q.z = z;
        q.c = c;
        long long me;
        return pt_cell_residual<T, D>(q, gf, u, f, bx, by, bz, s, me);
    }, fcoarse);
}

template <typename T, int D>
__device__ __forceinline__ void d_cell_restrict(const Ex& ex, Geom gf, Geom gc, Space sp,
                                                       const T* __restrict__ r,
                                                       T* __restrict__ fcoarse) {
    Pt p;
    if (!map_point(ex, sp, p)) return;
    pt_cell_restrict<T, D>(p, gf, gc, sp, r, fcoarse);
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_cell_restrict(Geom gf, Geom gc, Space sp,
                                                       const T* __restrict__ r,
                                                       T* __restrict__ fcoarse) {
    d_cell_restrict<T, D>(solo_ex(), gf, gc, sp, r, fcoarse);
}

// Cell-centred linear interpolation: per axis fine(2I) = 3/4 e[I] + 1/4 e[I-1],
// fine(2I+1) = 3/4 e[I] + 1/4 e[I+1], ghost -e[I] (Dirichlet) or e[I]
// (Neumann) beyond a wall; x first, then y, then z; then u += P e.
template <typename T, int D>
__device__ __forceinline__ void pt_cell_prolong(const Pt& p, Geom gf, Geom gc, Space sp, T* __restrict__ u,
                                                      const T* __restrict__ ec) {
    const int par = (p.y + p.z + p.c) & 1;
    const int x = 2 * p.xs + par, y = p.y, z = p.z;
    const int Nc = gc.n;
    const T a = T(0.75), b = T(0.25);
    const int I = x >> 1, In = (x & 1) ? I + 1 : I - 1;
    const int J = y >> 1, Jn = (y & 1) ? J + 1 : J - 1;
    const int K = z >> 1, Kn = (z & 1) ? K + 1 : K - 1;
    const bool wI = In < 0 || In >= Nc, wJ = Jn < 0 || Jn >= Nc, wK = Kn < 0 || Kn >= Nc;
    const T sg = gc.neu ? T(1) : T(-1);
    auto E = [&](int X, int Y, int Z) -> T {
        return ec[(long long)((X + Y + Z) & 1) * gc.cs + row_off(gc, Y, Z) + (X >> 1)];
    };
    auto ix = [&](int Y, int Z) -> T {
        const T c0 = E(I, Y, Z);
        const T c1 = wI ? sg * c0 : E(In, Y, Z);
        return a * c0 + b * c1;
    };
    auto iy = [&](int Z) -> T {
        const T c0 = ix(J, Z);
        const T c1 = wJ ? sg * c0 : ix(Jn, Z);
        return a * c0 + b * c1;
    };
    T e;
    if (D == 3) {
        const T c0 = iy(K);
        const T c1 = wK ? sg * c0 : iy(Kn);
        e = a * c0 + b * c1;
    } else {
        e = iy(0);
    }
    const long long me = (long long)p.c * gf.cs + row_off(gf, y, z) + p.xs;
    u[me] = u[me] + e;
}

// Cell-centred interpolation + correction on large 3-D cell levels, one
// thread per (x >> 1, y) column of one colour marching a chunk of planes.
// Along the column the fine x parity alternates with z, so plane 2K uses the
// coarse planes K and K - 1 at one parity and plane 2K + 1 the planes K and
// K + 1 at the other: each y-interpolated coarse value serves two fine planes
// and is formed once (half the coarse loads of the point kernel).  Every fine
// cell takes pt_cell_prolong's operands in its order (bitwise equal).
template <typename T>
__global__ __launch_bounds__(256) void k_cell_prolong_zm(Geom gf, Geom gc, ZSpace zs, int colour,
                                                         T* __restrict__ u, const T* __restrict__ ec) {
    int tx, ty, tz;
    zm_tile(zs, (int)blockIdx.x, tx, ty, tz);
    const int xs = tx * 64 + (int)threadIdx.x;
    const int y = ty * zs.rows + (int)threadIdx.y;
    if (xs >= zs.xr || y >= gf.n) return;
    const int z0 = tz * zs.zc, z1 = min(z0 + zs.zc, gf.n);
    const int Nc = gc.n;
    const T a = T(0.75), b = T(0.25);
    const T sg = gc.neu ? T(1) : T(-1);
    const int J = y >> 1, Jn = (y & 1) ? J + 1 : J - 1;
    const bool wJ = Jn < 0 || Jn >= Nc;
    const int pe = (y + colour) & 1, po = 1 - pe;   // x parity on even and odd planes
    auto E = [&](int X, int Y, int Z) -> T {
        return ec[(long long)((X + Y + Z) & 1) * gc.cs + row_off(gc, Y, Z) + (X >> 1)];
    };
    // x- then y-interpolated coarse value of plane Z for x parity p
    auto iyp = [&](int Z, int p) -> T {
        const int In = p ? xs + 1 : xs - 1;
        const bool wI = In < 0 || In >= Nc;
        auto ix = [&](int Y) -> T {
            const T c0 = E(xs, Y, Z);
            const T c1 = wI ? sg * c0 : E(In, Y, Z);
            return a * c0 + b * c1;
        };
        const T c0 = ix(J);
        const T c1 = wJ ? sg * c0 : ix(Jn);
        return a * c0 + b * c1;
    };
    const long long pl = gf.plane;
    const long long ro0 = (long long)colour * gf.cs + row_off(gf, y, z0) + xs;
    // the column's iterate for the whole chunk, loaded before any store
    T uv[kZChunk];
#pragma unroll
    for (int k = 0; k < kZChunk; ++k) uv[k] = z0 + k < z1 ? u[ro0 + k * pl] : T(0);
    int K = z0 >> 1;
    T ecur = iyp(K, pe);
    T eprev = K >= 1 ? iyp(K - 1, pe) : T(0);
    T ocur = iyp(K, po);
#pragma unroll
    for (int k = 0; k < kZChunk; k += 2, ++K) {
        if (z0 + k >= z1) break;
        {   // plane 2K: coarse K and K - 1
            const T c0 = ecur;
            const T c1 = K - 1 < 0 ? sg * c0 : eprev;
            u[ro0 + k * pl] = uv[k] + (a * c0 + b * c1);
        }
        const bool top = K + 1 >= Nc;
        const T onext = top ? T(0) : iyp(K + 1, po);
        {   // plane 2K + 1: coarse K and K + 1
            const T c0 = ocur;
            const T c1 = top ? sg * c0 : onext;
            u[ro0 + (k + 1) * pl] = uv[k + 1] + (a * c0 + b * c1);
        }
        eprev = ecur;
        ecur = top ? T(0) : iyp(K + 1, pe);
        ocur = onext;
    }
}

template <typename T, int D>
__device__ __forceinline__ void d_cell_prolong(const Ex& ex, Geom gf, Geom gc, Space sp, T* __restrict__ u,
                                                      const T* __restrict__ ec) {
    Pt p;
    if (!map_point(ex, sp, p)) return;
    pt_cell_prolong<T, D>(p, gf, gc, sp, u, ec);
}

template <typename T, int D>
__global__ __launch_bounds__(256) void k_cell_prolong(Geom gf, Geom gc, Space sp, T* __restrict__ u,
                                                      const T* __restrict__ ec) {
    d_cell_prolong<T, D>(solo_ex(), gf, gc, sp, u, ec);
}

// ------------------------------------------------------ coarsest, reductions
// Exact coarsest solve: gather the m unknowns (C order), L y = b and
// L^T x = y column by column in FP64, scatter x.  One block of 64 threads.
template <typename T>
__device__ __forceinline__ void d_coarse(const Ex& ex, Geom g, const T* __restrict__ f, T* __restrict__ u,
                                               const double* __restrict__ L, int m) {
    __shared__ double b[64];
    const int t = ex.t;
    const int side = g.cell ? g.n : g.n - 2, off = g.cell ? 0 : 1;
    long long idx = 0;
    if (t < m) {
        const int x = t % side + off, y = (t / side) % side + off;
        const int z = (g.dim == 3) ? t / (side * side) + off : 0;
        idx = (long long)((x + y + z) & 1) * g.cs + row_off(g, y, z) + (x >> 1);
        b[t] = (double)f[idx];
    }
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (t == j) b[j] = b[j] / L[j * m + j];
        __syncthreads();
        if (t > j && t < m) b[t] = b[t] - L[t * m + j] * b[j];
        __syncthreads();
    }
    for (int j = m - 1; j >= 0; --j) {
        if (t == j) b[j] = b[j] / L[j * m + j];
        __syncthreads();
        if (t < j) b[t] = b[t] - L[j * m + t] * b[j];
        __syncthreads();
    }
    if (t < m) u[idx] = (T)b[t];
}

template <typename T>
__global__ __launch_bounds__(64) void k_coarse(Geom g, const T* __restrict__ f, T* __restrict__ u,
                                               const double* __restrict__ L, int m) {
    d_coarse<T>(solo_ex(), g, f, u, L, m);
}

// ------------------------------------------- coarse levels in one workgroup
// The V-cycle from level lg[0] down to the coarsest and back, run by one
// workgroup on LDS copies of the levels' fields: each operation is the
// per-level kernels' point function, wavefronts taking rows of the level
// in turn, so every point takes the same operands in the same order as in
// the separate launches (and in the oracle); a barrier separates operations.
// Small levels otherwise cost a launch per operation for a few hundred
// points each.
// Every point of a space: a wavefront covers 64 >> lx consecutive rows with
// 1 << lx lanes each (lx = the space's x tiling, log2 of xr rounded up, at
// most 6); the row groups (y block fastest, then plane, then colour) are
// split into 16 contiguous runs, one per wavefront, which steps through its
// run with increments instead of divisions (the uniform index arithmetic
// otherwise dominates these small passes).
template <typename F>
__device__ __forceinline__ void tail_points(const Space& sp, F&& fn) {
    const int lane = (int)threadIdx.x & 63;
    const int lg = sp.lx, rpw = 64 >> lg;
    const int nyb = (sp.yr + rpw - 1) / rpw;
    const int groups = nyb * sp.zr * sp.ncol;
    constexpr int W = kTailThreads / 64;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int per = (groups + W - 1) / W;
    const int g0 = w * per, g1 = min(g0 + per, groups);
    if (g0 >= g1) return;
    int yb = g0 % nyb, t = g0 / nyb;
    int z = t % sp.zr, c = t / sp.zr;
    const int ylane = lane >> lg, x0 = lane & ((1 << lg) - 1);
    for (int b = g0; b < g1; ++b) {
        const int y = yb * rpw + ylane;
        if (y < sp.yr) {
            Pt p;
            p.y = sp.y0 + y;
            p.z = sp.z0 + z;
            p.c = sp.col0 + c;
            for (p.xs = x0; p.xs < sp.xr; p.xs += 1 << lg) fn(p);
        }
        if (++yb == nyb) {
            yb = 0;
            if (++z == sp.zr) {
                z = 0;
                ++c;
            }
        }
    }
}

// Coarsest solve in LDS by the first wavefront: lane t holds b[t] in a
// register, the factor L (m x m, row major) sits in LDS; forward and
// backward substitution take the same operations in the same order as
// d_coarse.
template <typename T>
__device__ __forceinline__ void tail_coarse(const Geom& g, const T* __restrict__ f, T* __restrict__ u,
                                            const double* __restrict__ L, int m) {
    if (threadIdx.x >= 64) return;
    const int t = (int)threadIdx.x;
    const int side = g.cell ? g.n : g.n - 2, off = g.cell ? 0 : 1;
    long long idx = 0;
    double bt = 0.0;
    if (t < m) {
        const int x = t % side + off, y = (t / side) % side + off;
        const int z = (g.dim == 3) ? t / (side * side) + off : 0;
        idx = (long long)((x + y + z) & 1) * g.cs + row_off(g, y, z) + (x >> 1);
        bt = (double)f[idx];
    }
    for (int j = 0; j < m; ++j) {
        if (t == j) bt = bt / L[j * m + j];
        const double bj = __shfl(bt, j, 64);
        if (t > j && t < m) bt = bt - L[t * m + j] * bj;
    }
    for (int j = m - 1; j >= 0; --j) {
        if (t == j) bt = bt / L[j * m + j];
        const double bj = __shfl(bt, j, 64);
        if (t < j) bt = bt - L[j * m + t] * bj;
    }
    if (t < m) u[idx] = (T)bt;
}

// Copy a node field between two colour-split layouts of the same level
// (device memory and LDS rows of `half` entries).
template <typename T>
__device__ __forceinline__ void tail_copy(const Geom& gs, const T* __restrict__ src, const Geom& gd,
                                          T* __restrict__ dst) {
    const int lane = (int)threadIdx.x & 63;
    constexpr int W = kTailThreads / 64;
    const int rows = 2 * gs.nz * gs.ny;
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int per = (rows + W - 1) / W;
    const int r0 = w * per, r1 = min(r0 + per, rows);
    if (r0 >= r1) return;
    int y = r0 % gs.ny, t = r0 / gs.ny;
    int z = t % gs.nz, c = t / gs.nz;
    for (int r = r0; r < r1; ++r) {
        const long long so = (long long)c * gs.cs + (long long)z * gs.plane + (long long)y * gs.pitch;
        const long long d = (long long)c * gd.cs + (long long)z * gd.plane + (long long)y * gd.pitch;
        for (int xs = lane; xs < gs.half; xs += 64) dst[d + xs] = src[so + xs];
        if (++y == gs.ny) {
            y = 0;
            if (++z == gs.nz) {
                z = 0;
                ++c;
            }
        }
    }
}

template <typename T, int D, bool CELL>
__device__ void tail_smooth(const TailPlan& P, T* A, unsigned& sw, int i, int sweeps, bool zero, int c0,
                            bool first_done = false) {
    const Geom g = P.lg[i];
    const T s = (T)P.s[i];
    const T rs = (T)P.rs[i];   // exact when P.p2
    const T* f = A + P.of[i];
    const T* bx = static_cast<const T*>(P.beta[i][0]);
    const T* by = static_cast<const T*>(P.beta[i][1]);
    const T* bz = static_cast<const T*>(P.beta[i][2]);
    // first_done: the first sweep's first (pointwise, from zero) operation
    // already ran with the restriction into this level
    for (int k = (first_done && !P.rbgs) ? 1 : 0; k < sweeps; ++k) {
        const bool z = zero && k == 0;
        T* u = A + (((sw >> i) & 1u) ? P.ob[i] : P.oa[i]);
        if (P.rbgs) {
            for (int h = (first_done && k == 0) ? 1 : 0; h < 2; ++h) {
                const int c = h == 0 ? c0 : 1 - c0;
                const Space sp = P.one[i][c];
                T* me = u + (long long)c * g.cs;
                const T* other = u + (long long)(1 - c) * g.cs;
                const T* fc = f + (long long)c * g.cs;
                if constexpr (CELL) {
                    if (z && h == 0)
                        tail_points(sp, [&](const Pt& p) {
                            pt_cell_gs<T, D, true>(p, g, sp, me, other, fc, bx, by, bz, s);
                        });
                    else
                        tail_points(sp, [&](const Pt& p) {
                            pt_cell_gs<T, D, false>(p, g, sp, me, other, fc, bx, by, bz, s);
                        });
                } else {
                    if (z && h == 0)
                        tail_points(sp, [&](const Pt& p) {
                            if (P.p2) pt_node_gs<T, D, true, true>(p, g, sp, me, other, fc, s, rs);
                            else pt_node_gs<T, D, true>(p, g, sp, me, other, fc, s);
                        });
                    else
                        tail_points(sp, [&](const Pt& p) {
                            if (P.p2) pt_node_gs<T, D, false, true>(p, g, sp, me, other, fc, s, rs);
                            else pt_node_gs<T, D, false>(p, g, sp, me, other, fc, s);
                        });
                }
                __syncthreads();
            }
        } else {
            T* out = A + (((sw >> i) & 1u) ? P.oa[i] : P.ob[i]);
            const Space sp = P.all[i];
            const T om = (T)P.omega;
            if constexpr (CELL) {
                if (z)
                    tail_points(sp, [&](const Pt& p) {
                        pt_cell_jacobi<T, D, true>(p, g, sp, u, f, out, bx, by, bz, s, om);
                    });
                else
                    tail_points(sp, [&](const Pt& p) {
                        pt_cell_jacobi<T, D, false>(p, g, sp, u, f, out, bx, by, bz, s, om);
                    });
            } else {
                if (P.p2) {
                    if (z)
                        tail_points(sp, [&](const Pt& p) {
                            pt_node_jacobi<T, D, true, true>(p, g, sp, u, f, out, s, om, rs);
                        });
                    else
                        tail_points(sp, [&](const Pt& p) {
                            pt_node_jacobi<T, D, false, true>(p, g, sp, u, f, out, s, om, rs);
                        });
                } else {
                    if (z)
                        tail_points(sp, [&](const Pt& p) { pt_node_jacobi<T, D, true>(p, g, sp, u, f, out, s, om); });
                    else
                        tail_points(sp, [&](const Pt& p) { pt_node_jacobi<T, D, false>(p, g, sp, u, f, out, s, om); });
                }
            }
            __syncthreads();
            sw ^= 1u << i;
        }
    }
}

template <typename T, int D, bool CELL>
__global__ __launch_bounds__(kTailThreads) void k_tail(TailPlan P, const T* __restrict__ f0, T* __restrict__ u0) {
    __shared__ double arena[kTailLdsBytes / 8];
    T* A = reinterpret_cast<T*>(arena);
    for (int i = (int)threadIdx.x; i < P.elems; i += kTailThreads) A[i] = T(0);
    // the coarsest factor after the fields (8-byte aligned)
    double* Ls = arena + (P.elems * (int)sizeof(T) + 7) / 8;
    for (int i = (int)threadIdx.x; i < P.m * P.m; i += kTailThreads) Ls[i] = P.chol[i];
    __syncthreads();
    tail_copy<T>(P.g0, f0, P.lg[0], A + P.of[0]);
    if (!P.from_zero) tail_copy<T>(P.g0, u0, P.lg[0], A + P.oa[0]);
    __syncthreads();
    unsigned sw = 0;   // bit i set: level i's iterate is in its second buffer
    const int last = P.nl - 1;
    bool first_done = false;
    for (int i = 0; i < last; ++i) {
        tail_smooth<T, D, CELL>(P, A, sw, i, P.nu1, i > 0 || P.from_zero, 0, first_done);
        // the residual of level i restricted to level i + 1 and, when level
        // i + 1 is smoothed before its own restriction, that smoothing's
        // first operation, pointwise from zero, at the same coarse point
        const Geom g = P.lg[i], gc = P.lg[i + 1];
        const T* u = A + (((sw >> i) & 1u) ? P.ob[i] : P.oa[i]);
        const T* f = A + P.of[i];
        const T s = (T)P.s[i];
        const Space sc = P.all[i + 1];
        T* fco = A + P.of[i + 1];
        const bool pre = i + 1 < last && P.nu1 > 0;
        T* uc = A + P.oa[i + 1];           // level i + 1 is untouched: its iterate is in oa
        T* oc = A + P.ob[i + 1];
        const T sc1 = (T)P.s[i + 1], om = (T)P.omega;
        if constexpr (CELL) {
            const T* bx = static_cast<const T*>(P.beta[i][0]);
            const T* by = static_cast<const T*>(P.beta[i][1]);
            const T* bz = static_cast<const T*>(P.beta[i][2]);
            const T* cx = static_cast<const T*>(P.beta[i + 1][0]);
            const T* cy = static_cast<const T*>(P.beta[i + 1][1]);
            const T* cz = static_cast<const T*>(P.beta[i + 1][2]);
            // (cell residuals read six faces from device memory each: stored
            // once by their own pass rather than formed eight times per
            // coarse cell)
            T* r = A + (((sw >> i) & 1u) ? P.oa[i] : P.ob[i]);
            const Space sa = P.all[i];
            tail_points(sa, [&](const Pt& p) {
                long long me;
                const T rv = pt_cell_residual<T, D>(p, g, u, f, bx, by, bz, s, me);
                r[me] = rv;
            });
            __syncthreads();
            tail_points(sc, [&](const Pt& p) {
                pt_cell_restrict_by<T, D>(p, gc, [&](int c, int xs, int y, int z) -> T {
                    return r[(long long)c * g.cs + row_off(g, y, z) + xs];
                }, fco);
                if (!pre) return;
                if (P.rbgs) {
                    if (p.c == 0) pt_cell_gs<T, D, true>(p, gc, sc, uc, uc + gc.cs, fco, cx, cy, cz, sc1);
                } else {
                    pt_cell_jacobi<T, D, true>(p, gc, sc, uc, fco, oc, cx, cy, cz, sc1, om);
                }
            });
        } else {
            // 2-D: the residual formed as the restriction needs it (nine
            // terms per coarse point); 3-D: stored once by its own pass (27
            // terms per coarse point measured slower than the extra pass)
            T* r = A + (((sw >> i) & 1u) ? P.oa[i] : P.ob[i]);
            if constexpr (D == 3) {
                const Space sa = P.all[i];
                tail_points(sa, [&](const Pt& p) {
                    long long me;
                    T rv;
                    if (pt_node_residual<T, D>(p, g, u, f, s, me, rv)) r[me] = rv;
                });
                __syncthreads();
            }
            tail_points(sc, [&](const Pt& p) {
                const bool in = pt_node_restrict_by<T, D>(p, gc, [&](int c, int xs, int y, int z) -> T {
                    if constexpr (D == 3) {
                        return r[(long long)c * g.cs + row_off(g, y, z) + xs];
                    } else {
                        Pt q;
                        q.xs = xs;
                        q.y = y;
                        q.z = z;
                        q.c = c;
                        long long me;
                        T rv = T(0);
                        pt_node_residual<T, D>(q, g, u, f, s, me, rv);
                        return rv;
                    }
                }, fco);
                if (!in || !pre) return;
                if (P.rbgs) {
                    if (p.c == 0) {
                        if (P.p2) pt_node_gs<T, D, true, true>(p, gc, sc, uc, uc + gc.cs, fco, sc1, (T)P.rs[i + 1]);
                        else pt_node_gs<T, D, true>(p, gc, sc, uc, uc + gc.cs, fco, sc1);
                    }
                } else {
                    if (P.p2) pt_node_jacobi<T, D, true, true>(p, gc, sc, uc, fco, oc, sc1, om, (T)P.rs[i + 1]);
                    else pt_node_jacobi<T, D, true>(p, gc, sc, uc, fco, oc, sc1, om);
                }
            });
        }
        __syncthreads();
        if (pre && !P.rbgs) sw ^= 1u << (i + 1);
        first_done = pre;
    }
    tail_coarse<T>(P.lg[last], A + P.of[last], A + P.oa[last], Ls, P.m);
    __syncthreads();
    for (int i = last - 1; i >= 0; --i) {
        const Geom g = P.lg[i], gc = P.lg[i + 1];
        T* u = A + (((sw >> i) & 1u) ? P.ob[i] : P.oa[i]);
        const T* e = A + (((sw >> (i + 1)) & 1u) ? P.ob[i + 1] : P.oa[i + 1]);
        const Space sp = P.pro[i];
        if constexpr (CELL)
            tail_points(sp, [&](const Pt& p) { pt_cell_prolong<T, D>(p, g, gc, sp, u, e); });
        else
            tail_points(sp, [&](const Pt& p) { pt_node_prolong<T, D>(p, g, gc, sp, u, e); });
        __syncthreads();
        tail_smooth<T, D, CELL>(P, A, sw, i, P.nu2, false, P.post_order);
    }
    tail_copy<T>(P.lg[0], A + ((sw & 1u) ? P.ob[0] : P.oa[0]), P.g0, u0);
}

__device__ __forceinline__ void d_reduce(const Ex& ex, const double* __restrict__ in, long long count,
                                                double* __restrict__ out, double* mx_copy = nullptr) {
    const long long i0 = (long long)ex.b * kReduceChunk;
    const long long i1 = i0 + kReduceChunk < count ? i0 + kReduceChunk : count;
    double sq = 0.0, mx = 0.0;
    for (long long i = i0 + ex.t; i < i1; i += ex.nt) {
        sq = sq + in[2 * i];
        mx = fmax(mx, in[2 * i + 1]);
    }
    block_sum_max(sq, mx, out + 2 * (long long)ex.b, mx_copy);
}

__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ in, long long count,
                                                double* __restrict__ out, double* mx_copy,
                                                const double* __restrict__ move_src, double* __restrict__ move_dst) {
    d_reduce(solo_ex(), in, count, out, mx_copy);
    if (move_dst && blockIdx.x == 0 && threadIdx.x == 0) *move_dst = *move_src;
}

// ------------------------------------------------------ layout conversion
__device__ __forceinline__ bool nat_to_split(const Geom& g, long long i, long long& s) {
    const int n = g.n;
    const int x = (int)(i % n);
    const int y = (int)((i / n) % n);
    const int z = g.dim == 3 ? (int)(i / ((long long)n * n)) : 0;
    s = (long long)((x + y + z) & 1) * g.cs + row_off(g, y, z) + (x >> 1);
    if (g.cell) return true;
    const bool bx = x == 0 || x == n - 1, by = y == 0 || y == n - 1;
    const bool bz = g.dim == 3 && (z == 0 || z == n - 1);
    return !(bx || by || bz);
}

template <typename T>
__device__ __forceinline__ void d_pack(const Ex& ex, Geom g, long long total, const double* __restrict__ nat,
                                              T* __restrict__ split) {
    const long long i = (long long)ex.b * ex.nt + ex.t;
    if (i >= total) return;
    long long s;
    if (nat_to_split(g, i, s)) split[s] = (T)nat[i];
}

template <typename T>
__global__ __launch_bounds__(256) void k_pack(Geom g, long long total, const double* __restrict__ nat,
                                              T* __restrict__ split) {
    d_pack<T>(solo_ex(), g, total, nat, split);
}

template <typename T>
__device__ __forceinline__ void d_unpack(const Ex& ex, Geom g, long long total, const T* __restrict__ split,
                                                double* __restrict__ nat) {
    const long long i = (long long)ex.b * ex.nt + ex.t;
    if (i >= total) return;
    long long s;
    nat[i] = nat_to_split(g, i, s) ? (double)split[s] : 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_unpack(Geom g, long long total, const T* __restrict__ split,
                                                double* __restrict__ nat) {
    d_unpack<T>(solo_ex(), g, total, split, nat);
}

// ------------------------------------------------------ mixed precision
__device__ __forceinline__ double pow2_floor(double v) {
    if (!(v > 0.0)) return 1.0;
    int e;
    frexp(v, &e);              // v = m 2^e, m in [0.5, 1)
    return ldexp(1.0, e - 1);
}

// The cast and the update run over whole level fields as flat streams, four
// elements per thread: boundary nodes and row padding of r64 and of the
// single-precision iterate are zero and stay zero, so a flat pass computes
// the same values at every unknown as a pass over the unknowns.
__device__ __forceinline__ void d_cast(const Ex& ex, long long n4, const double* __restrict__ r,
                                       float* __restrict__ f32, const double* __restrict__ red,
                                       double* __restrict__ sigma_out) {
    const double sigma = pow2_floor(red[1]);
    if (ex.b == 0 && ex.t == 0) *sigma_out = sigma;
    const long long i = (long long)ex.b * ex.nt + ex.t;
    if (i >= n4) return;
    const double2 a = reinterpret_cast<const double2*>(r)[2 * i];
    const double2 b = reinterpret_cast<const double2*>(r)[2 * i + 1];
    float4 o;
    o.x = (float)(a.x / sigma);
    o.y = (float)(a.y / sigma);
    o.z = (float)(b.x / sigma);
    o.w = (float)(b.y / sigma);
    reinterpret_cast<float4*>(f32)[i] = o;
}

// The residual and the cast of a refinement step in one pass: sigma comes
// from the previous residual's maximum (*basis), so it is known before r is.
template <int U, bool NT>
__global__ __launch_bounds__(1024) void k_node_res_cast_zm(Geom g, ZSpace zs, const double* __restrict__ u,
                                                           const double* __restrict__ f, float* __restrict__ r32,
                                                           double s, const double* __restrict__ basis,
                                                           double* __restrict__ sigma_out,
                                                           double* __restrict__ part) {
    const double sigma = pow2_floor(basis[0]);
    const Ex ex = solo_ex();
    if (ex.b == 0 && ex.t == 0) *sigma_out = sigma;
    d_node_res_zm<double, U, NT, true, true, true>(ex, g, zs, u, f, nullptr, s, part, r32, sigma);
}

// The update of one refinement step and the residual and cast of the next in
// one pass (3-D node levels): u' = u + sigma_old fl64(c) is formed once per
// point and plane, written out of place (a block's neighbours still read
// the old iterate at its halo), and the residual of u', fl32(r / sigma_new)
// and the norm partials follow.  A block is 64 positions of x >> 1 by
// kUrRows rows plus one halo row on either side (threads that only form
// u'), marching a chunk of planes; the current plane of u' (both colours,
// with one halo position left and right, formed by the edge lanes) sits in
// LDS for the x and y neighbours, planes z - 1 and z + 1 of the thread's own
// column in registers, and the next plane's loads are issued one step
// ahead across LDS-only barriers.  Every value takes the operations of the
// separate update, residual and cast in their order (neighbours x-, x+, y-,
// y+, z-, z+), so the iterate and the cast are bitwise theirs.  sigma_old is
// red[2] (the scale of the cast that made c's right-hand side), sigma_new =
// 2^floor(log2 red[3]) goes to red[5] (moved to red[2] by the reduction that
// follows, once every block has read the old one).
constexpr int kUrRows = 14;
constexpr int kUrChunk = 16;

template <bool NT>
__global__ __launch_bounds__(64 * (kUrRows + 2)) void k_node_upd_res_cast(
    Geom g, int ntx, int nty, int zc, const double* __restrict__ u, const float* __restrict__ c32,
    const double* __restrict__ f, double* __restrict__ uo, float* __restrict__ r32, double s,
    double* __restrict__ red, double* __restrict__ part) {
    __shared__ double pl[2][2][kUrRows + 2][66];
    const Ex ex = solo_ex();
    const int lane = (int)threadIdx.x, row = (int)threadIdx.y;
    const int tx = ex.b % ntx, rest = ex.b / ntx;
    const int ty = rest % nty, tz = rest / nty;
    const int xr = (g.n - 1) / 2;
    const int xs = tx * 64 + lane;
    const int y = ty * kUrRows + row;                 // row 0: the halo row below the block
    const int z0 = 1 + tz * zc;
    const int z1 = min(z0 + zc, g.n - 1);
    const double so = red[2];
    const double sn = pow2_floor(red[3]);
    if (ex.b == 0 && ex.t == 0) red[5] = sn;
    const long long cs = g.cs, plane = g.plane;
    const bool inrow = y <= g.n - 1;
    const bool interior = row >= 1 && row <= kUrRows && y <= g.n - 2 && xs < xr;
    // the edge lanes also form the halo positions xs - 1 (lane 0) and xs + 1 (lane 63)
    const int hx = lane == 0 ? xs - 1 : xs + 1;
    const bool edge = (lane == 0 || lane == 63) && inrow && hx >= 0 && hx <= xr;
    const bool own = inrow && xs <= xr;
    const long long ro = (long long)y * g.pitch + xs;
    const long long rh = (long long)y * g.pitch + hx;
    const int hcol = lane == 0 ? 0 : 65;
    // raw loads of one plane: own position and halo position, both colours
    double uR = 0.0, uB = 0.0, hR = 0.0, hB = 0.0;
    float cR = 0.f, cB = 0.f, gR = 0.f, gB = 0.f;
    auto load = [&](int zq) {
        const long long o = (long long)zq * plane + ro;
        if (own) {
            uR = u[o];
            uB = u[cs + o];
            cR = c32[o];
            cB = c32[cs + o];
        }
        if (edge) {
            const long long oh = (long long)zq * plane + rh;
            hR = u[oh];
            hB = u[cs + oh];
            gR = c32[oh];
            gB = c32[cs + oh];
        }
    };
    // u' of the loaded plane into LDS buffer b (and, for the own position, registers)
    double vR = 0.0, vB = 0.0;
    auto form = [&](int b) {
        vR = uR + so * (double)cR;
        vB = uB + so * (double)cB;
        pl[b][0][row][lane + 1] = vR;
        pl[b][1][row][lane + 1] = vB;
        if (lane == 0 || lane == 63) {
            pl[b][0][row][hcol] = edge ? hR + so * (double)gR : 0.0;
            pl[b][1][row][hcol] = edge ? hB + so * (double)gB : 0.0;
        }
    };
    double sq = 0.0, mx = 0.0;
    // planes z0 - 1 and z0
    load(z0 - 1);
    form(1);
    double pR = vR, pB = vB;
    load(z0);
    form(0);
    double qR = vR, qB = vB;           // plane z
    double fR = 0.0, fB = 0.0;
    if (interior) {
        fR = ld_stream<NT>(f + (long long)z0 * plane + ro);
        fB = ld_stream<NT>(f + cs + (long long)z0 * plane + ro);
    }
    load(z0 + 1);
    lds_barrier();
    for (int z = z0; z < z1; ++z) {
        const int b = (z - z0) & 1;
        // u' of plane z + 1 (loaded one step ahead) into the other buffer
        form(b ^ 1);
        const double nR = vR, nB = vB;
        const double fr = fR, fb = fB;
        if (z + 2 <= g.n - 1) load(z + 2);
        if (interior && z + 1 < z1) {
            fR = ld_stream<NT>(f + (long long)(z + 1) * plane + ro);
            fB = ld_stream<NT>(f + cs + (long long)(z + 1) * plane + ro);
        }
        if (interior) {
            const long long at = (long long)z * plane + ro;
            const int pr = (y + z) & 1;
            const double(*P)[66] = pl[b][0];
            const double(*Q)[66] = pl[b][1];
            auto point = [&](double xm, double xp, double ym, double yp, double zm, double zp, double uc, double fv,
                             long long o) {
                double nb = xm;
                nb = nb + xp;
                nb = nb + ym;
                nb = nb + yp;
                nb = nb + zm;
                nb = nb + zp;
                const double v = fv - (6.0 * uc - nb) * s;
                st_stream<NT>(r32 + o, (float)(v / sn));
                st_stream<NT>(uo + o, uc);
                sq = sq + v * v;
                mx = fmax(mx, fabs(v));
            };
            if (pr | xs)
                point(pr ? Q[row][lane + 1] : Q[row][lane], pr ? Q[row][lane + 2] : Q[row][lane + 1],
                      Q[row - 1][lane + 1], Q[row + 1][lane + 1], pB, nB, qR, fr, at);
            if ((1 - pr) | xs)
                point(pr ? P[row][lane] : P[row][lane + 1], pr ? P[row][lane + 1] : P[row][lane + 2],
                      P[row - 1][lane + 1], P[row + 1][lane + 1], pR, nR, qB, fb, cs + at);
        }
        pR = qR;
        pB = qB;
        qR = nR;
        qB = nB;
        lds_barrier();
    }
    block_sum_max(sq, mx, part + 2 * (long long)ex.b);
}

__global__ __launch_bounds__(256) void k_cast(long long n4, const double* __restrict__ r, float* __restrict__ f32,
                                              const double* __restrict__ basis, double* __restrict__ sigma_out) {
    Ex ex;
    ex.b = (int)blockIdx.x;
    ex.t = (int)threadIdx.x;
    ex.nt = (int)blockDim.x;
    d_cast(ex, n4, r, f32, basis, sigma_out);
}

__device__ __forceinline__ void d_update(const Ex& ex, long long n4, double* __restrict__ u,
                                         const float* __restrict__ c32, const double* __restrict__ sigma_p) {
    const long long i = (long long)ex.b * ex.nt + ex.t;
    if (i >= n4) return;
    const double sigma = *sigma_p;
    const float4 c = reinterpret_cast<const float4*>(c32)[i];
    double2 a = reinterpret_cast<double2*>(u)[2 * i];
    double2 b = reinterpret_cast<double2*>(u)[2 * i + 1];
    a.x = a.x + sigma * (double)c.x;
    a.y = a.y + sigma * (double)c.y;
    b.x = b.x + sigma * (double)c.z;
    b.y = b.y + sigma * (double)c.w;
    reinterpret_cast<double2*>(u)[2 * i] = a;
    reinterpret_cast<double2*>(u)[2 * i + 1] = b;
}

__global__ __launch_bounds__(256) void k_update(long long n4, double* __restrict__ u, const float* __restrict__ c32,
                                                const double* __restrict__ sigma_p) {
    Ex ex;
    ex.b = (int)blockIdx.x;
    ex.t = (int)threadIdx.x;
    ex.nt = (int)blockDim.x;
    d_update(ex, n4, u, c32, sigma_p);
}

// ------------------------------------------------ preconditioned CG vectors
// Flat FP64 kernels over whole level fields (boundary nodes and padding are
// zero in every vector involved, so they add nothing).  The dot product uses
// a fixed grid of at most kDotBlocks blocks striding over the field: a fixed
// assignment of elements to threads, hence a deterministic sum.
constexpr int kDotBlocks = 2048;

__global__ __launch_bounds__(256) void k_dot(long long n2, const double* __restrict__ a,
                                             const double* __restrict__ b, double* __restrict__ part) {
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n2; i += (long long)gridDim.x * 256) {
        const double2 x = reinterpret_cast<const double2*>(a)[i];
        const double2 y = reinterpret_cast<const double2*>(b)[i];
        acc = acc + x.x * y.x;
        acc = acc + x.y * y.y;
    }
    block_sum_max(acc, 0.0, part + 2 * (long long)blockIdx.x);
}

// x += alpha p, r += alpha q with q = -A p and alpha = rho / (p . A p):
// sc[0] = rho, sc[2] = p . q
__global__ __launch_bounds__(256) void k_pcg_step(long long n2, double* __restrict__ x, const double* __restrict__ p,
                                                  double* __restrict__ r, const double* __restrict__ q,
                                                  const double* __restrict__ sc) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n2) return;
    const double alpha = -(sc[0] / sc[2]);
    const double2 pv = reinterpret_cast<const double2*>(p)[i];
    const double2 qv = reinterpret_cast<const double2*>(q)[i];
    double2 xv = reinterpret_cast<double2*>(x)[i];
    double2 rv = reinterpret_cast<double2*>(r)[i];
    xv.x = xv.x + alpha * pv.x;
    xv.y = xv.y + alpha * pv.y;
    rv.x = rv.x + alpha * qv.x;
    rv.y = rv.y + alpha * qv.y;
    reinterpret_cast<double2*>(x)[i] = xv;
    reinterpret_cast<double2*>(r)[i] = rv;
}

// p = z + beta p with beta = rho_new / rho: sc[4] = rho_new, sc[0] = rho
__global__ __launch_bounds__(256) void k_pcg_dir(long long n2, double* __restrict__ p, const double* __restrict__ z,
                                                 const double* __restrict__ sc) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n2) return;
    const double beta = sc[4] / sc[0];
    const double2 zv = reinterpret_cast<const double2*>(z)[i];
    double2 pv = reinterpret_cast<double2*>(p)[i];
    pv.x = zv.x + beta * pv.x;
    pv.y = zv.y + beta * pv.y;
    reinterpret_cast<double2*>(p)[i] = pv;
}

// ------------------------------------ 3^d-point node stencils (Galerkin)
// Sum of W[o] u[x + o] over the 3^d offsets, z offset slowest, x fastest; the
// neighbour (X, Y, Z) is colour (X + Y + Z) & 1 at X >> 1 (boundary nodes hold
// zero, and an interior node's neighbours are inside the array).
template <int D>
__device__ __forceinline__ double stencil27_sum(const Geom& g, const double* __restrict__ u, int x, int y, int z,
                                                const Stencil27& W) {
    double acc = 0.0;
#pragma unroll
    for (int oz = (D == 3 ? -1 : 0); oz <= (D == 3 ? 1 : 0); ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                const int k = (D == 3 ? 9 * (oz + 1) : 0) + 3 * (oy + 1) + (ox + 1);
                const int X = x + ox, Y = y + oy, Z = z + oz;
                const double t = W.w[k] * u[(long long)((X + Y + Z) & 1) * g.cs + row_off(g, Y, Z) + (X >> 1)];
                acc = k == 0 ? t : acc + t;
            }
    return acc;
}

template <int D, bool NORM, bool STORE>
__global__ __launch_bounds__(256) void k_node27_residual(Geom g, Space sp, const double* __restrict__ u,
                                                         const double* __restrict__ f, double* __restrict__ r,
                                                         Stencil27 W, double* __restrict__ part) {
    const Ex ex = solo_ex();
    double sq = 0.0, mx = 0.0;
    Pt p;
    if (map_point(ex, sp, p)) {
        const int x = 2 * p.xs + ((p.y + p.z + p.c) & 1);
        if (x >= 1 && x <= g.n - 2) {
            const long long me = (long long)p.c * g.cs + row_off(g, p.y, p.z) + p.xs;
            const double v = f[me] - stencil27_sum<D>(g, u, x, p.y, p.z, W);
            if (STORE) r[me] = v;
            sq = v * v;
            mx = fabs(v);
        }
    }
    if (NORM) block_sum_max(sq, mx, part + 2 * (long long)ex.b);
}

template <int D, bool ZERO>
__global__ __launch_bounds__(256) void k_node27_jacobi(Geom g, Space sp, const double* __restrict__ u,
                                                       const double* __restrict__ f, double* __restrict__ out,
                                                       Stencil27 W, double omega) {
    Pt p;
    if (!map_point(solo_ex(), sp, p)) return;
    const int x = 2 * p.xs + ((p.y + p.z + p.c) & 1);
    if (x < 1 || x > g.n - 2) return;
    const long long me = (long long)p.c * g.cs + row_off(g, p.y, p.z) + p.xs;
    const double wc = W.w[D == 3 ? 13 : 4];
    if (ZERO) {
        out[me] = 0.0 + (omega * f[me]) / wc;     // r = f when u = 0
    } else {
        const double r = f[me] - stencil27_sum<D>(g, u, x, p.y, p.z, W);
        out[me] = u[me] + (omega * r) / wc;
    }
}

// ------------------------------------------- zero-mean projection (Neumann)
// Sum over all cells of a cell-grid FP64 field into per-block partials
// (fixed assignment of cells to threads: deterministic), then a -= sum / count.
__global__ __launch_bounds__(256) void k_cell_sum(Geom g, Space sp, const double* __restrict__ a,
                                                  double* __restrict__ part) {
    const Ex ex = solo_ex();
    Pt p;
    double v = 0.0;
    if (map_point(ex, sp, p)) v = a[(long long)p.c * g.cs + row_off(g, p.y, p.z) + p.xs];
    block_sum_max(v, 0.0, part + 2 * (long long)ex.b);
}

// The same per-block sums on large 3-D cell levels: each thread first adds
// its (x >> 1, y) column of both colours over a chunk of planes (colour 0,
// then 1, plane by plane), so a block of 256 threads reduces 16 values per
// thread instead of one and the partials are 16 times fewer.
__global__ __launch_bounds__(256) void k_cell_sum_zm(Geom g, ZSpace zs, const double* __restrict__ a,
                                                     double* __restrict__ part) {
    const Ex ex = solo_ex();
    int tx, ty, tz;
    zm_tile(zs, ex.b, tx, ty, tz);
    const int xs = tx * 64 + (ex.t & 63);
    const int y = ty * zs.rows + (ex.t >> 6);
    double v = 0.0;
    if (xs < zs.xr && y < g.n) {
        const int z0 = tz * zs.zc, z1 = min(z0 + zs.zc, g.n);
        long long ro = row_off(g, y, z0) + xs;
        for (int z = z0; z < z1; ++z, ro += g.plane) {
            v = v + a[ro];
            v = v + a[g.cs + ro];
        }
    }
    block_sum_max(v, 0.0, part + 2 * (long long)ex.b);
}

__global__ __launch_bounds__(256) void k_cell_shift(Geom g, Space sp, double* __restrict__ a,
                                                    const double* __restrict__ sum, double count) {
    Pt p;
    if (!map_point(solo_ex(), sp, p)) return;
    const double mean = sum[0] / count;
    const long long i = (long long)p.c * g.cs + row_off(g, p.y, p.z) + p.xs;
    a[i] = a[i] - mean;
}

__global__ void k_scalar_copy(double* __restrict__ dst, const double* __restrict__ src) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

__global__ __launch_bounds__(256) void k_copy(uint4* __restrict__ dst, const uint4* __restrict__ src, long long n16) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_zero(uint4* __restrict__ p, long long n16) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ------------------------------------------------------------- spaces
static long long nat_count(const Geom& g) {
    return (long long)g.n * g.n * (g.dim == 3 ? g.n : 1);
}

// Points of one or both colours over the unknowns of a level.
Space space_of(const Geom& g, int ncol, int col0) {
    if (g.cell)
        return make_space(g.n / 2, 0, g.n, 0, g.dim == 3 ? g.n : 1, ncol, col0);
    // node grid: interior rows/planes; xs in [0, (n-1)/2) covers interior x
    return make_space((g.n - 1) / 2, 1, g.n - 2, g.dim == 3 ? 1 : 0, g.dim == 3 ? g.n - 2 : 1, ncol, col0);
}

// ------------------------------------------------------------ batched ops
__device__ void run_item(const BItem& it, const Ex& ex) {
    switch (it.op) {
        case BOP_PACK:
            d_pack<double>(ex, it.g, it.n, static_cast<const double*>(it.io[0]), static_cast<double*>(it.a));
            break;
        case BOP_ZERO: {
            const long long i = (long long)ex.b * ex.nt + ex.t;
            if (i < it.n) static_cast<uint4*>(it.a)[i] = make_uint4(0u, 0u, 0u, 0u);
            break;
        }
        case BOP_RES64:
            if (it.dim == 3)
                d_node_residual<double, 3, true, true>(ex, it.g, it.sp, static_cast<const double*>(it.a),
                                                       static_cast<const double*>(it.b),
                                                       static_cast<double*>(it.c), it.s, it.part);
            else
                d_node_residual<double, 2, true, true>(ex, it.g, it.sp, static_cast<const double*>(it.a),
                                                       static_cast<const double*>(it.b),
                                                       static_cast<double*>(it.c), it.s, it.part);
            break;
        case BOP_REDUCE: {
            double sq = 0.0, mx = 0.0;
            for (long long i = ex.t; i < it.n; i += ex.nt) {
                sq = sq + it.part[2 * i];
                mx = fmax(mx, it.part[2 * i + 1]);
            }
            // m: the maximum also becomes the scale basis of the next cast
            block_sum_max(sq, mx, it.red, it.m ? it.red + 3 : nullptr);
            if (ex.t == 0 && it.res) {
                it.res[0] = it.red[0];
                it.res[1] = it.red[1];
            }
            break;
        }
        case BOP_CAST:
            d_cast(ex, it.n, static_cast<const double*>(it.a), static_cast<float*>(it.b), it.red + 3, it.red + 2);
            break;
        case BOP_GS:
        case BOP_GS_ZERO: {
            float* me = static_cast<float*>(it.a);
            const float* ot = static_cast<const float*>(it.b);
            const float* f = static_cast<const float*>(it.c);
            const float s = (float)it.s;
            if (it.op == BOP_GS_ZERO) {
                if (it.dim == 3) d_node_gs<float, 3, true>(ex, it.g, it.sp, me, ot, f, s);
                else d_node_gs<float, 2, true>(ex, it.g, it.sp, me, ot, f, s);
            } else {
                if (it.dim == 3) d_node_gs<float, 3, false>(ex, it.g, it.sp, me, ot, f, s);
                else d_node_gs<float, 2, false>(ex, it.g, it.sp, me, ot, f, s);
            }
            break;
        }
        case BOP_JAC:
        case BOP_JAC_ZERO: {
            const float* u = static_cast<const float*>(it.a);
            const float* f = static_cast<const float*>(it.b);
            float* out = static_cast<float*>(it.c);
            const float s = (float)it.s, om = (float)it.omega;
            if (it.op == BOP_JAC_ZERO) {
                if (it.dim == 3) d_node_jacobi<float, 3, true, false>(ex, it.g, it.sp, u, f, out, s, om, 0.f);
                else d_node_jacobi<float, 2, true, false>(ex, it.g, it.sp, u, f, out, s, om, 0.f);
            } else {
                if (it.dim == 3) d_node_jacobi<float, 3, false, false>(ex, it.g, it.sp, u, f, out, s, om, 0.f);
                else d_node_jacobi<float, 2, false, false>(ex, it.g, it.sp, u, f, out, s, om, 0.f);
            }
            break;
        }
        case BOP_RES32:
            if (it.dim == 3)
                d_node_residual<float, 3, false, true>(ex, it.g, it.sp, static_cast<const float*>(it.a),
                                                       static_cast<const float*>(it.b), static_cast<float*>(it.c),
                                                       (float)it.s, nullptr);
            else
                d_node_residual<float, 2, false, true>(ex, it.g, it.sp, static_cast<const float*>(it.a),
                                                       static_cast<const float*>(it.b), static_cast<float*>(it.c),
                                                       (float)it.s, nullptr);
            break;
        case BOP_RESTRICT:
            if (it.dim == 3)
                d_node_restrict<float, 3>(ex, it.g, it.gc, it.sp, static_cast<const float*>(it.a),
                                          static_cast<float*>(it.b));
            else
                d_node_restrict<float, 2>(ex, it.g, it.gc, it.sp, static_cast<const float*>(it.a),
                                          static_cast<float*>(it.b));
            break;
        case BOP_PROLONG:
            if (it.dim == 3)
                d_node_prolong<float, 3>(ex, it.g, it.gc, it.sp, static_cast<float*>(it.a),
                                         static_cast<const float*>(it.b));
            else
                d_node_prolong<float, 2>(ex, it.g, it.gc, it.sp, static_cast<float*>(it.a),
                                         static_cast<const float*>(it.b));
            break;
        case BOP_COARSE:
            d_coarse<float>(ex, it.g, static_cast<const float*>(it.a), static_cast<float*>(it.b), it.L, it.m);
            break;
        case BOP_UPDATE:
            d_update(ex, it.n, static_cast<double*>(it.a), static_cast<const float*>(it.b), it.red + 2);
            break;
        case BOP_UNPACK:
            d_unpack<double>(ex, it.g, it.n, static_cast<const double*>(it.a), static_cast<double*>(it.io[1]));
            break;
        case BOP_GS_M:
            d_node_gs_zm<float, 2, false>(ex, it.g, it.zs, static_cast<float*>(it.a), static_cast<const float*>(it.b),
                                          static_cast<const float*>(it.c), (float)it.s, it.m);
            break;
        case BOP_JAC_M:
            d_node_jac_ym<float, false>(ex, it.g, it.ys, static_cast<const float*>(it.a),
                                        static_cast<const float*>(it.b), static_cast<float*>(it.c), (float)it.s,
                                        (float)it.omega);
            break;
        case BOP_JAC_ZERO_M:
            d_node_jac_ym<float, true>(ex, it.g, it.ys, static_cast<const float*>(it.a),
                                       static_cast<const float*>(it.b), static_cast<float*>(it.c), (float)it.s,
                                       (float)it.omega);
            break;
        case BOP_RES32_M:
            if (it.dim == 3)
                d_node_res_zm<float, 2, false, false, true>(ex, it.g, it.zs, static_cast<const float*>(it.a),
                                                            static_cast<const float*>(it.b),
                                                            static_cast<float*>(it.c), (float)it.s, nullptr);
            else
                d_node_res_ym<float, false, true>(ex, it.g, it.ys, static_cast<const float*>(it.a),
                                                  static_cast<const float*>(it.b), static_cast<float*>(it.c),
                                                  (float)it.s, nullptr);
            break;
        case BOP_RES64_M:
            if (it.dim == 3)
                d_node_res_zm<double, 1, false, true, true>(ex, it.g, it.zs, static_cast<const double*>(it.a),
                                                            static_cast<const double*>(it.b),
                                                            static_cast<double*>(it.c), it.s, it.part);
            else
                d_node_res_ym<double, true, true>(ex, it.g, it.ys, static_cast<const double*>(it.a),
                                                  static_cast<const double*>(it.b), static_cast<double*>(it.c), it.s,
                                                  it.part);
            break;
        default:
            break;
    }
}

// Persistent: block b owns the work-unit range [b c, (b + 1) c) of the launch,
// c = ceil(total / gridDim.x), and runs every tile that starts in it.  A tile
// of entry e covers w units, so blocks get equal work whatever mix of light
// (one point per thread) and heavy (marching) tiles the launch holds.  Entry
// prefixes sit in LDS; the descriptor of the current entry is copied to LDS
// once and reused for all its tiles in the range.
constexpr int kBatchLds = 1024;

// at most 128 VGPRs: four waves per SIMD whatever op the launch holds
__global__ __launch_bounds__(256, 4) void k_batch(const BEntry* __restrict__ ent, int n, long long total) {
    __shared__ long long s_pre[kBatchLds];
    __shared__ BItem s_item;
    const bool in_lds = n <= kBatchLds;
    if (in_lds)
        for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) s_pre[i] = ent[i].prefix;
    __syncthreads();
    const long long chunk = (total + gridDim.x - 1) / gridDim.x;
    const long long g0 = (long long)blockIdx.x * chunk;
    const long long g1 = g0 + chunk < total ? g0 + chunk : total;
    long long lo_u = 0, hi_u = -1;
    unsigned w = 1;
    long long u = g0;
    while (u < g1) {
        if (u >= hi_u) {
            int lo = 0, hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                const long long pm = in_lds ? s_pre[mid] : ent[mid].prefix;
                if (pm <= u) lo = mid;
                else hi = mid - 1;
            }
            lo_u = in_lds ? s_pre[lo] : ent[lo].prefix;
            hi_u = lo + 1 < n ? (in_lds ? s_pre[lo + 1] : ent[lo + 1].prefix) : total;
            const unsigned* src = reinterpret_cast<const unsigned*>(ent[lo].item);
            unsigned* dst = reinterpret_cast<unsigned*>(&s_item);
            __syncthreads();   // every thread is done with the previous descriptor
            for (int i = (int)threadIdx.x; i < (int)(sizeof(BItem) / 4); i += (int)blockDim.x) dst[i] = src[i];
            __syncthreads();
            w = s_item.w > 1 ? (unsigned)s_item.w : 1u;
        }
        // first tile of the entry that starts at or after u (an entry spans < 2^32 units)
        const unsigned t = ((unsigned)(u - lo_u) + w - 1) / w;
        const long long start = lo_u + (long long)t * w;
        if (start >= hi_u) {
            u = hi_u;
            continue;
        }
        if (start >= g1) break;
        Ex ex;
        ex.b = (int)t;
        ex.t = (int)threadIdx.x;
        ex.nt = (int)blockDim.x;
        run_item(s_item, ex);
        __syncthreads();
        u = start + w;
    }
}

dim3 grid_of(const Space& sp) { return dim3((unsigned)sp.blocks()); }
dim3 block_of(const Space& sp) { return dim3((unsigned)sp.threads()); }

template <typename T>
const T* cp(const void* p) { return static_cast<const T*>(p); }
template <typename T>
T* mp(void* p) { return static_cast<T*>(p); }

}  // namespace

// =================================================================== launchers
#define MG_DISPATCH_DIM(g, ...)      \
    if ((g).dim == 3) {              \
        constexpr int D = 3;         \
        __VA_ARGS__;                 \
    } else {                         \
        constexpr int D = 2;         \
        __VA_ARGS__;                 \
    }

template <typename T>
static hipError_t gs_t(const Geom& g, int colour, bool zero, void* u, const void* f, const Faces& fc,
                       double s, hipStream_t st) {
    const Space sp = space_of(g, 1, colour);
    T* me = mp<T>(u) + (long long)colour * g.cs;
    const T* other = cp<T>(u) + (long long)(1 - colour) * g.cs;
    const T* fm = cp<T>(f) + (long long)colour * g.cs;
    if (sizeof(T) == 8 && g.cell && fc.k && use_cell_zm(g)) {
        const ZSpace zs = make_czspace(g);
        const dim3 grid((unsigned)zs.blocks()), block(64, zs.rows);
        const double* km = cp<double>(fc.k) + (long long)colour * g.cs;
        const double* ko = cp<double>(fc.k) + (long long)(1 - colour) * g.cs;
        double* m64 = reinterpret_cast<double*>(me);
        const double* o64 = reinterpret_cast<const double*>(other);
        const double* f64 = reinterpret_cast<const double*>(fm);
        const bool nt = streams_from_hbm(g, 8);
        if (zero && nt) k_cell_gs_zmk<true, true><<<grid, block, 0, st>>>(g, zs, m64, o64, f64, km, ko, s, colour);
        else if (zero) k_cell_gs_zmk<false, true><<<grid, block, 0, st>>>(g, zs, m64, o64, f64, km, ko, s, colour);
        else if (nt) k_cell_gs_zmk<true, false><<<grid, block, 0, st>>>(g, zs, m64, o64, f64, km, ko, s, colour);
        else k_cell_gs_zmk<false, false><<<grid, block, 0, st>>>(g, zs, m64, o64, f64, km, ko, s, colour);
    } else if (g.cell) {
        MG_DISPATCH_DIM(g, if (zero) k_cell_gs<T, D, true><<<grid_of(sp), block_of(sp), 0, st>>>(
                               g, sp, me, other, fm, cp<T>(fc.b[0]), cp<T>(fc.b[1]), cp<T>(fc.b[2]), (T)s);
                           else k_cell_gs<T, D, false><<<grid_of(sp), block_of(sp), 0, st>>>(
                               g, sp, me, other, fm, cp<T>(fc.b[0]), cp<T>(fc.b[1]), cp<T>(fc.b[2]), (T)s));
    } else if (!zero && use_zmarch(g)) {
        const ZSpace zs = make_zspace(g);
        const dim3 grid((unsigned)zs.blocks()), block(64, zs.rows);
        // planes in flight per thread: 2 x 8 B (FP64) or 4 x 4 B (FP32) columns
        constexpr int U = sizeof(T) == 8 ? 2 : 4;
        const bool nt = streams_from_hbm(g, sizeof(T)), p2 = pow2_scale(s);
        const T rs = (T)(1.0 / s);
        if (nt && p2) k_node_gs_zm<T, U, true, true><<<grid, block, 0, st>>>(g, zs, me, other, fm, (T)s, colour, rs);
        else if (nt) k_node_gs_zm<T, U, true, false><<<grid, block, 0, st>>>(g, zs, me, other, fm, (T)s, colour, rs);
        else if (p2) k_node_gs_zm<T, U, false, true><<<grid, block, 0, st>>>(g, zs, me, other, fm, (T)s, colour, rs);
        else k_node_gs_zm<T, U, false, false><<<grid, block, 0, st>>>(g, zs, me, other, fm, (T)s, colour, rs);
    } else {
        const T rs = (T)(1.0 / s);
#define MG_NGS(Z, P)                                                                                   \
    MG_DISPATCH_DIM(g, k_node_gs<T, D, Z, P><<<grid_of(sp), block_of(sp), 0, st>>>(g, sp, me, other, fm, \
                                                                                (T)s, rs))
        if (pow2_scale(s)) {
            if (zero) {
                MG_NGS(true, true);
            } else {
                MG_NGS(false, true);
            }
        } else {
            if (zero) {
                MG_NGS(true, false);
            } else {
                MG_NGS(false, false);
            }
        }
#undef MG_NGS
    }
    return hipGetLastError();
}

hipError_t launch_gs(const Geom& g, int prec, int colour, bool zero, void* u, const void* f,
                     const Faces& fc, double s, hipStream_t st) {
    return prec ? gs_t<float>(g, colour, zero, u, f, fc, s, st)
                : gs_t<double>(g, colour, zero, u, f, fc, s, st);
}

// FP64 levels run the rolled march (k_node_gs_tb), FP32 levels the
// pair-unrolled one (k_node_gs_tbu): with FP64 values the unrolled march
// needs more registers than three wavefronts per SIMD leave and measured
// slower, while on FP32 fields it is 20 % (513^3) to 40 % (257^3) faster.
template <typename T, int S, int R, int NW, int PF>
static void gs_tb_launch(const Geom& g, int c1, int z, const void* u, const void* f, void* out, double s,
                         hipStream_t st) {
    const TbSpace ts = make_tbspace(g, S, NW * R);
    const dim3 grid((unsigned)ts.blocks()), block(64 * NW);
    int e;
    const bool p2 = s > 0.0 && std::frexp(s, &e) == 0.5;   // s = 2^(e - 1)
    const bool buf = 2 * g.cs * (long long)sizeof(T) < (1LL << 31);
    const T rs = (T)(1.0 / s);
#define MG_TB(KERNEL)                                                                                        \
    if (p2 && buf)                                                                                           \
        KERNEL<T, S, R, NW, PF, true, true><<<grid, block, 0, st>>>(g, ts, cp<T>(u), cp<T>(f), mp<T>(out), (T)s, \
                                                                    rs, c1, z);                             \
    else if (p2)                                                                                             \
        KERNEL<T, S, R, NW, PF, true, false><<<grid, block, 0, st>>>(g, ts, cp<T>(u), cp<T>(f), mp<T>(out),    \
                                                                     (T)s, rs, c1, z);                      \
    else if (buf)                                                                                            \
        KERNEL<T, S, R, NW, PF, false, true><<<grid, block, 0, st>>>(g, ts, cp<T>(u), cp<T>(f), mp<T>(out),    \
                                                                     (T)s, rs, c1, z);                      \
    else                                                                                                     \
        KERNEL<T, S, R, NW, PF, false, false><<<grid, block, 0, st>>>(g, ts, cp<T>(u), cp<T>(f), mp<T>(out),   \
                                                                      (T)s, rs, c1, z);
    if constexpr (sizeof(T) == 8) {
        MG_TB(k_node_gs_tb)
    } else {
        MG_TB(k_node_gs_tbu)
    }
#undef MG_TB
}

template <typename T>
static hipError_t gs_tb_t(const Geom& g, int sweeps, int c1, bool zero, const void* u, const void* f, void* out,
                          double s, hipStream_t st) {
    // rows per thread and wavefronts per block: registers (two planes of
    // every stage per row, plus the operands in flight) and LDS (one plane of
    // every stage) grow with S x R; these shapes measured fastest among those
    // that do not spill
    constexpr bool dp = sizeof(T) == 8;
    const int z = zero ? 1 : 0;
    switch (sweeps) {
        case 1: gs_tb_launch<T, 2, 3, 16, 2>(g, c1, z, u, f, out, s, st); break;
        case 2: gs_tb_launch<T, 4, dp ? 3 : 4, 16, 4>(g, c1, z, u, f, out, s, st); break;
        case 3: gs_tb_launch<T, 6, 3, dp ? 12 : 16, 6>(g, c1, z, u, f, out, s, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gs_tb(const Geom& g, int prec, int sweeps, int first_colour, bool zero, const void* u,
                        const void* f, void* out, double s, hipStream_t st) {
    if (!use_tb(g) || sweeps < 1 || sweeps > 3 || (first_colour & ~1)) return hipErrorInvalidValue;
    return prec ? gs_tb_t<float>(g, sweeps, first_colour, zero, u, f, out, s, st)
                : gs_tb_t<double>(g, sweeps, first_colour, zero, u, f, out, s, st);
}

template <typename T>
static hipError_t jacobi_t(const Geom& g, bool zero, const void* u, const void* f, void* out,
                           const Faces& fc, double s, double omega, hipStream_t st) {
    if (use_ymarch(g)) {
        const YSpace ys = make_yspace(g);
        if (zero)
            k_node_jac_ym<T, true><<<(unsigned)ys.blocks(), 256, 0, st>>>(g, ys, cp<T>(u), cp<T>(f), mp<T>(out),
                                                                         (T)s, (T)omega);
        else
            k_node_jac_ym<T, false><<<(unsigned)ys.blocks(), 256, 0, st>>>(g, ys, cp<T>(u), cp<T>(f), mp<T>(out),
                                                                          (T)s, (T)omega);
        return hipGetLastError();
    }
    if (!zero && !g.cell && use_zmarch(g)) {
        const ZSpace zs = make_zspace(g);
        const dim3 grid((unsigned)zs.blocks()), block(64, zs.rows);
        constexpr int U = sizeof(T) == 8 ? 2 : 4;
        const bool nt = streams_from_hbm(g, sizeof(T)), p2 = pow2_scale(s);
        const T rs = (T)(1.0 / s);
#define MG_JZ(N, P) \
    k_node_jac_zm<T, U, N, P><<<grid, block, 0, st>>>(g, zs, cp<T>(u), cp<T>(f), mp<T>(out), (T)s, (T)omega, rs)
        if (nt && p2) MG_JZ(true, true);
        else if (nt) MG_JZ(true, false);
        else if (p2) MG_JZ(false, true);
        else MG_JZ(false, false);
#undef MG_JZ
        return hipGetLastError();
    }
    const Space sp = space_of(g, 2, 0);
    if (g.cell) {
        MG_DISPATCH_DIM(g, if (zero) k_cell_jacobi<T, D, true><<<grid_of(sp), block_of(sp), 0, st>>>(
                               g, sp, cp<T>(u), cp<T>(f), mp<T>(out), cp<T>(fc.b[0]), cp<T>(fc.b[1]),
                               cp<T>(fc.b[2]), (T)s, (T)omega);
                           else k_cell_jacobi<T, D, false><<<grid_of(sp), block_of(sp), 0, st>>>(
                               g, sp, cp<T>(u), cp<T>(f), mp<T>(out), cp<T>(fc.b[0]), cp<T>(fc.b[1]),
                               cp<T>(fc.b[2]), (T)s, (T)omega));
    } else {
        const T rs = (T)(1.0 / s);
#define MG_NJAC(Z, P)                                                                                  \
    MG_DISPATCH_DIM(g, k_node_jacobi<T, D, Z, P><<<grid_of(sp), block_of(sp), 0, st>>>(                \
                           g, sp, cp<T>(u), cp<T>(f), mp<T>(out), (T)s, (T)omega, rs))
        if (pow2_scale(s)) {
            if (zero) {
                MG_NJAC(true, true);
            } else {
                MG_NJAC(false, true);
            }
        } else {
            if (zero) {
                MG_NJAC(true, false);
            } else {
                MG_NJAC(false, false);
            }
        }
#undef MG_NJAC
    }
    return hipGetLastError();
}

hipError_t launch_jacobi(const Geom& g, int prec, bool zero, const void* u, const void* f, void* out,
                         const Faces& fc, double s, double omega, hipStream_t st) {
    return prec ? jacobi_t<float>(g, zero, u, f, out, fc, s, omega, st)
                : jacobi_t<double>(g, zero, u, f, out, fc, s, omega, st);
}

long long residual_blocks(const Geom& g) {
    // the stand-alone path may march columns or rows; the batched path may use one point per thread
    const long long a = use_zmarch(g)    ? make_zspace(g).blocks()
                        : use_ymarch_batched(g) ? make_yspace(g).blocks()
                        : use_cell_zm(g) ? make_czspace(g).blocks()
                                         : 0;
    const long long b = space_of(g, 2, 0).blocks();
    return a > b ? a : b;
}

template <typename T, bool NORM, bool STORE>
static void residual_tt(const Geom& g, const Space& sp, const void* u, const void* f, void* r,
                        const Faces& fc, double s, double* part, hipStream_t st) {
    if (g.cell) {
        MG_DISPATCH_DIM(g, k_cell_residual<T, D, NORM, STORE><<<grid_of(sp), block_of(sp), 0, st>>>(
                               g, sp, cp<T>(u), cp<T>(f), mp<T>(r), cp<T>(fc.b[0]), cp<T>(fc.b[1]),
                               cp<T>(fc.b[2]), (T)s, part));
    } else {
        MG_DISPATCH_DIM(g, k_node_residual<T, D, NORM, STORE><<<grid_of(sp), block_of(sp), 0, st>>>(
                               g, sp, cp<T>(u), cp<T>(f), mp<T>(r), (T)s, part));
    }
}

template <typename T>
static hipError_t residual_t(const Geom& g, const void* u, const void* f, void* r, const Faces& fc,
                             double s, bool norm, bool store, double* part, long long* nb,
                             hipStream_t st) {
    if (sizeof(T) == 8 && g.cell && fc.k && use_cell_zm(g)) {
        const ZSpace zs = make_czspace(g);
        if (nb) *nb = zs.blocks();
        const dim3 grid((unsigned)zs.blocks()), block(64, zs.rows);
        const double* u64 = cp<double>(u);
        const double* f64 = cp<double>(f);
        double* r64 = reinterpret_cast<double*>(r);
        const double* kk = cp<double>(fc.k);
#define MG_CRES(NT)                                                                                         \
    if (norm && store)                                                                                      \
        k_cell_res_zmk<NT, true, true><<<grid, block, 0, st>>>(g, zs, u64, f64, r64, kk, s, part);          \
    else if (norm)                                                                                          \
        k_cell_res_zmk<NT, true, false><<<grid, block, 0, st>>>(g, zs, u64, f64, r64, kk, s, part);         \
    else                                                                                                    \
        k_cell_res_zmk<NT, false, true><<<grid, block, 0, st>>>(g, zs, u64, f64, r64, kk, s, part);
        if (streams_from_hbm(g, 8)) {
            MG_CRES(true)
        } else {
            MG_CRES(false)
        }
#undef MG_CRES
        return hipGetLastError();
    }
    if (use_ymarch(g)) {
        const YSpace ys = make_yspace(g);
        if (nb) *nb = ys.blocks();
        const unsigned grid = (unsigned)ys.blocks();
        if (norm && store)
            k_node_res_ym<T, true, true><<<grid, 256, 0, st>>>(g, ys, cp<T>(u), cp<T>(f), mp<T>(r), (T)s, part);
        else if (norm)
            k_node_res_ym<T, true, false><<<grid, 256, 0, st>>>(g, ys, cp<T>(u), cp<T>(f), mp<T>(r), (T)s, part);
        else
            k_node_res_ym<T, false, true><<<grid, 256, 0, st>>>(g, ys, cp<T>(u), cp<T>(f), mp<T>(r), (T)s, part);
        return hipGetLastError();
    }
    if (use_zmarch(g)) {
        const ZSpace zs = make_zspace(g);
        if (nb) *nb = zs.blocks();
        const dim3 grid((unsigned)zs.blocks()), block(64, zs.rows);
        constexpr int U = sizeof(T) == 8 ? 2 : 4;
        if (streams_from_hbm(g, sizeof(T))) {
            if (norm && store)
                k_node_res_zm<T, U, true, true, true><<<grid, block, 0, st>>>(g, zs, cp<T>(u), cp<T>(f), mp<T>(r),
                                                                             (T)s, part);
            else if (norm)
                k_node_res_zm<T, U, true, true, false><<<grid, block, 0, st>>>(g, zs, cp<T>(u), cp<T>(f), mp<T>(r),
                                                                              (T)s, part);
            else
                k_node_res_zm<T, U, true, false, true><<<grid, block, 0, st>>>(g, zs, cp<T>(u), cp<T>(f), mp<T>(r),
                                                                              (T)s, part);
        } else {
            if (norm && store)
                k_node_res_zm<T, U, false, true, true><<<grid, block, 0, st>>>(g, zs, cp<T>(u), cp<T>(f), mp<T>(r),
                                                                              (T)s, part);
            else if (norm)
                k_node_res_zm<T, U, false, true, false><<<grid, block, 0, st>>>(g, zs, cp<T>(u), cp<T>(f),
                                                                               mp<T>(r), (T)s, part);
            else
                k_node_res_zm<T, U, false, false, true><<<grid, block, 0, st>>>(g, zs, cp<T>(u), cp<T>(f),
                                                                               mp<T>(r), (T)s, part);
        }
        return hipGetLastError();
    }
    const Space sp = space_of(g, 2, 0);
    if (nb) *nb = sp.blocks();
    if (norm && store) residual_tt<T, true, true>(g, sp, u, f, r, fc, s, part, st);
    else if (norm) residual_tt<T, true, false>(g, sp, u, f, r, fc, s, part, st);
    else residual_tt<T, false, true>(g, sp, u, f, r, fc, s, part, st);
    return hipGetLastError();
}

hipError_t launch_residual(const Geom& g, int prec, const void* u, const void* f, void* r,
                           const Faces& fc, double s, bool norm, bool store, double* partials,
                           long long* nblocks, hipStream_t st) {
    return prec ? residual_t<float>(g, u, f, r, fc, s, norm, store, partials, nblocks, st)
                : residual_t<double>(g, u, f, r, fc, s, norm, store, partials, nblocks, st);
}

template <typename T>
static hipError_t restrict_t(const Geom& gf, const Geom& gc, const void* r, void* fco, hipStream_t st) {
    const Space sp = space_of(gc, 2, 0);
    if (gf.cell) {
        MG_DISPATCH_DIM(gf, k_cell_restrict<T, D><<<grid_of(sp), block_of(sp), 0, st>>>(gf, gc, sp, cp<T>(r),
                                                                                         mp<T>(fco)));
    } else {
        MG_DISPATCH_DIM(gf, k_node_restrict<T, D><<<grid_of(sp), block_of(sp), 0, st>>>(gf, gc, sp, cp<T>(r),
                                                                                         mp<T>(fco)));
    }
    return hipGetLastError();
}

bool fused_transfers(const Geom& gf) { return use_zmarch(gf); }

template <typename T>
static hipError_t res_restrict_t(const Geom& gf, const Geom& gc, const void* u, const void* f, void* fco,
                                 double s, hipStream_t st) {
    // 256-thread blocks of 3 (FP64) or 4 (FP32) rows per thread measured
    // fastest among 2-4 rows and 4 or 8 wavefronts; chunks of 8 coarse
    // planes, shorter on small levels so that at least 512 blocks run
    constexpr int R = sizeof(T) == 8 ? 3 : 4, NW = 4, CY = (R * NW - 1) / 2;
    const int ntx = (gc.n - 2 + kRrCX - 1) / kRrCX, nty = (gc.n - 2 + CY - 1) / CY;
    int KC = 8;
    while (KC > 1 && (long long)ntx * nty * ((gc.n - 2 + KC - 1) / KC) < 512) KC /= 2;
    const int ntz = (gc.n - 2 + KC - 1) / KC;
    const unsigned nb = (unsigned)((long long)ntx * nty * ntz);
    k_node_res_restrict_zm<T, R, NW><<<nb, 64 * NW, 0, st>>>(gf, gc, ntx, nty, KC, cp<T>(u), cp<T>(f), mp<T>(fco),
                                                             (T)s);
    return hipGetLastError();
}

hipError_t launch_residual_restrict(const Geom& gf, const Geom& gc, int prec, const void* u, const void* f,
                                    void* fcoarse, double s, hipStream_t st) {
    if (!fused_transfers(gf)) return hipErrorInvalidValue;
    return prec ? res_restrict_t<float>(gf, gc, u, f, fcoarse, s, st)
                : res_restrict_t<double>(gf, gc, u, f, fcoarse, s, st);
}

// 2-D node levels that run point kernels: residual + full weighting, and
// interpolation + correction + the first damped-Jacobi sweep, one launch each.
bool fused_point_transfers(const Geom& gf) { return gf.dim == 2 && !gf.cell && !use_ymarch(gf); }

template <typename T>
static hipError_t res_restrict_pt_t(const Geom& gf, const Geom& gc, const void* u, const void* f, void* fco,
                                    double s, hipStream_t st) {
    const Space sp = space_of(gc, 2, 0);
    k_node_res_restrict_pt<T, 2><<<grid_of(sp), block_of(sp), 0, st>>>(gf, gc, sp, cp<T>(u), cp<T>(f), mp<T>(fco),
                                                                       (T)s);
    return hipGetLastError();
}

hipError_t launch_residual_restrict_pt(const Geom& gf, const Geom& gc, int prec, const void* u, const void* f,
                                       void* fcoarse, double s, hipStream_t st) {
    if (!fused_point_transfers(gf)) return hipErrorInvalidValue;
    return prec ? res_restrict_pt_t<float>(gf, gc, u, f, fcoarse, s, st)
                : res_restrict_pt_t<double>(gf, gc, u, f, fcoarse, s, st);
}

template <typename T>
static hipError_t prolong_jacobi_t(const Geom& gf, const Geom& gc, const void* u, const void* ec, const void* f,
                                   void* out, double s, double omega, hipStream_t st) {
    const Space sp = space_of(gf, 2, 0);
    const T rs = (T)(1.0 / s);
    if (pow2_scale(s))
        k_node_prolong_jacobi<T, 2, true><<<grid_of(sp), block_of(sp), 0, st>>>(gf, gc, sp, cp<T>(u), cp<T>(ec),
                                                                                 cp<T>(f), mp<T>(out), (T)s,
                                                                                 (T)omega, rs);
    else
        k_node_prolong_jacobi<T, 2, false><<<grid_of(sp), block_of(sp), 0, st>>>(gf, gc, sp, cp<T>(u), cp<T>(ec),
                                                                                  cp<T>(f), mp<T>(out), (T)s,
                                                                                  (T)omega, rs);
    return hipGetLastError();
}

hipError_t launch_prolong_jacobi(const Geom& gf, const Geom& gc, int prec, const void* u, const void* ec,
                                 const void* f, void* out, double s, double omega, hipStream_t st) {
    if (!fused_point_transfers(gf)) return hipErrorInvalidValue;
    return prec ? prolong_jacobi_t<float>(gf, gc, u, ec, f, out, s, omega, st)
                : prolong_jacobi_t<double>(gf, gc, u, ec, f, out, s, omega, st);
}

template <typename T>
static hipError_t jacobi2_t(const Geom& g, const Geom* gc, bool zero, const void* u, const void* ec, const void* f,
                            void* out, void* fco, double s, double omega, hipStream_t st) {
    const int ntx = (g.n + kJ2 - 1) / kJ2;
    const unsigned nb = (unsigned)(ntx * ntx);
    const T rs = (T)(1.0 / s);
    const Geom gcc = gc ? *gc : g;
#define MG_J2(P, Z, R, Q)                                                                                      \
    k_node_jacobi2<T, P, Z, R, Q><<<nb, 256, 0, st>>>(g, gcc, ntx, cp<T>(u), cp<T>(ec), cp<T>(f), mp<T>(out), \
                                                      mp<T>(fco), (T)s, (T)omega, rs)
    const bool p2 = pow2_scale(s);
    if (fco) {   // sweeps, residual and restriction
        if (zero) {
            if (p2) MG_J2(true, true, false, true);
            else MG_J2(false, true, false, true);
        } else {
            if (p2) MG_J2(true, false, false, true);
            else MG_J2(false, false, false, true);
        }
    } else if (ec) {
        if (p2) MG_J2(true, false, true, false);
        else MG_J2(false, false, true, false);
    } else if (zero) {
        if (p2) MG_J2(true, true, false, false);
        else MG_J2(false, true, false, false);
    } else {
        if (p2) MG_J2(true, false, false, false);
        else MG_J2(false, false, false, false);
    }
#undef MG_J2
    return hipGetLastError();
}

hipError_t launch_jacobi2(const Geom& g, const Geom* gc, int prec, bool zero, const void* u, const void* ec,
                          const void* f, void* out, void* fco, double s, double omega, hipStream_t st) {
    if (!fused_point_transfers(g) || (ec && (zero || fco)) || ((ec || fco) && !gc)) return hipErrorInvalidValue;
    return prec ? jacobi2_t<float>(g, gc, zero, u, ec, f, out, fco, s, omega, st)
                : jacobi2_t<double>(g, gc, zero, u, ec, f, out, fco, s, omega, st);
}

template <typename T>
static hipError_t cell_res_restrict_pt_t(const Geom& gf, const Geom& gc, const void* u, const void* f,
                                         const Faces& fc, void* fco, double s, hipStream_t st) {
    const Space sp = space_of(gc, 2, 0);
    MG_DISPATCH_DIM(gf, k_cell_res_restrict_pt<T, D><<<grid_of(sp), block_of(sp), 0, st>>>(
                            gf, gc, sp, cp<T>(u), cp<T>(f), cp<T>(fc.b[0]), cp<T>(fc.b[1]), cp<T>(fc.b[2]),
                            mp<T>(fco), (T)s));
    return hipGetLastError();
}

hipError_t launch_cell_res_restrict_pt(const Geom& gf, const Geom& gc, int prec, const void* u, const void* f,
                                       const Faces& fc, void* fco, double s, hipStream_t st) {
    if (!gf.cell || !fc.b[0] || !fc.b[1] || (gf.dim == 3 && !fc.b[2])) return hipErrorInvalidValue;
    return prec ? cell_res_restrict_pt_t<float>(gf, gc, u, f, fc, fco, s, st)
                : cell_res_restrict_pt_t<double>(gf, gc, u, f, fc, fco, s, st);
}

bool cell_res_restrict_fused(const Geom& gf) { return use_cell_zm(gf) && kZChunk % 2 == 0; }

hipError_t launch_cell_res_restrict(const Geom& gf, const Geom& gc, const void* u, const void* f, const void* k,
                                    void* fco, double s, hipStream_t st) {
    if (!cell_res_restrict_fused(gf) || !k) return hipErrorInvalidValue;
    ZSpace zs = make_czspace(gf);
    zs.nty = (gf.n / 2 + zs.rows - 1) / zs.rows;   // tiles of coarse rows
    const dim3 grid((unsigned)zs.blocks()), block(64, zs.rows);
    if (streams_from_hbm(gf, 8))
        k_cell_res_restrict_zmk<true><<<grid, block, 0, st>>>(gf, gc, zs, cp<double>(u), cp<double>(f), cp<double>(k),
                                                              mp<double>(fco), s);
    else
        k_cell_res_restrict_zmk<false><<<grid, block, 0, st>>>(gf, gc, zs, cp<double>(u), cp<double>(f),
                                                               cp<double>(k), mp<double>(fco), s);
    return hipGetLastError();
}

hipError_t launch_restrict(const Geom& gf, const Geom& gc, int prec, const void* r, void* fcoarse,
                           hipStream_t st) {
    return prec ? restrict_t<float>(gf, gc, r, fcoarse, st) : restrict_t<double>(gf, gc, r, fcoarse, st);
}

template <typename T>
static hipError_t prolong_t(const Geom& gf, const Geom& gc, void* u, const void* ec, int mask,
                            hipStream_t st) {
    if (use_zmarch(gf)) {
        const ZSpace zs = make_zspace(gf);
        for (int c = 0; c < 2; ++c)
            if (mask & (1 << c))
                k_node_prolong_zm<T><<<dim3((unsigned)zs.blocks()), dim3(64, zs.rows), 0, st>>>(
                    gf, gc, zs, c, mp<T>(u), cp<T>(ec));
        return hipGetLastError();
    }
    if (gf.cell && gf.dim == 3 && use_cell_zm(gf) && kZChunk % 2 == 0) {
        const ZSpace zs = make_czspace(gf);
        for (int c = 0; c < 2; ++c)
            if (mask & (1 << c))
                k_cell_prolong_zm<T><<<dim3((unsigned)zs.blocks()), dim3(64, zs.rows), 0, st>>>(
                    gf, gc, zs, c, mp<T>(u), cp<T>(ec));
        return hipGetLastError();
    }
    const int ncol = (mask == 3) ? 2 : 1;
    const int col0 = (mask == 2) ? 1 : 0;
    const Space sp = space_of(gf, ncol, col0);
    if (gf.cell) {
        MG_DISPATCH_DIM(gf, k_cell_prolong<T, D><<<grid_of(sp), block_of(sp), 0, st>>>(gf, gc, sp, mp<T>(u),
                                                                                        cp<T>(ec)));
    } else {
        MG_DISPATCH_DIM(gf, k_node_prolong<T, D><<<grid_of(sp), block_of(sp), 0, st>>>(gf, gc, sp, mp<T>(u),
                                                                                        cp<T>(ec)));
    }
    return hipGetLastError();
}

hipError_t launch_prolong(const Geom& gf, const Geom& gc, int prec, void* u, const void* ec,
                          int colour_mask, hipStream_t st) {
    if (colour_mask < 1 || colour_mask > 3) return hipErrorInvalidValue;
    return prec ? prolong_t<float>(gf, gc, u, ec, colour_mask, st)
                : prolong_t<double>(gf, gc, u, ec, colour_mask, st);
}

hipError_t launch_coarse(const Geom& g, int prec, const void* f, void* u, const double* L, int m,
                         hipStream_t st) {
    if (m < 1 || m > 64) return hipErrorInvalidValue;
    if (prec)
        k_coarse<float><<<1, 64, 0, st>>>(g, cp<float>(f), mp<float>(u), L, m);
    else
        k_coarse<double><<<1, 64, 0, st>>>(g, cp<double>(f), mp<double>(u), L, m);
    return hipGetLastError();
}

hipError_t launch_tail(const TailPlan& P, int prec, const void* f, void* u, hipStream_t st) {
    if (P.nl < 2 || P.nl > kTailMax || P.m < 1 || P.m > 64 || P.g0.neu ||
        ((long long)P.elems * (prec ? 4 : 8) + 7) / 8 * 8 + 8LL * P.m * P.m > kTailLdsBytes)
        return hipErrorInvalidValue;
#define MG_TAIL(T, D, C) k_tail<T, D, C><<<1, kTailThreads, 0, st>>>(P, cp<T>(f), mp<T>(u))
    const bool c = P.g0.cell != 0, d3 = P.g0.dim == 3;
    if (prec) {
        if (c) {
            if (d3) MG_TAIL(float, 3, true); else MG_TAIL(float, 2, true);
        } else {
            if (d3) MG_TAIL(float, 3, false); else MG_TAIL(float, 2, false);
        }
    } else {
        if (c) {
            if (d3) MG_TAIL(double, 3, true); else MG_TAIL(double, 2, true);
        } else {
            if (d3) MG_TAIL(double, 3, false); else MG_TAIL(double, 2, false);
        }
    }
#undef MG_TAIL
    return hipGetLastError();
}

long long reduce_scratch_pairs(long long count) {
    long long total = 0;
    while (count > 1) {
        count = (count + kReduceChunk - 1) / kReduceChunk;
        total += count;
    }
    return total + 1;
}

hipError_t launch_jacobi27(const Geom& g, bool zero, const void* u, const void* f, void* out, const Stencil27& W,
                           double omega, hipStream_t st) {
    if (g.cell) return hipErrorInvalidValue;
    const Space sp = space_of(g, 2, 0);
    MG_DISPATCH_DIM(g, if (zero) k_node27_jacobi<D, true><<<grid_of(sp), block_of(sp), 0, st>>>(
                           g, sp, cp<double>(u), cp<double>(f), mp<double>(out), W, omega);
                       else k_node27_jacobi<D, false><<<grid_of(sp), block_of(sp), 0, st>>>(
                           g, sp, cp<double>(u), cp<double>(f), mp<double>(out), W, omega));
    return hipGetLastError();
}

hipError_t launch_residual27(const Geom& g, const void* u, const void* f, void* r, const Stencil27& W, bool norm,
                             bool store, double* partials, long long* nblocks, hipStream_t st) {
    if (g.cell) return hipErrorInvalidValue;
    const Space sp = space_of(g, 2, 0);
    if (nblocks) *nblocks = sp.blocks();
    if (norm && store) {
        MG_DISPATCH_DIM(g, k_node27_residual<D, true, true><<<grid_of(sp), block_of(sp), 0, st>>>(
                               g, sp, cp<double>(u), cp<double>(f), mp<double>(r), W, partials));
    } else if (norm) {
        MG_DISPATCH_DIM(g, k_node27_residual<D, true, false><<<grid_of(sp), block_of(sp), 0, st>>>(
                               g, sp, cp<double>(u), cp<double>(f), mp<double>(r), W, partials));
    } else {
        MG_DISPATCH_DIM(g, k_node27_residual<D, false, true><<<grid_of(sp), block_of(sp), 0, st>>>(
                               g, sp, cp<double>(u), cp<double>(f), mp<double>(r), W, partials));
    }
    return hipGetLastError();
}

hipError_t launch_project(const Geom& g, double* a, double* partials, double* scratch, double* out,
                          hipStream_t st) {
    if (!g.cell) return hipErrorInvalidValue;
    const Space sp = space_of(g, 2, 0);
    long long nparts = sp.blocks();
    if (g.dim == 3 && use_cell_zm(g)) {
        const ZSpace zs = make_czspace(g);
        nparts = zs.blocks();
        k_cell_sum_zm<<<(unsigned)zs.blocks(), dim3(64, zs.rows), 0, st>>>(g, zs, a, partials);
    } else {
        k_cell_sum<<<grid_of(sp), block_of(sp), 0, st>>>(g, sp, a, partials);
    }
    hipError_t e = launch_reduce(partials, nparts, scratch, out, st);
    if (e != hipSuccess) return e;
    k_cell_shift<<<grid_of(sp), block_of(sp), 0, st>>>(g, sp, a, out, (double)nat_count(g));
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, long long count, double* scratch, double* out,
                         hipStream_t st, double* mx_copy, const double* move_src, double* move_dst) {
    const double* in = partials;
    double* buf = scratch;
    if (count < 1) return hipErrorInvalidValue;
    while (count > 1) {
        const long long nb = (count + kReduceChunk - 1) / kReduceChunk;
        double* dst = (nb == 1) ? out : buf;
        k_reduce<<<(unsigned)nb, 256, 0, st>>>(in, count, dst, nb == 1 ? mx_copy : nullptr,
                                                nb == 1 ? move_src : nullptr, nb == 1 ? move_dst : nullptr);
        in = dst;
        buf += 2 * nb;
        count = nb;
    }
    if (in != out) {   // a single partial pair: copy it through the reduce kernel
        k_reduce<<<1, 256, 0, st>>>(in, 1, out, mx_copy, move_src, move_dst);
    }
    return hipGetLastError();
}

hipError_t launch_pack(const Geom& g, int prec, const double* nat, void* split, hipStream_t st) {
    const long long tot = nat_count(g);
    const unsigned nb = (unsigned)((tot + 255) / 256);
    if (prec)
        k_pack<float><<<nb, 256, 0, st>>>(g, tot, nat, mp<float>(split));
    else
        k_pack<double><<<nb, 256, 0, st>>>(g, tot, nat, mp<double>(split));
    return hipGetLastError();
}

hipError_t launch_unpack(const Geom& g, int prec, const void* split, double* nat, hipStream_t st) {
    const long long tot = nat_count(g);
    const unsigned nb = (unsigned)((tot + 255) / 256);
    if (prec)
        k_unpack<float><<<nb, 256, 0, st>>>(g, tot, cp<float>(split), nat);
    else
        k_unpack<double><<<nb, 256, 0, st>>>(g, tot, cp<double>(split), nat);
    return hipGetLastError();
}

long long field_quads(const Geom& g) { return g.cs / 2; }   // 2 cs elements, 4 per thread

hipError_t launch_cast(const Geom& g, const double* r64, float* f32, const double* basis, double* sigma,
                       hipStream_t st) {
    const long long n4 = field_quads(g);
    k_cast<<<(unsigned)((n4 + 255) / 256), 256, 0, st>>>(n4, r64, f32, basis, sigma);
    return hipGetLastError();
}

hipError_t launch_residual_cast(const Geom& g, const void* u, const void* f, float* f32, double s,
                                const double* basis, double* sigma, double* partials, long long* nblocks,
                                hipStream_t st) {
    if (!use_zmarch(g)) return hipErrorInvalidValue;
    const ZSpace zs = make_zspace(g);
    if (nblocks) *nblocks = zs.blocks();
    const dim3 grid((unsigned)zs.blocks()), block(64, zs.rows);
    if (streams_from_hbm(g, sizeof(double)))
        k_node_res_cast_zm<2, true><<<grid, block, 0, st>>>(g, zs, cp<double>(u), cp<double>(f), f32, s, basis,
                                                           sigma, partials);
    else
        k_node_res_cast_zm<2, false><<<grid, block, 0, st>>>(g, zs, cp<double>(u), cp<double>(f), f32, s, basis,
                                                            sigma, partials);
    return hipGetLastError();
}

hipError_t launch_update_residual_cast(const Geom& g, const double* u, const float* c32, const double* f, double* uo,
                                       float* f32, double s, double* red, double* partials, long long* nblocks,
                                       hipStream_t st) {
    if (!use_zmarch(g)) return hipErrorInvalidValue;
    const int ntx = ((g.n - 1) / 2 + 63) / 64, nty = (g.n - 2 + kUrRows - 1) / kUrRows;
    const int ntz = (g.n - 2 + kUrChunk - 1) / kUrChunk;
    const long long nb = (long long)ntx * nty * ntz;
    if (nblocks) *nblocks = nb;
    const dim3 grid((unsigned)nb), block(64, kUrRows + 2);
    if (streams_from_hbm(g, sizeof(double)))
        k_node_upd_res_cast<true><<<grid, block, 0, st>>>(g, ntx, nty, kUrChunk, u, c32, f, uo, f32, s, red, partials);
    else
        k_node_upd_res_cast<false><<<grid, block, 0, st>>>(g, ntx, nty, kUrChunk, u, c32, f, uo, f32, s, red, partials);
    return hipGetLastError();
}

hipError_t launch_update(const Geom& g, double* u64, const float* c32, const double* sigma,
                         hipStream_t st) {
    const long long n4 = field_quads(g);
    k_update<<<(unsigned)((n4 + 255) / 256), 256, 0, st>>>(n4, u64, c32, sigma);
    return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes % 16) return hipErrorInvalidValue;
    const long long n16 = (long long)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    k_copy<<<(unsigned)((n16 + 255) / 256), 256, 0, st>>>(static_cast<uint4*>(dst), static_cast<const uint4*>(src),
                                                          n16);
    return hipGetLastError();
}

long long dot_blocks(size_t bytes) {
    const long long n2 = (long long)(bytes / 16);
    const long long nb = (n2 + 255) / 256;
    return nb < kDotBlocks ? (nb > 0 ? nb : 1) : kDotBlocks;
}

hipError_t launch_dot(const double* a, const double* b, size_t bytes, double* partials, hipStream_t st) {
    if (bytes % 16) return hipErrorInvalidValue;
    k_dot<<<(unsigned)dot_blocks(bytes), 256, 0, st>>>((long long)(bytes / 16), a, b, partials);
    return hipGetLastError();
}

hipError_t launch_pcg_step(double* x, const double* p, double* r, const double* q, const double* sc, size_t bytes,
                           hipStream_t st) {
    if (bytes % 16) return hipErrorInvalidValue;
    const long long n2 = (long long)(bytes / 16);
    k_pcg_step<<<(unsigned)((n2 + 255) / 256), 256, 0, st>>>(n2, x, p, r, q, sc);
    return hipGetLastError();
}

hipError_t launch_pcg_dir(double* p, const double* z, const double* sc, size_t bytes, hipStream_t st) {
    if (bytes % 16) return hipErrorInvalidValue;
    const long long n2 = (long long)(bytes / 16);
    k_pcg_dir<<<(unsigned)((n2 + 255) / 256), 256, 0, st>>>(n2, p, z, sc);
    return hipGetLastError();
}

hipError_t launch_scalar_copy(double* dst, const double* src, hipStream_t st) {
    k_scalar_copy<<<1, 64, 0, st>>>(dst, src);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
    if (bytes % 16) return hipErrorInvalidValue;
    const long long n16 = (long long)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    k_zero<<<(unsigned)((n16 + 255) / 256), 256, 0, st>>>(static_cast<uint4*>(p), n16);
    return hipGetLastError();
}

Space level_space(const Geom& g, int ncol, int col0) { return space_of(g, ncol, col0); }

hipError_t launch_batch(const BEntry* d_entries, int n, long long total, hipStream_t st) {
    if (n < 1 || total < 1) return hipSuccess;
    // ~8 resident blocks per CU on 256 CUs; smaller batches get one block per work unit
    const long long grid = total < 2048 ? total : 2048;
    k_batch<<<(unsigned)grid, 256, 0, st>>>(d_entries, n, total);
    return hipGetLastError();
}

}  // namespace mg
