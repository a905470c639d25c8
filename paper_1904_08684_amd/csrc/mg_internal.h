// Internal layout and launch descriptors shared by the kernels and the runtime.
//
// Colour-split storage.  Every level field keeps its two colours (red = even
// index sum, black = odd) in separate half arrays: the entry at grid index
// (x, y, z) lives in colour plane c = (x + y + z) & 1 at (z, y, x >> 1).
// A red-black Gauss-Seidel half-sweep then reads one whole colour, writes the
// other, and touches no byte it does not need (8 B read of the other colour,
// 8 B read of f, 8 B write per updated point, FP64), where an interleaved
// layout drags both colours through HBM on every half-sweep.  All six axis
// neighbours of a point sit in the other colour plane: the y and z
// neighbours at the same x >> 1, the x neighbours at x >> 1 - 1 + p and
// x >> 1 + p where p = x & 1.
//
// Node grids keep their boundary nodes (always zero); cell grids have no
// boundary entries and handle walls with mirror ghosts inside the kernels.
#pragma once

#include <cmath>
#include <cstdint>

namespace mg {

// Geometry of one level in colour-split storage (element strides).
struct Geom {
    int dim;          // 2 or 3
    int n;            // nodes (node grid) or cells (cell grid) per axis
    int cell;         // 1 for a cell grid
    int nz, ny;       // array extents in z (1 in 2-D) and y
    int half;         // entries per colour row actually used
    int pitch;        // row pitch in elements (>= half)
    long long plane;  // ny * pitch
    long long cs;     // colour stride: nz * plane
    // face-coefficient arrays (cell grids): natural layout, [z][y][x]
    int fpitch;       // row pitch, >= n + 1
    long long fplane; // (n + 1) * fpitch
    long long fsize;  // elements per face array (nz_f * fplane)
    int neu;          // cell grid with zero-flux (Neumann) walls
};

// Iteration space of one launch over colour-split points and its tiling into
// blocks of (1<<lx) x (1<<ly) x (1<<lz) threads.
struct Space {
    int xr, y0, yr, z0, zr;  // xs in [0, xr), y in [y0, y0+yr), z in [z0, z0+zr)
    int ncol, col0;          // colours col0 .. col0+ncol-1
    int lx, ly, lz;          // log2 tile extents
    int ntx, nty, ntz;       // tiles per axis
    long long blocks() const { return (long long)ntx * ncol * nty * ntz; }
    int threads() const { return 1 << (lx + ly + lz); }
};

static inline int ilog2ceil(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Tile a space: x extent up to 64 lanes (one wavefront per row), the rest of
// a 256-thread block over y, then z, each clipped to the space.
static inline Space make_space(int xr, int y0, int yr, int z0, int zr, int ncol, int col0) {
    Space s;
    s.xr = xr; s.y0 = y0; s.yr = yr; s.z0 = z0; s.zr = zr; s.ncol = ncol; s.col0 = col0;
    s.lx = ilog2ceil(xr) < 6 ? ilog2ceil(xr) : 6;
    int rem = 8 - s.lx;
    int ly = ilog2ceil(yr);
    s.ly = ly < rem ? ly : rem;
    rem -= s.ly;
    int lz = ilog2ceil(zr);
    s.lz = lz < rem ? lz : rem;
    s.ntx = (xr + (1 << s.lx) - 1) >> s.lx;
    s.nty = (yr + (1 << s.ly) - 1) >> s.ly;
    s.ntz = (zr + (1 << s.lz) - 1) >> s.lz;
    return s;
}

// Column-marching tiling of a 3-D node level: blocks of 64 x rows threads
// over (x >> 1, y); each thread walks `zc` consecutive planes of its column
// and keeps the z-1 / z / z+1 values of the colour it reads in registers, so
// every plane of that colour is fetched once per launch instead of three
// times (the plane distance exceeds what one XCD's L2 keeps).
struct ZSpace {
    int xr;          // xs in [0, xr)
    int rows;        // y extent of a block (blockDim.y)
    int zc;          // planes per block
    int ntx, nty, ntz;
    long long blocks() const { return (long long)ntx * nty * ntz; }
};

// Planes per block and rows per block, measured on MI355X at 513^3: 8-plane
// chunks keep ~16 K blocks in flight with little halo re-read; 4 rows of 64
// lanes per block.
constexpr int kZChunk = 8;
constexpr int kZRows = 4;

// A field larger than the 256 MB Infinity Cache streams from HBM: such
// levels read f and write the updated colour with non-temporal accesses;
// smaller levels keep default caching so that consecutive sweeps hit in cache.
static inline bool streams_from_hbm(const Geom& g, size_t elem_bytes) {
    return (size_t)(2 * g.cs) * elem_bytes > (size_t(256) << 20);
}

static inline bool use_zmarch(const Geom& g) {
    return g.dim == 3 && !g.cell && (g.n - 1) / 2 >= 64;
}

static inline ZSpace make_zspace(const Geom& g) {
    ZSpace z;
    z.xr = (g.n - 1) / 2;
    z.rows = kZRows;
    const int planes = g.n - 2;
    int zc = kZChunk;
    if (zc > planes) zc = planes;
    z.zc = zc;
    z.ntx = (z.xr + 63) / 64;
    z.nty = (g.n - 2 + z.rows - 1) / z.rows;
    z.ntz = (planes + zc - 1) / zc;
    return z;
}

// Column-marching tiling of a 3-D cell level (all cells are unknowns):
// (x >> 1, y) columns over chunks of kZChunk planes, blocks of 64 x kZRows.
static inline bool use_cell_zm(const Geom& g) {
    return g.dim == 3 && g.cell && g.n / 2 >= 64;
}

static inline ZSpace make_czspace(const Geom& g) {
    ZSpace z;
    z.xr = g.n / 2;
    z.rows = kZRows;
    z.zc = kZChunk < g.n ? kZChunk : g.n;
    z.ntx = (z.xr + 63) / 64;
    z.nty = (g.n + z.rows - 1) / z.rows;
    z.ntz = (g.n + z.zc - 1) / z.zc;
    return z;
}

// Row-marching tiling of a 2-D node level: 256-thread blocks of 64 lanes
// over x >> 1 times `rows` row chunks; each thread walks `yc` consecutive rows
// of its column and keeps rows y-1, y, y+1 of both colours in registers.
struct YSpace {
    int xr;          // xs in [0, xr)
    int yc;          // rows per thread
    int rows;        // row chunks per block
    int ntx, nty;
    long long blocks() const { return (long long)ntx * nty; }
};

constexpr int kYChunk = 16;
constexpr int kYRows = 4;

// Stand-alone 2-D levels run a thread per point: it spreads a level over
// more workgroups and measured faster than row marching at every size (a
// Jacobi V(2,2)-cycle at 129^2 78 against 120 us, 513^2 114 against 255 us,
// 1025^2 173 against 372 us).  The batched server keeps the row-marching
// forms for its large 2-D requests (use_ymarch_batched), where a launch
// holds many requests and fewer, larger tiles pay.
static inline bool use_ymarch(const Geom& g) {
    (void)g;
    return false;
}

static inline bool use_ymarch_batched(const Geom& g) {
    return g.dim == 2 && !g.cell && (g.n - 1) / 2 >= 64;
}

static inline YSpace make_yspace(const Geom& g) {
    YSpace y;
    y.xr = (g.n - 1) / 2;
    y.yc = kYChunk;
    y.rows = kYRows;
    y.ntx = (y.xr + 63) / 64;
    y.nty = (g.n - 2 + y.yc * y.rows - 1) / (y.yc * y.rows);
    return y;
}

// Temporally blocked red-black GS on a 3-D node level: a block owns a region
// of 64 x R positions (x >> 1, y) with a halo of ceil(S/2) positions in
// x >> 1 and S rows in y, and marches z over a chunk of `zc` output planes
// plus S planes of wavefront lead-in and lead-out on either side.
struct TbSpace {
    int S, R;        // half-sweeps fused, region rows
    int ntx, nty, ntz, zc;
    long long blocks() const { return (long long)ntx * nty * ntz; }
};

constexpr int kTbLanes = 64;

static inline bool use_tb(const Geom& g) {
    return g.dim == 3 && !g.cell && g.n >= 257;
}

static inline TbSpace make_tbspace(const Geom& g, int S, int rows) {
    TbSpace t;
    t.S = S;
    t.R = rows;
    const int H = (S + 1) / 2;
    t.ntx = (g.half + kTbLanes - 2 * H - 1) / (kTbLanes - 2 * H);
    const int ry = rows - 2 * S;
    t.nty = (g.n + ry - 1) / ry;
    // one resident block per CU: pick the chunk length that minimises
    // (rounds of 256 blocks) x (wavefront steps per block)
    const int planes = g.n - 2;
    long long best = -1;
    t.zc = planes;
    t.ntz = 1;
    for (int c = 1; c <= 64; ++c) {
        const int zc = (planes + c - 1) / c;
        const int nz = (planes + zc - 1) / zc;
        const long long nb = (long long)t.ntx * t.nty * nz;
        const long long cost = ((nb + 255) / 256) * (zc + 2 * S);
        if (best < 0 || cost < best) {
            best = cost;
            t.zc = zc;
            t.ntz = nz;
        }
    }
    return t;
}

// The lower part of a V-cycle in one workgroup: every level from
// lg[0] down to the coarsest keeps its iterate, a second buffer (Jacobi's
// output and the residual) and its right-hand side in LDS, in colour-split
// layout with rows of exactly `half` entries.  Offsets are in elements of
// the hierarchy's precision; the spaces are those of the per-level launches
// (one colour each, both colours, and the prolongation's colour mask).  The
// coarsest level's Cholesky factor follows the fields in LDS.
constexpr int kTailMax = 6;
// Largest 2-D level of a damped-Jacobi tail: a 129^2 Jacobi V(2,2) cycle
// measured 64.3 us with the tail from 65^2, 54.6 from 33^2, 53.8 from 17^2
// and 55.9 us from 9^2.
constexpr int kTail2DJacobiMax = 17;
constexpr int kTailThreads = 1024;
constexpr int kTailLdsBytes = 156 * 1024;

struct TailPlan {
    int nl;                       // levels, the last one the coarsest
    int rbgs;                     // 1 red-black Gauss-Seidel, 0 damped Jacobi
    int nu1, nu2, post_order;
    int from_zero;                // the top level starts from a zero iterate
    int m;                        // coarsest unknowns
    int elems;                    // LDS elements in use
    double omega;
    const double* chol;           // Cholesky factor of the coarsest matrix
    const void* beta[kTailMax][3];  // face coefficients (cell grids), device memory
    Geom g0;                      // the top level in device memory
    Geom lg[kTailMax];            // every level in LDS
    Space one[kTailMax][2], all[kTailMax], pro[kTailMax];
    int oa[kTailMax], ob[kTailMax], of[kTailMax];
    double s[kTailMax];
    double rs[kTailMax];          // 1 / s
    int p2;                       // every s is a power of two (rs exact)
};

// Is the operator scale s = 1 / h^2 a power of two (its reciprocal exact)?
static inline bool pow2_scale(double s) {
    int e;
    return s > 0.0 && std::frexp(s, &e) == 0.5;
}

// LDS geometry of a level: rows of exactly `half` entries (face arrays keep
// their device-memory layout).
static inline Geom tail_geom(const Geom& g) {
    Geom l = g;
    l.pitch = g.half;
    l.plane = (long long)g.ny * g.half;
    l.cs = (long long)g.nz * l.plane;
    return l;
}

}  // namespace mg
