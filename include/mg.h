/*
 * mg.h - C ABI of the MI355X geometric-multigrid V-cycle library (libmg.so).
 *
 * The library solves the elliptic problems that ExaStencils-style generated
 * programs solve iteratively on regular grids with stencil operators (paper,
 * Sec. 1): -Laplace(u) = f with the 5-point (2-D) or 7-point (3-D) stencil on
 * a node grid, and -div(k grad u) = f with harmonic-mean face coefficients on
 * a cell-centred grid (a per-point stencil field, ExaSlang's StencilField),
 * both on the unit square/cube with zero Dirichlet data (the paper assumes
 * Dirichlet boundaries, Sec. 2.1).  The solver is the textbook geometric
 * multigrid V-cycle named by the ExaSlang vocabulary that accompanies the
 * paper's listings: per-level stencils on coarser/coarsest levels, restriction
 * and prolongation, jacobi or color-ed relax-ation, a coarsest-level solve,
 * repeat ... until a residual criterion.
 *
 * Conventions shared by every call:
 *  - Arrays crossing the ABI are dense FP64 in C order with x fastest:
 *    a[z][y][x] (3-D) or a[y][x] (2-D).  Node grids pass n^d values including
 *    the boundary nodes (ignored on input, returned as 0); cell grids pass
 *    N^d cell values.
 *  - `on_device` = 1: the pointer is HIP device memory on the context's
 *    device; 0: ordinary host memory.  Host transfers are synchronous.
 *  - The caller owns every buffer, including the device workspace passed to
 *    mg_setup; the library never frees caller memory and allocates only small
 *    host-side metadata.  A context is bound to one HIP stream and is not
 *    thread-safe; distinct contexts may be used from distinct threads.
 *  - Every int-returning call returns MG_OK (0) or a negative MG_E* code;
 *    no C++ exception or abort crosses the ABI.  mg_last_error() returns the
 *    message of the last failure on a context.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum {
    MG_OK = 0,
    MG_EINVAL = -1,      /* bad argument: sizes, kinds, null pointers      */
    MG_ENOMEM = -2,      /* workspace too small / admission budget exceeded */
    MG_EDEVICE = -3,     /* a HIP call failed or no device is present       */
    MG_ENOTCONV = -4,    /* max_cycles reached before the tolerance         */
    MG_ENONFINITE = -5,  /* residual norm is NaN or Inf                     */
    MG_EDIVERGED = -6,   /* residual grew in 3 consecutive cycles           */
    MG_EBUSY = -7,       /* server queue full                               */
    MG_ECANCELED = -8,   /* server request cancelled by mg_server_cancel    */
    MG_ETIMEDOUT = -9    /* server request not converged by its deadline    */
};

enum { MG_NODE = 0, MG_CELL = 1 };              /* field location           */
enum { MG_LAPLACE = 0, MG_VARCOEF = 1 };        /* operator kind            */
enum { MG_DIRICHLET0 = 0, MG_NEUMANN0 = 1 };   /* boundary kind            */
enum { MG_JACOBI = 0, MG_RBGS = 1 };            /* smoother                 */
enum { MG_FP64 = 0, MG_MIXED = 1 };             /* arithmetic               */
enum { MG_CYCLE_V = 0, MG_CYCLE_W = 1, MG_CYCLE_F = 2 };   /* cycle type      */
enum { MG_PREC_FP64 = 0, MG_PREC_FP32 = 1 };    /* which level hierarchy    */
enum { MG_FIELD_U = 0, MG_FIELD_F = 1, MG_FIELD_R = 2 };

/* Grid: the domain is [0,1]^dim.
 *  MG_NODE: n[a] = nodes per axis, (coarsest_n - 1) * 2^L + 1, boundary included;
 *           coarsest_n = 5 means 3^dim unknowns on the coarsest level.
 *  MG_CELL: n[a] = cells per axis, coarsest_n * 2^L; coarsest_n = 4 typical.
 *  All axes must have the same size.  dim is 2 or 3. */
typedef struct mg_grid {
    int dim;
    int n[3];
    int centering;
    int coarsest_n;
} mg_grid;

/* Operator.  MG_LAPLACE: -Laplace.  MG_VARCOEF (cell grids only): k holds N^dim
 * positive cell coefficients (host or device per k_on_device); face
 * coefficients are their harmonic means, wall faces take the inner cell's k,
 * coarse faces are the mean of the fine faces that tile them.  k is read
 * during mg_setup only. */
typedef struct mg_stencil {
    int kind;
    const double* k;
    int k_on_device;
} mg_stencil;

/* Boundary condition.  MG_DIRICHLET0: u = 0 on the boundary (node grids:
 * the boundary nodes; cell grids: on the walls, odd ghosts).  MG_NEUMANN0:
 * zero normal flux on the walls of a cell grid (the ExaSlang `Neumann`
 * boundary): wall faces drop out of the stencil, interpolation uses even
 * ghosts; the operator annihilates constants, so mg_set_rhs projects f to
 * zero mean, every restricted right-hand side is projected likewise, the
 * coarsest solve returns the zero-mean solution (Cholesky of A + a 1 1^T)
 * and the finest iterate is projected to zero mean after every cycle.
 * Neumann needs cell centring and FP64 precision, and no krylov vectors.
 * NULL means MG_DIRICHLET0. */
typedef struct mg_bc {
    int kind;                  /* MG_DIRICHLET0 or MG_NEUMANN0 */
} mg_bc;

/* Cycle options.  omega is the Jacobi damping; nu1/nu2 pre/post sweeps;
 * post_order 0 = red (even index sum) first, 1 = black first; max_cycles caps
 * mg_solve (cycles in MG_FP64, refinement steps in MG_MIXED, each one
 * single-precision cycle).  cycle: MG_CYCLE_V (cycle index 1), MG_CYCLE_W
 * (cycle index 2: each coarser level is visited twice, the second visit
 * continuing from the first) or MG_CYCLE_F (an F-cycle from zero, then a
 * V-cycle, on each coarser level); a level directly above the coarsest is
 * visited once (Trottenberg, Oosterlee, Schueller, Multigrid, Sec. 2.4).
 * The solve server runs V-cycles only.  krylov = 1 reserves the vectors of
 * mg_pcg (five FP64 fields of the finest level; FP64 contexts).  coarse_op:
 * MG_COARSE_REDISCRETISE (every level the 5/7-point stencil with its own
 * mesh width) or MG_COARSE_GALERKIN (every coarser level the Galerkin
 * operator R A P of the next finer one, a constant 9/27-point stencil;
 * node grids, damped Jacobi, FP64). */
enum { MG_COARSE_REDISCRETISE = 0, MG_COARSE_GALERKIN = 1 };

typedef struct mg_opts {
    int smoother;
    double omega;
    int nu1, nu2;
    int precision;
    int max_cycles;
    int post_order;
    int cycle;
    int krylov;
    int coarse_op;
} mg_opts;

typedef struct mg_ctx mg_ctx;

/* ---------------------------------------------------------------- setup */
const char* mg_version(void);

/* Fill *o with the defaults: RB-GS, omega 0.8, V(2,2), FP64, 100 cycles, red first, V-cycle. */
void mg_default_opts(mg_opts* o);

/* Device workspace bytes mg_setup needs for this problem (host-only call). */
int mg_workspace_bytes(const mg_grid* g, const mg_stencil* st, const mg_opts* o, size_t* bytes);

/* Build the level hierarchy inside the caller's device workspace (256-byte
 * aligned, >= mg_workspace_bytes), upload per-level constants, face
 * coefficients and the FP64 Cholesky factor of the coarsest matrix, and zero
 * all fields.  hip_stream is a hipStream_t (NULL = default stream); every
 * later call on the context is ordered on it.  On success *out owns host
 * metadata only; release it with mg_destroy. */
int mg_setup(const mg_grid* g, const mg_stencil* st, const mg_bc* bc, const mg_opts* o,
             void* d_workspace, size_t bytes, void* hip_stream, mg_ctx** out);

void mg_destroy(mg_ctx* c);                     /* NULL-safe */

/* ---------------------------------------------------------- data in/out */
int mg_set_rhs(mg_ctx* c, const double* f, int on_device);
int mg_set_initial(mg_ctx* c, const double* u0, int on_device);   /* u0 NULL = zero */
int mg_get_solution(mg_ctx* c, double* u, int on_device);

/* -------------------------------------------------------------- compute */
/* Enqueue ncycles V(nu1,nu2)-cycles on the stream (MG_MIXED: ncycles FP64
 * refinement steps, each with one single-precision V-cycle); asynchronous.
 * Each cycle is replayed from a captured HIP graph unless profiling is on. */
int mg_vcycle(mg_ctx* c, int ncycles);

/* Full multigrid (Trottenberg, Oosterlee, Schueller, Multigrid, Sec. 2.6):
 * the right-hand side is restricted to every level, the coarsest level is
 * solved exactly, and each finer level starts from the interpolated coarser
 * solution and receives cycles_per_level cycles of the context's type; the
 * finest result becomes the iterate (a following mg_solve continues from it).
 * Overwrites the coarse levels' fields.  FP64 contexts only (MG_EINVAL
 * otherwise); asynchronous. */
int mg_fmg(mg_ctx* c, int cycles_per_level);

/* Conjugate gradients preconditioned by one cycle from zero (Saad, Iterative
 * Methods for Sparse Linear Systems, Alg. 9.1; Trottenberg et al. Sec. 7.8),
 * from the current iterate until ||f - A u||_2 / ||f - A u0||_2 <= tol or
 * max_it iterations; the result becomes the iterate and f is kept.  The
 * cycle must be symmetric: nu1 = nu2 and, with red-black GS, post_order = 1
 * (MG_EINVAL otherwise, and without krylov = 1 in the options).  FP64
 * contexts; synchronous (one 16-byte read-back per iteration).  Returns
 * MG_OK, MG_ENOTCONV or MG_ENONFINITE; the history is kept for mg_history. */
int mg_pcg(mg_ctx* c, double tol, int max_it, int* its_out, double* relres_out);

/* Cycle until ||f - A u||_2 / ||f - A u0||_2 <= tol over the unknowns;
 * synchronous.  Returns MG_OK, MG_ENOTCONV, MG_ENONFINITE or MG_EDIVERGED;
 * cycles_out / relres_out may be NULL.  Each iteration (cycle or refinement
 * step, then the residual norm) is captured once as a HIP graph on a private
 * stream and replayed on the context's stream; the results are those of the
 * same launches issued one by one.  While profiling is enabled, or if
 * capture is unavailable, the launches are issued one by one. */
int mg_solve(mg_ctx* c, double tol, int* cycles_out, double* relres_out);

/* Number of graph replays mg_solve and mg_vcycle have made on this context. */
int mg_graph_launches(const mg_ctx* c, long long* n);

/* ||f - A u||_2 over the unknowns of the finest level (FP64); synchronous. */
int mg_residual_norm(mg_ctx* c, double* out);

/* Relative residual history of the last mg_solve, starting with 1.0. */
int mg_history(const mg_ctx* c, double* buf, int cap, int* n);

/* --------------------------------------------- level access and single ops
 * For kernel-level verification and custom cycles.  Level 0 is the finest.
 * prec selects the FP64 or the single-precision hierarchy (the latter exists
 * only with MG_MIXED, where the FP64 hierarchy has level 0 only).  Values
 * cross the ABI as FP64 and are rounded to FP32 on the way in. */
int mg_levels(const mg_ctx* c, int* nlevels);
int mg_level_size(const mg_ctx* c, int level, int* n);
int mg_level_set(mg_ctx* c, int level, int field, int prec, const double* a, int on_device);
int mg_level_get(mg_ctx* c, int level, int field, int prec, double* a, int on_device);

enum {
    MG_OP_GS_RED = 0,     /* u <- GS update of red unknowns                       */
    MG_OP_GS_BLACK = 1,   /* u <- GS update of black unknowns                     */
    MG_OP_JACOBI = 2,     /* u <- u + omega D^-1 (f - A u)                        */
    MG_OP_RESIDUAL = 3,   /* r <- f - A u                                         */
    MG_OP_RESTRICT = 4,   /* f(level+1) <- R r(level)                             */
    MG_OP_PROLONG = 5,    /* u(level) <- u(level) + P u(level+1)                  */
    MG_OP_COARSE = 6,     /* u <- A^-1 f on the coarsest level (FP64 Cholesky)    */
    MG_OP_VCYCLE = 7,     /* one V-cycle starting at `level` (u, f of that level) */
    MG_OP_RESIDUAL_RESTRICT = 8, /* f(level+1) <- R (f - A u); r is not written where a
                                    fused kernel exists (3-D node levels with n >= 129,
                                    2-D node levels, the finest 3-D cell level with k,
                                    cell levels with n <= 64) */
    MG_OP_PRESMOOTH = 9,  /* u <- nu1 smoothing sweeps, as the V-cycle's pre-smoothing
                             (red-black: red first); on 3-D node levels with
                             n >= 257 up to three red-black sweeps run as one fused
                             pass, on 2-D node levels two damped-Jacobi sweeps per
                             launch, bitwise equal to the separate sweeps        */
    MG_OP_POSTSMOOTH = 10, /* u <- nu2 sweeps, as the post-smoothing (post_order)    */
    MG_OP_PRESMOOTH_RESTRICT = 11 /* MG_OP_PRESMOOTH then MG_OP_RESIDUAL_RESTRICT, as the
                             V-cycle runs them (2-D node levels with damped Jacobi
                             and nu1 >= 2: the last two sweeps, the residual and the
                             restriction in one launch, bitwise equal)           */
};
int mg_apply(mg_ctx* c, int op, int level, int prec);

/* -------------------------------------------------------------- profiling
 * When enabled, every kernel launch is bracketed by HIP events on the
 * context's stream.  mg_profile_read synchronises the stream and returns the
 * launch count and summed milliseconds of one kernel class on one level
 * (level -1 = all levels). */
enum {
    MG_K_SMOOTH = 0, MG_K_RESIDUAL = 1, MG_K_RESTRICT = 2, MG_K_PROLONG = 3,
    MG_K_COARSE = 4, MG_K_REDUCE = 5, MG_K_CAST = 6, MG_K_UPDATE = 7, MG_K_COPY = 8,
    MG_K_COUNT = 9
};
int mg_profile(mg_ctx* c, int enable);          /* enabling clears the record */
int mg_profile_read(mg_ctx* c, int kclass, int level, int* count, double* ms);

/* ---------------------------------------------------------------- serving
 * A solve server keeps level hierarchies resident in one caller-owned device
 * arena and runs many mixed-precision solves at once.  Work advances in
 * rounds: in each round every in-flight request performs one FP64
 * refinement step (a newly admitted request also loads its right-hand side
 * and computes its initial residual), and launch k of the round runs op k
 * of every in-flight request in one persistent batched kernel.  One host
 * synchronisation per round reads all residual norms; converged requests
 * write their solution and retire, and queued requests are admitted in FIFO
 * order as slots and arena bytes free up (their footprint is checked against
 * the arena before admission).  Idle hierarchies stay resident for reuse by
 * later requests of the same shape and are evicted, least recently used
 * first, when a different shape needs the memory.
 *
 * A request's arithmetic does not depend on what else is in flight: it runs
 * the same kernels on its own hierarchy with per-request reductions, so its
 * result is bitwise the same alone and in any mix. */
typedef struct mg_server mg_server;

typedef struct mg_server_opts {
    void* d_arena;          /* caller-owned device buffer, 256-byte aligned   */
    size_t arena_bytes;     /* HBM budget of the server                       */
    int max_slots;          /* requests in flight at most (1 .. 4096)         */
    int max_queue;          /* queued requests at most; submit beyond: MG_EBUSY */
    void* hip_stream;       /* hipStream_t for all server work (NULL default)  */
} mg_server_opts;

/* A solve request.  grid: MG_NODE, dim 2 or 3; opts: smoother, omega, nu1,
 * nu2, max_cycles (refinement steps); precision is always MG_MIXED.  f and
 * u_out are device arrays of n^dim doubles (C order, boundary included);
 * the caller keeps them valid until the request's result is polled.
 * t_arrive is the arrival time on the server clock (mg_server_clock).
 * deadline (server clock, <= 0 = none): a request not converged when a round
 * ends at or after it is retired with MG_ETIMEDOUT (u_out receives its
 * iterate so far, relres its residual); one still queued at its deadline is
 * retired unadmitted (steps 0, u_out untouched). */
typedef struct mg_request {
    uint64_t id;
    mg_grid grid;
    mg_opts opts;
    double tol;
    const double* f;
    double* u_out;
    double t_arrive;
    double deadline;
} mg_request;

typedef struct mg_result {
    uint64_t id;
    uint64_t ticket;        /* the ticket mg_server_submit returned           */
    int status;             /* MG_OK, MG_ENOTCONV, MG_ENONFINITE, MG_ECANCELED,
                               MG_ETIMEDOUT                                   */
    int steps;              /* refinement steps (single-precision V-cycles)   */
    double relres;          /* ||f - A u|| / ||f|| of the returned solution   */
    double t_arrive, t_admit, t_done;   /* server clock, seconds               */
} mg_result;

typedef struct mg_server_stats {
    long long rounds, launches, admitted, completed, hierarchies_built, evictions;
    size_t arena_peak_bytes, arena_used_bytes;
    int in_flight, queued, resident;
    /* algorithmic device-memory bytes of the batched launches so far: each
     * op's compulsory reads and writes (e.g. 12 B per point of an FP32
     * Jacobi sweep, 24 B of an FP64 residual), summed over every op run */
    double algorithmic_bytes;
} mg_server_stats;

/* Device bytes one resident hierarchy of this grid and options occupies. */
int mg_server_footprint(const mg_grid* g, const mg_opts* o, size_t* bytes);
int mg_server_create(const mg_server_opts* o, mg_server** out);
/* A server whose rounds run through host callbacks instead of the batched
 * device kernels, and which makes no HIP call: the scheduler is the one
 * above (FIFO queue, tickets, footprint admission against arena_bytes,
 * resident hierarchies reused by shape and evicted least recently used
 * first, one step per request per round, deadlines, cancellation, the
 * clock), so that its logic runs on machines without a GPU.  The library
 * computes nothing on this path; its own tests drive it with the CPU
 * reference implementation as the executor.  d_arena and hip_stream are
 * ignored, and f and u_out are whatever the executor takes them to be.
 * A callback returning an MG_E* code aborts the round (mg_server_step
 * returns it). */
typedef struct mg_server_executor {
    void* user;
    /* a hierarchy of r's shape now occupies slot (0 .. 4 max_slots - 1),
     * which later requests of the same shape reuse; 0 or an MG_E* code */
    int (*build)(void* user, int slot, const mg_request* r);
    /* one round: request reqs[i] runs its next refinement step on the
     * hierarchy in slots[i] (first loading f and forming its initial
     * residual when first[i] != 0); norms[2 i] receives the sum of squares
     * of that initial residual (first steps only), norms[2 i + 1] that of
     * the residual after the step */
    int (*step)(void* user, int count, const int* slots, const int* first, const mg_request* reqs,
                double* norms);
    /* the request in slot retired after at least one step (converged, out
     * of steps or past its deadline): its iterate goes to r->u_out */
    int (*finish)(void* user, int slot, const mg_request* r);
    /* the hierarchy in slot was evicted (NULL: not told) */
    void (*release)(void* user, int slot);
} mg_server_executor;
int mg_server_create_hosted(const mg_server_opts* o, const mg_server_executor* ex, mg_server** out);
void mg_server_destroy(mg_server* s);                  /* NULL-safe */
double mg_server_clock(const mg_server* s);           /* seconds since create */
/* Queue a request (copies the descriptor, not the arrays).  *ticket (if not
 * NULL) receives the server's sequence number of the request, 0, 1, 2, ...
 * in submission order, unique for the server's lifetime and echoed in its
 * result.  MG_EBUSY when the queue is full, MG_EINVAL for unsupported
 * grids/options, MG_ENOMEM when the request alone cannot fit the arena (no
 * ticket is issued then).  The server does no work between calls: rounds
 * run in mg_server_step, on the caller's thread. */
int mg_server_submit(mg_server* s, const mg_request* r, uint64_t* ticket);
/* Run one round; *in_flight receives the requests still in flight and
 * *queued those waiting.  Synchronous. */
int mg_server_step(mg_server* s, int* in_flight, int* queued);
/* Cancel the request with this ticket: a queued one is retired at once, one
 * in flight at the start of the next round (its slot freed, no further
 * work); either way its result carries MG_ECANCELED and u_out is left as
 * it is.  MG_EINVAL for a ticket that is unknown or already finished. */
int mg_server_cancel(mg_server* s, uint64_t ticket);
/* Move up to cap finished results to out; *n receives the count. */
int mg_server_poll(mg_server* s, mg_result* out, int cap, int* n);
int mg_server_get_stats(const mg_server* s, mg_server_stats* st);
const char* mg_server_last_error(const mg_server* s);

/* ------------------------------------------------------------------ errors */
const char* mg_strerror(int code);
const char* mg_last_error(const mg_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* MG_H */
