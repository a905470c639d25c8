// Host-side state of a multigrid context (internal to libmg).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "mg.h"
#include "mg_internal.h"
#include "mg_kernels.h"

namespace mg {

constexpr int kMaxLevels = 16;

// Byte offsets of one level's fields inside the workspace, per precision
// (0 = FP64, 1 = FP32); SIZE_MAX = absent.
struct LevelPlan {
    Geom g;
    bool has[2] = {false, false};
    size_t u[2] = {SIZE_MAX, SIZE_MAX}, f[2] = {SIZE_MAX, SIZE_MAX}, r[2] = {SIZE_MAX, SIZE_MAX};
    size_t utmp[2] = {SIZE_MAX, SIZE_MAX};
    size_t beta[2][3] = {{SIZE_MAX, SIZE_MAX, SIZE_MAX}, {SIZE_MAX, SIZE_MAX, SIZE_MAX}};
    size_t k = SIZE_MAX;          // FP64 cell values, colour-split (finest 3-D cell level)
};

struct Plan {
    int L = 0, m = 0;
    std::vector<LevelPlan> lv;
    long long partial_pairs = 0;
    size_t partials = 0, reduce_scratch = 0, red = 0, chol = 0, staging = 0, total = 0;
    size_t pcg = SIZE_MAX;        // x, p, q, saved f, zero (finest FP64 fields), partials, scratch, scalars
};

// Workspace layout for a problem; returns the total byte count.
size_t plan_workspace(const mg_grid* g, const mg_stencil* st, const mg_opts* o, Plan* out, bool staging);

struct Ctx;
// Validate, lay out and initialise a context inside d_workspace (staging:
// reserve a host-transfer buffer for host-pointer I/O).
int setup_ctx(const mg_grid* g, const mg_stencil* st, const mg_opts* o, void* d_workspace, size_t bytes,
              hipStream_t stream, bool staging, Ctx** out, std::string* errmsg, int bc_kind = MG_DIRICHLET0);

struct Level {
    Geom g;
    bool has[2] = {false, false};
    void* u[2] = {nullptr, nullptr};
    void* f[2] = {nullptr, nullptr};
    void* r[2] = {nullptr, nullptr};
    void* utmp[2] = {nullptr, nullptr};
    void* beta[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    void* k = nullptr;            // FP64 cell values, colour-split (finest 3-D cell level)
    size_t field_bytes[2] = {0, 0};
    bool gal = false;             // Galerkin stencil W instead of the 5/7-point operator
    Stencil27 W{};
};

struct Rec {
    int kclass, level;
    hipEvent_t e0, e1;
};

struct Ctx {
    mg_grid grid{};
    mg_opts opts{};
    int kind = MG_LAPLACE;
    bool neu = false;             // Neumann walls (cell grids, FP64)
    void* base = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    int L = 0, m = 0;
    std::vector<Level> lv;
    long long partial_pairs = 0;
    double* partials = nullptr;
    double* reduce_scratch = nullptr;
    double* red = nullptr;        // [sum r^2, max |r|, sigma, scale basis, projection sum, next sigma]
    double* chol = nullptr;
    double* staging = nullptr;
    // preconditioned CG (krylov = 1): finest-level FP64 vectors and scalars
    void* pcg_v[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // x, p, q = -A p, saved f, zero
    double* pcg_part = nullptr;
    double* pcg_scratch = nullptr;
    double* pcg_s = nullptr;      // [rho, -, p.q, -, rho_new, -, r.r, -]
    std::vector<double> hist;
    std::string err;
    std::vector<std::vector<double>> coarse_beta_host;
    // profiling
    bool prof = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double agg_ms[MG_K_COUNT][kMaxLevels] = {};
    int agg_n[MG_K_COUNT][kMaxLevels] = {};
    // recording mode (batched execution): ops append descriptors here
    std::vector<BItem>* rec = nullptr;
    double* rec_res = nullptr;    // extra destination of recorded norm reductions
    long long last_partials = 0;  // norm partial pairs of the last residual
    // mixed precision: red[3] holds the largest |r| of the latest finest
    // residual, the scale basis of the next refinement step's cast; false
    // after a new right-hand side, iterate or level write
    bool scale_known = false;
    // per precision: the level from which a V-cycle runs in one workgroup
    // with its fields in LDS (-1: none), and that launch's plan
    int tail_l[2] = {-1, -1};
    TailPlan tail[2] = {};
    BItem item(int op, int l) const;
    int push(BItem it);
    int rec_check(int pr, bool want_fp32);

    int fail(int code, const std::string& msg);
    int dev(hipError_t e, const char* what);
    void* at(size_t off) const;
    Faces faces(int l, int pr) const;
    double scale(int l) const;
    hipEvent_t begin();
    hipEvent_t event();
    int record(int kclass, int level, hipError_t e, hipEvent_t e0, const char* what);

    int gs(int l, int pr, int colour, bool zero);
    int jacobi(int l, int pr, bool zero);
    int smooth(int l, int pr, int sweeps, bool from_zero, int first_colour);
    int residual(int l, int pr, bool norm, bool store, bool reduce = true);
    int reduce_norm(int l);
    int residual_cast(bool first);
    int restrict_to(int l, int pr);
    int residual_restrict(int l, int pr);
    int presmooth_restrict(int l, int pr, bool from_zero);
    int prolong(int l, int pr, int mask);
    int coarse(int pr);
    int vcycle(int l, int pr, bool from_zero);
    int cycle(int l, int pr, bool from_zero, int kind);
    void plan_tail();
    int tail_cycle(int l, int pr, bool from_zero);
    int fmg(int cpl);
    int project(int l, void* a);
    int pcg(double tol, int max_it, int* its_out, double* relres_out);
    int refine_step(bool defer = false);
    bool fused_update() const;
    int update_residual_cast();
    int read_red(double* sq, double* mx);
    int norm(double* out);
    int step(int k);
    int solve(double tol, int* cycles_out, double* relres_out);

    // One solve iteration (a V-cycle, or a refinement step in mixed mode)
    // followed by the residual norm, replayed from a captured HIP graph when
    // profiling is off: the ~100 launches of a cycle cost one graph launch.
    // Operations swap level buffers on the host (Jacobi and fused sweeps run
    // out of place), so a graph is keyed by the buffer assignment it was
    // captured from and restores the assignment it leaves.
    // With profiling on the launches are issued one by one, bracketed by
    // events (elapsed times of events recorded by graph nodes are not
    // available from the runtime).
    struct Graph {
        int kind = 0;   // 0: iteration + norm copied to h_red (mg_solve); 1: one step (mg_vcycle)
        std::vector<void*> pre, post;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;
    hipStream_t cap_stream = nullptr;
    double* h_red = nullptr;    // pinned copy of red[0..1] written by the graph
    bool graphs_off = false;
    long long graph_launches = 0;
    void add_times(const std::vector<Rec>& rs);
    std::vector<void*> buffers() const;
    void set_buffers(const std::vector<void*>& b);
    const Graph* capture(int kind);
    const Graph* replayable(int kind);
    int iterate(double* nr);
    int step_once();
    ~Ctx();
};

}  // namespace mg
