/* Host-only checks of libmg for an AddressSanitizer + UndefinedBehaviorSanitizer
 * build (host code instrumented, no GPU needed): the workspace and footprint
 * planners over many grids and options, argument validation of every entry
 * point that rejects before touching a device, the exact DG tables and the
 * basis values, and the server's scheduler driven by a host executor.  Exits non-zero on the first unexpected return code; the
 * sanitizers abort on any memory or undefined-behaviour error. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "dg.h"
#include "mg.h"

static int fails = 0;

static void expect(int got, int want, const char* what) {
    if (got != want) {
        fprintf(stderr, "%s: returned %d, expected %d\n", what, got, want);
        ++fails;
    }
}

static void planners(void) {
    static const int sizes2[] = {9, 17, 33, 129, 1025};
    static const int sizes3[] = {9, 17, 65, 257, 513};
    static const int cells[] = {8, 16, 32, 256};
    for (int prec = 0; prec < 2; ++prec)
        for (int sm = 0; sm < 2; ++sm)
            for (int kry = 0; kry < 2; ++kry)
                for (int dim = 2; dim <= 3; ++dim)
                    for (int i = 0; i < 5; ++i) {
                        mg_opts o;
                        mg_default_opts(&o);
                        o.precision = prec ? MG_MIXED : MG_FP64;
                        o.smoother = sm ? MG_RBGS : MG_JACOBI;
                        o.krylov = prec ? 0 : kry;
                        const int n = dim == 2 ? sizes2[i] : sizes3[i];
                        mg_grid g = {dim, {n, n, dim == 3 ? n : 1}, MG_NODE, 5};
                        size_t b = 0, fb = 0;
                        expect(mg_workspace_bytes(&g, NULL, &o, &b), MG_OK, "workspace (node)");
                        if (b == 0) expect(1, 0, "workspace bytes > 0");
                        if (prec && sm == 0 && dim == 2) expect(mg_server_footprint(&g, &o, &fb), MG_OK, "footprint");
                        if (!prec && !kry) {
                            o.coarse_op = MG_COARSE_GALERKIN;
                            o.smoother = MG_JACOBI;
                            expect(mg_workspace_bytes(&g, NULL, &o, &b), MG_OK, "workspace (Galerkin)");
                        }
                    }
    /* cell grids, variable coefficient */
    for (int i = 0; i < 4; ++i) {
        const int n = cells[i];
        double* k = (double*)malloc(sizeof(double) * (size_t)n * n * n);
        for (long long j = 0; j < (long long)n * n * n; ++j) k[j] = 1.0 + 0.5 * (double)(j % 7);
        mg_stencil st = {MG_VARCOEF, k, 0};
        mg_grid g = {3, {n, n, n}, MG_CELL, 4};
        mg_opts o;
        mg_default_opts(&o);
        size_t b = 0;
        expect(mg_workspace_bytes(&g, &st, &o, &b), MG_OK, "workspace (cell)");
        o.precision = MG_MIXED;
        expect(mg_workspace_bytes(&g, &st, &o, &b), MG_OK, "workspace (cell, mixed)");
        free(k);
    }
    /* rejected before any device work */
    mg_opts o;
    mg_default_opts(&o);
    size_t b = 0;
    mg_grid bad = {4, {9, 9, 9}, MG_NODE, 5};
    expect(mg_workspace_bytes(&bad, NULL, &o, &b), MG_EINVAL, "workspace: dim 4");
    mg_grid odd = {2, {10, 10, 1}, MG_NODE, 5};
    expect(mg_workspace_bytes(&odd, NULL, &o, &b), MG_EINVAL, "workspace: n = 10");
    expect(mg_workspace_bytes(NULL, NULL, &o, &b), MG_EINVAL, "workspace: no grid");
    mg_ctx* c = NULL;
    expect(mg_setup(&bad, NULL, NULL, &o, NULL, 0, NULL, &c), MG_EINVAL, "setup: dim 4");
    if (c) expect(1, 0, "setup left a context");
    expect(mg_server_create(NULL, NULL), MG_EINVAL, "server: no options");
    for (int code = 0; code >= -12; --code)
        if (!mg_strerror(code)) expect(1, 0, "strerror");
}

static void dg_tables(void) {
    for (int k = 0; k <= 3; ++k) {
        const long long nr = dg_reference_size(k), np = dg_product_size(k), ne = dg_edge_table_size(k);
        if (nr <= 0 || np <= 0 || ne <= 0) expect(1, 0, "DG table sizes");
        double* r = (double*)malloc(sizeof(double) * (size_t)nr);
        double* p = (double*)malloc(sizeof(double) * (size_t)np);
        double* e = (double*)malloc(sizeof(double) * (size_t)ne);
        expect(dg_reference_integrals(k, r), MG_OK, "reference integrals");
        expect(dg_product_integrals(k, p), MG_OK, "product integrals");
        expect(dg_edge_integrals(k, e), MG_OK, "edge integrals");
        const int K = (k + 1) * (k + 2) / 2;
        double x[5] = {0.1, 0.2, 0.3, 0.0, 1.0}, y[5] = {0.1, 0.5, 0.3, 0.0, 0.0};
        double* v = (double*)malloc(sizeof(double) * 5 * (size_t)K);
        expect(dg_basis_values(k, 5, x, y, v), MG_OK, "basis values");
        free(r);
        free(p);
        free(e);
        free(v);
    }
    expect(dg_reference_integrals(4, NULL), MG_EINVAL, "reference integrals: k = 4");
    expect((int)(dg_reference_size(-1) > 0), 0, "reference size: k = -1");
    /* device entry points: rejected (or empty) before touching a device */
    expect(dg_volume_integrals(7, 1, NULL, NULL, NULL, NULL, 9.81, NULL, NULL, NULL), MG_EINVAL, "volume: k = 7");
    expect(dg_volume_integrals(1, 0, NULL, NULL, NULL, NULL, 9.81, NULL, NULL, NULL), MG_OK, "volume: no elements");
    expect(dg_velocity_projection(2, 5, NULL, NULL, NULL, NULL, NULL, NULL), MG_EINVAL, "projection: null arrays");
    expect(dg_edge_terms(3, 4, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, NULL, 9.81, NULL, NULL, NULL), MG_EINVAL,
           "edges: null arrays");
    expect(dg_ssp_rk3_step_noalloc(1, 10, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL, NULL, 9.81, 0.0, 0.0, NULL, NULL,
                                   NULL, NULL, 0.5, NULL),
           MG_EINVAL, "noalloc step: null arrays");
}

/* The server's scheduler with a host executor whose requests "converge" by
 * a factor 10 per step: queue, admission against a budget of two
 * hierarchies, reuse, eviction, cancellation and deadlines under the
 * sanitizers. */
static int steps_of[64];
static int ex_build(void* user, int slot, const mg_request* r) {
    (void)user;
    return (slot < 0 || r->grid.n[0] < 9) ? MG_EINVAL : MG_OK;
}
static int ex_step(void* user, int count, const int* slots, const int* first, const mg_request* reqs, double* norms) {
    (void)user;
    (void)slots;
    for (int i = 0; i < count; ++i) {
        const int id = (int)reqs[i].id;
        if (first[i]) steps_of[id] = 0;
        ++steps_of[id];
        double v = 1.0;
        for (int k = 0; k < steps_of[id]; ++k) v *= 0.01;
        norms[2 * i] = first[i] ? 1.0 : 0.0;
        norms[2 * i + 1] = v;
    }
    return MG_OK;
}
static int ex_finish(void* user, int slot, const mg_request* r) {
    (void)user;
    (void)slot;
    r->u_out[0] = (double)steps_of[r->id];
    return MG_OK;
}
static void ex_release(void* user, int slot) {
    (void)user;
    (void)slot;
}

static void hosted_server(void) {
    static const int shapes[4][2] = {{2, 33}, {3, 17}, {2, 65}, {3, 9}};
    size_t fp[4], big = 0;
    for (int s = 0; s < 4; ++s) {
        mg_grid g = {shapes[s][0], {shapes[s][1], shapes[s][1], shapes[s][0] == 3 ? shapes[s][1] : 1}, MG_NODE, 5};
        mg_opts o;
        mg_default_opts(&o);
        o.precision = MG_MIXED;
        expect(mg_server_footprint(&g, &o, &fp[s]), MG_OK, "server footprint");
        if (fp[s] > big) big = fp[s];
    }
    mg_server_opts so;
    memset(&so, 0, sizeof(so));
    so.arena_bytes = 2 * big;
    so.max_slots = 3;
    so.max_queue = 64;
    mg_server_executor ex = {NULL, ex_build, ex_step, ex_finish, ex_release};
    mg_server* srv = NULL;
    expect(mg_server_create_hosted(&so, &ex, &srv), MG_OK, "hosted server");
    if (!srv) return;
    static double f[64], u[64];
    uint64_t tk[40];
    for (int i = 0; i < 40; ++i) {
        const int s = i % 4;
        mg_request r;
        memset(&r, 0, sizeof(r));
        r.id = (uint64_t)i;
        r.grid = (mg_grid){shapes[s][0], {shapes[s][1], shapes[s][1], shapes[s][0] == 3 ? shapes[s][1] : 1}, MG_NODE,
                           5};
        mg_default_opts(&r.opts);
        r.opts.precision = MG_MIXED;
        r.tol = 1e-7;
        r.f = &f[i];
        r.u_out = &u[i];
        r.deadline = (i % 13 == 5) ? 1e-12 : 0.0;   /* past at the first round */
        expect(mg_server_submit(srv, &r, &tk[i]), MG_OK, "hosted submit");
    }
    expect(mg_server_cancel(srv, tk[7]), MG_OK, "hosted cancel");
    int in_flight = 1, queued = 1, rounds = 0, got = 0, ok = 0;
    mg_result res[64];
    while ((in_flight || queued) && rounds < 1000) {
        expect(mg_server_step(srv, &in_flight, &queued), MG_OK, "hosted step");
        int n = 0;
        expect(mg_server_poll(srv, res, 64, &n), MG_OK, "hosted poll");
        for (int k = 0; k < n; ++k) ok += res[k].status == MG_OK;
        got += n;
        ++rounds;
    }
    int n = 0;
    expect(mg_server_poll(srv, res, 64, &n), MG_OK, "hosted poll");
    got += n;
    mg_server_stats st;
    expect(mg_server_get_stats(srv, &st), MG_OK, "hosted stats");
    expect(got, 40, "hosted: every request retired");
    expect(ok, 40 - 1 - 3, "hosted: converged requests");
    expect((int)(st.arena_peak_bytes <= so.arena_bytes), 1, "hosted: budget respected");
    expect((int)(st.evictions > 0), 1, "hosted: idle hierarchies evicted");
    mg_server_destroy(srv);
    expect(mg_server_create_hosted(&so, NULL, &srv), MG_EINVAL, "hosted: no executor");
}

int main(void) {
    printf("%s\n", mg_version());
    planners();
    dg_tables();
    hosted_server();
    if (fails) {
        fprintf(stderr, "%d unexpected return codes\n", fails);
        return 1;
    }
    printf("host checks passed\n");
    return 0;
}
