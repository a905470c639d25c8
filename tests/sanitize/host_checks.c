/* Host-only checks of libmg for an AddressSanitizer + UndefinedBehaviorSanitizer
 * build (host code instrumented, no GPU needed): the workspace and footprint
 * planners over many grids and options, argument validation of every entry
 * point that rejects before touching a device, the exact DG tables and the
 * basis values.  Exits non-zero on the first unexpected return code; the
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

int main(void) {
    printf("%s\n", mg_version());
    planners();
    dg_tables();
    if (fails) {
        fprintf(stderr, "%d unexpected return codes\n", fails);
        return 1;
    }
    printf("host checks passed\n");
    return 0;
}
