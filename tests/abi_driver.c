/* Drives the C ABI of libjgs2 end to end on a small generated beam, checking
 * every status: mesh, material, the exact variant's precompute and steps (also
 * with FP16 tiles),
 * energy (also without allocation), residual, device-state round trip, the
 * coloured plain sweeps, a rollout and its adjoint, the precompute cache file
 * (when a directory is given as the first argument), and the documented error
 * paths.  Built against a host-sanitised library (AddressSanitizer and
 * UndefinedBehaviorSanitizer on the host code) by
 * `python -m paper_2506_06494_amd.build --sanitize`; exits 0 when every call
 * returns what its documentation states. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "jgs2.h"

static int failures = 0;

#define EXPECT(call, want)                                                                  \
    do {                                                                                    \
        int32_t got_ = (call);                                                              \
        if (got_ != (want)) {                                                               \
            fprintf(stderr, "FAIL %s:%d %s -> %d (want %d): %s\n", __FILE__, __LINE__, #call, \
                    got_, (want), s ? jgs2_last_error(s) : "");                             \
            ++failures;                                                                     \
        }                                                                                   \
    } while (0)

/* Hexahedral grid of nx x ny x nz cells (cell h), six tets per cube around
 * the cube's main diagonal, each ordered to positive volume. */
static void beam(int nx, int ny, int nz, double h, double** X, int* nV, int32_t** tets, int* nT) {
    const int vx = nx + 1, vy = ny + 1, vz = nz + 1;
    *nV = vx * vy * vz;
    *nT = 6 * nx * ny * nz;
    *X = (double*)malloc(sizeof(double) * 3 * (size_t)*nV);
    *tets = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)*nT);
    for (int k = 0; k < vz; ++k)
        for (int j = 0; j < vy; ++j)
            for (int i = 0; i < vx; ++i) {
                const int v = (k * vy + j) * vx + i;
                (*X)[3 * v] = i * h;
                (*X)[3 * v + 1] = j * h;
                (*X)[3 * v + 2] = k * h;
            }
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int t = 0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                for (int p = 0; p < 6; ++p) {
                    int c[3] = {i, j, k}, id[4];
                    id[0] = (c[2] * vy + c[1]) * vx + c[0];
                    for (int q = 0; q < 3; ++q) {
                        c[perm[p][q]] += 1;
                        id[q + 1] = (c[2] * vy + c[1]) * vx + c[0];
                    }
                    double e[3][3];
                    for (int q = 0; q < 3; ++q)
                        for (int d = 0; d < 3; ++d) e[q][d] = (*X)[3 * id[q + 1] + d] - (*X)[3 * id[0] + d];
                    const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                                       e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                                       e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
                    if (det < 0) {
                        const int tmp = id[1];
                        id[1] = id[2];
                        id[2] = tmp;
                    }
                    memcpy(*tets + 4 * t, id, sizeof(id));
                    ++t;
                }
}

int main(int argc, char** argv) {
    jgs2_solver* s = NULL;
    double* X;
    int32_t* tets;
    int nV, nT;
    beam(4, 4, 12, 0.05, &X, &nV, &tets, &nT);
    uint8_t* pinned = (uint8_t*)calloc((size_t)nV, 1);
    for (int v = 0; v < nV; ++v) pinned[v] = X[3 * v + 2] == 0.0;
    double *E = malloc(sizeof(double) * nT), *nu = malloc(sizeof(double) * nT), *rho = malloc(sizeof(double) * nT);
    for (int t = 0; t < nT; ++t) {
        E[t] = 1e6;
        nu[t] = 0.4;
        rho[t] = 1000.0;
    }
    double *x = malloc(sizeof(double) * 3 * nV), *v = calloc(3 * (size_t)nV, sizeof(double));
    memcpy(x, X, sizeof(double) * 3 * nV);

    jgs2_params p;
    jgs2_default_params(&p);
    p.gravity[0] = 0.0;
    p.gravity[1] = -9.8;
    p.variant = JGS2_EXACT;
    p.check_every = 1;
    EXPECT(jgs2_create(&p, &s), JGS2_OK);
    if (!s) return 1;

    /* calls out of order and bad arguments */
    EXPECT(jgs2_step(s, NULL), JGS2_E_NOT_READY);
    EXPECT(jgs2_upload_mesh(s, 0, X, nT, tets, pinned), JGS2_E_INVALID);
    EXPECT(jgs2_upload_mesh(s, nV, NULL, nT, tets, pinned), JGS2_E_INVALID);

    EXPECT(jgs2_upload_mesh(s, nV, X, nT, tets, pinned), JGS2_OK);
    EXPECT(jgs2_set_material(s, E, nu, rho), JGS2_OK);
    EXPECT(jgs2_set_state(s, x, v), JGS2_OK);
    EXPECT(jgs2_step(s, NULL), JGS2_E_NOT_READY); /* exact variant without its precompute */
    EXPECT(jgs2_precompute(s, 4, 64, 0), JGS2_OK);
    int64_t n_tiles = 0, n_live = 0;
    double live_bytes = 0, part_bytes = 0;
    EXPECT(jgs2_exact_tiles(s, &n_tiles, &n_live, &live_bytes, &part_bytes), JGS2_OK);

    /* precompute cache: the first call computes and writes, the second loads */
    int32_t loaded = -1;
    if (argc > 1) {
        char path[1024];
        snprintf(path, sizeof path, "%s/abi_driver_precompute.bin", argv[1]);
        EXPECT(jgs2_precompute_cached(s, 4, 64, 0, path, &loaded), JGS2_OK);
        if (loaded != 0) {
            fprintf(stderr, "FAIL first cached precompute loaded=%d\n", loaded);
            ++failures;
        }
        EXPECT(jgs2_precompute_cached(s, 4, 64, 0, path, &loaded), JGS2_OK);
        if (loaded != 1) {
            fprintf(stderr, "FAIL second cached precompute loaded=%d\n", loaded);
            ++failures;
        }
        EXPECT(jgs2_precompute_cached(s, 0, 64, 0, path, &loaded), JGS2_E_INVALID);
    }

    /* exact variant: three steps, then two more with the tiles in FP16 (a second
     * conversion does nothing); the production library has no bounds record */
    jgs2_step_stats st;
    for (int k = 0; k < 3; ++k) EXPECT(jgs2_step(s, &st), JGS2_OK);
    EXPECT(jgs2_exact_tiles_fp16(s), JGS2_OK);
    EXPECT(jgs2_exact_tiles_fp16(s), JGS2_OK);
    double half_bytes = 0;
    EXPECT(jgs2_exact_tiles(s, NULL, NULL, &half_bytes, NULL), JGS2_OK);
    if (half_bytes * 2.0 != live_bytes) {
        fprintf(stderr, "FAIL FP16 live bytes %.0f, FP32 %.0f\n", half_bytes, live_bytes);
        ++failures;
    }
    for (int k = 0; k < 2; ++k) EXPECT(jgs2_step(s, &st), JGS2_OK);
    int32_t line = -1;
    EXPECT(jgs2_bounds_report(s, &line, NULL, NULL, 0), JGS2_E_INVALID);
    EXPECT(jgs2_bounds_selftest(s), JGS2_E_INVALID);
    double e0 = 0, e1 = 0, ra = 0, rr = 0;
    EXPECT(jgs2_energy(s, &e0), JGS2_OK);
    EXPECT(jgs2_energy_noalloc(s, &e1), JGS2_OK);
    if (e0 != e1) {
        fprintf(stderr, "FAIL energy %.17g != allocation-free energy %.17g\n", e0, e1);
        ++failures;
    }
    EXPECT(jgs2_residual(s, &ra, &rr), JGS2_OK);
    EXPECT(jgs2_get_state(s, x, v), JGS2_OK);
    for (int i = 0; i < 3 * nV; ++i)
        if (!isfinite(x[i]) || !isfinite(v[i])) {
            fprintf(stderr, "FAIL non-finite state\n");
            ++failures;
            break;
        }

    /* plain coloured GS on the same handle */
    p.variant = JGS2_PLAIN;
    p.order = JGS2_GS;
    p.check_every = 16;
    EXPECT(jgs2_set_params(s, &p), JGS2_OK);
    int32_t* color = malloc(sizeof(int32_t) * nV);
    int32_t n_colors = 0;
    EXPECT(jgs2_get_coloring(s, color, &n_colors), JGS2_OK);
    for (int k = 0; k < 2; ++k) EXPECT(jgs2_step(s, &st), JGS2_OK);

    /* rollout and its adjoint with the plain variant */
    EXPECT(jgs2_set_state(s, X, v), JGS2_OK);
    EXPECT(jgs2_rollout(s, 4, 2, &st), JGS2_OK);
    double *xbar = calloc(3 * (size_t)nV, sizeof(double)), *thbar = malloc(sizeof(double) * nT);
    double *xb0 = malloc(sizeof(double) * 3 * nV), *vb0 = malloc(sizeof(double) * 3 * nV), ub[3];
    xbar[3 * (nV - 1) + 1] = 1.0;
    jgs2_adjoint_stats as;
    EXPECT(jgs2_rollout_backward(s, xbar, NULL, thbar, xb0, vb0, ub, &as), JGS2_OK);

    /* a non-finite start and a bad parameter */
    x[3 * (nV - 1)] = NAN;
    EXPECT(jgs2_set_state(s, x, v), JGS2_E_INVALID);
    p.omega = -1.0;
    EXPECT(jgs2_set_params(s, &p), JGS2_E_INVALID);

    jgs2_destroy(s);
    free(X); free(tets); free(pinned); free(E); free(nu); free(rho); free(x); free(v); free(color);
    free(xbar); free(thbar); free(xb0); free(vb0);
    printf("abi driver: %d tets, %d colours, %lld of %lld tiles live, %d failures\n", nT, n_colors,
           (long long)n_live, (long long)n_tiles, failures);
    return failures == 0 ? 0 : 1;
}
