/* A C program that drives the lbrd library through its C ABI (include/lbrd.h)
 * and nothing else: every entry point, the error paths, tiny and ragged
 * lattices in every storage form and reaction, batches and the server.
 *
 * Test infrastructure.  Two builds:
 *   - "stub": linked with the host-only build of the library and a host-memory
 *     stand-in for the HIP runtime, under AddressSanitizer and
 *     UndefinedBehaviorSanitizer (no GPU; kernels run nothing, so only
 *     statuses and host-side state are checked);
 *   - "gpu": linked with liblbrd.so and the HIP runtime on a GPU; then the
 *     numbers are checked too (mass conservation without reaction, exact
 *     forward Euler on uniform fields, round trips of the state).
 * Prints "<n> failures" and exits with their count (capped at 100). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbrd.h"

/* The few HIP runtime calls the driver needs (C linkage, int status). */
int hipMalloc(void **p, size_t n);
int hipFree(void *p);
int hipMemcpy(void *dst, const void *src, size_t n, int kind);
int hipDeviceSynchronize(void);
#define H2D 1
#define D2H 2

static int g_fail = 0;
static int g_gpu = 0;

#define CHECK(cond, ...)                                              \
    do {                                                              \
        if (!(cond)) {                                                \
            ++g_fail;                                                 \
            printf("FAIL %s:%d: ", __FILE__, __LINE__);               \
            printf(__VA_ARGS__);                                      \
            printf("\n");                                             \
        }                                                             \
    } while (0)
#define EXPECT(call, want) CHECK((call) == (want), "%s -> %d, want %d", #call, (int)(call), (int)(want))

static lbrd_config base(int ns, int nx, int ny, int storage, int reaction) {
    lbrd_config c;
    memset(&c, 0, sizeof c);
    c.nspecies = ns;
    c.nx = nx;
    c.ny = ny;
    c.storage = storage;
    c.reaction = reaction;
    for (int s = 0; s < LBRD_MAX_SPECIES; ++s) c.tau[s] = 0.7 + 0.2 * s;
    if (reaction == LBRD_REACT_GRAY_SCOTT) {
        c.F = 0.04;
        c.k = 0.06;
        c.tau[0] = 1.0;
        c.tau[1] = 0.75;
        c.rho_ref[0] = 1.0;
    }
    if (reaction == LBRD_REACT_LINEAR)
        for (int s = 0; s < ns; ++s) c.K[s * ns + s] = -0.001 * (s + 1);
    if (storage == LBRD_F16_SHIFTED || storage == LBRD_BF16_SHIFTED)
        for (int s = 0; s < ns; ++s) c.rho_ref[s] = reaction == LBRD_REACT_GRAY_SCOTT ? (s == 0 ? 1.0 : 0.0) : 0.8;
    return c;
}

static void *dalloc(size_t n) {
    void *p = NULL;
    if (hipMalloc(&p, n) != 0) return NULL;
    return p;
}

static double *densities(const lbrd_config *c, int uniform) {
    const size_t n = (size_t)c->nspecies * c->nx * c->ny;
    double *r = malloc(n * sizeof(double));
    for (size_t j = 0; j < n; ++j) r[j] = uniform ? 0.75 : 0.5 + 0.5 * (double)((j * 2654435761u) % 1000) / 1000.0;
    return r;
}

static void check_validation(void) {
    lbrd_config ok = base(2, 8, 6, LBRD_F32, LBRD_REACT_GRAY_SCOTT);
    EXPECT(lbrd_validate(&ok), LBRD_OK);
    EXPECT(lbrd_validate(NULL), LBRD_EINVAL);
    lbrd_config c;
    c = ok; c.nspecies = 0; EXPECT(lbrd_validate(&c), LBRD_EINVAL);
    c = ok; c.nspecies = 5; EXPECT(lbrd_validate(&c), LBRD_EINVAL);
    c = ok; c.nspecies = 3; EXPECT(lbrd_validate(&c), LBRD_EINVAL);          /* Gray-Scott needs N = 2 */
    c = ok; c.nx = 0; EXPECT(lbrd_validate(&c), LBRD_EINVAL);
    c = ok; c.ny = -3; EXPECT(lbrd_validate(&c), LBRD_EINVAL);
    c = ok; c.tau[1] = 0.5; EXPECT(lbrd_validate(&c), LBRD_EINVAL);
    c = ok; c.tau[0] = NAN; EXPECT(lbrd_validate(&c), LBRD_EINVAL);
    c = ok; c.storage = 4; EXPECT(lbrd_validate(&c), LBRD_EINVAL);
    c = ok; c.reaction = 3; EXPECT(lbrd_validate(&c), LBRD_EINVAL);
    c = ok; c.reserved = 1; EXPECT(lbrd_validate(&c), LBRD_EINVAL);
    c = ok; c.u[0] = 0.6; EXPECT(lbrd_validate(&c), LBRD_EINVAL);            /* u.u >= 1/3 */
    c = ok; c.storage = LBRD_F16_SHIFTED; c.shear[0] = 0.1; c.shear[1] = 1;
    EXPECT(lbrd_validate(&c), LBRD_EINVAL);                                  /* shear needs FP64/FP32 */
    c = ok; c.shear[0] = 0.1; c.shear[1] = 1.5; EXPECT(lbrd_validate(&c), LBRD_EINVAL);   /* m whole */
    size_t bytes = 0;
    EXPECT(lbrd_workspace_size(&ok, &bytes), LBRD_OK);
    CHECK(bytes > 2 * 9 * 2 * 8 * 6 * 4, "workspace %zu too small", bytes);
    EXPECT(lbrd_workspace_size(&ok, NULL), LBRD_EINVAL);
    for (int st = -8; st <= 1; ++st) CHECK(lbrd_strerror(st) != NULL, "strerror(%d)", st);
    CHECK(lbrd_version() != NULL && lbrd_last_error() != NULL, "version / last_error");
}

/* One solver through every call; numbers checked on a GPU. */
static void solver_case(lbrd_config c) {
    size_t bytes = 0;
    EXPECT(lbrd_workspace_size(&c, &bytes), LBRD_OK);
    char *ws = dalloc(bytes);
    lbrd_solver *h = NULL;
    EXPECT(lbrd_create(&c, ws, bytes - 1, NULL, &h), LBRD_ENOMEM);
    EXPECT(lbrd_create(&c, ws + 8, bytes, NULL, &h), LBRD_EINVAL);           /* misaligned */
    EXPECT(lbrd_create(&c, ws, bytes, NULL, NULL), LBRD_EINVAL);
    EXPECT(lbrd_create(&c, ws, bytes, NULL, &h), LBRD_OK);
    if (!h) {
        hipFree(ws);
        return;
    }
    const int ns = c.nspecies;
    const size_t sites = (size_t)c.nx * c.ny, nrho = ns * sites, npop = 9 * nrho;
    EXPECT(lbrd_step(h, 1), LBRD_ESTATE);
    EXPECT(lbrd_moments(h, NULL, LBRD_DTYPE_F64, NULL), LBRD_ESTATE);
    double *rho0 = densities(&c, c.reaction == LBRD_REACT_NONE ? 0 : 1);
    EXPECT(lbrd_init(h, rho0, LBRD_DTYPE_F64, 0), LBRD_OK);
    EXPECT(lbrd_init(h, rho0, 7, 0), LBRD_EINVAL);
    double m0[LBRD_MAX_SPECIES], m1[LBRD_MAX_SPECIES], err[LBRD_MAX_SPECIES];
    EXPECT(lbrd_moments(h, NULL, LBRD_DTYPE_F64, m0), LBRD_OK);
    EXPECT(lbrd_step(h, -1), LBRD_EINVAL);
    EXPECT(lbrd_step(h, 0), LBRD_OK);
    EXPECT(lbrd_step(h, 7), LBRD_OK);
    EXPECT(lbrd_step(h, 1), LBRD_OK);
    int64_t t = -1;
    EXPECT(lbrd_time(h, &t), LBRD_OK);
    CHECK(t == 8, "time %lld", (long long)t);
    double *drho = dalloc(nrho * sizeof(double));
    float *drho32 = dalloc(nrho * sizeof(float));
    EXPECT(lbrd_moments(h, drho, LBRD_DTYPE_F64, m1), LBRD_OK);
    EXPECT(lbrd_moments(h, drho32, LBRD_DTYPE_F32, NULL), LBRD_OK);
    EXPECT(lbrd_rel_l2(h, drho, LBRD_DTYPE_F64, err), LBRD_OK);
    EXPECT(lbrd_rel_l2(h, NULL, LBRD_DTYPE_F64, err), LBRD_EINVAL);
    if (g_gpu) {
        for (int s = 0; s < ns; ++s) CHECK(err[s] == 0.0, "rel_l2 against itself %g", err[s]);
        double *host = malloc(nrho * sizeof(double));
        hipMemcpy(host, drho, nrho * sizeof(double), D2H);
        const double tol = c.storage == LBRD_F64 ? 1e-12 : (c.storage == LBRD_F32 ? 1e-5 : 2e-2);
        if (c.reaction == LBRD_REACT_NONE && c.u[0] == 0.0 && c.shear[0] == 0.0)
            for (int s = 0; s < ns; ++s)
                CHECK(fabs(m1[s] - m0[s]) <= tol * fabs(m0[s]), "mass %g -> %g", m0[s], m1[s]);
        if (c.reaction == LBRD_REACT_LINEAR && c.storage == LBRD_F64) {
            /* a uniform field under R = K rho is forward Euler: (1 + K_ss)^8 */
            for (int s = 0; s < ns; ++s) {
                const double want = 0.75 * pow(1.0 + c.K[s * ns + s], 8);
                for (size_t j = 0; j < sites; j += 7)
                    CHECK(fabs(host[s * sites + j] - want) <= 1e-13, "uniform decay %g vs %g", host[s * sites + j],
                          want);
            }
        }
        free(host);
    }
    /* populations: read, write back, read again */
    double *pop = dalloc(npop * sizeof(double));
    double *pop2 = dalloc(npop * sizeof(double));
    EXPECT(lbrd_get_populations(h, pop, LBRD_DTYPE_F64), LBRD_OK);
    EXPECT(lbrd_set_populations(h, pop, LBRD_DTYPE_F64, 1), LBRD_OK);
    EXPECT(lbrd_get_populations(h, pop2, LBRD_DTYPE_F64), LBRD_OK);
    EXPECT(lbrd_time(h, &t), LBRD_OK);
    CHECK(t == 0, "time after set_populations %lld", (long long)t);
    if (g_gpu) {
        double *a = malloc(npop * sizeof(double)), *b = malloc(npop * sizeof(double));
        hipMemcpy(a, pop, npop * sizeof(double), D2H);
        hipMemcpy(b, pop2, npop * sizeof(double), D2H);
        CHECK(memcmp(a, b, npop * sizeof(double)) == 0, "population round trip");
        free(a);
        free(b);
    }
    double *hpop = malloc(npop * sizeof(double));
    for (size_t j = 0; j < npop; ++j) hpop[j] = 0.05 + 0.001 * (double)(j % 17);
    EXPECT(lbrd_set_populations(h, hpop, LBRD_DTYPE_F64, 0), LBRD_OK);
    /* spectrum */
    size_t wbytes = 0;
    EXPECT(lbrd_spectrum_work_size(c.nx, c.ny, &wbytes), LBRD_OK);
    void *work = dalloc(wbytes);
    double *spec = dalloc(sites * sizeof(double));
    EXPECT(lbrd_spectrum(h, 0, spec, work, wbytes), LBRD_OK);
    EXPECT(lbrd_spectrum(h, ns, spec, work, wbytes), LBRD_EINVAL);
    EXPECT(lbrd_spectrum(h, 0, spec, work, wbytes ? wbytes - 1 : 0), wbytes ? LBRD_ENOMEM : LBRD_OK);
    /* the variant that allocates nothing: the same numbers */
    double *spec2 = dalloc(sites * sizeof(double));
    EXPECT(lbrd_spectrum(h, ns - 1, spec, work, wbytes), LBRD_OK);
    EXPECT(lbrd_spectrum_static(h, ns - 1, spec2), LBRD_OK);
    EXPECT(lbrd_spectrum_static(h, ns, spec2), LBRD_EINVAL);
    EXPECT(lbrd_spectrum_static(h, 0, (char *)spec2 + 4), LBRD_EINVAL);
    EXPECT(lbrd_spectrum_static(NULL, 0, spec2), LBRD_EINVAL);
    if (g_gpu) {
        double *a = malloc(sites * sizeof(double)), *b2 = malloc(sites * sizeof(double));
        hipMemcpy(a, spec, sites * sizeof(double), D2H);
        hipMemcpy(b2, spec2, sites * sizeof(double), D2H);
        CHECK(memcmp(a, b2, sites * sizeof(double)) == 0, "static-scratch spectrum differs");
        free(a);
        free(b2);
    }
    hipFree(spec2);
    /* launch shapes */
    lbrd_tuning tu, bad;
    EXPECT(lbrd_get_tuning(h, &tu), LBRD_OK);
    bad = tu; bad.waves = 3; EXPECT(lbrd_set_tuning(h, &bad), LBRD_EINVAL);
    bad = tu; bad.graph_steps = 3; EXPECT(lbrd_set_tuning(h, &bad), LBRD_EINVAL);
    bad = tu; bad.fused_steps = 9; EXPECT(lbrd_set_tuning(h, &bad), LBRD_EINVAL);
    bad = tu; bad.fused_steps = 1; bad.graph_steps = 4; EXPECT(lbrd_set_tuning(h, &bad), LBRD_OK);
    EXPECT(lbrd_step(h, 9), LBRD_OK);
    EXPECT(lbrd_set_tuning(h, &tu), LBRD_OK);
    double ms = -1;
    EXPECT(lbrd_time_steps(h, 5, &ms), LBRD_OK);
    CHECK(ms >= 0, "time_steps %g", ms);
    hipDeviceSynchronize();
    EXPECT(lbrd_destroy(h), LBRD_OK);
    free(rho0);
    free(hpop);
    hipFree(drho);
    hipFree(drho32);
    hipFree(pop);
    hipFree(pop2);
    hipFree(work);
    hipFree(spec);
    hipFree(ws);
}

/* The multi-step kernels form row offsets with 24-bit multiplies: a lattice
 * taller than 2^24 rows must take one-step launches.  The solver is created
 * on a workspace pointer that is never touched (nothing is stepped). */
static void tall_lattice_gate(void) {
    for (int tall = 0; tall < 2; ++tall) {
        lbrd_config c = base(1, 16, tall ? (1 << 24) + 1 : (1 << 24), LBRD_F32, LBRD_REACT_NONE);
        size_t bytes = 0;
        EXPECT(lbrd_workspace_size(&c, &bytes), LBRD_OK);
        lbrd_solver *h = NULL;
        EXPECT(lbrd_create(&c, (void *)(uintptr_t)0x100000000ull, bytes, NULL, &h), LBRD_OK);
        if (!h) continue;
        lbrd_tuning tu;
        EXPECT(lbrd_get_tuning(h, &tu), LBRD_OK);
        double spec_out = 0;
        EXPECT(lbrd_spectrum_static(h, 0, &spec_out), LBRD_ENOMEM);          /* beyond the fixed scratch */
        if (tall) {
            CHECK(tu.fused_steps == 1, "tall lattice takes %d steps per launch", tu.fused_steps);
            tu.fused_steps = 4;
            tu.tile_cols = 32;
            tu.tile_rows = 4;
            EXPECT(lbrd_set_tuning(h, &tu), LBRD_EINVAL);
        } else {
            CHECK(tu.fused_steps > 1, "2^24 rows: %d steps per launch", tu.fused_steps);
        }
        EXPECT(lbrd_destroy(h), LBRD_OK);
    }
}

static void autotune_case(void) {
    lbrd_config c = base(2, 40, 24, LBRD_F32, LBRD_REACT_GRAY_SCOTT);
    size_t bytes = 0;
    lbrd_workspace_size(&c, &bytes);
    void *ws = dalloc(bytes);
    lbrd_solver *h = NULL;
    EXPECT(lbrd_create(&c, ws, bytes, NULL, &h), LBRD_OK);
    lbrd_tuning chosen;
    EXPECT(lbrd_autotune(h, 1, NULL, &chosen), LBRD_EINVAL);
    EXPECT(lbrd_autotune(h, 2, NULL, &chosen), LBRD_OK);
    EXPECT(lbrd_step(h, 1), LBRD_ESTATE);                                     /* state overwritten */
    double *rho0 = densities(&c, 1);
    EXPECT(lbrd_init(h, rho0, LBRD_DTYPE_F64, 0), LBRD_OK);
    EXPECT(lbrd_step(h, 3), LBRD_OK);
    EXPECT(lbrd_destroy(h), LBRD_OK);
    free(rho0);
    hipFree(ws);
}

static void batch_case(int serve_mix) {
    lbrd_config cfg[4];
    if (serve_mix) {
        cfg[0] = base(2, 37, 20, LBRD_F32, LBRD_REACT_GRAY_SCOTT);
        cfg[1] = base(1, 64, 9, LBRD_F16_SHIFTED, LBRD_REACT_LINEAR);
        cfg[2] = base(2, 5, 3, LBRD_BF16_SHIFTED, LBRD_REACT_GRAY_SCOTT);
        cfg[3] = base(1, 1, 1, LBRD_F32, LBRD_REACT_LINEAR);
    } else {
        cfg[0] = base(3, 17, 13, LBRD_F64, LBRD_REACT_LINEAR);
        cfg[1] = base(2, 33, 7, LBRD_F32, LBRD_REACT_GRAY_SCOTT);
        cfg[2] = base(4, 3, 5, LBRD_F32, LBRD_REACT_NONE);
        cfg[3] = base(1, 70, 2, LBRD_F64, LBRD_REACT_NONE);
    }
    size_t bytes = 0;
    EXPECT(lbrd_batch_workspace_size(cfg, 4, &bytes), LBRD_OK);
    EXPECT(lbrd_batch_workspace_size(cfg, 0, &bytes), LBRD_EINVAL);
    void *ws = dalloc(bytes);
    lbrd_batch *b = NULL;
    EXPECT(lbrd_batch_create(cfg, 4, ws, bytes - 1, NULL, &b), LBRD_ENOMEM);
    EXPECT(lbrd_batch_create(cfg, 4, ws, bytes, NULL, &b), LBRD_OK);
    if (!b) {
        hipFree(ws);
        return;
    }
    EXPECT(lbrd_batch_step(b, 2), LBRD_ESTATE);
    for (int i = 0; i < 4; ++i) {
        double *r = densities(&cfg[i], 0);
        EXPECT(lbrd_batch_init(b, i, r, LBRD_DTYPE_F64, 0), LBRD_OK);
        free(r);
    }
    EXPECT(lbrd_batch_init(b, 4, NULL, LBRD_DTYPE_F64, 0), LBRD_EINVAL);
    EXPECT(lbrd_batch_step(b, 11), LBRD_OK);
    int64_t counts[4] = {0, 3, 12, 1};
    EXPECT(lbrd_batch_advance(b, counts), LBRD_OK);
    int64_t t = 0;
    EXPECT(lbrd_batch_time(b, 2, &t), LBRD_OK);
    CHECK(t == 23, "batch time %lld", (long long)t);
    for (int i = 0; i < 4; ++i) {
        const size_t nrho = (size_t)cfg[i].nspecies * cfg[i].nx * cfg[i].ny;
        double *d = dalloc(nrho * sizeof(double)), *p = dalloc(9 * nrho * sizeof(double));
        double m[LBRD_MAX_SPECIES], e[LBRD_MAX_SPECIES];
        EXPECT(lbrd_batch_moments(b, i, d, LBRD_DTYPE_F64, m), LBRD_OK);
        EXPECT(lbrd_batch_rel_l2(b, i, d, LBRD_DTYPE_F64, e), LBRD_OK);
        EXPECT(lbrd_batch_get_populations(b, i, p, LBRD_DTYPE_F32), LBRD_OK);
        size_t wb = 0;
        lbrd_spectrum_work_size(cfg[i].nx, cfg[i].ny, &wb);
        void *w = dalloc(wb);
        double *sp = dalloc((size_t)cfg[i].nx * cfg[i].ny * sizeof(double));
        EXPECT(lbrd_batch_spectrum(b, i, 0, sp, w, wb), LBRD_OK);
        if (g_gpu)
            for (int s = 0; s < cfg[i].nspecies; ++s) CHECK(e[s] == 0.0 && isfinite(m[s]), "batch read-outs");
        hipFree(d);
        hipFree(p);
        hipFree(w);
        hipFree(sp);
    }
    lbrd_tuning tu, bad;
    EXPECT(lbrd_batch_get_tuning(b, &tu), LBRD_OK);
    bad = tu; bad.waves = 17; EXPECT(lbrd_batch_set_tuning(b, &bad), LBRD_EINVAL);
    bad = tu; bad.nontemporal = 2; EXPECT(lbrd_batch_set_tuning(b, &bad), LBRD_EINVAL);
    double ms = -1;
    EXPECT(lbrd_batch_time_steps(b, 4, &ms), LBRD_OK);
    lbrd_tuning chosen;
    EXPECT(lbrd_batch_autotune(b, 2, &chosen), LBRD_OK);
    EXPECT(lbrd_batch_step(b, 1), LBRD_ESTATE);
    EXPECT(lbrd_batch_destroy(b), LBRD_OK);
    hipFree(ws);
}

static void server_case(void) {
    const size_t arena_bytes = (size_t)24 << 20;
    void *arena = dalloc(arena_bytes);
    lbrd_server_config sc = {16, 8, 64, 0};
    lbrd_server *srv = NULL;
    lbrd_server_config badc = sc;
    badc.chunk_steps = 0;
    EXPECT(lbrd_server_create(&badc, arena, arena_bytes, NULL, &srv), LBRD_EINVAL);
    EXPECT(lbrd_server_create(&sc, arena, arena_bytes, NULL, &srv), LBRD_OK);
    if (!srv) {
        hipFree(arena);
        return;
    }
    lbrd_config cfgs[6] = {
        base(2, 64, 64, LBRD_F32, LBRD_REACT_GRAY_SCOTT), base(1, 80, 48, LBRD_F16_SHIFTED, LBRD_REACT_LINEAR),
        base(2, 33, 70, LBRD_BF16_SHIFTED, LBRD_REACT_GRAY_SCOTT), base(1, 1, 1, LBRD_F32, LBRD_REACT_LINEAR),
        base(1, 128, 96, LBRD_F32, LBRD_REACT_LINEAR), base(2, 1024, 1024, LBRD_F32, LBRD_REACT_GRAY_SCOTT)};
    int64_t tickets[6];
    for (int i = 0; i < 6; ++i) {
        size_t fp = 0;
        EXPECT(lbrd_server_footprint(&cfgs[i], &fp), LBRD_OK);
        double *r = densities(&cfgs[i], 1);
        const int rc = lbrd_server_submit(srv, &cfgs[i], r, 20 + 7 * i, &tickets[i]);
        if (fp > arena_bytes) EXPECT(rc, LBRD_ENOMEM);
        else EXPECT(rc, LBRD_OK);
        free(r);
    }
    lbrd_config shear = base(1, 16, 16, LBRD_F32, LBRD_REACT_LINEAR);
    shear.shear[0] = 0.05;
    shear.shear[1] = 1;
    double r1[16 * 16];
    for (int j = 0; j < 256; ++j) r1[j] = 1.0;
    int64_t tk = 0;
    EXPECT(lbrd_server_submit(srv, &shear, r1, 5, &tk), LBRD_EINVAL);
    for (int i = 0; i < 5; ++i) {
        EXPECT(lbrd_server_wait(srv, tickets[i], 120.0), LBRD_OK);
        lbrd_request_info info;
        EXPECT(lbrd_server_info(srv, tickets[i], &info), LBRD_OK);
        CHECK(info.state == 2 && info.steps == 20 + 7 * i, "request %d state %d", i, info.state);
        const size_t nrho = (size_t)cfgs[i].nspecies * cfgs[i].nx * cfgs[i].ny;
        double *out = malloc(nrho * sizeof(double)), mass[LBRD_MAX_SPECIES];
        EXPECT(lbrd_server_take(srv, tickets[i], out, mass, &info), LBRD_OK);
        if (g_gpu) {
            /* uniform start 0.75: Gray-Scott u, v and the linear decay stay uniform */
            for (size_t j = 1; j < nrho / cfgs[i].nspecies; ++j)
                CHECK(out[j] == out[0], "request %d not uniform", i);
        }
        free(out);
        EXPECT(lbrd_server_info(srv, tickets[i], &info), LBRD_ENOTFOUND);
    }
    EXPECT(lbrd_server_wait(srv, 987654321, 0.01), LBRD_ENOTFOUND);
    lbrd_server_stats st;
    EXPECT(lbrd_server_stats_get(srv, &st), LBRD_OK);
    CHECK(st.arena_used == 0 && st.arena_used_byte_s >= 0.0 && st.resident == 0, "arena after all retired: %lld",
          (long long)st.arena_used);
    /* the 1024^2 request exceeds the whole arena: refused at submit, counted */
    CHECK(st.completed == 5 && st.rejected == 1 && st.submitted == 5 && st.arena_peak_used <= (int64_t)arena_bytes,
          "server stats: completed %lld rejected %lld submitted %lld peak %lld", (long long)st.completed,
          (long long)st.rejected, (long long)st.submitted, (long long)st.arena_peak_used);
    /* requests still queued or resident at destroy */
    for (int i = 0; i < 3; ++i) {
        double *r = densities(&cfgs[0], 1);
        EXPECT(lbrd_server_submit(srv, &cfgs[0], r, 100000, &tk), LBRD_OK);
        free(r);
    }
    EXPECT(lbrd_server_destroy(srv), LBRD_OK);
    hipFree(arena);
}

int main(int argc, char **argv) {
    g_gpu = argc > 1 && strcmp(argv[1], "gpu") == 0;
    check_validation();
    const int shapes[][2] = {{1, 1}, {3, 5}, {40, 9}, {130, 33}};
    for (size_t k = 0; k < sizeof shapes / sizeof shapes[0]; ++k) {
        const int nx = shapes[k][0], ny = shapes[k][1];
        for (int storage = LBRD_F64; storage <= LBRD_BF16_SHIFTED; ++storage) {
            solver_case(base(2, nx, ny, storage, LBRD_REACT_GRAY_SCOTT));
            for (int ns = 1; ns <= 4; ++ns) solver_case(base(ns, nx, ny, storage, LBRD_REACT_LINEAR));
            solver_case(base(3, nx, ny, storage, LBRD_REACT_NONE));
            lbrd_config adv = base(1, nx, ny, storage, LBRD_REACT_LINEAR);
            adv.u[0] = 0.1;
            adv.u[1] = -0.05;
            solver_case(adv);
            if (storage <= LBRD_F32) {
                lbrd_config sh = base(2, nx, ny, storage, LBRD_REACT_GRAY_SCOTT);
                sh.shear[0] = 0.08;
                sh.shear[1] = 2;
                solver_case(sh);
            }
        }
    }
    tall_lattice_gate();
    autotune_case();
    batch_case(0);
    batch_case(1);
    server_case();
    printf("%d failures\n", g_fail);
    return g_fail > 100 ? 100 : g_fail;
}
