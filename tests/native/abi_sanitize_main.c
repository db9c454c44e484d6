/* Driver for the library's host code under AddressSanitizer and
 * UndefinedBehaviorSanitizer (the library's host side built with
 * -fsanitize=address,undefined, its device code as usual).
 *
 *   abi_sanitize          host checks only: every entry point is called with
 *                         invalid arguments (which must be rejected before
 *                         any device work) and every size query with sizes
 *                         up to INT32_MAX (no overflow may be undefined).
 *   abi_sanitize gpu      the host checks, then every entry point on a small
 *                         mixture of spheres and rods in a periodic box and on
 *                         a sphere cluster with the RPY mobility in a walled
 *                         box: build, canonical order, assembly, the solves
 *                         (matrix, chain, no-alloc, async), the adjoints, the
 *                         time-stepping calls, a batch (plain, built on the
 *                         device, through its graph), then sc_release.
 *
 * Only the return codes and a few consistency checks are tested here; the
 * numbers themselves are compared with the oracle by the parity tests. Any
 * sanitizer report ends the run with a non-zero status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "sc_api.h"

static int g_fail = 0;

#define EXPECT(cond)                                                              \
    do {                                                                          \
        if (!(cond)) {                                                            \
            fprintf(stderr, "%s:%d: expected %s\n", __FILE__, __LINE__, #cond);  \
            g_fail = 1;                                                           \
        }                                                                         \
    } while (0)

#define OK(call)                                                                  \
    do {                                                                          \
        int rc_ = (call);                                                         \
        if (rc_ != SC_OK) {                                                       \
            fprintf(stderr, "%s:%d: %s returned %d (%s)\n", __FILE__, __LINE__,   \
                    #call, rc_, sc_strerror(rc_));                                \
            exit(2);                                                              \
        }                                                                         \
    } while (0)

#define SOLVED(call)                                                              \
    do {                                                                          \
        int rc_ = (call);                                                         \
        if (rc_ != SC_OK && rc_ != SC_NOT_CONVERGED) {                            \
            fprintf(stderr, "%s:%d: %s returned %d (%s)\n", __FILE__, __LINE__,   \
                    #call, rc_, sc_strerror(rc_));                                \
            exit(2);                                                              \
        }                                                                         \
    } while (0)

#define HIP(call)                                                                 \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s:%d: %s: %s\n", __FILE__, __LINE__, #call,        \
                    hipGetErrorString(e_));                                       \
            exit(3);                                                              \
        }                                                                         \
    } while (0)

/* ------------------------------------------------------------ host checks */

static void host_checks(void) {
    static const int32_t sizes[] = {0, 1, 7, 64, 1000, 1 << 20, 1 << 28, INT32_MAX};
    const int ns = (int)(sizeof sizes / sizeof sizes[0]);
    for (int a = 0; a < ns; ++a) {
        (void)sc_rpy_work_bytes(sizes[a]);
        for (int b = 0; b < ns; ++b) {
            const int32_t n = sizes[a], cap = sizes[b];
            size_t all = sc_workspace_bytes(n, cap, SC_WS_ALL);
            for (int w = SC_WS_BUILD; w <= SC_WS_ADJOINT; ++w)
                EXPECT(sc_workspace_bytes(n, cap, w) <= all);
            (void)sc_plan_bytes(n, cap);
            (void)sc_matrix_bytes(cap, (int64_t)cap * 40);
            (void)sc_matrix_bytes(cap, INT64_MAX / 2);
            (void)sc_solve_mob_work_bytes(n, cap);
            (void)sc_solve_rpy_work_bytes(n, cap);
            (void)sc_adjoint_mob_work_bytes(n, cap);
        }
    }
    EXPECT(sc_workspace_bytes(-1, 10, SC_WS_ALL) == 0);
    EXPECT(sc_workspace_bytes(10, -1, SC_WS_ALL) == 0);
    EXPECT(sc_workspace_bytes(10, 10, 9) == 0);
    EXPECT(sc_batch_workspace_bytes(1, NULL, NULL) == 0);
    EXPECT(sc_batch_workspace_bytes(-3, NULL, NULL) == 0);
    for (int code = -8; code <= 2; ++code) EXPECT(sc_strerror(code) != NULL);
    EXPECT(sc_version() >= 100);

    sc_particles p0 = {0};
    sc_particles pneg = {0};
    pneg.n = -5;
    sc_contacts c = {0};
    sc_box box = {{0, 0, 0}, {1, 1, 1}, 1, 0};
    sc_solve_opts o = {1e-6, 100, 1, 0, 0, 0, 0, 0, 0, 0, 0};
    sc_adjoint_opts ao = {1e-10, 100, 0, 0, 0, 0, 0, 0};
    sc_stats st;
    memset(&st, 0, sizeof st);

    EXPECT(sc_apply_mobility(&pneg, NULL, NULL, NULL) == SC_ERR_INVALID);
    EXPECT(sc_apply_mobility(NULL, NULL, NULL, NULL) == SC_ERR_INVALID);
    EXPECT(sc_build_contacts(NULL, NULL, 0.1, NULL, 1e-3, NULL, NULL, 0, NULL) == SC_ERR_INVALID);
    EXPECT(sc_build_contacts(&p0, &box, 0.1, NULL, 1e-3, &c, NULL, 0, NULL) == SC_ERR_INVALID);
    EXPECT(sc_build_contacts(&pneg, &box, 0.1, NULL, 1e-3, &c, NULL, 0, NULL) == SC_ERR_INVALID);
    EXPECT(sc_canonical_order(3, NULL, NULL, NULL, 0, NULL) == SC_ERR_INVALID);
    EXPECT(sc_assemble_matrix(NULL, &c, NULL) == SC_ERR_INVALID);
    EXPECT(sc_assemble_matrix(&pneg, &c, NULL) == SC_ERR_INVALID);
    EXPECT(sc_mvop(NULL, &c, NULL, NULL, NULL, 0, NULL) == SC_ERR_INVALID);

    c.capacity = 5;
    c.count = 10; /* beyond capacity */
    EXPECT(sc_solve_lcp(&p0, &c, &o, NULL, NULL, NULL, NULL, &st, NULL, 0, NULL) ==
           SC_ERR_INVALID);
    EXPECT(sc_solve_lcp_noalloc(&p0, &c, &o, NULL, NULL, NULL, NULL, &st, NULL) ==
           SC_ERR_INVALID);
    EXPECT(sc_solve_lcp_async(&p0, &c, &o, NULL, NULL, NULL, NULL, NULL, NULL, 0, NULL) ==
           SC_ERR_INVALID);
    EXPECT(sc_canonical_order(3, &c, NULL, NULL, 0, NULL) == SC_ERR_INVALID);
    c.count = 0;
    {
        sc_solve_opts bad[8];
        for (int k = 0; k < 8; ++k) bad[k] = o;
        bad[0].tol = -1.0;
        bad[1].bb = 7;
        bad[2].slices_per_wave = 3;
        bad[3].lds_entries_per_wave = -2;
        bad[4].lanes_per_particle = 16;
        bad[5].block = 768;
        bad[6].op = 3;
        bad[7].spin_limit = -1;
        for (int k = 0; k < 8; ++k) {
            EXPECT(sc_solve_lcp(&p0, &c, &bad[k], NULL, NULL, NULL, NULL, &st, NULL, 0, NULL) ==
                   SC_ERR_INVALID);
            EXPECT(sc_solve_lcp_noalloc(&p0, &c, &bad[k], NULL, NULL, NULL, NULL, &st, NULL) ==
                   SC_ERR_INVALID);
        }
    }
    {
        sc_particles pbig = {0};
        pbig.n = 100000;
        sc_contacts cbig = {0};
        cbig.capacity = 4000000;
        EXPECT(sc_solve_lcp_noalloc(&pbig, &cbig, &o, NULL, NULL, NULL, NULL, &st, NULL) ==
               SC_ERR_WORKSPACE);
    }
    EXPECT(sc_solve_lcp_adjoint(NULL, &box, &c, NULL, 1e-3, NULL, NULL, NULL, NULL, NULL, &ao,
                                &st, NULL, 0, NULL) == SC_ERR_INVALID);
    EXPECT(sc_solve_lcp_mob(NULL, &c, &o, sc_dry_apply, NULL, 0, NULL, NULL, NULL, NULL, &st,
                            NULL, 0, NULL) == SC_ERR_INVALID);
    EXPECT(sc_solve_lcp_mob(&p0, &c, &o, NULL, NULL, 0, NULL, NULL, NULL, NULL, &st, NULL, 0,
                            NULL) == SC_ERR_INVALID);
    EXPECT(sc_solve_lcp_rpy(&p0, &c, NULL, &o, NULL, NULL, NULL, NULL, &st, NULL, 0, NULL) ==
           SC_ERR_INVALID);
    EXPECT(sc_solve_lcp_adjoint_mob(NULL, &box, &c, NULL, NULL, 1e-3, NULL, NULL, NULL,
                                    sc_dry_apply, NULL, NULL, NULL, &ao, 0, NULL, NULL, &st,
                                    NULL, 0, NULL) == SC_ERR_INVALID);
    {
        sc_rpy r = {0};
        r.n = 4;
        r.mu = -1.0;
        EXPECT(sc_rpy_apply(&r, 4, NULL, NULL, NULL) == SC_ERR_INVALID);
        EXPECT(sc_rpy_apply(&r, 3, NULL, NULL, NULL) == SC_ERR_INVALID);
        EXPECT(sc_rpy_grad(&r, 4, NULL, NULL, NULL, NULL) == SC_ERR_INVALID);
        EXPECT(sc_rpy_apply(NULL, 4, NULL, NULL, NULL) == SC_ERR_INVALID);
        EXPECT(sc_dry_apply(NULL, 4, NULL, NULL, NULL) == SC_ERR_INVALID);
    }
    EXPECT(sc_polish_lcp(NULL, &c, NULL, NULL, NULL, NULL, &ao, 0, &st, NULL, 0, NULL) ==
           SC_ERR_INVALID);
    EXPECT(sc_polish_lcp(&p0, &c, NULL, NULL, NULL, NULL, &ao, -1, &st, NULL, 0, NULL) ==
           SC_ERR_INVALID);
    EXPECT(sc_advance(-1, NULL, NULL, NULL, NULL, NULL, 0.1, NULL) == SC_ERR_INVALID);
    EXPECT(sc_advance(4, NULL, NULL, NULL, NULL, NULL, 0.0, NULL) == SC_ERR_INVALID);
    EXPECT(sc_advance(4, NULL, NULL, NULL, NULL, NULL, 0.1, NULL) == SC_ERR_INVALID);
    EXPECT(sc_advance(0, NULL, NULL, NULL, NULL, NULL, 0.1, NULL) == SC_OK);
    EXPECT(sc_quat_from_axis(-1, NULL, NULL, NULL) == SC_ERR_INVALID);
    EXPECT(sc_map_gamma(3, NULL, NULL, NULL, NULL, NULL) == SC_ERR_INVALID);
    {
        sc_batch *b = (sc_batch *)0x1;
        sc_batch_opts bo;
        memset(&bo, 0, sizeof bo);
        EXPECT(sc_batch_create(0, NULL, &bo, NULL, 0, NULL, &b) == SC_ERR_INVALID && !b);
        EXPECT(sc_batch_create(-1, NULL, &bo, NULL, 0, NULL, &b) == SC_ERR_INVALID);
        EXPECT(sc_batch_solve(NULL, NULL) == SC_ERR_INVALID);
        EXPECT(sc_batch_graph_launch(NULL, NULL) == SC_ERR_INVALID);
        EXPECT(sc_batch_stats(NULL, NULL, NULL, NULL, NULL) == SC_ERR_INVALID);
        EXPECT(sc_batch_contacts(NULL, NULL, NULL, NULL, NULL) == SC_ERR_INVALID);
        sc_batch_destroy(NULL);
    }
    printf("host checks: %s\n", g_fail ? "FAILED" : "ok");
}

/* ------------------------------------------------------------- GPU pass */

static uint64_t g_rng = 0x9E3779B97F4A7C15ull;

static double urand(void) { /* xorshift64*, uniform in [0, 1) */
    g_rng ^= g_rng >> 12;
    g_rng ^= g_rng << 25;
    g_rng ^= g_rng >> 27;
    return (double)((g_rng * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static void *dev_alloc(size_t bytes) {
    void *p = NULL;
    HIP(hipMalloc(&p, bytes ? bytes : 256));
    HIP(hipMemset(p, 0, bytes ? bytes : 256));
    return p;
}

static void *dev_copy(const void *h, size_t bytes) {
    void *p = dev_alloc(bytes);
    HIP(hipMemcpy(p, h, bytes, hipMemcpyHostToDevice));
    return p;
}

typedef struct {
    int n;
    double *pos, *axis, *radius, *half_len, *mob, *f, *quat; /* device */
    sc_particles p;
} system_t;

/* n particles on a jittered cubic lattice of spacing 1 (side m), radius 0.5;
 * every third a rod of half length 0.3 with a random axis unless spheres_only. */
static system_t make_system(int m, int spheres_only) {
    system_t s;
    const int n = m * m * m;
    s.n = n;
    double *pos = malloc(sizeof(double) * 3 * n), *axis = malloc(sizeof(double) * 3 * n);
    double *rad = malloc(sizeof(double) * n), *hl = malloc(sizeof(double) * n);
    double *mob = malloc(sizeof(double) * 4 * n), *f = malloc(sizeof(double) * 6 * n);
    for (int i = 0; i < n; ++i) {
        const int x = i % m, y = (i / m) % m, z = i / (m * m);
        pos[3 * i + 0] = x + 0.5 + 0.1 * (urand() - 0.5);
        pos[3 * i + 1] = y + 0.5 + 0.1 * (urand() - 0.5);
        pos[3 * i + 2] = z + 0.5 + 0.1 * (urand() - 0.5);
        double a[3] = {urand() - 0.5, urand() - 0.5, urand() - 0.5}, nr = 0.0;
        for (int k = 0; k < 3; ++k) nr += a[k] * a[k];
        nr = nr > 0.0 ? 1.0 / __builtin_sqrt(nr) : 0.0;
        for (int k = 0; k < 3; ++k) axis[3 * i + k] = nr > 0.0 ? a[k] * nr : (k == 2);
        rad[i] = 0.5;
        hl[i] = (!spheres_only && i % 3 == 0) ? 0.3 : 0.0;
        mob[4 * i + 0] = 1.0;
        mob[4 * i + 1] = hl[i] > 0.0 ? 0.8 : 1.0;
        mob[4 * i + 2] = 3.0;
        mob[4 * i + 3] = hl[i] > 0.0 ? 2.0 : 3.0;
        for (int k = 0; k < 6; ++k) f[6 * i + k] = urand() - 0.5;
    }
    s.pos = dev_copy(pos, sizeof(double) * 3 * n);
    s.axis = dev_copy(axis, sizeof(double) * 3 * n);
    s.radius = dev_copy(rad, sizeof(double) * n);
    s.half_len = dev_copy(hl, sizeof(double) * n);
    s.mob = dev_copy(mob, sizeof(double) * 4 * n);
    s.f = dev_copy(f, sizeof(double) * 6 * n);
    s.quat = dev_alloc(sizeof(double) * 4 * n);
    free(pos), free(axis), free(rad), free(hl), free(mob), free(f);
    s.p.n = n;
    s.p.reserved = 0;
    s.p.pos = s.pos;
    s.p.axis = s.axis;
    s.p.radius = s.radius;
    s.p.half_len = s.half_len;
    s.p.mob = s.mob;
    return s;
}

static void free_system(system_t *s) {
    HIP(hipFree(s->pos)); HIP(hipFree(s->axis)); HIP(hipFree(s->radius));
    HIP(hipFree(s->half_len)); HIP(hipFree(s->mob)); HIP(hipFree(s->f)); HIP(hipFree(s->quat));
}

typedef struct {
    sc_contacts c;
    void *ws;
    size_t ws_bytes;
} contacts_t;

static contacts_t alloc_contacts(int n, int cap, size_t nnz_cap) {
    contacts_t k;
    memset(&k, 0, sizeof k);
    k.c.capacity = cap;
    k.c.ci = dev_alloc(sizeof(int32_t) * cap);
    k.c.cj = dev_alloc(sizeof(int32_t) * cap);
    k.c.phi = dev_alloc(sizeof(double) * cap);
    k.c.q = dev_alloc(sizeof(double) * cap);
    k.c.frame = dev_alloc(sizeof(double) * 9 * cap);
    k.c.plan_bytes = sc_plan_bytes(n, cap);
    k.c.plan = dev_alloc(k.c.plan_bytes);
    if (nnz_cap) {
        k.c.nnz = (int64_t)nnz_cap;
        k.c.mat_bytes = sc_matrix_bytes(cap, (int64_t)nnz_cap);
        k.c.mat = dev_alloc(k.c.mat_bytes);
    }
    k.ws_bytes = sc_workspace_bytes(n, cap, SC_WS_ALL);
    k.ws = dev_alloc(k.ws_bytes);
    return k;
}

static void free_contacts(contacts_t *k) {
    HIP(hipFree(k->c.ci)); HIP(hipFree(k->c.cj)); HIP(hipFree(k->c.phi)); HIP(hipFree(k->c.q));
    HIP(hipFree(k->c.frame)); HIP(hipFree(k->c.plan)); HIP(hipFree(k->ws));
    if (k->c.mat) HIP(hipFree(k->c.mat));
}

static void gpu_dry(hipStream_t s) {
    const double dt = 1e-3, delta = 0.05;
    system_t S = make_system(10, 0); /* 1000 particles, a third of them rods */
    const int n = S.n, cap = 20 * n;
    sc_box box = {{0, 0, 0}, {10, 10, 10}, 1, 0};
    double *u_nc = dev_alloc(sizeof(double) * 6 * n);
    OK(sc_apply_mobility(&S.p, S.f, u_nc, s));
    contacts_t K = alloc_contacts(n, cap, 0);
    OK(sc_build_contacts(&S.p, &box, delta, u_nc, dt, &K.c, K.ws, K.ws_bytes, s));
    const int nc = K.c.count;
    EXPECT(nc > n);
    printf("[dry] contacts built: %d\n", nc);
    K.c.mat_bytes = sc_matrix_bytes(nc, K.c.nnz);
    K.c.mat = dev_alloc(K.c.mat_bytes);
    OK(sc_assemble_matrix(&S.p, &K.c, s));
    EXPECT(K.c.mat_ready == 1);

    int32_t *perm = dev_alloc(sizeof(int32_t) * nc);
    OK(sc_canonical_order(n, &K.c, perm, K.ws, K.ws_bytes, s));

    double *x = dev_alloc(sizeof(double) * nc), *y = dev_alloc(sizeof(double) * nc);
    double *gamma = dev_alloc(sizeof(double) * nc), *g = dev_alloc(sizeof(double) * nc);
    double *gamma2 = dev_alloc(sizeof(double) * nc), *g2 = dev_alloc(sizeof(double) * nc);
    double *f_c = dev_alloc(sizeof(double) * 6 * n), *u_c = dev_alloc(sizeof(double) * 6 * n);
    OK(sc_mvop(&S.p, &K.c, K.c.q, y, K.ws, K.ws_bytes, s));

    sc_solve_opts o = {1e-6, 20000, 1, 0, 0, 0, 0, SC_OP_MATRIX, 0, 0, 0};
    sc_stats st;
    for (int bb = 1; bb <= 3; ++bb) {
        o.bb = bb;
        SOLVED(sc_solve_lcp(&S.p, &K.c, &o, gamma, g, f_c, u_c, &st, K.ws, K.ws_bytes, s));
        EXPECT(st.status == SC_OK);
    }
    printf("[dry] matrix solves done\n");
    o.bb = 1;
    o.op = SC_OP_CHAIN;
    SOLVED(sc_solve_lcp(&S.p, &K.c, &o, gamma2, g2, NULL, NULL, &st, K.ws, K.ws_bytes, s));
    /* the chain's LDS copy of pass A's data: none, capped, one workgroup */
    o.lds_entries_per_wave = -1;
    SOLVED(sc_solve_lcp(&S.p, &K.c, &o, gamma2, g2, NULL, NULL, &st, K.ws, K.ws_bytes, s));
    o.lds_entries_per_wave = 5;
    SOLVED(sc_solve_lcp(&S.p, &K.c, &o, gamma2, g2, NULL, NULL, &st, K.ws, K.ws_bytes, s));
    EXPECT(st.lds_entries_per_wave == 5);
    o.lds_entries_per_wave = 0;
    o.grid = 1;
    SOLVED(sc_solve_lcp(&S.p, &K.c, &o, gamma2, g2, NULL, NULL, &st, K.ws, K.ws_bytes, s));
    EXPECT(st.grid == 1);
    o.grid = 0;
    o.op = SC_OP_AUTO;
    o.warm_start = 1;
    SOLVED(sc_solve_lcp(&S.p, &K.c, &o, gamma2, g2, NULL, NULL, &st, K.ws, K.ws_bytes, s));
    o.warm_start = 0;
    SOLVED(sc_solve_lcp_noalloc(&S.p, &K.c, &o, gamma2, g2, f_c, u_c, &st, s));
    EXPECT(st.status == SC_OK);
    {
        sc_stats *st_dev = dev_alloc(sizeof(sc_stats));
        OK(sc_solve_lcp_async(&S.p, &K.c, &o, gamma2, g2, f_c, u_c, st_dev, K.ws, K.ws_bytes,
                              s));
        HIP(hipMemcpyAsync(&st, st_dev, sizeof st, hipMemcpyDeviceToHost, s));
        HIP(hipStreamSynchronize(s));
        EXPECT(st.status == SC_OK);
        HIP(hipFree(st_dev));
    }
    o.spin_limit = 1; /* the timeout path: every workgroup leaves its loop */
    {
        int rc = sc_solve_lcp(&S.p, &K.c, &o, gamma2, g2, NULL, NULL, &st, K.ws, K.ws_bytes, s);
        EXPECT(rc == SC_ERR_TIMEOUT || rc == SC_OK);
    }
    o.spin_limit = 0;
    SOLVED(sc_solve_lcp(&S.p, &K.c, &o, gamma, g, f_c, u_c, &st, K.ws, K.ws_bytes, s));

    printf("[dry] chain, no-alloc, async and time-out solves done\n");
    /* adjoint of L = 1/2 ||F_c||^2 */
    double *dq = dev_alloc(sizeof(double) * nc), *dpos = dev_alloc(sizeof(double) * 3 * n);
    sc_adjoint_opts ao = {1e-10, 10000, 0, 0, 0, 0, 0, 0};
    SOLVED(sc_solve_lcp_adjoint(&S.p, &box, &K.c, u_nc, dt, gamma, NULL, f_c, dq, dpos, &ao, &st,
                                K.ws, K.ws_bytes, s));
    ao.op = SC_OP_CHAIN;
    SOLVED(sc_solve_lcp_adjoint(&S.p, &box, &K.c, u_nc, dt, gamma, gamma, NULL, dq, dpos, &ao,
                                &st, K.ws, K.ws_bytes, s));

    {
        /* the active-set polish of the solve, in place on a copy */
        sc_adjoint_opts po = {1e-13, 10000, 0, 0, 0, 0, 0, 0};
        HIP(hipMemcpy(gamma2, gamma, sizeof(double) * nc, hipMemcpyDeviceToDevice));
        SOLVED(sc_polish_lcp(&S.p, &K.c, gamma2, g2, f_c, u_c, &po, 0, &st, K.ws, K.ws_bytes, s));
    }
    printf("[dry] adjoints and polish done\n");
    /* the dry mobility through the function interface */
    {
        size_t wb = sc_solve_mob_work_bytes(n, cap), wa = sc_adjoint_mob_work_bytes(n, cap);
        void *w = dev_alloc(wb > wa ? wb : wa);
        sc_solve_opts mo = {1e-6, 20000, 3, 0, 0, 0, 0, 0, 0, 0, 0};
        SOLVED(sc_solve_lcp_mob(&S.p, &K.c, &mo, sc_dry_apply, &S.p, 0, gamma2, g2, f_c, u_c,
                                &st, w, wb > wa ? wb : wa, s));
        SOLVED(sc_solve_lcp_adjoint_mob(&S.p, &box, &K.c, u_nc, S.f, dt, gamma2, NULL, f_c,
                                        sc_dry_apply, &S.p, NULL, NULL, &ao, 0, dq, dpos, &st, w,
                                        wb > wa ? wb : wa, s));
        HIP(hipFree(w));
    }

    printf("[dry] function-mobility solve and adjoint done\n");
    /* time stepping: warm start across a step */
    OK(sc_quat_from_axis(n, S.axis, S.quat, s));
    OK(sc_advance(n, S.pos, S.quat, S.axis, u_nc, u_c, dt, s));
    contacts_t K2 = alloc_contacts(n, cap, 0);
    OK(sc_build_contacts(&S.p, &box, delta, u_nc, dt, &K2.c, K2.ws, K2.ws_bytes, s));
    double *g0 = dev_alloc(sizeof(double) * (K2.c.count ? K2.c.count : 1));
    OK(sc_map_gamma(n, &K.c, gamma, &K2.c, g0, s));
    HIP(hipStreamSynchronize(s));

    /* a batch of two instances on the first contacts (plain, then its graph,
     * with the adjoint), and one built on the device */
    {
        double *gb[2], *gg[2], *dqb[2], *dpb[2];
        sc_batch_item it[2];
        memset(it, 0, sizeof it);
        for (int k = 0; k < 2; ++k) {
            gb[k] = dev_alloc(sizeof(double) * nc), gg[k] = dev_alloc(sizeof(double) * nc);
            dqb[k] = dev_alloc(sizeof(double) * nc);
            dpb[k] = dev_alloc(sizeof(double) * 3 * n);
            it[k].p = S.p;
            it[k].c = K.c;
            it[k].gamma = gb[k];
            it[k].g = gg[k];
            it[k].box = box;
            it[k].u_nc = u_nc;
            it[k].dt = dt;
            it[k].dL_dq = dqb[k];
            it[k].dL_dpos = dpb[k];
        }
        sc_batch_opts bo;
        memset(&bo, 0, sizeof bo);
        bo.tol = 1e-6, bo.max_iter = 20000, bo.bb = 1, bo.team = 0, bo.adjoint = 1;
        bo.adjoint_tol = 1e-10, bo.adjoint_max_iter = 10000;
        size_t wb = sc_batch_workspace_bytes(2, it, &bo);
        EXPECT(wb > 0);
        void *w = dev_alloc(wb);
        sc_batch *b = NULL;
        printf("[dry] time step done; batch of two\n");
        OK(sc_batch_create(2, it, &bo, w, wb, s, &b));
        OK(sc_batch_solve(b, s));
        OK(sc_batch_graph_launch(b, s));
        OK(sc_batch_graph_launch(b, s));
        sc_stats bst[2], bad[2];
        sc_batch_info info;
        OK(sc_batch_stats(b, bst, bad, &info, s));
        EXPECT(bst[0].status == SC_OK && bst[1].status == SC_OK);
        EXPECT(sc_batch_contacts(b, NULL, NULL, NULL, s) == SC_ERR_INVALID);
        sc_batch_destroy(b);
        HIP(hipFree(w));

        printf("[dry] batch (eager, graph) done\n");
        /* built on the device: its own output buffers */
        contacts_t KB = alloc_contacts(n, cap, (size_t)K.c.nnz * 2);
        sc_batch_item ib = it[0];
        ib.c = KB.c;
        ib.delta = delta;
        bo.build = 1, bo.team = 1, bo.adjoint = 0;
        wb = sc_batch_workspace_bytes(1, &ib, &bo);
        w = dev_alloc(wb);
        double *gbb = dev_alloc(sizeof(double) * cap), *ggb = dev_alloc(sizeof(double) * cap);
        ib.gamma = gbb, ib.g = ggb;
        OK(sc_batch_create(1, &ib, &bo, w, wb, s, &b));
        OK(sc_batch_solve(b, s));
        int32_t cnt = -1, bs = -1;
        int64_t nz = -1;
        OK(sc_batch_contacts(b, &cnt, &nz, &bs, s));
        EXPECT(bs == SC_OK && cnt == K2.c.count);
        OK(sc_batch_stats(b, bst, NULL, NULL, s));
        sc_batch_destroy(b);
        HIP(hipFree(w)); HIP(hipFree(gbb)); HIP(hipFree(ggb));
        free_contacts(&KB);
        for (int k = 0; k < 2; ++k) {
            HIP(hipFree(gb[k])); HIP(hipFree(gg[k])); HIP(hipFree(dqb[k])); HIP(hipFree(dpb[k]));
        }
    }

    HIP(hipFree(g0));
    free_contacts(&K2);
    HIP(hipFree(dq)); HIP(hipFree(dpos)); HIP(hipFree(perm)); HIP(hipFree(x)); HIP(hipFree(y));
    HIP(hipFree(gamma)); HIP(hipFree(g)); HIP(hipFree(gamma2)); HIP(hipFree(g2));
    HIP(hipFree(f_c)); HIP(hipFree(u_c)); HIP(hipFree(u_nc));
    free_contacts(&K);
    free_system(&S);
    printf("dry mobility: %d particles, %d contacts: %s\n", n, nc, g_fail ? "FAILED" : "ok");
}

static void gpu_rpy(hipStream_t s) {
    const double dt = 1e-3, delta = 0.05;
    system_t S = make_system(6, 1); /* 216 spheres */
    const int n = S.n, cap = 20 * n;
    sc_box box = {{0, 0, 0}, {6, 6, 6}, 0, 0x3}; /* walls on both x faces */
    sc_rpy r = {0};
    r.n = n;
    r.pos = S.pos;
    r.radius = S.radius;
    r.mu = 1.0;
    r.work_bytes = sc_rpy_work_bytes(n);
    r.work = dev_alloc(r.work_bytes);
    double *u_nc = dev_alloc(sizeof(double) * 6 * n);
    OK(sc_rpy_apply(&r, n, S.f, u_nc, s));
    contacts_t K = alloc_contacts(n, cap, 0);
    OK(sc_build_contacts(&S.p, &box, delta, u_nc, dt, &K.c, K.ws, K.ws_bytes, s));
    const int nc = K.c.count;
    EXPECT(nc > 0);
    double *gamma = dev_alloc(sizeof(double) * nc), *g = dev_alloc(sizeof(double) * nc);
    double *f_c = dev_alloc(sizeof(double) * 6 * n), *u_c = dev_alloc(sizeof(double) * 6 * n);
    double *dq = dev_alloc(sizeof(double) * nc), *dpos = dev_alloc(sizeof(double) * 3 * n);
    double *gr = dev_alloc(sizeof(double) * 3 * n);
    size_t wb = sc_solve_mob_work_bytes(n, cap), wr = sc_solve_rpy_work_bytes(n, cap),
           wa = sc_adjoint_mob_work_bytes(n, cap);
    size_t wmax = wb > wr ? wb : wr;
    wmax = wmax > wa ? wmax : wa;
    void *w = dev_alloc(wmax);
    sc_solve_opts o = {1e-6, 20000, 1, 0, 0, 0, 0, 0, 0, 0, 0};
    sc_stats st;
    SOLVED(sc_solve_lcp_mob(&S.p, &K.c, &o, sc_rpy_apply, &r, 0, gamma, g, f_c, u_c, &st, w,
                            wmax, s));
    printf("[rpy] %d contacts; function-mobility solve done\n", nc);
    SOLVED(sc_solve_lcp_rpy(&S.p, &K.c, &r, &o, gamma, g, f_c, u_c, &st, w, wmax, s));
    printf("[rpy] persistent solve done\n");
    OK(sc_rpy_grad(&r, n, f_c, S.f, gr, s));
    sc_adjoint_opts ao = {1e-10, 10000, 0, 0, 0, 0, 0, 0};
    SOLVED(sc_solve_lcp_adjoint_mob(&S.p, &box, &K.c, u_nc, S.f, dt, gamma, NULL, f_c,
                                    sc_rpy_apply, &r, sc_rpy_grad, &r, &ao, 0, dq, dpos, &st, w,
                                    wmax, s));
    HIP(hipStreamSynchronize(s));
    HIP(hipFree(w)); HIP(hipFree(gamma)); HIP(hipFree(g)); HIP(hipFree(f_c)); HIP(hipFree(u_c));
    HIP(hipFree(dq)); HIP(hipFree(dpos)); HIP(hipFree(gr)); HIP(hipFree(u_nc)); HIP(hipFree(r.work));
    free_contacts(&K);
    free_system(&S);
    printf("RPY mobility: %d spheres, %d contacts: %s\n", n, nc, g_fail ? "FAILED" : "ok");
}

int main(int argc, char **argv) {
    setvbuf(stdout, NULL, _IONBF, 0); /* the progress lines survive an abort */
    host_checks();
    if (argc > 1 && strcmp(argv[1], "gpu") == 0) {
        hipStream_t s;
        HIP(hipStreamCreate(&s));
        gpu_dry(s);
        gpu_rpy(s);
        OK(sc_release());
        HIP(hipStreamDestroy(s));
    }
    printf("%s\n", g_fail ? "FAILED" : "all ok");
    return g_fail;
}
