/*
 * sc_api.h -- C ABI of the MI355X (gfx950) collision-resolution library.
 *
 * The library implements the data-parallel core of the collision method of
 * Yan, Corona, Malhotra, Veerapaneni and Shelley, "A scalable computational
 * platform for particulate Stokes suspensions" (arXiv:1909.06623), section 3:
 * the close-pair set A(C, delta), the contact Jacobian D, the LCP data
 * q = Phi/dt + D^T U_nc, and the Barzilai-Borwein projected gradient descent
 * (Algorithm 1) of min 1/2 gamma^T M gamma + q^T gamma over gamma >= 0 with
 * M = D^T Mob D, where Mob is a block-diagonal per-particle ("dry") mobility.
 * An implicit adjoint of the converged solve is provided as well.
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers (hipMalloc'd or equivalent) in
 *     FP64 unless typed otherwise; indices are int32. Arrays are row-major.
 *     Structs themselves are passed by host pointer.
 *   - The caller owns every buffer. No entry point allocates device memory:
 *     scratch comes from a caller-provided workspace of at least
 *     sc_workspace_bytes(n, capacity, what) bytes, 256-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the null stream). Work is enqueued on
 *     it in order. Entry points that must report a count or a status to the
 *     host (build_contacts, solve_lcp, solve_lcp_adjoint) synchronise that
 *     stream before returning; the others do not. sc_solve_lcp_async is the
 *     solve with its status left on the device (capturable into a graph).
 *   - A particle's 6-vectors (velocity, force) are (x, y, z, wx, wy, wz):
 *     translational part, then rotational part (section 2 stacks U and F
 *     per particle in this order).
 *   - Return value: one of the SC_* codes below. On an error return nothing
 *     is guaranteed about output arrays unless stated.
 */
#ifndef SC_API_H
#define SC_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define SC_OK                0  /* success */
#define SC_NOT_CONVERGED     1  /* max_iter reached; outputs hold the last iterate */
#define SC_ERR_INVALID      -1  /* NULL pointer, negative size, bad option */
#define SC_ERR_CAPACITY     -2  /* more contacts than capacity; count holds the need */
#define SC_ERR_NONFINITE    -3  /* NaN/Inf in an input or an iterate */
#define SC_ERR_BOX          -4  /* periodic side < 2 x interaction range */
#define SC_ERR_HIP          -5  /* a HIP runtime call failed */
#define SC_ERR_WORKSPACE    -6  /* workspace too small or misaligned */
#define SC_ERR_TIMEOUT      -7  /* a grid barrier of a persistent kernel timed out */

/* ---------------------------------------------------------------- data */

/* Rigid particles (section 3.1: each particle has a centre c and an
 * orientation; a spherocylinder needs only its unit axis p). A sphere is a
 * particle with half_len == 0 (its axis is ignored). */
typedef struct sc_particles {
    int32_t n;              /* number of particles, >= 0 */
    int32_t reserved;
    const double *pos;      /* [n][3] centres c */
    const double *axis;     /* [n][3] unit axes p */
    const double *radius;   /* [n] radius R > 0 (spheres: the radius; rods: D/2) */
    const double *half_len; /* [n] half segment length h >= 0 (0 = sphere) */
    const double *mob;      /* [n][4] dry mobility (a_par, a_perp, b_par, b_perp) > 0:
                               U = a_par pp^T F + a_perp (I - pp^T) F,
                               W = b_par pp^T T + b_perp (I - pp^T) T */
} sc_particles;

/* Simulation box. periodic != 0: minimum-image convention on [lo, lo+len)
 * (positions may lie anywhere; they are wrapped for binning only).
 * periodic == 0: free space; len only sizes the search grid (particles
 * outside [lo, lo+len) are still found), and `walls` may close faces of the
 * box with planar walls (section 3.3's boundary extension: a particle
 * within delta of a wall gets a constraint whose column of D holds its own
 * 6 entries only). */
typedef struct sc_box {
    double lo[3];
    double len[3];
    int32_t periodic;
    int32_t walls;          /* periodic == 0 only: bit 2a = wall at x_a = lo[a], bit
                               2a + 1 = wall at x_a = lo[a] + len[a]; a wall contact has
                               cj = -1 - face and tau_j = 0 */
} sc_box;

/* Contacts: one constraint per close pair i < j (section 3.1).
 * Caller-allocated; every per-contact array has `capacity` rows. Column l of
 * D (Eq. Dmatdef) places (-n_l, -tau_i,l) on particle ci and (+n_l, +tau_j,l)
 * on particle cj, where n_l is the unit normal from ci's closest core point to
 * cj's and tau_k,l = (x_k,l - c_k) x n_l is the moment arm of contact point
 * x_k,l; then D_l^T U = dPhi_l/dt under rigid velocities U (Eq. Dtranspose).
 *
 * Order ("solver order"): particles are ranked by search cell (row-major over
 * the grid reported in `grid`) and, within a cell, by index; contacts are
 * grouped by the rank of their lower-ranked particle, partners by increasing
 * rank. The order is a deterministic function of the inputs, keeps every
 * gather of the solve local, and is the order of gamma and g;
 * sc_canonical_order gives the permutation to the canonical (ci, cj) order.
 *
 * `plan` is a caller-allocated device buffer of at least
 * sc_plan_bytes(n, capacity) bytes (256-byte aligned) in which
 * sc_build_contacts stores the solver layout (ranking, incidence lists and
 * signed column entries) read by sc_solve_lcp, sc_mvop and
 * sc_solve_lcp_adjoint; its contents are private to the library. */
typedef struct sc_contacts {
    int32_t capacity;       /* rows allocated (>= 0) */
    int32_t count;          /* OUT (host): number of contacts n_c */
    int32_t *ci;            /* [capacity] particle i (caller index) */
    int32_t *cj;            /* [capacity] particle j (> i) */
    double *phi;            /* [capacity] minimum separation Phi_l (<= delta) */
    double *q;              /* [capacity] LCP vector q_l = Phi_l/dt + D_l^T U_nc */
    double *frame;          /* [capacity][9]: n (x y z), tau_i (x y z), tau_j (x y z) */
    void *plan;             /* [plan_bytes] device, solver layout (private) */
    size_t plan_bytes;
    int32_t n_parallel;     /* OUT (host): pairs resolved by the parallel-axes rule */
    int32_t n_zero_dist;    /* OUT (host): pairs with coincident cores (n := +x) */
    int32_t n_borderline;   /* OUT (host): pairs with |Phi - delta| < 1e-12 */
    int32_t grid[3];        /* OUT (host): search cells per axis used */
    int64_t nnz;            /* OUT (host): nonzeros of M = D^T Mob D (set by build) */
    void *mat;              /* optional device buffer of sc_matrix_bytes(count, nnz)
                               bytes (256-byte aligned) for the assembled M */
    size_t mat_bytes;
    int32_t mat_ready;      /* OUT (host): 1 once sc_assemble_matrix filled mat */
    int32_t reserved;
} sc_contacts;

#define SC_OP_AUTO   0      /* assembled M if c->mat_ready, else the matrix-free chain */
#define SC_OP_CHAIN  1      /* matrix-free: gather D x, apply Mob, gather D^T U */
#define SC_OP_MATRIX 2      /* assembled sparse M (requires c->mat_ready) */
#define SC_OP_CALLBACK 3    /* reported by sc_solve_lcp_mob only: D x, the caller's
                               mobility, D^T U */
#define SC_OP_RPY 4         /* reported by sc_solve_lcp_rpy only: one persistent launch
                               with the RPY mobility inside */

typedef struct sc_solve_opts {
    double tol;             /* absolute tolerance on ||min(gamma, g)||_2 (> 0) */
    int32_t max_iter;       /* j_max of Algorithm 1 (>= 0) */
    int32_t bb;             /* step rule: 1 = BB1, 2 = BB2, 3 = BB1 odd / BB2 even */
    int32_t warm_start;     /* 1: gamma holds gamma_0 on entry; 0: gamma_0 = 0 */
    int32_t lanes_per_particle; /* chain product: 0 (default 4), 1, 2, 4 or 8 lanes sharing
                                   a particle's incidence list */
    int32_t grid;           /* workgroups of the persistent kernel (0 = chosen: for the
                               assembled M about sqrt(nnz) / 5, a multiple of 8, which
                               is every CU from about 1.5 million nonzeros; for the
                               chain one per CU; clamped to at most one per CU and
                               to what is co-resident) */
    int32_t block;          /* threads per workgroup: 0 (default 1024), 256, 512 or 1024 */
    int32_t op;             /* product M x: SC_OP_AUTO (assembled M when ready, else the
                               matrix-free chain), SC_OP_CHAIN or SC_OP_MATRIX */
    int32_t slices_per_wave; /* assembled-M product: 0 (default 1), 1, 2 or 4 slices of 64
                                rows that one wave works on at once */
    int32_t lds_entries_per_wave; /* assembled-M product: entries of M each wave keeps in
                                LDS for the whole solve; matrix-free chain: incidences
                                (code and D column) per wave of the workgroup's share
                                kept in LDS; 0 = as many as fit, -1 = none, > 0 = at
                                most that many. Iterates do not depend on it. */
    int32_t spin_limit;     /* 0: a wait at a grid barrier gives up after 2^21 polls
                               (SC_ERR_TIMEOUT, every workgroup leaves its loop);
                               > 0: after this many (a small value forces the timeout
                               path, for tests of it) */
} sc_solve_opts;

typedef struct sc_stats {
    int32_t status;         /* SC_OK, SC_NOT_CONVERGED or SC_ERR_NONFINITE */
    int32_t iters;          /* descent steps taken (j at exit) */
    int32_t mvops;          /* products M x evaluated (section 6.2 accounting) */
    int32_t n_active;       /* |{l : gamma_l > 0}| at exit */
    double residual;        /* ||min(gamma, g)||_2 at exit */
    double alpha;           /* last step size */
    int32_t n_degenerate;   /* step sizes kept because a BB denominator was <= 0 */
    int32_t grid;           /* workgroups of the persistent kernel used */
    double kernel_ms;       /* GPU time of the persistent kernel (HIP events on `stream`) */
    int32_t lanes_per_particle; /* gather lanes per particle (chain; 0 for the matrix) */
    int32_t block;          /* threads per workgroup used */
    int32_t op;             /* SC_OP_CHAIN or SC_OP_MATRIX: the product used */
    int32_t slices_per_wave; /* slices per wave (matrix; 0 for the chain) */
    int32_t lds_entries_per_wave; /* entries of M (matrix) or incidences (chain) per wave
                                     held in LDS */
    int32_t reserved;
} sc_stats;

typedef struct sc_adjoint_opts {
    double tol;             /* CG stopping tolerance, relative to ||b_A|| */
    int32_t max_iter;       /* CG iteration cap */
    int32_t lanes_per_particle; /* as in sc_solve_opts */
    int32_t grid;           /* as in sc_solve_opts */
    int32_t block;          /* as in sc_solve_opts */
    int32_t op;             /* as in sc_solve_opts */
    int32_t slices_per_wave; /* as in sc_solve_opts */
    int32_t lds_entries_per_wave; /* as in sc_solve_opts */
} sc_adjoint_opts;

/* ---------------------------------------------------------------- calls */

/* What a workspace is for (sc_workspace_bytes' `what`). */
#define SC_WS_ALL      0    /* any entry point below */
#define SC_WS_BUILD    1    /* sc_build_contacts, sc_canonical_order */
#define SC_WS_SOLVE    2    /* sc_solve_lcp, sc_solve_lcp_async, sc_mvop */
#define SC_WS_ADJOINT  3    /* sc_solve_lcp_adjoint, sc_polish_lcp */

/* Bytes of workspace the entry points named by `what` need for n particles
 * and `capacity` contact rows (SC_WS_ALL: the largest of them). Pure host
 * arithmetic; 0 for negative sizes or an unknown `what`. */
size_t sc_workspace_bytes(int32_t n, int32_t capacity, int32_t what);

/* Bytes of the plan buffer of sc_contacts for n particles and `capacity`
 * contact rows. Pure host arithmetic. */
size_t sc_plan_bytes(int32_t n, int32_t capacity);

/* Bytes of the assembled-matrix buffer for `count` contact rows and `nnz`
 * nonzeros (both as reported in sc_contacts after sc_build_contacts). Pure
 * host arithmetic; 0 if nnz does not fit 32-bit column offsets. */
size_t sc_matrix_bytes(int32_t count, int64_t nnz);

/* u[k] = Mob_k f[k] for every particle (the dry block-diagonal mobility that
 * stands in for the paper's mobility solve, section 2). f, u: [n][6].
 * Does not synchronise. */
int sc_apply_mobility(const sc_particles *p, const double *f, double *u,
                      void *stream);

/* Close-pair set A(C, delta) = {(i, j), i < j : Phi_ij <= delta} (section
 * 3.2), its contact frames (Eq. Dmatdef, Eq. Dtranspose), the solver layout
 * in c->plan and q = Phi/dt + D^T u_nc (LCP LCPdef, scaled by 1/dt). Phi is
 * the minimum separation of the two cores (a point for a sphere, the segment
 * c +- h p for a spherocylinder) minus both radii.
 * u_nc: [n][6] non-collisional velocities. Writes c->count; if it exceeds
 * c->capacity returns SC_ERR_CAPACITY with c->count = the required rows and
 * no contact written. SC_ERR_BOX if periodic and a side is below twice the
 * interaction range 2 max(R + h) + delta. Synchronises `stream` (a batch of
 * one system created with build = 1 builds without host synchronisation). */
int sc_build_contacts(const sc_particles *p, const sc_box *box, double delta,
                      const double *u_nc, double dt, sc_contacts *c,
                      void *ws, size_t ws_bytes, void *stream);

/* The canonical order of the close-pair set (section 3.1: one constraint per
 * pair i < j; section 3.2's set listed by ci, then cj, with a wall contact's
 * negative cj = -1 - face before the particle's pairs): perm[t] = the
 * solver-order index of the t-th contact in that order, for t < c->count,
 * so that ci[perm[t]], cj[perm[t]] enumerate the pairs as a plain loop over
 * i < j would. n: the particles c was built for (sc_build_contacts' plan is
 * read). perm: device int32 [c->count], OUT. ws: device workspace of at
 * least sc_workspace_bytes(n, c->capacity, SC_WS_BUILD) bytes, 256-byte aligned.
 * Deterministic (no sort, no atomics). Enqueues only; returns SC_OK,
 * SC_ERR_INVALID, SC_ERR_WORKSPACE or SC_ERR_HIP. */
int sc_canonical_order(int32_t n, const sc_contacts *c, int32_t *perm, void *ws,
                       size_t ws_bytes, void *stream);

/* Assemble M = D^T Mob D (LCP LCPdef) into c->mat as a sparse matrix with
 * one row per contact: row l holds M_lm for every contact m sharing a
 * particle with l (deg(ci) + deg(cj) - 1 entries, the diagonal first; rows
 * are stored in slices of 64, each slice depth by depth, layout private),
 * M_lm = a_lk^T Mob_k a_mk with a_lk the signed column entries of contact l
 * on the shared particle k. For a block-diagonal mobility this is exact and
 * replaces the two-pass product inside the solve. Requires a prior
 * sc_build_contacts and c->mat_bytes >= sc_matrix_bytes(count, nnz); sets
 * c->mat_ready. Synchronises `stream`. */
int sc_assemble_matrix(const sc_particles *p, sc_contacts *c, void *stream);

/* y = M x = D^T Mob D x for x, y of c->count entries: one matrix-free
 * product ("MVOP", LCP LCPdef and section 6.2). Does not synchronise. */
int sc_mvop(const sc_particles *p, const sc_contacts *c, const double *x,
            double *y, void *ws, size_t ws_bytes, void *stream);

/* BBPGD, Algorithm 1 (section 3.3.1), as one persistent cooperative launch:
 * from gamma_0 (zero, or the contents of gamma if opts->warm_start), g_0 = M gamma_0 + q, alpha_0 = g0^T g0 /
 * g0^T M g0, then gamma_j = max(0, gamma_{j-1} - alpha_{j-1} g_{j-1}),
 * g_j = M gamma_j + q, stopping when ||min(gamma_j, g_j)||_2 < tol (Eq.
 * mmapnorm), with the BB1/BB2 step size of Algorithm 1. A non-positive
 * BB denominator keeps the previous step (g0^T M g0 <= 0 takes 1/max_l
 * M_ll). gamma, g: [c->count], OUT: the last iterate and M gamma + q.
 * f_c, u_c: [n][6] or NULL; OUT: contact forces D gamma and velocities
 * Mob D gamma (computed with gamma, as section 3.2's procedure asks). st: host pointer, OUT.
 * Returns SC_OK, SC_NOT_CONVERGED (outputs hold the last iterate) or an
 * error. Iterates are bitwise reproducible for a given launch shape (grid,
 * lanes_per_particle). Synchronises `stream`. */
int sc_solve_lcp(const sc_particles *p, const sc_contacts *c,
                 const sc_solve_opts *opts, double *gamma, double *g,
                 double *f_c, double *u_c, sc_stats *st, void *ws,
                 size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * sc_solve_lcp with the same arguments, kernels and results, except that its
 * workspace is a library-owned device array of SC_NOALLOC_SCRATCH_BYTES bytes
 * instead of a caller buffer, and st->kernel_ms is 0 (no HIP events are
 * created). The array is static device memory of the library: each GPU the
 * library runs on holds one copy until the process ends. The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); its device
 * address is looked up on the first call on each device. Every call on one
 * GPU shares that GPU's array, which keeps the last call's contents (what
 * must start at zero is cleared by the call): calls that overlap on one GPU,
 * on any streams, race and give undefined results. Returns
 * SC_ERR_WORKSPACE, before any device work, when the solve needs more than
 * the array holds, i.e. when sc_workspace_bytes(n, capacity, SC_WS_SOLVE)
 * (about 32 capacity + 64 n + 72 KiB) exceeds SC_NOALLOC_SCRATCH_BYTES, so
 * for example n = 100,000 particles with capacity up to about 1.8 million
 * contacts; otherwise as sc_solve_lcp. Synchronises `stream`. */
#define SC_NOALLOC_SCRATCH_BYTES (64u << 20)
int sc_solve_lcp_noalloc(const sc_particles *p, const sc_contacts *c,
                         const sc_solve_opts *opts, double *gamma, double *g, double *f_c,
                         double *u_c, sc_stats *st, void *stream);

/* sc_solve_lcp (Algorithm 1, section 3.3.1) without any host
 * synchronisation, for stream-ordered pipelines and HIP graph capture: the
 * same checks, kernels and results, but the call only enqueues work on
 * `stream` (gamma_0, the barrier block and the control block are cleared by
 * a kernel, no memset), and the statistics are written by a kernel to
 * `st_dev`, a DEVICE pointer to one sc_stats (status, iters, mvops,
 * n_active, residual, alpha, n_degenerate and the launch fields;
 * kernel_ms = 0). The return value reports only argument and launch errors
 * (SC_OK, SC_ERR_INVALID, SC_ERR_WORKSPACE, SC_ERR_HIP); the solve's own
 * outcome (SC_OK, SC_NOT_CONVERGED, SC_ERR_NONFINITE, SC_ERR_TIMEOUT) is
 * st_dev->status once the stream reaches it. Inside a stream capture the
 * persistent kernel's graph node is marked cooperative by the call. A
 * replayed graph repeats the captured solve on the buffers it was captured
 * with, bitwise as an eager call. */
int sc_solve_lcp_async(const sc_particles *p, const sc_contacts *c,
                       const sc_solve_opts *opts, double *gamma, double *g, double *f_c,
                       double *u_c, sc_stats *st_dev, void *ws, size_t ws_bytes, void *stream);

/* Implicit adjoint of a converged solve (not in the paper: it differentiates
 * the LCP of LCP LCPdef on its active set A = {gamma > 0}, section 3.2).
 * Given dL/dgamma [count] and dL/dF_c [n][6] (either may be NULL = zero),
 * solves M_AA w_A = b_A with b = dL/dgamma + D^T dL/dF_c and w = 0 off A by
 * conjugate gradients, then writes dL_dq = -w [count] and dL_dpos [n][3],
 * the gradient with respect to the centres with orientations, radii,
 * mobility and u_nc held fixed. gamma must be the solve's output for the
 * same contacts. st (host, OUT): iters = CG iterations, residual = final
 * relative CG residual, n_active = |A|, kernel_ms = GPU time of the
 * persistent CG kernel (HIP events on `stream`). Synchronises `stream`. */
int sc_solve_lcp_adjoint(const sc_particles *p, const sc_box *box,
                         const sc_contacts *c, const double *u_nc, double dt,
                         const double *gamma, const double *dL_dgamma,
                         const double *dL_df, double *dL_dq, double *dL_dpos,
                         const sc_adjoint_opts *opts, sc_stats *st, void *ws,
                         size_t ws_bytes, void *stream);

/* Active-set polish of a solve (not in the paper; it makes a converged
 * iterate of Algorithm 1 exact on its active set, section 3.2's LCP): with
 * A = {gamma > 0} of the input, solves M_AA gamma_A = -q_A by conjugate
 * gradients (to ||r|| <= opts->tol ||q_A||, at most opts->max_iter
 * iterations; the other fields of opts choose the product as for the
 * adjoint), sets gamma = 0 off A and g = M gamma + q, then moves the
 * violators (gamma_l < 0 leaves A, g_l < 0 joins A) and repeats, at most
 * max_pass times (0 = 20). gamma: [c->count] device, IN: the solve's
 * output, OUT: the polished point if a pass ends with no violator, else
 * unchanged. g: [c->count] device, OUT: M gamma + q of the returned gamma.
 * f_c, u_c: [n][6] or NULL, OUT: D gamma and Mob D gamma of it. st (host,
 * OUT): status SC_OK when polished, SC_NOT_CONVERGED when no pass settled
 * or an active block's CG did not converge (outputs are then the input's),
 * or the CG's error; iters = CG iterations over all passes; mvops = passes;
 * n_active = |A| of the polished point; residual = ||min(gamma, g)||_2 of
 * the returned point; kernel_ms = GPU time of the CG launches. ws: device
 * workspace of at least sc_workspace_bytes(n, c->capacity, SC_WS_ADJOINT)
 * bytes, 256-byte aligned. Synchronises `stream` once per pass. */
int sc_polish_lcp(const sc_particles *p, const sc_contacts *c, double *gamma, double *g,
                  double *f_c, double *u_c, const sc_adjoint_opts *opts, int32_t max_pass,
                  sc_stats *st, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------- batched */

/* One LCP of a batch (an independent suspension): its particles, its
 * contacts from sc_build_contacts with the assembled M (c.mat_ready == 1),
 * and device buffers for gamma (IN: gamma_0 when warm-starting) and g,
 * [c.count] each. For the adjoint (opts->adjoint != 0) also the box, u_nc
 * and dt the contacts were built with, an optional dL/dgamma [c.count]
 * (NULL = 0) and the outputs dL_dq [c.count] and dL_dpos [p.n][3], as in
 * sc_solve_lcp_adjoint.
 *
 * With opts->build = 1 the batch builds the contacts itself on every solve
 * (section 3.2's close-pair set, the frames of Eq. Dmatdef, q of LCP LCPdef
 * and M, as sc_build_contacts + sc_assemble_matrix do) from the particles'
 * current positions: box, delta, u_nc and dt are then the build's inputs, c
 * holds caller-allocated OUTPUT buffers of c.capacity rows (ci, cj, phi, q,
 * frame; plan of sc_plan_bytes(p.n, c.capacity) bytes; mat of
 * sc_matrix_bytes(c.capacity, c.nnz) bytes with c.nnz the nonzero capacity),
 * and gamma, g, dL_dgamma and dL_dq have c.capacity rows. c.count is
 * ignored; the contacts of the last solve are counted on the device
 * (sc_batch_contacts). The search grid of each suspension is fixed when the
 * batch is created (from its particles' largest R + h); positions may change
 * between solves, radii and lengths may not grow.
 *
 * The batch keeps the pointers, not the structs' owners: every buffer must
 * outlive the batch. */
typedef struct sc_batch_item {
    sc_particles p;
    sc_contacts c;
    double *gamma;
    double *g;
    sc_box box;
    const double *u_nc;
    double dt;
    double delta;           /* build only: pair threshold on Phi (>= 0) */
    const double *dL_dgamma;
    double *dL_dq;
    double *dL_dpos;
} sc_batch_item;

typedef struct sc_batch_opts {
    double tol;             /* epsilon_tol of Algorithm 1 for every instance */
    int32_t max_iter;       /* j_max */
    int32_t bb;             /* 1 = BB1, 2 = BB2, 3 = alternating */
    int32_t warm_start;     /* 1: gamma holds gamma_0 on entry */
    int32_t team;           /* workgroups per instance, all on one XCD: 1, 2, 4, 8,
                               16 or 32 for every instance; 0 = size classes (see
                               nnz_per_workgroup) */
    int32_t block;          /* threads per workgroup of the forward launch: 0 (1024),
                               256, 512 or 1024 */
    int32_t adjoint;        /* 0: solve only; 1: then the adjoint of
                               L = 1/2 ||D gamma||^2 + dL_dgamma . gamma; 2: of the
                               linear loss dL_dgamma . gamma only */
    double adjoint_tol;     /* CG tolerance relative to ||b_A|| */
    int32_t adjoint_max_iter;
    int32_t build;          /* 1: each solve first builds every instance's contacts
                               and M on the device (see sc_batch_item) */
    int32_t adjoint_team;   /* the adjoint launch's team (values as team); with
                               adjoint_nnz_per_workgroup also 0: the forward's policy,
                               tuned on its own when the forward's is tuned */
    int32_t nnz_per_workgroup; /* team == 0: instance k runs on t_k workgroups, the
                               smallest power of two with t_k * nnz_per_workgroup >=
                               its nonzeros of M, at most 32 (teams of 32 per XCD
                               halve as the queue, largest first, reaches smaller
                               classes); 0 with team == 0 = autotune: the batch is
                               solved once with classes for each of 4096, 8192, ...,
                               131072 and once with each single team size, and the
                               fastest policy kept, for the forward and the adjoint
                               launch apart (overwrites gamma and g) */
    int32_t adjoint_nnz_per_workgroup; /* the same for the adjoint launch (0: see
                               adjoint_team) */
    int32_t adjoint_block;  /* threads per workgroup of the adjoint launch: 0 (512),
                               256, 512 or 1024 */
} sc_batch_opts;

typedef struct sc_batch_info {
    int32_t team, block, grid;      /* launch used (team: the forward launch's team size,
                                       or 32 with size classes) */
    int32_t lds_entries_per_wave;   /* entries of M per wave kept in LDS */
    float tune_ms[12];              /* autotuner: build + forward time for size classes
                                       with nnz_per_workgroup = 4096, 8192, ..., 131072,
                                       then for one team size 1, 2, ..., 32 (0: skipped) */
    int32_t team_adjoint;           /* the adjoint launch's team size (32 with classes) */
    float tune_adjoint_ms[12];      /* autotuner: adjoint launch time, same policies */
    int32_t nnz_per_workgroup;      /* size classes' target used (0: one team size) */
    int32_t adjoint_nnz_per_workgroup;
    int32_t adjoint_block;          /* threads per workgroup of the adjoint launch */
} sc_batch_info;

typedef struct sc_batch sc_batch;   /* opaque plan (host memory) */

/* Workspace bytes of a batch (device memory, 256-byte aligned) for these
 * items and options (adjoint and build matter). 0 on invalid arguments. */
size_t sc_batch_workspace_bytes(int32_t count, const sc_batch_item *items,
                                const sc_batch_opts *opts);

/* Plans a batch of `count` LCPs (Algorithm 1 per instance, section 3.3.1): checks
 * every item, writes the instance table and the work order (by nonzeros,
 * largest first) into ws, and sets each launch's team policy (autotuning
 * if opts->team and opts->nnz_per_workgroup are 0). *out receives a plan
 * to free with sc_batch_destroy.
 * Synchronises `stream`. */
int sc_batch_create(int32_t count, const sc_batch_item *items, const sc_batch_opts *opts,
                    void *ws, size_t ws_bytes, void *stream, sc_batch **out);

/* Solves every instance of the batch in one persistent launch (preceded by a
 * small reset kernel; with the adjoint enabled, a second persistent launch
 * differentiates every solution; with build, the contact build of every
 * instance comes first, as one sequence of launches over the whole batch).
 * Enqueues only: no synchronisation, no allocation. An instance whose build
 * fails (SC_ERR_NONFINITE, SC_ERR_BOX: a particle grew past the planned grid,
 * SC_ERR_CAPACITY: contacts or nonzeros beyond c.capacity / c.nnz) reports
 * that status and is not solved; the others are unaffected. */
int sc_batch_solve(sc_batch *b, void *stream);

/* As sc_batch_solve, through a HIP graph captured on the first call (the
 * persistent kernels' nodes are marked cooperative) and replayed after. */
int sc_batch_graph_launch(sc_batch *b, void *stream);

/* Per-instance results of the last solve (st: host array of count; grid
 * holds the instance's team size), of its adjoint (adj: host array of count or NULL;
 * iters = CG iterations, residual = relative CG residual) and the launch
 * used (info may be NULL). Synchronises `stream`. */
int sc_batch_stats(const sc_batch *b, sc_stats *st, sc_stats *adj, sc_batch_info *info,
                   void *stream);

/* Build mode: per-instance contact count, nonzeros of M and build status of
 * the last solve (host arrays of count; any may be NULL). Synchronises
 * `stream`. SC_ERR_INVALID if the batch does not build its contacts. */
int sc_batch_contacts(const sc_batch *b, int32_t *count, int64_t *nnz, int32_t *status,
                      void *stream);

void sc_batch_destroy(sc_batch *b);

/* ------------------------------------------------------- time stepping */

/* One first-order Euler step of the configuration (section 3.2, Eq.
 * time-step; orientation kinematics of section 2): with U = u_nc + u_c per
 * particle ([n][6] each, u_c may be NULL = 0),
 *   c     += dt U[0:3]
 *   theta += dt Psi(theta) U[3:6],  Psi = 1/2 [-p^T; s I - [p]x]
 * for the unit quaternion theta = (s, p) ([n][4], s first), which is then
 * normalised (reading: the paper's update leaves the norm free), and
 * axis = R(theta) e_z ([n][3], written for every particle). pos, quat and
 * axis are device arrays updated in place. Enqueues only. SC_ERR_INVALID on
 * n < 0, dt <= 0 or a missing array. */
int sc_advance(int32_t n, double *pos, double *quat, double *axis, const double *u_nc,
               const double *u_c, double dt, void *stream);

/* quat [n][4] = the unit quaternion of the shortest rotation taking e_z to
 * the unit axis [n][3] (the half turn about x for axis = -e_z), the state
 * sc_advance starts from. Enqueues only. */
int sc_quat_from_axis(int32_t n, const double *axis, double *quat, void *stream);

/* Warm start of a step's LCP (the previous step's collision forces as
 * gamma_0 of Algorithm 1): gamma0[l] for each contact l = (i, j) of `cur` is
 * gamma_prev of the same pair in `prev` (the previous step's contacts of the
 * same n particles, from sc_build_contacts), or 0 if the pair is new. Pairs
 * are matched through prev's incidence lists, so the cost is the degree of
 * i per contact. All arrays device; gamma_prev [prev->count], gamma0
 * [cur->count]. Enqueues only. */
int sc_map_gamma(int32_t n, const sc_contacts *prev, const double *gamma_prev,
                 const sc_contacts *cur, double *gamma0, void *stream);

/* ---- Algorithm 1 behind a general mobility --------------------------------
 * Section 2 defines the mobility Mob as a dense SPD map from forces and
 * torques to velocities; in section 3.3 each product M x = D^T Mob D x is one
 * mobility problem for the force D x, and section 8 allows any mobility
 * solver that keeps Mob SPD. The entry points below take the mobility as a
 * function. */

/* A mobility: enqueue u = Mob f on `stream` (no host synchronisation needed)
 * for device arrays f, u of [n][6] in caller particle order (force xyz,
 * torque xyz -> velocity xyz, angular velocity xyz). Mob must be symmetric
 * positive definite. Returns SC_OK or an error code; an error ends the solve
 * that called it with that code. f and u belong to the caller of the
 * function and are valid until the enqueued work completes. */
typedef int (*sc_mobility_fn)(void *ctx, int32_t n, const double *f, double *u,
                              void *stream);

/* The Rotne-Prager-Yamakawa mobility of n spheres in unbounded fluid (the
 * approximation the abstract and section 1 name), in the form of Zuk,
 * Wajnryb, Mizerski and Szymczak (J. Fluid Mech. 2014) for unequal radii a_i,
 * a_j at centre distance r:
 *   r > a_i + a_j:   (1/(8 pi mu r)) [(1 + (a_i^2 + a_j^2)/(3 r^2)) I
 *                                     + (1 - (a_i^2 + a_j^2)/r^2) rr/r^2],
 *   |a_i - a_j| < r <= a_i + a_j: the overlap form
 *     (1/(6 pi mu a_i a_j)) [(16 r^3 (a_i + a_j) - ((a_i - a_j)^2 + 3 r^2)^2)/(32 r^3) I
 *                            + 3 ((a_i - a_j)^2 - r^2)^2/(32 r^3) rr/r^2],
 *   r <= |a_i - a_j|: I / (6 pi mu max(a_i, a_j)),
 * with the self term I / (6 pi mu a_i). Rotations take the single-sphere
 * mobility I / (8 pi mu a_i^3) and do not couple between spheres, which keeps
 * Mob SPD. The pair sum is evaluated directly (O(n^2), FP64). */
typedef struct sc_rpy {
    int32_t n;              /* number of spheres */
    int32_t reserved;
    const double *pos;      /* [n][3] device: centres */
    const double *radius;   /* [n] device: hydrodynamic radii > 0 (may differ from the
                               collision radii of sc_particles) */
    double mu;              /* viscosity > 0 */
    void *work;             /* device, 256-byte aligned, >= sc_rpy_work_bytes(n) bytes */
    size_t work_bytes;
} sc_rpy;

/* Device bytes of sc_rpy.work for n spheres. */
size_t sc_rpy_work_bytes(int32_t n);

/* sc_mobility_fn for ctx = const sc_rpy *: u = Mob f. n must equal ctx->n.
 * Enqueues only. Returns SC_OK, SC_ERR_INVALID (n mismatch, NULL pointer,
 * mu <= 0), SC_ERR_WORKSPACE or SC_ERR_HIP. Calls that overlap on one
 * stream's work buffer race. */
int sc_rpy_apply(void *ctx, int32_t n, const double *f, double *u, void *stream);

/* sc_mobility_fn for ctx = const sc_particles *: the dry block-diagonal
 * mobility of sc_apply_mobility. */
int sc_dry_apply(void *ctx, int32_t n, const double *f, double *u, void *stream);

/* The centre gradient of a mobility: enqueue g[k] = d/dc_k (a^T Mob(c) f)
 * for device arrays a, f of [n][6] (caller order) into g of [n][3]. Used by
 * the adjoint behind a mobility that depends on the centres; returns SC_OK
 * or an error code. */
typedef int (*sc_mobility_grad_fn)(void *ctx, int32_t n, const double *a, const double *f,
                                   double *g, void *stream);

/* sc_mobility_grad_fn for ctx = const sc_rpy *: the gradient of the RPY
 * translational couplings (from the r-derivatives of each branch's
 * coefficient functions; rotations and self terms do not depend on the
 * centres). Uses ctx->work like sc_rpy_apply (calls on one work buffer must
 * not overlap). Enqueues only. */
int sc_rpy_grad(void *ctx, int32_t n, const double *a, const double *f, double *g,
                void *stream);

/* Device bytes of the workspace of sc_solve_lcp_mob. */
size_t sc_solve_mob_work_bytes(int32_t n, int32_t capacity);

/* Algorithm 1 (section 3.3.1) as sc_solve_lcp computes it, with every
 * product M x = D^T Mob D x taking Mob from `mob(mob_ctx, ...)`: gamma_0,
 * g_0 = M gamma_0 + q, alpha_0 = g0^T g0 / g0^T M g0 (if that denominator is
 * <= 0: 1 / max_l of D_l^T Mob_self D_l from the particles' own `mob`
 * blocks), then projected BB steps until ||min(gamma, g)||_2 < opts->tol
 * (Eq. mmapnorm) or opts->max_iter steps. Uses opts->tol, max_iter, bb and
 * warm_start; the launch-shape fields are ignored. c: contacts from
 * sc_build_contacts (the plan is used; M need not be assembled).
 * The iterations are enqueued in chunks of `check_every` (0 = 4) and the
 * host reads the stop decision one chunk behind, so up to about two chunks
 * of mobility calls run after the decision to stop (their results are
 * ignored, and they are not counted in mvops). gamma, g: [c->count] device,
 * OUT (gamma holds gamma_0 on entry if warm_start). f_c, u_c: [n][6] device
 * or NULL: D gamma and Mob D gamma of the result. st: host, OUT (kernel_ms:
 * GPU time from the first product to the stop decision; op =
 * SC_OP_CALLBACK). work: device, 256-byte aligned, >=
 * sc_solve_mob_work_bytes(n, c->capacity). Returns SC_OK, SC_NOT_CONVERGED,
 * SC_ERR_NONFINITE, SC_ERR_INVALID, SC_ERR_WORKSPACE, SC_ERR_HIP or the
 * mobility's own error code. Synchronises `stream` before returning. */
int sc_solve_lcp_mob(const sc_particles *p, const sc_contacts *c, const sc_solve_opts *opts,
                     sc_mobility_fn mob, void *mob_ctx, int32_t check_every, double *gamma,
                     double *g, double *f_c, double *u_c, sc_stats *st, void *work,
                     size_t work_bytes, void *stream);

/* Device bytes of the workspace of sc_solve_lcp_rpy. */
size_t sc_solve_rpy_work_bytes(int32_t n, int32_t capacity);

/* Algorithm 1 with the RPY mobility of `rpy` (same arithmetic definition as
 * sc_solve_lcp_mob with sc_rpy_apply) in one persistent cooperative launch
 * (one 1024-thread workgroup per CU, two grid barriers per iteration:
 * after the RPY pair sum, whose work units form F = D gamma of their
 * sources from the previous iterate, and after g = D^T U + q and its
 * partial sums). For systems small enough that the
 * launches of the function-based solve dominate (measured faster for cold
 * solves up to about 2000 spheres, slower beyond). Sums run in fixed orders:
 * a given grid gives bitwise repeatable iterates, which differ from
 * sc_solve_lcp_mob's by rounding only. Uses opts->tol, max_iter,
 * bb, warm_start, grid (0 = one workgroup per CU) and spin_limit (as
 * sc_solve_lcp: a grid barrier that times out ends the solve with
 * SC_ERR_TIMEOUT). rpy->work holds the pair sums' split partials. gamma, g,
 * f_c, u_c, st as sc_solve_lcp_mob (st->op = SC_OP_RPY; mvops counts only
 * the products evaluated). work: device, 256-byte aligned, >=
 * sc_solve_rpy_work_bytes(n, c->capacity). Returns SC_OK, SC_NOT_CONVERGED,
 * SC_ERR_NONFINITE, SC_ERR_TIMEOUT, SC_ERR_INVALID, SC_ERR_WORKSPACE or
 * SC_ERR_HIP. Synchronises `stream`. */
int sc_solve_lcp_rpy(const sc_particles *p, const sc_contacts *c, const sc_rpy *rpy,
                     const sc_solve_opts *opts, double *gamma, double *g, double *f_c,
                     double *u_c, sc_stats *st, void *work, size_t work_bytes, void *stream);

/* Device bytes of the workspace of sc_solve_lcp_adjoint_mob. */
size_t sc_adjoint_mob_work_bytes(int32_t n, int32_t capacity);

/* Implicit adjoint of a converged solve behind a general mobility (not in the
 * paper; sc_solve_lcp_adjoint's derivation, which holds for any symmetric
 * mobility, plus the mobility's own dependence on the centres). With A =
 * {gamma > 0} and b = dL/dgamma + D^T dL/dF_c: M_AA w_A = b_A by conjugate
 * gradients with every product through `mob` (to ||r|| <= opts->tol ||b_A||
 * or opts->max_iter iterations, enqueued in chunks of `check_every` (0 = 4)
 * like sc_solve_lcp_mob); dL/dq = -w on A, 0 elsewhere; dL/dc = the
 * per-contact geometric terms of sc_solve_lcp_adjoint with V_w = Mob D w and
 * U = u_nc + Mob D gamma, minus d/dc [(D w)^T Mob(c) (D gamma + f_ext)] from
 * `mob_grad` (NULL: the mobility does not depend on the centres, f_ext may
 * be NULL). u_nc, f_ext: [n][6] device, u_nc = Mob f_ext at these centres.
 * gamma, dL_dgamma: [c->count]; dL_df: [n][6] or NULL; dL_dq: [c->count];
 * dL_dpos: [n][3]; all device. st: host, OUT (mvops = CG iterations; the
 * two products for V_w and U_c are extra). work: device, 256-byte aligned,
 * >= sc_adjoint_mob_work_bytes(n, c->capacity). Returns SC_OK,
 * SC_NOT_CONVERGED, SC_ERR_NONFINITE, SC_ERR_INVALID, SC_ERR_WORKSPACE,
 * SC_ERR_HIP or a mobility function's error code. Synchronises `stream`. */
int sc_solve_lcp_adjoint_mob(const sc_particles *p, const sc_box *box, const sc_contacts *c,
                             const double *u_nc, const double *f_ext, double dt,
                             const double *gamma, const double *dL_dgamma, const double *dL_df,
                             sc_mobility_fn mob, void *mob_ctx, sc_mobility_grad_fn mob_grad,
                             void *mob_grad_ctx, const sc_adjoint_opts *opts,
                             int32_t check_every, double *dL_dq, double *dL_dpos, sc_stats *st,
                             void *work, size_t work_bytes, void *stream);

/* Releases the host-side resources the calling thread's earlier calls keep
 * for reuse (the HIP events that time sc_solve_lcp, the pinned host slots
 * of the general-mobility solves), after waiting for the current device to
 * finish its work. Later calls create them again, so it may be called at any
 * time; a program calls it before it exits so that nothing of the library
 * is left for the HIP runtime's own teardown. Batches are released by
 * sc_batch_destroy. Returns SC_OK or SC_ERR_HIP. */
int sc_release(void);

/* Static string describing a return code. */
const char *sc_strerror(int code);

/* Library ABI version (major * 100 + minor). */
int sc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SC_API_H */
