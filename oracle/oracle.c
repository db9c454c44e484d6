/*
 * oracle.c -- plain, serial, FP64 reference implementation of the collision
 * resolution path of Yan, Corona, Malhotra, Veerapaneni and Shelley, "A
 * scalable computational platform for particulate Stokes suspensions"
 * (arXiv:1909.06623): close-pair detection, the contact Jacobian D, the LCP
 * data q, the matrix-free product M gamma = D^T Mob D gamma, the
 * Barzilai-Borwein projected gradient descent of Algorithm 1, and the
 * per-contact geometric derivatives used by the implicit adjoint.
 *
 * TEST INFRASTRUCTURE. This library is the parity checker. Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it;
 * the product path never calls it and shares no code, header or table with
 * it. Everything here is written for a reader checking it against the paper:
 * plain loops, serial sums in index order, no blocking, no fusion.
 *
 * Conventions (all arrays row-major, particle-major):
 *   pos[n][3] centres; axis[n][3] unit axis p; radius[n]; half_len[n]
 *   (0 for a sphere); mob[n][4] = (a_par, a_perp, b_par, b_perp), the dry
 *   per-particle mobility block diag(A, B) with A = a_par pp^T + a_perp
 *   (I - pp^T) and B likewise; 6-vectors per particle are (Ux,Uy,Uz,Wx,Wy,Wz).
 *   Contact l joins particles i < j; nrm[l][3] points from i to j.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no FMA
 * contraction, so every product and sum is rounded exactly as written).
 *
 * Threads. orc_set_threads(T) (default 1) lets the close-pair search and
 * the BBPGD loop use T OpenMP threads, for timing the oracle on all host
 * cores. With T = 1 every function computes exactly what the serial loops
 * below compute. With T > 1 the close pairs are searched per particle in T
 * contiguous ranges of i and concatenated in range order (the same list),
 * D gamma is gathered per particle over its contacts in increasing contact
 * order (the same sums as the contact-order scatter), the per-particle and
 * per-contact steps are independent, and only the sums over contacts are
 * formed as T partial sums over contiguous ranges, added in range order.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* threads                                                             */
/* ------------------------------------------------------------------ */
#define ORC_MAX_THREADS 256
static int g_threads = 1;

void orc_set_threads(int t)
{
    g_threads = t < 1 ? 1 : (t > ORC_MAX_THREADS ? ORC_MAX_THREADS : t);
}

int orc_get_threads(void)
{
    return g_threads;
}

/* Range [lo, hi) of `total` items taken by thread t of T. */
static void thread_range(long total, int t, int T, long *lo, long *hi)
{
    *lo = total * t / T;
    *hi = total * (t + 1) / T;
}

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double clampd(double x, double lo, double hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

/* ------------------------------------------------------------------ */
/* Geometry: minimum separation Phi of a pair (section 3.1: Phi_l is    */
/* the minimal separation distance of the pair, >= 0 without overlap). */
/* Shapes: a sphere is a point core of radius R; a spherocylinder is    */
/* the segment c + s p, |s| <= h, swept by radius R.                    */
/* ------------------------------------------------------------------ */

/* Minimum-image displacement r = c_j - c_i in a periodic box of sides L. */
static void min_image(const double *ci, const double *cj, const double *L,
                      int periodic, double *r)
{
    for (int k = 0; k < 3; ++k) {
        double d = cj[k] - ci[k];
        if (periodic)
            d = d - L[k] * nearbyint(d / L[k]);
        r[k] = d;
    }
}

/* Closest points between core i (parameter s) and core j (parameter t)
 * given r = c_j - c_i. Returns 1 if the parallel-segment rule was used.
 * The minimised quantity is |r + t p_j - s p_i|^2. */
static int closest_params(const double *r, const double *pi, double hi,
                          const double *pj, double hj, double *s_out,
                          double *t_out)
{
    double s = 0.0, t = 0.0;
    int parallel = 0;
    if (hi == 0.0 && hj == 0.0) {
        /* sphere-sphere: both cores are points */
    } else if (hi == 0.0) {
        /* sphere i against rod j: nearest point of segment j to c_i */
        t = clampd(-dot3(pj, r), -hj, hj);
    } else if (hj == 0.0) {
        /* rod i against sphere j: nearest point of segment i to c_j */
        s = clampd(dot3(pi, r), -hi, hi);
    } else {
        double b = dot3(pi, pj);
        double c = dot3(pi, r);
        double f = dot3(pj, r);
        double x[3];
        cross3(pi, pj, x);
        double den = dot3(x, x); /* = 1 - b^2 for unit axes */
        if (den < 1e-12) {
            /* (Near-)parallel cores: the closest points are not unique.
             * Take the midpoint of the overlap of the two segments'
             * projections on p_i; without overlap, the end of i nearest to
             * j's projection. */
            double ab = fabs(b);
            double lo = fmax(-hi, c - hj * ab);
            double hi2 = fmin(hi, c + hj * ab);
            double s0;
            if (lo <= hi2)
                s0 = 0.5 * (lo + hi2);
            else
                s0 = (c > 0.0) ? hi : -hi;
            t = clampd(b * s0 - f, -hj, hj);
            s = clampd(c + b * t, -hi, hi);
            parallel = 1;
        } else {
            /* stationary point of the quadratic: s = c + b t, t = b s - f */
            s = clampd((c - b * f) / (1.0 - b * b), -hi, hi);
            t = b * s - f;
            if (t < -hj) {
                t = -hj;
                s = clampd(c + b * t, -hi, hi);
            } else if (t > hj) {
                t = hj;
                s = clampd(c + b * t, -hi, hi);
            }
        }
    }
    *s_out = s;
    *t_out = t;
    return parallel;
}

/* Full pair geometry. out[12] = phi, n[3], s, t, tau_i[3], tau_j[3] with
 * tau_i = (x_i - c_i) x n = (s p_i) x n and tau_j = (t p_j) x n (the radial
 * part of the contact point drops out of the moment because n x n = 0).
 * Return value: bit 0 = parallel rule used, bit 1 = zero core distance
 * (n set to +e_x). */
static int pair_geometry(const double *ci, const double *pi, double Ri,
                         double hi, const double *cj, const double *pj,
                         double Rj, double hj, const double *L, int periodic,
                         double *out)
{
    double r[3], s, t, d[3], n[3];
    min_image(ci, cj, L, periodic, r);
    int flags = closest_params(r, pi, hi, pj, hj, &s, &t);
    for (int k = 0; k < 3; ++k)
        d[k] = r[k] + t * pj[k] - s * pi[k];
    double dist = sqrt(dot3(d, d));
    if (dist > 0.0) {
        for (int k = 0; k < 3; ++k)
            n[k] = d[k] / dist;
    } else {
        n[0] = 1.0; n[1] = 0.0; n[2] = 0.0;
        flags |= 2;
    }
    out[0] = dist - Ri - Rj;
    out[1] = n[0]; out[2] = n[1]; out[3] = n[2];
    out[4] = s; out[5] = t;
    double sp[3] = {s * pi[0], s * pi[1], s * pi[2]};
    double tp[3] = {t * pj[0], t * pj[1], t * pj[2]};
    cross3(sp, n, out + 6);
    cross3(tp, n, out + 9);
    return flags;
}

int orc_pair_geometry(const double *ci, const double *pi, double Ri, double hi,
                      const double *cj, const double *pj, double Rj, double hj,
                      const double *L, int periodic, double *out)
{
    return pair_geometry(ci, pi, Ri, hi, cj, pj, Rj, hj, L, periodic, out);
}

/* Particle-wall geometry (the boundary constraints of section 3.3's
 * extensions: a column of D with the 6 entries of the particle only). Face
 * f = 2a + side is the plane x_a = lo_a (side 0) or x_a = lo_a + L_a
 * (side 1) of a non-periodic box; its inward normal m is +e_a or -e_a. The
 * core point closest to the plane is c + s p with s = -h sign(m.p) (s = 0 if
 * the rod lies parallel to the plane, the midpoint reading), so
 * Phi = m.(c - x_face) - h |m.p| - R. The contact normal points from the
 * particle to the wall, n = -m, and tau_i = (s p) x n. Output as
 * pair_geometry's g with tau_j = 0; returns the parallel flag. */
static int wall_geometry(const double *c, const double *p, double R, double h,
                         const double *lo, const double *L, int face, double *g)
{
    int a = face / 2, up = face % 2;
    double sg = up ? -1.0 : 1.0;
    double d = up ? lo[a] + L[a] - c[a] : c[a] - lo[a];
    double mp = sg * p[a];
    double s = 0.0;
    int par = 0;
    if (h > 0.0) {
        if (fabs(mp) < 1e-12)
            par = 1;
        else
            s = mp > 0.0 ? -h : h;
    }
    double n[3] = {0.0, 0.0, 0.0};
    n[a] = -sg;
    double sp[3] = {s * p[0], s * p[1], s * p[2]}, ti[3];
    cross3(sp, n, ti);
    g[0] = d + s * mp - R;
    for (int b = 0; b < 3; ++b) {
        g[1 + b] = n[b];
        g[6 + b] = ti[b];
        g[9 + b] = 0.0;
    }
    g[4] = s;
    g[5] = 0.0;
    return par;
}

/* Wall contacts of particle i (faces in decreasing order, so that their
 * codes j = -1 - face come out increasing). */
static void push_walls(int i, const double *pos, const double *axis, const double *radius,
                       const double *half_len, const double *lo, const double *L, int walls,
                       double delta, void (*push)(void *, int, int, const double *, int),
                       void *k)
{
    double g[12];
    for (int f = 5; f >= 0; --f) {
        if (!(walls & (1 << f)))
            continue;
        int fl = wall_geometry(pos + 3 * i, axis + 3 * i, radius[i], half_len[i], lo, L, f, g);
        if (g[0] <= delta)
            push(k, i, -1 - f, g, fl);
    }
}

/* ------------------------------------------------------------------ */
/* Close-pair set A(C, delta) = { l : Phi_l <= delta } (section 3.2),   */
/* one constraint per pair i < j, in canonical order (by i, then j).    */
/* ------------------------------------------------------------------ */

typedef struct {
    long cap, count;
    int *ci, *cj;
    double *phi, *nrm, *tau_i, *tau_j, *st;
    long nflag_parallel, nflag_zero;
    int grow; /* 1: the arrays are the sink's own and grow on demand */
} contact_sink;

static void sink_reserve(contact_sink *k, long need)
{
    long cap = k->cap > 0 ? k->cap : 64;
    while (cap < need)
        cap *= 2;
    k->ci = realloc(k->ci, sizeof(int) * (size_t)cap);
    k->cj = realloc(k->cj, sizeof(int) * (size_t)cap);
    k->phi = realloc(k->phi, sizeof(double) * (size_t)cap);
    k->nrm = realloc(k->nrm, sizeof(double) * 3 * (size_t)cap);
    k->tau_i = realloc(k->tau_i, sizeof(double) * 3 * (size_t)cap);
    k->tau_j = realloc(k->tau_j, sizeof(double) * 3 * (size_t)cap);
    k->st = realloc(k->st, sizeof(double) * 2 * (size_t)cap);
    k->cap = cap;
}

static void sink_push(contact_sink *k, int i, int j, const double *g, int flags)
{
    long l = k->count++;
    if (flags & 1) k->nflag_parallel++;
    if (flags & 2) k->nflag_zero++;
    if (l >= k->cap && k->grow)
        sink_reserve(k, l + 1);
    if (l >= k->cap)
        return;
    k->ci[l] = i;
    k->cj[l] = j;
    k->phi[l] = g[0];
    for (int a = 0; a < 3; ++a) {
        k->nrm[3 * l + a] = g[1 + a];
        k->tau_i[3 * l + a] = g[6 + a];
        k->tau_j[3 * l + a] = g[9 + a];
    }
    k->st[2 * l] = g[4];
    k->st[2 * l + 1] = g[5];
}

static void sink_push_v(void *k, int i, int j, const double *g, int flags)
{
    sink_push((contact_sink *)k, i, j, g, flags);
}

/* O(N^2) enumeration of every pair i < j (each particle's wall contacts
 * first). */
static void contacts_brute(int n, const double *pos, const double *axis,
                           const double *radius, const double *half_len,
                           const double *lo, const double *L, int periodic, int walls,
                           double delta, contact_sink *k)
{
    double g[12];
    for (int i = 0; i < n; ++i) {
        push_walls(i, pos, axis, radius, half_len, lo, L, walls, delta, sink_push_v, k);
        for (int j = i + 1; j < n; ++j) {
            int fl = pair_geometry(pos + 3 * i, axis + 3 * i, radius[i],
                                   half_len[i], pos + 3 * j, axis + 3 * j,
                                   radius[j], half_len[j], L, periodic, g);
            if (g[0] <= delta)
                sink_push(k, i, j, g, fl);
        }
    }
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

typedef struct {
    const int *nc;
    const long *start;
    const int *members, *cell;
} cell_grid;

typedef struct {
    int cap_list;
    int *list;
} cell_scan;

/* The close pairs (i, j > i) of particle i from the distinct neighbour
 * cells of its own cell (and i's wall contacts first), in increasing j. */
static void cell_pairs_of(int i, const cell_grid *grid, cell_scan *scan, const double *pos,
                          const double *axis, const double *radius, const double *half_len,
                          const double *lo, const double *L, int periodic, int walls,
                          double delta, contact_sink *k)
{
    const int *nc = grid->nc, *cell = grid->cell, *members = grid->members;
    const long *start = grid->start;
    double g[12];
    int cx = cell[i] % nc[0];
    int cy = (cell[i] / nc[0]) % nc[1];
    int cz = cell[i] / (nc[0] * nc[1]);
    /* distinct neighbour cells along each axis */
    int off[3][3], noff[3];
    int cidx[3] = {cx, cy, cz};
    for (int a = 0; a < 3; ++a) {
        noff[a] = 0;
        for (int d = -1; d <= 1; ++d) {
            int c = cidx[a] + d;
            if (periodic) {
                c = (c + nc[a]) % nc[a];
            } else if (c < 0 || c >= nc[a]) {
                continue;
            }
            int dup = 0;
            for (int e = 0; e < noff[a]; ++e)
                if (off[a][e] == c) dup = 1;
            if (!dup) off[a][noff[a]++] = c;
        }
    }
    int cnt = 0;
    for (int az = 0; az < noff[2]; ++az)
        for (int ay = 0; ay < noff[1]; ++ay)
            for (int ax = 0; ax < noff[0]; ++ax) {
                long c = ((long)off[2][az] * nc[1] + off[1][ay]) * nc[0] + off[0][ax];
                for (long m = start[c]; m < start[c + 1]; ++m) {
                    int j = members[m];
                    if (j <= i) continue;
                    if (cnt == scan->cap_list) {
                        scan->cap_list *= 2;
                        scan->list = realloc(scan->list, sizeof(int) * (size_t)scan->cap_list);
                    }
                    scan->list[cnt++] = j;
                }
            }
    qsort(scan->list, (size_t)cnt, sizeof(int), cmp_int);
    push_walls(i, pos, axis, radius, half_len, lo, L, walls, delta, sink_push_v, k);
    for (int m = 0; m < cnt; ++m) {
        int j = scan->list[m];
        int fl = pair_geometry(pos + 3 * i, axis + 3 * i, radius[i],
                               half_len[i], pos + 3 * j, axis + 3 * j,
                               radius[j], half_len[j], L, periodic, g);
        if (g[0] <= delta)
            sink_push(k, i, j, g, fl);
    }
}

/* Cell list (section 5.2 names cell lists as a standard near-neighbour
 * method): cells of side >= the interaction range, each particle checks the
 * distinct neighbour cells around its own; pairs are emitted per i in
 * increasing j. Non-periodic boxes clamp cell indices into the grid, which
 * keeps nearby particles in the same or adjacent cells. */
static void contacts_cells(int n, const double *pos, const double *axis,
                           const double *radius, const double *half_len,
                           const double *lo, const double *L, int periodic, int walls,
                           double delta, contact_sink *k)
{
    double rmax = 0.0;
    for (int i = 0; i < n; ++i) {
        double e = radius[i] + half_len[i];
        if (e > rmax) rmax = e;
    }
    rmax = 2.0 * rmax + delta;
    int nc[3];
    long ncell = 1;
    for (int a = 0; a < 3; ++a) {
        int m = (int)floor(L[a] / rmax);
        if (m < 1) m = 1;
        if (m > 1024) m = 1024;
        nc[a] = m;
        ncell *= m;
    }
    double side[3] = {L[0] / nc[0], L[1] / nc[1], L[2] / nc[2]};
    int *cell = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    long *start = calloc((size_t)ncell + 1, sizeof(long));
    int *members = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        int cc[3];
        for (int a = 0; a < 3; ++a) {
            double x = pos[3 * i + a] - lo[a];
            if (periodic)
                x = x - L[a] * floor(x / L[a]);
            int c = (int)floor(x / side[a]);
            if (c < 0) c = 0;
            if (c >= nc[a]) c = nc[a] - 1;
            cc[a] = c;
        }
        cell[i] = (cc[2] * nc[1] + cc[1]) * nc[0] + cc[0];
        start[cell[i] + 1]++;
    }
    for (long c = 0; c < ncell; ++c)
        start[c + 1] += start[c];
    long *fill = malloc(sizeof(long) * (size_t)ncell);
    memcpy(fill, start, sizeof(long) * (size_t)ncell);
    for (int i = 0; i < n; ++i)
        members[fill[cell[i]]++] = i;
    free(fill);

    cell_grid grid = {nc, start, members, cell};
    int T = g_threads;
    if (T == 1) {
        cell_scan scan = {64, malloc(sizeof(int) * 64)};
        for (int i = 0; i < n; ++i)
            cell_pairs_of(i, &grid, &scan, pos, axis, radius, half_len, lo, L, periodic,
                          walls, delta, k);
        free(scan.list);
    } else {
        /* T contiguous ranges of i, each into a sink of its own, then
         * concatenated in range order: the same list as the loop above */
        contact_sink part[ORC_MAX_THREADS];
        memset(part, 0, sizeof(part));
#pragma omp parallel num_threads(T)
        {
            int t = omp_get_thread_num(), nt = omp_get_num_threads();
#pragma omp single
            T = nt;
            long i0, i1;
            thread_range(n, t, nt, &i0, &i1);
            contact_sink *mine = &part[t];
            mine->grow = 1;
            cell_scan scan = {64, malloc(sizeof(int) * 64)};
            for (long i = i0; i < i1; ++i)
                cell_pairs_of((int)i, &grid, &scan, pos, axis, radius, half_len, lo, L,
                              periodic, walls, delta, mine);
            free(scan.list);
        }
        for (int t = 0; t < T; ++t) {
            contact_sink *p = &part[t];
            for (long l = 0; l < p->count; ++l) {
                long d = k->count++;
                if (d >= k->cap)
                    continue;
                k->ci[d] = p->ci[l];
                k->cj[d] = p->cj[l];
                k->phi[d] = p->phi[l];
                memcpy(k->nrm + 3 * d, p->nrm + 3 * l, 3 * sizeof(double));
                memcpy(k->tau_i + 3 * d, p->tau_i + 3 * l, 3 * sizeof(double));
                memcpy(k->tau_j + 3 * d, p->tau_j + 3 * l, 3 * sizeof(double));
                memcpy(k->st + 2 * d, p->st + 2 * l, 2 * sizeof(double));
            }
            k->nflag_parallel += p->nflag_parallel;
            k->nflag_zero += p->nflag_zero;
            free(p->ci);
            free(p->cj);
            free(p->phi);
            free(p->nrm);
            free(p->tau_i);
            free(p->tau_j);
            free(p->st);
        }
    }
    free(cell);
    free(start);
    free(members);
}

/* method 0 = brute force, 1 = cell list. walls: bit f set = wall on face f
 * (non-periodic boxes only). Writes min(count, cap) contacts and returns the
 * full count; a wall contact has j = -1 - face. flags_out[2] =
 * (#parallel-rule pairs, #zero-distance pairs) among the emitted contacts. */
long orc_find_contacts(int method, int n, const double *pos,
                       const double *axis, const double *radius,
                       const double *half_len, const double *lo,
                       const double *L, int periodic, int walls, double delta, long cap,
                       int *ci, int *cj, double *phi, double *nrm,
                       double *tau_i, double *tau_j, double *st,
                       long *flags_out)
{
    contact_sink k = {cap, 0, ci, cj, phi, nrm, tau_i, tau_j, st, 0, 0, 0};
    if (periodic)
        walls = 0;
    if (method == 0)
        contacts_brute(n, pos, axis, radius, half_len, lo, L, periodic, walls, delta, &k);
    else
        contacts_cells(n, pos, axis, radius, half_len, lo, L, periodic, walls,
                       delta, &k);
    if (flags_out) {
        flags_out[0] = k.nflag_parallel;
        flags_out[1] = k.nflag_zero;
    }
    return k.count;
}

/* ------------------------------------------------------------------ */
/* Mobility, D and D^T (Eqs. Dmatdef and Dtranspose; LCP LCPdef).       */
/* Column l of D puts (-n, -tau_i) on particle i and (+n, +tau_j) on    */
/* particle j, so that D_l^T U = dPhi_l/dt for rigid velocities U. A    */
/* wall contact (j < 0) has the particle's 6 entries only.              */
/* ------------------------------------------------------------------ */

/* U = Mob F, per particle. */
void orc_mobility(int n, const double *axis, const double *mob,
                  const double *F, double *U)
{
    for (int k = 0; k < n; ++k) {
        const double *p = axis + 3 * k;
        const double *f = F + 6 * k;
        double *u = U + 6 * k;
        double pf = dot3(p, f);
        double pt = dot3(p, f + 3);
        for (int a = 0; a < 3; ++a) {
            u[a] = mob[4 * k + 1] * f[a] + (mob[4 * k + 0] - mob[4 * k + 1]) * pf * p[a];
            u[3 + a] = mob[4 * k + 3] * f[3 + a] + (mob[4 * k + 2] - mob[4 * k + 3]) * pt * p[a];
        }
    }
}

/* F = D gamma: accumulate each column in contact order. */
void orc_D_apply(int n, long nc, const int *ci, const int *cj,
                 const double *nrm, const double *tau_i, const double *tau_j,
                 const double *gamma, double *F)
{
    memset(F, 0, sizeof(double) * 6 * (size_t)n);
    for (long l = 0; l < nc; ++l) {
        double *fi = F + 6 * (size_t)ci[l];
        for (int a = 0; a < 3; ++a) {
            fi[a] -= nrm[3 * l + a] * gamma[l];
            fi[3 + a] -= tau_i[3 * l + a] * gamma[l];
        }
        if (cj[l] < 0)
            continue;
        double *fj = F + 6 * (size_t)cj[l];
        for (int a = 0; a < 3; ++a) {
            fj[a] += nrm[3 * l + a] * gamma[l];
            fj[3 + a] += tau_j[3 * l + a] * gamma[l];
        }
    }
}

/* out_l = D_l^T U. */
void orc_DT_apply(long nc, const int *ci, const int *cj, const double *nrm,
                  const double *tau_i, const double *tau_j, const double *U,
                  double *out)
{
    for (long l = 0; l < nc; ++l) {
        const double *ui = U + 6 * (size_t)ci[l];
        const double *nn = nrm + 3 * l;
        double v = -dot3(nn, ui) - dot3(tau_i + 3 * l, ui + 3);
        if (cj[l] >= 0) {
            const double *uj = U + 6 * (size_t)cj[l];
            v = v + dot3(nn, uj) + dot3(tau_j + 3 * l, uj + 3);
        }
        out[l] = v;
    }
}

/* q = Phi/dt + D^T U_nc (LCP LCPdef, scaled by 1/dt). */
void orc_build_q(long nc, const int *ci, const int *cj, const double *phi,
                 const double *nrm, const double *tau_i, const double *tau_j,
                 const double *u_nc, double dt, double *q)
{
    orc_DT_apply(nc, ci, cj, nrm, tau_i, tau_j, u_nc, q);
    for (long l = 0; l < nc; ++l)
        q[l] = phi[l] / dt + q[l];
}

typedef struct {
    int n;
    long nc;
    const int *ci, *cj;
    const double *nrm, *tau_i, *tau_j, *axis, *mob;
    double *F, *U; /* scratch [n][6] */
    long *inc_ptr, *inc; /* T > 1: contacts of each particle, 2 l + side (0: i, 1: j) */
} mvop_ctx;

/* For T > 1 threads: each particle's contacts in increasing contact order. */
static void mvop_incidence(mvop_ctx *c)
{
    c->inc_ptr = calloc((size_t)c->n + 1, sizeof(long));
    c->inc = malloc(sizeof(long) * 2 * (size_t)(c->nc > 0 ? c->nc : 1));
    for (long l = 0; l < c->nc; ++l) {
        c->inc_ptr[c->ci[l] + 1]++;
        if (c->cj[l] >= 0) c->inc_ptr[c->cj[l] + 1]++;
    }
    for (int k = 0; k < c->n; ++k)
        c->inc_ptr[k + 1] += c->inc_ptr[k];
    long *fill = malloc(sizeof(long) * (size_t)(c->n > 0 ? c->n : 1));
    memcpy(fill, c->inc_ptr, sizeof(long) * (size_t)c->n);
    for (long l = 0; l < c->nc; ++l) {
        c->inc[fill[c->ci[l]]++] = 2 * l;
        if (c->cj[l] >= 0) c->inc[fill[c->cj[l]]++] = 2 * l + 1;
    }
    free(fill);
}

/* F = D x gathered per particle: the same operations, in the same order per
 * particle, as orc_D_apply's scatter in contact order. */
static void d_apply_gather(const mvop_ctx *c, const double *x, double *F)
{
#pragma omp parallel for if (g_threads > 1) num_threads(g_threads) schedule(static)
    for (int k = 0; k < c->n; ++k) {
        double f[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (long e = c->inc_ptr[k]; e < c->inc_ptr[k + 1]; ++e) {
            long l = c->inc[e] / 2;
            if (c->inc[e] % 2 == 0) {
                for (int a = 0; a < 3; ++a) {
                    f[a] -= c->nrm[3 * l + a] * x[l];
                    f[3 + a] -= c->tau_i[3 * l + a] * x[l];
                }
            } else {
                for (int a = 0; a < 3; ++a) {
                    f[a] += c->nrm[3 * l + a] * x[l];
                    f[3 + a] += c->tau_j[3 * l + a] * x[l];
                }
            }
        }
        memcpy(F + 6 * (size_t)k, f, sizeof(f));
    }
}

/* out = M x = D^T Mob D x (one "MVOP" in the paper's accounting). */
static void mvop(mvop_ctx *c, const double *x, double *out)
{
    if (g_threads == 1) {
        orc_D_apply(c->n, c->nc, c->ci, c->cj, c->nrm, c->tau_i, c->tau_j, x, c->F);
        orc_mobility(c->n, c->axis, c->mob, c->F, c->U);
        orc_DT_apply(c->nc, c->ci, c->cj, c->nrm, c->tau_i, c->tau_j, c->U, out);
        return;
    }
    d_apply_gather(c, x, c->F);
#pragma omp parallel for if (g_threads > 1) num_threads(g_threads) schedule(static)
    for (int k = 0; k < c->n; ++k)
        orc_mobility(1, c->axis + 3 * k, c->mob + 4 * k, c->F + 6 * k, c->U + 6 * k);
    long T = g_threads;
#pragma omp parallel for if (g_threads > 1) num_threads(g_threads) schedule(static)
    for (long t = 0; t < T; ++t) {
        long l0, l1;
        thread_range(c->nc, (int)t, (int)T, &l0, &l1);
        orc_DT_apply(l1 - l0, c->ci + l0, c->cj + l0, c->nrm + 3 * l0, c->tau_i + 3 * l0,
                     c->tau_j + 3 * l0, c->U, out + l0);
    }
}

void orc_mvop(int n, long nc, const int *ci, const int *cj, const double *nrm,
              const double *tau_i, const double *tau_j, const double *axis,
              const double *mob, const double *x, double *out)
{
    mvop_ctx c = {n, nc, ci, cj, nrm, tau_i, tau_j, axis, mob,
                  malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1)),
                  malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1)), NULL, NULL};
    if (g_threads > 1)
        mvop_incidence(&c);
    mvop(&c, x, out);
    free(c.F);
    free(c.U);
    free(c.inc_ptr);
    free(c.inc);
}

/* Diagonal of M: M_ll = D_l^T Mob D_l. */
void orc_M_diag(long nc, const int *ci, const int *cj, const double *nrm,
                const double *tau_i, const double *tau_j, const double *axis,
                const double *mob, double *diag)
{
    for (long l = 0; l < nc; ++l) {
        double acc = 0.0;
        for (int side = 0; side < 2; ++side) {
            int k = side ? cj[l] : ci[l];
            if (k < 0)
                continue;
            const double *tau = side ? tau_j + 3 * l : tau_i + 3 * l;
            double f[6], u[6];
            for (int a = 0; a < 3; ++a) {
                f[a] = nrm[3 * l + a];
                f[3 + a] = tau[a];
            }
            orc_mobility(1, axis + 3 * k, mob + 4 * k, f, u);
            acc += dot3(f, u) + dot3(f + 3, u + 3);
        }
        diag[l] = acc;
    }
}

/* ------------------------------------------------------------------ */
/* BBPGD, Algorithm 1 of section 3.3.1, with phi(gamma, g) =           */
/* ||min(gamma, g)||_2 (Eq. mmapnorm) as the absolute stopping test.    */
/* ------------------------------------------------------------------ */

/* The sums over contacts of the solver, sums[0..2] over l of
 *   what 0: min(a_l, b_l)^2 (and nothing else)
 *   what 1: a_l a_l, a_l b_l
 *   what 2: s_l s_l, s_l y_l, y_l y_l with s = a - c, y = b - d
 * as T partial sums over contiguous ranges of l added in range order (one
 * range, the plain left-to-right sum, when T = 1). */
static void contact_sums(int what, long nc, const double *a, const double *b,
                         const double *c, const double *d, double *sums)
{
    double part[ORC_MAX_THREADS][3];
    int T = g_threads;
#pragma omp parallel if (T > 1) num_threads(T)
    {
        int t = omp_get_thread_num(), nt = omp_get_num_threads();
#pragma omp single
        T = nt;
        long l0, l1;
        thread_range(nc, t, nt, &l0, &l1);
        double x0 = 0.0, x1 = 0.0, x2 = 0.0;
        for (long l = l0; l < l1; ++l) {
            if (what == 0) {
                double m = a[l] < b[l] ? a[l] : b[l];
                x0 += m * m;
            } else if (what == 1) {
                x0 += a[l] * a[l];
                x1 += a[l] * b[l];
            } else {
                double s = a[l] - c[l];
                double y = b[l] - d[l];
                x0 += s * s;
                x1 += s * y;
                x2 += y * y;
            }
        }
        part[t][0] = x0;
        part[t][1] = x1;
        part[t][2] = x2;
    }
    for (int k = 0; k < 3; ++k) {
        double acc = part[0][k];
        for (int t = 1; t < T; ++t)
            acc += part[t][k];
        sums[k] = acc;
    }
}

static double residual(long nc, const double *gamma, const double *g)
{
    double sums[3];
    contact_sums(0, nc, gamma, g, NULL, NULL, sums);
    return sqrt(sums[0]);
}

/* bb: 1 = BB1 every step, 2 = BB2 every step, 3 = BB1 on odd j and BB2 on
 * even j. gamma holds gamma_0 on entry (zero unless warm-started) and the
 * result on exit; g receives M gamma + q. stats[8] = (status, iterations,
 * MVOPs, residual, #active, #degenerate step sizes, alpha_last, 0) with
 * status 0 = converged, 1 = not converged within max_iter, 3 = non-finite.
 * A non-positive or non-finite BB denominator keeps the previous step size;
 * a non-positive g0^T M g0 uses 1/max_l M_ll. */
int orc_bbpgd(int n, long nc, const int *ci, const int *cj, const double *nrm,
              const double *tau_i, const double *tau_j, const double *axis,
              const double *mob, const double *q, double *gamma, double *g,
              double tol, int max_iter, int bb, double *stats)
{
    size_t sz = sizeof(double) * (size_t)(nc > 0 ? nc : 1);
    mvop_ctx c = {n, nc, ci, cj, nrm, tau_i, tau_j, axis, mob,
                  malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1)),
                  malloc(sizeof(double) * 6 * (size_t)(n > 0 ? n : 1)), NULL, NULL};
    if (g_threads > 1)
        mvop_incidence(&c);
    double *gamma_prev = malloc(sz), *g_prev = malloc(sz), *tmp = malloc(sz);
    int status = 0, iters = 0, mvops = 0;
    long ndegen = 0;
    double res, alpha = 0.0;

    /* g0 = M gamma0 + q */
    mvop(&c, gamma, g);
    mvops++;
#pragma omp parallel for if (g_threads > 1) num_threads(g_threads) schedule(static)
    for (long l = 0; l < nc; ++l)
        g[l] += q[l];
    res = residual(nc, gamma, g);
    if (!isfinite(res)) {
        status = 3;
        goto done;
    }
    /* gamma0 may already satisfy the tolerance */
    if (res < tol)
        goto done;
    /* initial step size alpha0 = g0^T g0 / g0^T M g0 */
    mvop(&c, g, tmp);
    mvops++;
    {
        double sums[3];
        contact_sums(1, nc, g, tmp, NULL, NULL, sums);
        double num = sums[0], den = sums[1];
        if (den > 0.0 && isfinite(den) && isfinite(num)) {
            alpha = num / den;
        } else {
            orc_M_diag(nc, ci, cj, nrm, tau_i, tau_j, axis, mob, tmp);
            double mx = 0.0;
            for (long l = 0; l < nc; ++l)
                if (tmp[l] > mx) mx = tmp[l];
            alpha = mx > 0.0 ? 1.0 / mx : 1.0;
            ndegen++;
        }
    }
    status = 1;
    for (int j = 1; j <= max_iter; ++j) {
        memcpy(gamma_prev, gamma, sz);
        memcpy(g_prev, g, sz);
        /* descent step, then projection onto gamma >= 0 */
#pragma omp parallel for if (g_threads > 1) num_threads(g_threads) schedule(static)
        for (long l = 0; l < nc; ++l) {
            double v = gamma_prev[l] - alpha * g_prev[l];
            gamma[l] = v < 0.0 ? 0.0 : v;
        }
        /* new gradient g = M gamma + q */
        mvop(&c, gamma, g);
        mvops++;
#pragma omp parallel for if (g_threads > 1) num_threads(g_threads) schedule(static)
        for (long l = 0; l < nc; ++l)
            g[l] += q[l];
        iters = j;
        res = residual(nc, gamma, g);
        if (!isfinite(res)) {
            status = 3;
            break;
        }
        /* stopping test */
        if (res < tol) {
            status = 0;
            break;
        }
        /* BB step size from s = gamma_j - gamma_{j-1}, y = g_j - g_{j-1} */
        double sums[3];
        contact_sums(2, nc, gamma, g, gamma_prev, g_prev, sums);
        double ss = sums[0], sy = sums[1], yy = sums[2];
        int use_bb2 = (bb == 2) || (bb == 3 && (j % 2 == 0));
        double num = use_bb2 ? sy : ss;
        double den = use_bb2 ? yy : sy;
        if (den > 0.0 && num > 0.0 && isfinite(num) && isfinite(den))
            alpha = num / den;
        else
            ndegen++;
    }
done:;
    long nact = 0;
    for (long l = 0; l < nc; ++l)
        if (gamma[l] > 0.0) nact++;
    stats[0] = status;
    stats[1] = iters;
    stats[2] = mvops;
    stats[3] = res;
    stats[4] = (double)nact;
    stats[5] = (double)ndegen;
    stats[6] = alpha;
    stats[7] = 0.0;
    free(gamma_prev);
    free(g_prev);
    free(tmp);
    free(c.F);
    free(c.U);
    free(c.inc_ptr);
    free(c.inc);
    return status;
}

/* ------------------------------------------------------------------ */
/* Geometric derivatives for the adjoint (not in the paper; derived by   */
/* differentiating the closest-point conditions of the pair geometry).   */
/* For contact l with weights E_i, E_j (6-vectors) and scalar c_phi,     */
/*   J(r) = D_l(r)^T [E_i; E_j] + c_phi * Phi_l(r)                       */
/*        = -n.E_i^F - tau_i.E_i^T + n.E_j^F + tau_j.E_j^T + c_phi Phi,  */
/* with r = c_j - c_i and orientations fixed. out[3] = dJ/dr; the        */
/* gradient is +dJ/dr on c_j and -dJ/dr on c_i.                           */
/* ------------------------------------------------------------------ */

static void matvecT(const double A[3][3], const double *v, double *out)
{ /* out = A^T v */
    for (int b = 0; b < 3; ++b)
        out[b] = A[0][b] * v[0] + A[1][b] * v[1] + A[2][b] * v[2];
}

void orc_contact_grad(const double *ci, const double *pi, double Ri, double hi,
                      const double *cj, const double *pj, double Rj, double hj,
                      const double *L, int periodic, const double *Ei,
                      const double *Ej, double c_phi, double *out)
{
    double r[3], s, t;
    (void)Ri; /* the radii shift Phi by a constant and drop out */
    (void)Rj;
    min_image(ci, cj, L, periodic, r);
    closest_params(r, pi, hi, pj, hj, &s, &t);
    /* which parameters sit strictly inside their segment */
    int s_free = (hi > 0.0) && (s > -hi) && (s < hi);
    int t_free = (hj > 0.0) && (t > -hj) && (t < hj);
    double b = dot3(pi, pj);
    double ds[3] = {0, 0, 0}, dt[3] = {0, 0, 0}; /* ds/dr, dt/dr */
    if (s_free && t_free) {
        double den = 1.0 - b * b;
        for (int a = 0; a < 3; ++a) {
            ds[a] = (pi[a] - b * pj[a]) / den;
            dt[a] = (b * pi[a] - pj[a]) / den;
        }
    } else if (t_free) {
        for (int a = 0; a < 3; ++a) dt[a] = -pj[a];
    } else if (s_free) {
        for (int a = 0; a < 3; ++a) ds[a] = pi[a];
    }
    double d[3], Jd[3][3]; /* d = r + t p_j - s p_i, Jd = dd/dr */
    for (int a = 0; a < 3; ++a) {
        d[a] = r[a] + t * pj[a] - s * pi[a];
        for (int bb = 0; bb < 3; ++bb)
            Jd[a][bb] = (a == bb ? 1.0 : 0.0) + pj[a] * dt[bb] - pi[a] * ds[bb];
    }
    double rho = sqrt(dot3(d, d));
    double n[3] = {d[0] / rho, d[1] / rho, d[2] / rho};
    double dphi[3], Jn[3][3];
    matvecT(Jd, n, dphi); /* dPhi/dr = n^T dd/dr */
    for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k)
                acc += ((a == k ? 1.0 : 0.0) - n[a] * n[k]) * Jd[k][bb];
            Jn[a][bb] = acc / rho;
        }
    /* tau_i = s (p_i x n): dtau_i/dr = (p_i x n) ds^T + s [p_i]x Jn */
    double pin[3], pjn[3];
    cross3(pi, n, pin);
    cross3(pj, n, pjn);
    double Jti[3][3], Jtj[3][3];
    for (int bb = 0; bb < 3; ++bb) {
        double col[3] = {Jn[0][bb], Jn[1][bb], Jn[2][bb]}, pc[3], qc[3];
        cross3(pi, col, pc);
        cross3(pj, col, qc);
        for (int a = 0; a < 3; ++a) {
            Jti[a][bb] = pin[a] * ds[bb] + s * pc[a];
            Jtj[a][bb] = pjn[a] * dt[bb] + t * qc[a];
        }
    }
    double dEF[3] = {Ej[0] - Ei[0], Ej[1] - Ei[1], Ej[2] - Ei[2]};
    double g1[3], g2[3], g3[3];
    matvecT(Jn, dEF, g1);
    matvecT(Jti, Ei + 3, g2);
    matvecT(Jtj, Ej + 3, g3);
    for (int a = 0; a < 3; ++a)
        out[a] = g1[a] - g2[a] + g3[a] + c_phi * dphi[a];
}

/* dL/dpos for the implicit adjoint: for every contact l,
 *   E_i = gamma_l (dLdF_i - Vw_i) - w_l Utot_i  (and likewise for j),
 *   c_phi = -w_l / dt,
 * and the gradient of J_l (orc_contact_grad) is added to particle j and
 * subtracted from particle i, in contact order. dLdpos[n][3] is
 * overwritten. dLdF may be NULL (taken as zero). */
void orc_adjoint_positions(int n, long nc, const double *pos,
                           const double *axis, const double *radius,
                           const double *half_len, const double *L,
                           int periodic, const int *ci, const int *cj,
                           const double *gamma, const double *w,
                           const double *dLdF, const double *Vw,
                           const double *Utot, double dt, double *dLdpos)
{
    memset(dLdpos, 0, sizeof(double) * 3 * (size_t)n);
    for (long l = 0; l < nc; ++l) {
        if (gamma[l] == 0.0 && w[l] == 0.0)
            continue;
        int i = ci[l], j = cj[l];
        double Ei[6], Ej[6], gr[3];
        if (j < 0) {
            /* a plane wall: n and tau_i do not move with c_i, and
             * dPhi/dc_i is the face's inward normal m = -n */
            int face = -1 - j, a = face / 2;
            double m = face % 2 ? -1.0 : 1.0;
            dLdpos[3 * (size_t)i + a] += (-w[l] / dt) * m;
            continue;
        }
        for (int a = 0; a < 6; ++a) {
            double fi = dLdF ? dLdF[6 * (size_t)i + a] : 0.0;
            double fj = dLdF ? dLdF[6 * (size_t)j + a] : 0.0;
            Ei[a] = gamma[l] * (fi - Vw[6 * (size_t)i + a]) - w[l] * Utot[6 * (size_t)i + a];
            Ej[a] = gamma[l] * (fj - Vw[6 * (size_t)j + a]) - w[l] * Utot[6 * (size_t)j + a];
        }
        orc_contact_grad(pos + 3 * i, axis + 3 * i, radius[i], half_len[i],
                         pos + 3 * j, axis + 3 * j, radius[j], half_len[j],
                         L, periodic, Ei, Ej, -w[l] / dt, gr);
        for (int a = 0; a < 3; ++a) {
            dLdpos[3 * (size_t)j + a] += gr[a];
            dLdpos[3 * (size_t)i + a] -= gr[a];
        }
    }
}
