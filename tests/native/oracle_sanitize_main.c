/*
 * Runs every entry point of the FP64 oracle (oracle/oracle.c) on a small
 * synthetic suspension of rods and spheres, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer: the close-pair search by
 * brute force and by cell list (one and three threads, periodic and walled
 * boxes), the contact geometry and its derivative, q, products with D, D^T
 * and M, the diagonal of M, Algorithm 1 for all three step rules, and the
 * geometric part of the adjoint. Exits non-zero if two searches disagree;
 * the sanitizers abort on any invalid access or undefined operation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_set_threads(int t);
int orc_pair_geometry(const double *ci, const double *pi, double Ri, double hi,
                      const double *cj, const double *pj, double Rj, double hj,
                      const double *L, int periodic, double *out);
long orc_find_contacts(int method, int n, const double *pos, const double *axis,
                       const double *radius, const double *half_len, const double *lo,
                       const double *L, int periodic, int walls, double delta, long cap,
                       int *ci, int *cj, double *phi, double *nrm, double *tau_i,
                       double *tau_j, double *st, long *flags_out);
void orc_mobility(int n, const double *axis, const double *mob, const double *F, double *U);
void orc_D_apply(int n, long nc, const int *ci, const int *cj, const double *nrm,
                 const double *tau_i, const double *tau_j, const double *gamma, double *F);
void orc_DT_apply(long nc, const int *ci, const int *cj, const double *nrm,
                  const double *tau_i, const double *tau_j, const double *U, double *out);
void orc_build_q(long nc, const int *ci, const int *cj, const double *phi,
                 const double *nrm, const double *tau_i, const double *tau_j,
                 const double *u_nc, double dt, double *q);
void orc_mvop(int n, long nc, const int *ci, const int *cj, const double *nrm,
              const double *tau_i, const double *tau_j, const double *axis,
              const double *mob, const double *x, double *out);
void orc_M_diag(long nc, const int *ci, const int *cj, const double *nrm,
                const double *tau_i, const double *tau_j, const double *axis,
                const double *mob, double *diag);
int orc_bbpgd(int n, long nc, const int *ci, const int *cj, const double *nrm,
              const double *tau_i, const double *tau_j, const double *axis,
              const double *mob, const double *q, double *gamma, double *g,
              double tol, int max_iter, int bb, double *stats);
void orc_contact_grad(const double *ci, const double *pi, double Ri, double hi,
                      const double *cj, const double *pj, double Rj, double hj,
                      const double *L, int periodic, const double *Ei, const double *Ej,
                      double c_phi, double *out);
void orc_adjoint_positions(int n, long nc, const double *pos, const double *axis,
                           const double *radius, const double *half_len, const double *L,
                           int periodic, const int *ci, const int *cj, const double *gamma,
                           const double *w, const double *dLdF, const double *Vw,
                           const double *Utot, double dt, double *dLdpos);

/* 64-bit linear congruential generator (Knuth's MMIX constants), top 53 bits */
static unsigned long long rng_state = 12345u;
static double uniform(void)
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

typedef struct {
    long nc;
    int *ci, *cj;
    double *phi, *nrm, *ti, *tj, *st;
} list;

static list search(int method, int n, const double *pos, const double *axis, const double *rad,
                   const double *hl, const double *lo, const double *L, int periodic, int walls,
                   double delta)
{
    list c;
    long cap = 64;
    for (;;) {
        c.ci = malloc(sizeof(int) * cap);
        c.cj = malloc(sizeof(int) * cap);
        c.phi = malloc(sizeof(double) * cap);
        c.nrm = malloc(sizeof(double) * 3 * cap);
        c.ti = malloc(sizeof(double) * 3 * cap);
        c.tj = malloc(sizeof(double) * 3 * cap);
        c.st = malloc(sizeof(double) * 2 * cap);
        long flags[2];
        c.nc = orc_find_contacts(method, n, pos, axis, rad, hl, lo, L, periodic, walls, delta,
                                 cap, c.ci, c.cj, c.phi, c.nrm, c.ti, c.tj, c.st, flags);
        if (c.nc <= cap)
            return c;
        cap = c.nc;
        free(c.ci); free(c.cj); free(c.phi); free(c.nrm); free(c.ti); free(c.tj); free(c.st);
    }
}

static void release(list *c)
{
    free(c->ci); free(c->cj); free(c->phi); free(c->nrm); free(c->ti); free(c->tj); free(c->st);
}

static int same(const list *a, const list *b)
{
    if (a->nc != b->nc) return 0;
    for (long l = 0; l < a->nc; ++l)
        if (a->ci[l] != b->ci[l] || a->cj[l] != b->cj[l] || a->phi[l] != b->phi[l]) return 0;
    return 1;
}

int main(void)
{
    const int nr = 300, ns = 100, n = nr + ns;
    double *pos = malloc(sizeof(double) * 3 * n), *axis = malloc(sizeof(double) * 3 * n);
    double *rad = malloc(sizeof(double) * n), *hl = malloc(sizeof(double) * n);
    double *mob = malloc(sizeof(double) * 4 * n), *F = malloc(sizeof(double) * 6 * n);
    double *U = malloc(sizeof(double) * 6 * n), *G = malloc(sizeof(double) * 3 * n);
    const double side = 3.0, lo[3] = {0.0, 0.0, 0.0}, L[3] = {side, side, side};
    for (int k = 0; k < n; ++k) {
        double p[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            pos[3 * k + a] = side * uniform();
            p[a] = 2.0 * uniform() - 1.0;
            r2 += p[a] * p[a];
        }
        for (int a = 0; a < 3; ++a) axis[3 * k + a] = p[a] / sqrt(r2 > 0.0 ? r2 : 1.0);
        rad[k] = k < nr ? 0.025 : 0.05;
        hl[k] = k < nr ? 0.5 : 0.0;
        for (int a = 0; a < 4; ++a) mob[4 * k + a] = 0.3 + 0.1 * a;
        for (int a = 0; a < 6; ++a) F[6 * k + a] = 2.0 * uniform() - 1.0;
    }
    int bad = 0;
    for (int box = 0; box < 2; ++box) {
        const int periodic = box == 0, walls = box == 0 ? 0 : 63;
        list b = search(0, n, pos, axis, rad, hl, lo, L, periodic, walls, 0.015);
        list c1 = search(1, n, pos, axis, rad, hl, lo, L, periodic, walls, 0.015);
        orc_set_threads(3);
        list c3 = search(1, n, pos, axis, rad, hl, lo, L, periodic, walls, 0.015);
        orc_set_threads(1);
        if (!same(&b, &c1) || !same(&c1, &c3)) {
            fprintf(stderr, "searches disagree (box %d)\n", box);
            bad = 1;
        }
        const long nc = c1.nc;
        double *q = malloc(sizeof(double) * (nc + 1)), *x = malloc(sizeof(double) * (nc + 1));
        double *y = malloc(sizeof(double) * (nc + 1)), *gam = malloc(sizeof(double) * (nc + 1));
        double *g = malloc(sizeof(double) * (nc + 1)), *w = malloc(sizeof(double) * (nc + 1));
        orc_mobility(n, axis, mob, F, U);
        orc_build_q(nc, c1.ci, c1.cj, c1.phi, c1.nrm, c1.ti, c1.tj, U, 1e-4, q);
        for (long l = 0; l < nc; ++l) x[l] = uniform();
        orc_D_apply(n, nc, c1.ci, c1.cj, c1.nrm, c1.ti, c1.tj, x, F);
        orc_DT_apply(nc, c1.ci, c1.cj, c1.nrm, c1.ti, c1.tj, U, y);
        orc_mvop(n, nc, c1.ci, c1.cj, c1.nrm, c1.ti, c1.tj, axis, mob, x, y);
        orc_M_diag(nc, c1.ci, c1.cj, c1.nrm, c1.ti, c1.tj, axis, mob, y);
        for (int bb = 1; bb <= 3; ++bb)
            for (int t = 1; t <= 3; t += 2) {
                double stats[8];
                orc_set_threads(t);
                memset(gam, 0, sizeof(double) * (nc + 1));
                orc_bbpgd(n, nc, c1.ci, c1.cj, c1.nrm, c1.ti, c1.tj, axis, mob, q, gam, g, 1e-8,
                          20000, bb, stats);
                orc_set_threads(1);
            }
        for (long l = 0; l < nc; ++l) w[l] = gam[l] > 0.0 ? uniform() : 0.0;
        orc_D_apply(n, nc, c1.ci, c1.cj, c1.nrm, c1.ti, c1.tj, gam, F);
        orc_adjoint_positions(n, nc, pos, axis, rad, hl, L, periodic, c1.ci, c1.cj, gam, w, F,
                              U, U, 1e-4, G);
        for (long l = 0; l < nc && l < 50; ++l) {
            const int i = c1.ci[l], j = c1.cj[l];
            double out[12], grad[3], Ei[6] = {1, 2, 3, 4, 5, 6}, Ej[6] = {6, 5, 4, 3, 2, 1};
            if (j < 0) continue;
            orc_pair_geometry(pos + 3 * i, axis + 3 * i, rad[i], hl[i], pos + 3 * j,
                              axis + 3 * j, rad[j], hl[j], L, periodic, out);
            orc_contact_grad(pos + 3 * i, axis + 3 * i, rad[i], hl[i], pos + 3 * j,
                             axis + 3 * j, rad[j], hl[j], L, periodic, Ei, Ej, 0.5, grad);
        }
        printf("box %d: %ld contacts\n", box, nc);
        free(q); free(x); free(y); free(gam); free(g); free(w);
        release(&b); release(&c1); release(&c3);
    }
    free(pos); free(axis); free(rad); free(hl); free(mob); free(F); free(U); free(G);
    return bad;
}
