// sc_build_dev.hpp -- per-particle, per-rank and per-contact steps of the
// close-pair build (section 3.2's A(C, delta) with a uniform cell list,
// section 5.2; contact frames for Eq. Dmatdef / Eq. Dtranspose; q of LCP
// LCPdef), shared by the single-suspension build and the batched build.
//
// A build works on one suspension's arrays with local indices (particle i,
// rank t, contact l). The batched build keeps the suspensions of a batch in
// one set of cells and ranks: a suspension's cells start at `cbase` and its
// ranks at `rbase` in those shared arrays, and both are 0 for a build of a
// single suspension. Every step is a pure function of the inputs, so the
// contacts of a suspension and their order do not depend on the batch it is
// built in.
#pragma once

#include <cmath>

#include "sc_common.hpp"
#include "sc_geometry.hpp"
#include "sc_plan.hpp"

namespace sc {

enum BuildFlag {
    kFlagBadInput = 0,   // non-finite or out-of-range particle data
    kFlagParallel = 1,   // pairs resolved by the parallel-axes rule
    kFlagZero = 2,       // coincident cores
    kFlagBorder = 3,     // |Phi - delta| < 1e-12
    kFlagNonfiniteQ = 4, // q not finite (bad u_nc)
    kFlagExtent = 5,     // a particle reaches further than the search grid allows
    kFlagWalls = 6,      // particle-wall contacts
    kFlagCount = 8,
};

struct Grid {
    double lo[3], len[3], side[3];
    int nc[3];
    int periodic;
    int walls;              // faces with a wall (bit 2a: x_a = lo_a, 2a + 1: x_a = lo_a + len_a)
    int npart;              // particles; partner code npart + f stands for the wall on face f
    double delta;
    __host__ __device__ PBox box() const { return PBox{{len[0], len[1], len[2]}, periodic}; }
};

struct Parts {
    int n;
    const double *pos, *axis, *radius, *half_len, *mob;
};

// Ranked (cell-ordered) copies used by the pair search: centre and radius in
// one 32-byte record, the half length, and the (local) cell of each rank;
// the axis comes from the plan record. Indexed by local rank.
struct Ranked {
    const double *prec;   // [n][4] x y z, R
    const double *hl;     // [n]
    const int *cell;      // [n]
};

__device__ __forceinline__ int cell_axis(double x, int a, const Grid &g) {
    double u = x - g.lo[a];
    if (g.periodic) u = u - g.len[a] * floor(u / g.len[a]);
    int c = static_cast<int>(floor(u / g.side[a]));
    return c < 0 ? 0 : (c >= g.nc[a] ? g.nc[a] - 1 : c);
}

// Distinct neighbour coordinates of cell coordinate c along axis a.
__device__ __forceinline__ int neighbours(int c, int a, const Grid &g, int out[3]) {
    int k = 0;
    for (int d = -1; d <= 1; ++d) {
        int x = c + d;
        if (g.periodic) {
            x = (x + g.nc[a]) % g.nc[a];
        } else if (x < 0 || x >= g.nc[a]) {
            continue;
        }
        bool dup = false;
        for (int e = 0; e < k; ++e) dup |= (out[e] == x);
        if (!dup) out[k++] = x;
    }
    return k;
}

// Non-finite or out-of-range data of particle k (radius and mobility > 0,
// half length >= 0, unit axis for rods).
__device__ __forceinline__ bool particle_bad(const Parts &P, int k) {
    bool bad = false;
    for (int a = 0; a < 3; ++a) bad |= !isfinite(P.pos[3 * k + a]) || !isfinite(P.axis[3 * k + a]);
    const double R = P.radius[k], h = P.half_len[k];
    bad |= !(R > 0.0) || !isfinite(R) || !(h >= 0.0) || !isfinite(h);
    for (int a = 0; a < 4; ++a) bad |= !(P.mob[4 * k + a] > 0.0) || !isfinite(P.mob[4 * k + a]);
    if (h > 0.0) {
        const V3 p = load3(P.axis + 3 * k);
        bad |= fabs(dot(p, p) - 1.0) > 1e-10;
    }
    return bad;
}

// Cell of particle k (cbase + row-major cell of the suspension's grid).
__device__ __forceinline__ int particle_cell(const Parts &P, int k, const Grid &g, int cbase) {
    const int cx = cell_axis(P.pos[3 * k + 0], 0, g);
    const int cy = cell_axis(P.pos[3 * k + 1], 1, g);
    const int cz = cell_axis(P.pos[3 * k + 2], 2, g);
    return cbase + (cz * g.nc[1] + cy) * g.nc[0] + cx;
}

// Rank of particle k (shared index gk = rbase + k): its cell's start plus the
// number of cell members with a smaller index, a deterministic order within
// each cell. Writes the permutation and the plan record (local ranks) and the
// ranked records (shared rank; the cell stored relative to cbase).
__device__ __forceinline__ void rank_particle(const Parts &P, int k, int rbase, int cbase,
                                              const int *cell_of, const int *cell_start,
                                              const int *members, const Plan &pl, double *prec,
                                              double *hl, int *cell_r) {
    const int gk = rbase + k;
    const int c = cell_of[gk];
    const int b0 = cell_start[c], b1 = cell_start[c + 1];
    int r = 0;
    for (int m = b0; m < b1; ++m) r += members[m] < gk;
    const int rg = b0 + r, rk = rg - rbase;
    pl.rank[k] = rk;
    pl.order[rk] = k;
    cell_r[rg] = c - cbase;
    double *rec = pl.pdat + 8 * static_cast<long long>(rk);
    rec[0] = P.axis[3 * k + 0];
    rec[1] = P.axis[3 * k + 1];
    rec[2] = P.axis[3 * k + 2];
    rec[3] = 0.0;
    for (int a = 0; a < 4; ++a) rec[4 + a] = P.mob[4 * k + a];
    double *pr = prec + 4 * static_cast<long long>(rg);
    pr[0] = P.pos[3 * k + 0];
    pr[1] = P.pos[3 * k + 1];
    pr[2] = P.pos[3 * k + 2];
    pr[3] = P.radius[k];
    hl[rg] = P.half_len[k];
}

// Geometry of ranks (ri, rj) evaluated as the pair (lower caller index, higher
// caller index), so a contact's normal and moment arms do not depend on the
// ranking.
__device__ __forceinline__ PairGeo ranked_geo(int a, int b, const Ranked &R, const Plan &pl,
                                              const PBox &box, bool &a_is_i) {
    a_is_i = pl.order[a] < pl.order[b];
    const int ri = a_is_i ? a : b, rj = a_is_i ? b : a;
    const double *pi_ = R.prec + 4 * static_cast<long long>(ri);
    const double *pj_ = R.prec + 4 * static_cast<long long>(rj);
    const double *ai = pl.pdat + 8 * static_cast<long long>(ri);
    const double *aj = pl.pdat + 8 * static_cast<long long>(rj);
    return pair_geo(min_image(v3(pi_[0], pi_[1], pi_[2]), v3(pj_[0], pj_[1], pj_[2]), box),
                    v3(ai[0], ai[1], ai[2]), pi_[3], R.hl[ri], v3(aj[0], aj[1], aj[2]),
                    pj_[3], R.hl[rj]);
}

// Particle-wall geometry (section 3.3's boundary extension: the constraint's
// column of D holds the particle's 6 entries only) for face f of a closed
// box. With m the face's inward normal, the core point nearest the plane is
// c + s p with s = -h sign(m.p) (s = 0 for a rod parallel to the plane: the
// midpoint), Phi = m.(c - plane) - h |m.p| - R, and the contact normal
// points from the particle to the wall, n = -m.
__device__ __forceinline__ PairGeo wall_geo(V3 c, V3 p, double R, double h, const Grid &g,
                                            int face) {
    const int a = face >> 1;
    const bool up = face & 1;
    const double sg = up ? -1.0 : 1.0;
    const double ca = a == 0 ? c.x : (a == 1 ? c.y : c.z);
    const double pa = a == 0 ? p.x : (a == 1 ? p.y : p.z);
    const double d = up ? g.lo[a] + g.len[a] - ca : ca - g.lo[a];
    const double mp = sg * pa;
    double s = 0.0;
    int par = 0;
    if (h > 0.0) {
        if (fabs(mp) < 1e-12)
            par = 1;
        else
            s = mp > 0.0 ? -h : h;
    }
    PairGeo G;
    G.phi = d + s * mp - R;
    G.n = v3(a == 0 ? -sg : 0.0, a == 1 ? -sg : 0.0, a == 2 ? -sg : 0.0);
    G.s = s;
    G.t = 0.0;
    G.flags = par;
    return G;
}

// Lanes that share one particle's 27-cell stencil in the pair search (lane j
// takes the neighbour cells whose index in (z, y, x) order is j modulo this).
constexpr int kPairLanes = 8;
// Partners each lane keeps from the count pass (a lane with more is searched
// again by the write pass).
constexpr int kLaneSlots = 8;

// Visit every partner u > t (by local rank) of rank t whose pair has
// Phi <= delta, calling fn(u, geo), and lane 0 also every wall within delta
// (u = npart + face). The candidates are the ranks of the 27
// neighbour cells: per (y, z) row the x-neighbours are merged into runs of
// consecutive cells, which are consecutive ranks (cells are row-major), and
// the kPairLanes lanes of rank t take every kPairLanes-th candidate of the
// runs laid end to end, so the lanes share the work evenly and neighbouring
// lanes read neighbouring records. cstart: the suspension's cell starts
// (shared ranks), rbase subtracted to make them local.
template <class Fn>
__device__ __forceinline__ void for_close_partners(int t, int lane, const Ranked &R,
                                                   const Plan &pl, const Grid &g,
                                                   const int *cstart, int rbase, Fn fn) {
    static_assert((kPairLanes & (kPairLanes - 1)) == 0, "lanes per rank: a power of two");
    const double *pt = R.prec + 4 * static_cast<long long>(t);
    const V3 ct = v3(pt[0], pt[1], pt[2]);
    const double Rt = pt[3], ht = R.hl[t];
    const int c = R.cell[t];
    const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    int nx[3], ny[3], nz[3];
    const int kx = neighbours(cx, 0, g, nx), ky = neighbours(cy, 1, g, ny),
              kz = neighbours(cz, 2, g, nz);
    // x-neighbours in increasing order, as runs [x0, x1) of consecutive cells
    for (int a = 1; a < kx; ++a)
        for (int b = a; b > 0 && nx[b - 1] > nx[b]; --b) {
            const int tmp = nx[b];
            nx[b] = nx[b - 1];
            nx[b - 1] = tmp;
        }
    int rx0[3], rx1[3], nrun = 0;
    for (int a = 0; a < kx; ++a) {
        if (nrun > 0 && rx1[nrun - 1] == nx[a]) {
            rx1[nrun - 1] = nx[a] + 1;
        } else {
            rx0[nrun] = nx[a];
            rx1[nrun] = nx[a] + 1;
            ++nrun;
        }
    }
    const PBox box = g.box();
    const double *at = pl.pdat + 8 * static_cast<long long>(t);
    const V3 pt_ax = v3(at[0], at[1], at[2]);
    int seen = 0;  // candidates in the runs before the current one
    for (int az = 0; az < kz; ++az)
        for (int ay = 0; ay < ky; ++ay) {
            const int row = (nz[az] * g.nc[1] + ny[ay]) * g.nc[0];
            for (int q = 0; q < nrun; ++q) {
                int u0 = cstart[row + rx0[q]] - rbase;
                const int end = cstart[row + rx1[q]] - rbase;
                if (u0 <= t) u0 = t + 1;
                if (end <= u0) continue;
                for (int u = u0 + ((lane - seen) & (kPairLanes - 1)); u < end; u += kPairLanes) {
                    const double *pu = R.prec + 4 * static_cast<long long>(u);
                    const V3 r = min_image(ct, v3(pu[0], pu[1], pu[2]), box);
                    // the core distance is at least |r| - ht - hu
                    const double hu = R.hl[u];
                    const double reach = ht + hu + Rt + pu[3] + g.delta;
                    if (dot(r, r) > reach * reach * (1.0 + 1e-9)) continue;
                    if (ht > 0.0 && hu > 0.0) {
                        // two segments are no closer than their lines: skip pairs
                        // whose lines are farther apart than R_t + R_u + delta
                        // (near-parallel axes give w ~ 0 and fall through to the
                        // exact test)
                        const double *au = pl.pdat + 8 * static_cast<long long>(u);
                        const V3 w = cross(pt_ax, v3(au[0], au[1], au[2]));
                        const double rw = dot(r, w), lim = Rt + pu[3] + g.delta;
                        if (rw * rw > lim * lim * dot(w, w) * (1.0 + 1e-9)) continue;
                    }
                    bool t_is_i;
                    const PairGeo G = ranked_geo(t, u, R, pl, box, t_is_i);
                    if (G.phi <= g.delta) fn(u, G);
                }
                seen += end - u0;
            }
        }
    if (g.walls && lane == 0)
        for (int f = 0; f < 6; ++f) {
            if (!(g.walls & (1 << f))) continue;
            const PairGeo G = wall_geo(ct, pt_ax, Rt, ht, g, f);
            if (G.phi <= g.delta) fn(g.npart + f, G);
        }
}

// Count pass of lane `lane` of rank t: the number of its partners goes to
// lane_cnt[0] and the first kLaneSlots of them (in search order) to slots,
// the rank's total (over the kPairLanes lanes, which must be consecutive
// threads) to cptr[t]; diagnostic counts to flags.
__device__ __forceinline__ void count_partners(int t, int lane, const Ranked &R, const Plan &pl,
                                               const Grid &g, const int *cstart, int rbase,
                                               int *lane_cnt, int *slots, int *flags) {
    int cnt = 0, npar = 0, nzero = 0, nborder = 0, nwall = 0;
    for_close_partners(t, lane, R, pl, g, cstart, rbase, [&](int u, const PairGeo &G) {
        if (cnt < kLaneSlots) slots[cnt] = u;
        ++cnt;
        nwall += u >= g.npart;
        npar += G.flags & 1;
        nzero += (G.flags >> 1) & 1;
        nborder += fabs(G.phi - g.delta) < 1e-12;
    });
    *lane_cnt = cnt;
    int tot = cnt;
#pragma unroll
    for (int off = kPairLanes / 2; off > 0; off >>= 1) tot += __shfl_xor(tot, off, kPairLanes);
    if (lane == 0) pl.cptr[t] = tot;
    if (npar) atomicAdd(flags + kFlagParallel, npar);
    if (nzero) atomicAdd(flags + kFlagZero, nzero);
    if (nborder) atomicAdd(flags + kFlagBorder, nborder);
    if (nwall) atomicAdd(flags + kFlagWalls, nwall);
}

// Write pass: lane `lane` of rank t stores its partners' ranks (even slots of
// cs) after those of the rank's lower lanes, from the count pass's slots, or
// by searching again if it had more than kLaneSlots. lane_cnt points at lane
// 0's count, slots at this lane's slots.
__device__ __forceinline__ void write_partners(int t, int lane, const Ranked &R, const Plan &pl,
                                               const Grid &g, const int *cstart, int rbase,
                                               const int *lane_cnt, const int *slots) {
    const int lim = lane_cnt[lane];
    int before = 0;
    for (int j = 0; j < lane; ++j) before += lane_cnt[j];
    int *part = pl.cs + 2 * static_cast<long long>(pl.cptr[t] + before);
    if (lim <= kLaneSlots) {
        for (int k = 0; k < lim; ++k) part[2 * k] = slots[k];
        return;
    }
    int k = 0;
    // the count pass used the same pure predicate, so k ends at lim; the
    // bound only guards the segment
    for_close_partners(t, lane, R, pl, g, cstart, rbase, [&](int u, const PairGeo &) {
        if (k < lim) part[2 * k] = u;
        ++k;
    });
}

// Contacts of rank t (partners of higher rank, ascending, then walls):
// caller indices, Phi, frame [l][9] = n, tau_i, tau_j oriented from ci
// (lower caller index) to cj, and cs[l] = the ranks of (ci, cj). A wall
// contact has cj = -1 - face, tau_j = 0 and no second rank (-1).
__device__ __forceinline__ void finish_partners(int t, const Ranked &R, const Plan &pl,
                                                const Grid &g, int *ci, int *cj, double *phi,
                                                double *frame) {
    const int base = pl.cptr[t], k = pl.cptr[t + 1] - base;
    int *part = pl.cs + 2 * static_cast<long long>(base);  // even slots: partner ranks
    for (int a = 1; a < k; ++a) {
        const int v = part[2 * a];
        int b = a - 1;
        while (b >= 0 && part[2 * b] > v) {
            part[2 * (b + 1)] = part[2 * b];
            --b;
        }
        part[2 * (b + 1)] = v;
    }
    const PBox box = g.box();
    const int ot = pl.order[t];
    for (int a = 0; a < k; ++a) {
        const long long l = base + a;
        const int u = part[2 * a];
        if (u >= g.npart) {
            const double *pr = R.prec + 4 * static_cast<long long>(t);
            const double *ax = pl.pdat + 8 * static_cast<long long>(t);
            const V3 p = v3(ax[0], ax[1], ax[2]);
            const PairGeo G = wall_geo(v3(pr[0], pr[1], pr[2]), p, pr[3], R.hl[t], g, u - g.npart);
            const V3 ti = cross(G.s * p, G.n);
            ci[l] = ot;
            cj[l] = -1 - (u - g.npart);
            phi[l] = G.phi;
            double *f = frame + 9 * l;
            f[0] = G.n.x; f[1] = G.n.y; f[2] = G.n.z;
            f[3] = ti.x;  f[4] = ti.y;  f[5] = ti.z;
            f[6] = 0.0;   f[7] = 0.0;   f[8] = 0.0;
            part[2 * a] = t;
            part[2 * a + 1] = -1;
            continue;
        }
        bool t_is_i;
        const PairGeo G = ranked_geo(t, u, R, pl, box, t_is_i);
        const int ri = t_is_i ? t : u, rj = t_is_i ? u : t;
        const double *ai = pl.pdat + 8 * static_cast<long long>(ri);
        const double *aj = pl.pdat + 8 * static_cast<long long>(rj);
        const int ou = pl.order[u];
        ci[l] = t_is_i ? ot : ou;
        cj[l] = t_is_i ? ou : ot;
        phi[l] = G.phi;
        // moment arms of the contact points: tau_i = (s p_i) x n, tau_j = (t p_j) x n
        const V3 ti = cross(G.s * v3(ai[0], ai[1], ai[2]), G.n);
        const V3 tj = cross(G.t * v3(aj[0], aj[1], aj[2]), G.n);
        double *f = frame + 9 * l;
        f[0] = G.n.x; f[1] = G.n.y; f[2] = G.n.z;
        f[3] = ti.x;  f[4] = ti.y;  f[5] = ti.z;
        f[6] = tj.x;  f[7] = tj.y;  f[8] = tj.z;
        part[2 * a] = ri;
        part[2 * a + 1] = rj;
    }
}

// Incidences of each rank: its contacts as the lower rank first, in contact
// order (these incidences own gamma_l), then its contacts as the higher rank,
// placed by an atomic cursor and sorted by contact index afterwards.
__device__ __forceinline__ void count_second(int l, const Plan &pl, int *deg) {
    const int a = pl.cs[2 * l], b = pl.cs[2 * l + 1];
    if (b < 0) return;  // a wall contact belongs to its particle only
    atomicAdd(deg + (a > b ? a : b), 1);
}

__device__ __forceinline__ void incidence_count(int k, const Plan &pl, const int *deg) {
    pl.inc_ptr[k] = (pl.cptr[k + 1] - pl.cptr[k]) + deg[k];
}

__device__ __forceinline__ void incidence_fill(int l, const Plan &pl, int *fill) {
    const int a = pl.cs[2 * l], b = pl.cs[2 * l + 1];
    if (b < 0) {  // wall contact: in its particle's own group
        pl.inc[pl.inc_ptr[a] + (l - pl.cptr[a])] = 2 * l + 1;
        return;
    }
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    pl.inc[pl.inc_ptr[lo] + (l - pl.cptr[lo])] = 2 * l + 1;
    const int first_hi = pl.cptr[hi + 1] - pl.cptr[hi];
    pl.inc[pl.inc_ptr[hi] + first_hi + atomicAdd(fill + hi, 1)] = 2 * l;
}

// Sort the higher-rank part of rank k's incidence list, then write the signed
// column entries: -(n, tau_i) on ci's rank, +(n, tau_j) on cj's rank.
__device__ __forceinline__ void incidence_finish(int k, const Plan &pl, const double *frame) {
    const int e0 = pl.inc_ptr[k] + (pl.cptr[k + 1] - pl.cptr[k]), e1 = pl.inc_ptr[k + 1];
    for (int a = e0 + 1; a < e1; ++a) {
        const int v = pl.inc[a];
        int b = a - 1;
        while (b >= e0 && pl.inc[b] > v) {
            pl.inc[b + 1] = pl.inc[b];
            --b;
        }
        pl.inc[b + 1] = v;
    }
    for (int e = pl.inc_ptr[k]; e < e1; ++e) {
        const long long l = pl.inc[e] >> 1;
        const double *f = frame + 9 * l;
        const bool is_i = pl.cs[2 * l] == k;
        const double sg = is_i ? -1.0 : 1.0;
        const double *tau = is_i ? f + 3 : f + 6;
        double *d = pl.dpm + 6 * static_cast<long long>(e);
        d[0] = sg * f[0];
        d[1] = sg * f[1];
        d[2] = sg * f[2];
        d[3] = sg * tau[0];
        d[4] = sg * tau[1];
        d[5] = sg * tau[2];
    }
}

// q_l = Phi_l / dt + D_l^T U_nc (LCP LCPdef, scaled by 1/dt).
__device__ __forceinline__ double contact_q(int l, const int *ci, const int *cj, const double *phi,
                                            const double *frame, const double *u_nc, double dt) {
    const double *f = frame + 9 * static_cast<long long>(l);
    const V3 n = load3(f), ti = load3(f + 3), tj = load3(f + 6);
    const double *ui = u_nc + 6 * static_cast<long long>(ci[l]);
    double v = -dot(n, load3(ui)) - dot(ti, load3(ui + 3));
    if (cj[l] >= 0) {
        const double *uj = u_nc + 6 * static_cast<long long>(cj[l]);
        v = v + dot(n, load3(uj)) + dot(tj, load3(uj + 3));
    }
    return phi[l] / dt + v;
}

// Search grid of one suspension for interaction range rmax (cells of side >=
// rmax, at most 1024 per axis, the total within `budget`). Returns false if a
// periodic side is shorter than 2 rmax (the minimum image would be
// ambiguous).
inline bool make_grid(const sc_box &box, int n, double delta, double rmax, size_t budget,
                      Grid &g) {
    g = Grid{};
    g.npart = n;
    g.walls = box.periodic ? 0 : box.walls;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = box.lo[a];
        g.len[a] = box.len[a];
        if (box.periodic && box.len[a] < 2.0 * rmax) return false;
        double m = std::floor(box.len[a] / rmax);
        g.nc[a] = m < 1.0 ? 1 : (m > 1024.0 ? 1024 : static_cast<int>(m));
    }
    // keep the grid within the cell budget (bigger cells stay correct)
    while (static_cast<size_t>(g.nc[0]) * g.nc[1] * g.nc[2] > budget) {
        int a = (g.nc[0] >= g.nc[1] && g.nc[0] >= g.nc[2]) ? 0 : (g.nc[1] >= g.nc[2] ? 1 : 2);
        g.nc[a] = g.nc[a] > 1 ? (g.nc[a] + 1) / 2 : 1;
    }
    for (int a = 0; a < 3; ++a) g.side[a] = box.len[a] / g.nc[a];
    g.periodic = box.periodic ? 1 : 0;
    g.delta = delta;
    return true;
}

// Cells the search grid of n particles may use.
inline size_t cell_budget(int32_t n) { return 2 * static_cast<size_t>(n) + 64; }

}  // namespace sc
