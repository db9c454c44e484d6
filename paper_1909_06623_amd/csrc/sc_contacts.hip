// sc_contacts.hip -- close-pair detection and LCP assembly on gfx950.
//
// Builds the set A(C, delta) = {(i, j), i < j : Phi_ij <= delta} of section
// 3.2 with a uniform cell list (section 5.2 names cell lists as the standard
// near-neighbour method), the contact frames that define the columns of D
// (Eq. Dmatdef; their entries follow from Eq. Dtranspose) and
// q = Phi/dt + D^T U_nc (LCP LCPdef), plus the solver layout (sc_plan.hpp).
//
// Pipeline (stream-ordered; two host synchronisations: the interaction range
// sizes the grid, and the pair count is checked against capacity):
//   validate + max extent -> bin -> scan -> scatter -> rank particles in
//   cell order (ties by caller index) -> count partners of higher rank ->
//   scan -> write contacts (partners sorted by rank) -> incidence lists and
//   signed column entries -> q.
// Every decision is a pure function of the inputs, so the contact list and
// its order are independent of thread scheduling.
#include <cmath>
#include <cstring>

#include "sc_common.hpp"
#include "sc_geometry.hpp"
#include "sc_plan.hpp"

namespace sc {

namespace {

enum Flag {
    kFlagBadInput = 0,   // non-finite or out-of-range particle data
    kFlagParallel = 1,   // pairs resolved by the parallel-axes rule
    kFlagZero = 2,       // coincident cores
    kFlagBorder = 3,     // |Phi - delta| < 1e-12
    kFlagNonfiniteQ = 4, // q not finite (bad u_nc)
    kFlagCount = 8,
};

struct Grid {
    double lo[3], len[3], side[3];
    int nc[3];
    int periodic;
    double delta;
    __host__ __device__ PBox box() const { return PBox{{len[0], len[1], len[2]}, periodic}; }
};

struct Parts {
    int n;
    const double *pos, *axis, *radius, *half_len, *mob;
};

// Ranked (cell-ordered) copies used by the pair search: centre and radius in
// one 32-byte record, the half length, and the cell of each rank; the axis
// comes from the plan record.
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

__global__ void k_validate(Parts P, unsigned long long *max_ext, int *flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    bool bad = false;
    for (int a = 0; a < 3; ++a) bad |= !isfinite(P.pos[3 * k + a]) || !isfinite(P.axis[3 * k + a]);
    const double R = P.radius[k], h = P.half_len[k];
    bad |= !(R > 0.0) || !isfinite(R) || !(h >= 0.0) || !isfinite(h);
    for (int a = 0; a < 4; ++a) bad |= !(P.mob[4 * k + a] > 0.0) || !isfinite(P.mob[4 * k + a]);
    if (h > 0.0) {
        const V3 p = load3(P.axis + 3 * k);
        bad |= fabs(dot(p, p) - 1.0) > 1e-10;
    }
    if (bad) {
        atomicOr(flags + kFlagBadInput, 1);
        return;
    }
    // non-negative doubles order like their bit patterns
    const double e = R + h;
    atomicMax(max_ext, static_cast<unsigned long long>(__double_as_longlong(e)));
}

__global__ void k_bin(Parts P, Grid g, int *cell_of, int *cell_count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    const int cx = cell_axis(P.pos[3 * k + 0], 0, g);
    const int cy = cell_axis(P.pos[3 * k + 1], 1, g);
    const int cz = cell_axis(P.pos[3 * k + 2], 2, g);
    const int c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
    cell_of[k] = c;
    atomicAdd(cell_count + c, 1);
}

__global__ void k_scatter(int n, const int *cell_of, const int *cell_start, int *cell_fill,
                          int *members) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int c = cell_of[k];
    members[cell_start[c] + atomicAdd(cell_fill + c, 1)] = k;
}

// Rank of particle k: its cell's start plus the number of cell members with
// a smaller caller index (a deterministic order within each cell). Writes the
// permutation and the ranked particle records.
__global__ void k_rank(Parts P, const int *cell_of, const int *cell_start, const int *members,
                       Plan pl, double *prec, double *hl, int *cell_r) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    const int c = cell_of[k];
    const int b0 = cell_start[c], b1 = cell_start[c + 1];
    int r = 0;
    for (int m = b0; m < b1; ++m) r += members[m] < k;
    const int rk = b0 + r;
    pl.rank[k] = rk;
    pl.order[rk] = k;
    cell_r[rk] = c;
    double *rec = pl.pdat + 8 * static_cast<long long>(rk);
    rec[0] = P.axis[3 * k + 0];
    rec[1] = P.axis[3 * k + 1];
    rec[2] = P.axis[3 * k + 2];
    rec[3] = 0.0;
    for (int a = 0; a < 4; ++a) rec[4 + a] = P.mob[4 * k + a];
    double *pr = prec + 4 * static_cast<long long>(rk);
    pr[0] = P.pos[3 * k + 0];
    pr[1] = P.pos[3 * k + 1];
    pr[2] = P.pos[3 * k + 2];
    pr[3] = P.radius[k];
    hl[rk] = P.half_len[k];
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

// Lanes that share one particle's 27-cell stencil in the pair search (lane j
// takes the neighbour cells whose index in (z, y, x) order is j modulo this).
constexpr int kPairLanes = 8;

// Visit every partner u > t (by rank) of rank t whose pair has Phi <= delta
// among the neighbour cells of lane `lane`'s share, calling fn(u, geo).
template <class Fn>
__device__ __forceinline__ void for_close_partners(int t, int lane, const Ranked &R,
                                                   const Plan &pl, const Grid &g,
                                                   const int *cell_start, Fn fn) {
    const double *pt = R.prec + 4 * static_cast<long long>(t);
    const V3 ct = v3(pt[0], pt[1], pt[2]);
    const double Rt = pt[3], ht = R.hl[t];
    const int c = R.cell[t];
    const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    int nx[3], ny[3], nz[3];
    const int kx = neighbours(cx, 0, g, nx), ky = neighbours(cy, 1, g, ny),
              kz = neighbours(cz, 2, g, nz);
    const PBox box = g.box();
    const double *at = pl.pdat + 8 * static_cast<long long>(t);
    const V3 pt_ax = v3(at[0], at[1], at[2]);
    for (int idx = lane; idx < kx * ky * kz; idx += kPairLanes) {
        const int ax = idx % kx, ay = (idx / kx) % ky, az = idx / (kx * ky);
        const int cc = (nz[az] * g.nc[1] + ny[ay]) * g.nc[0] + nx[ax];
        int u = cell_start[cc];
        const int end = cell_start[cc + 1];
        if (u <= t) u = t + 1;
        for (; u < end; ++u) {
            const double *pu = R.prec + 4 * static_cast<long long>(u);
            const V3 r = min_image(ct, v3(pu[0], pu[1], pu[2]), box);
            // the core distance is at least |r| - ht - hu
            const double hu = R.hl[u];
            const double reach = ht + hu + Rt + pu[3] + g.delta;
            if (dot(r, r) > reach * reach * (1.0 + 1e-9)) continue;
            if (ht > 0.0 && hu > 0.0) {
                // two segments are no closer than their lines: skip pairs whose
                // lines are farther apart than R_t + R_u + delta (near-parallel
                // axes give w ~ 0 and fall through to the exact test)
                const double *au = pl.pdat + 8 * static_cast<long long>(u);
                const V3 w = cross(pt_ax, v3(au[0], au[1], au[2]));
                const double rw = dot(r, w), lim = Rt + pu[3] + g.delta;
                if (rw * rw > lim * lim * dot(w, w) * (1.0 + 1e-9)) continue;
            }
            bool t_is_i;
            const PairGeo G = ranked_geo(t, u, R, pl, box, t_is_i);
            if (G.phi <= g.delta) fn(u, G);
        }
    }
}

// Count pass: kPairLanes consecutive threads per rank; per-lane counts go to
// lane_cnt, the rank's total to cptr.
__global__ void k_count_pairs(int n, Ranked R, Plan pl, Grid g, const int *cell_start,
                              int *lane_cnt, int *flags) {
    const long long gid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int t = static_cast<int>(gid / kPairLanes), lane = static_cast<int>(gid % kPairLanes);
    if (t >= n) return;  // whole groups of kPairLanes leave together
    int cnt = 0, npar = 0, nzero = 0, nborder = 0;
    for_close_partners(t, lane, R, pl, g, cell_start, [&](int, const PairGeo &G) {
        ++cnt;
        npar += G.flags & 1;
        nzero += (G.flags >> 1) & 1;
        nborder += fabs(G.phi - g.delta) < 1e-12;
    });
    lane_cnt[gid] = cnt;
    int tot = cnt;
#pragma unroll
    for (int off = kPairLanes / 2; off > 0; off >>= 1) tot += __shfl_xor(tot, off, kPairLanes);
    if (lane == 0) pl.cptr[t] = tot;
    if (npar) atomicAdd(flags + kFlagParallel, npar);
    if (nzero) atomicAdd(flags + kFlagZero, nzero);
    if (nborder) atomicAdd(flags + kFlagBorder, nborder);
}

// Write pass: each lane stores its partners' ranks (even slots of cs) after
// those of the lower lanes of its rank.
__global__ void k_write_pairs(int n, Ranked R, Plan pl, Grid g, const int *cell_start,
                              const int *lane_cnt) {
    const long long gid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int t = static_cast<int>(gid / kPairLanes), lane = static_cast<int>(gid % kPairLanes);
    if (t >= n) return;
    const int lim = lane_cnt[gid];
    int before = 0;
    for (int j = 0; j < lane; ++j) before += lane_cnt[gid - lane + j];
    int *part = pl.cs + 2 * static_cast<long long>(pl.cptr[t] + before);
    int k = 0;
    // the count pass used the same pure predicate, so k ends at lim; the
    // bound only guards the segment
    for_close_partners(t, lane, R, pl, g, cell_start, [&](int u, const PairGeo &) {
        if (k < lim) part[2 * k] = u;
        ++k;
    });
}

// Contacts of rank t (partners of higher rank, ascending): caller indices,
// Phi, frame [l][9] = n, tau_i, tau_j oriented from ci (lower caller index)
// to cj, and cs[l] = the ranks of (ci, cj).
__global__ void k_finish_pairs(int n, Ranked R, Plan pl, Grid g, int *ci, int *cj, double *phi,
                               double *frame) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
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
__global__ void k_second_degree(int nc, Plan pl, int *deg) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    const int a = pl.cs[2 * l], b = pl.cs[2 * l + 1];
    atomicAdd(deg + (a > b ? a : b), 1);
}

__global__ void k_inc_counts(int n, Plan pl, const int *deg) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    pl.inc_ptr[k] = (pl.cptr[k + 1] - pl.cptr[k]) + deg[k];
}

__global__ void k_inc_fill(int nc, Plan pl, int *fill) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    const int a = pl.cs[2 * l], b = pl.cs[2 * l + 1];
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    pl.inc[pl.inc_ptr[lo] + (l - pl.cptr[lo])] = 2 * l + 1;
    const int first_hi = pl.cptr[hi + 1] - pl.cptr[hi];
    pl.inc[pl.inc_ptr[hi] + first_hi + atomicAdd(fill + hi, 1)] = 2 * l;
}

// Sort the higher-rank part of each incidence list, then write the signed
// column entries: -(n, tau_i) on ci's rank, +(n, tau_j) on cj's rank.
__global__ void k_inc_finish(int n, Plan pl, const double *frame) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
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

// Nonzeros of M = D^T Mob D: contact rows l have deg(ci) + deg(cj) - 1
// entries, so the total is sum_k deg(k)^2 - n_c.
__global__ void k_deg_squares(int n, Plan pl, unsigned long long *sum) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long d2 = 0;
    if (k < n) {
        const unsigned long long d = pl.inc_ptr[k + 1] - pl.inc_ptr[k];
        d2 = d * d;
    }
    for (int off = kWave / 2; off > 0; off >>= 1)
        d2 += __shfl_xor(d2, off, kWave);
    __shared__ unsigned long long ws[kBlock / kWave];
    if (threadIdx.x % kWave == 0) ws[threadIdx.x / kWave] = d2;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += ws[w];
        if (t) atomicAdd(sum, t);
    }
}

// q_l = Phi_l / dt + D_l^T U_nc (LCP LCPdef, scaled by 1/dt).
__global__ void k_q(int nc, const int *ci, const int *cj, const double *phi,
                    const double *frame, const double *u_nc, double dt, double *q, int *flags) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    const double *f = frame + 9 * static_cast<long long>(l);
    const V3 n = load3(f), ti = load3(f + 3), tj = load3(f + 6);
    const double *ui = u_nc + 6 * static_cast<long long>(ci[l]);
    const double *uj = u_nc + 6 * static_cast<long long>(cj[l]);
    const double v = -dot(n, load3(ui)) - dot(ti, load3(ui + 3)) + dot(n, load3(uj)) +
                     dot(tj, load3(uj + 3));
    const double ql = phi[l] / dt + v;
    q[l] = ql;
    if (!isfinite(ql)) atomicOr(flags + kFlagNonfiniteQ, 1);
}

}  // namespace

size_t cell_budget(int32_t n) { return 2 * static_cast<size_t>(n) + 64; }

size_t contacts_ws_bytes(int32_t n, int32_t cap) {
    (void)cap;
    const size_t nn = static_cast<size_t>(n), nb = cell_budget(n);
    size_t b = 0;
    b += align_up(kFlagCount * sizeof(int), 256) + 256;     // flags, max extent
    b += 5 * align_up(nn * sizeof(int), 256);                // cell_of, members, cell_r, deg, fill
    b += align_up(kPairLanes * nn * sizeof(int), 256);       // per-lane pair counts
    b += align_up(4 * nn * sizeof(double), 256);             // ranked centre + radius
    b += align_up(nn * sizeof(double), 256);                 // ranked half length
    b += 2 * align_up((nb + 1) * sizeof(int), 256);          // cell_start, cell_fill
    const size_t sn = (nn + 1 > nb + 1 ? nn + 1 : nb + 1);
    b += align_up(static_cast<size_t>(scan_tmp_ints(static_cast<int>(sn))) * sizeof(int), 256);
    b += 256;                                                // host-read staging
    return b + 2048;
}

}  // namespace sc

using namespace sc;

extern "C" size_t sc_plan_bytes(int32_t n, int32_t capacity) {
    if (n < 0 || capacity < 0) return 0;
    return plan_bytes(n, capacity);
}

extern "C" int sc_build_contacts(const sc_particles *p, const sc_box *box, double delta,
                                 const double *u_nc, double dt, sc_contacts *c, void *ws,
                                 size_t ws_bytes, void *stream_) {
    if (!p || !box || !c || p->n < 0 || c->capacity < 0) return SC_ERR_INVALID;
    if (!(delta >= 0.0) || !std::isfinite(delta) || !(dt > 0.0) || !std::isfinite(dt))
        return SC_ERR_INVALID;
    for (int a = 0; a < 3; ++a)
        if (!(box->len[a] > 0.0) || !std::isfinite(box->len[a]) || !std::isfinite(box->lo[a]))
            return SC_ERR_INVALID;
    c->count = 0;
    c->n_parallel = c->n_zero_dist = c->n_borderline = 0;
    c->grid[0] = c->grid[1] = c->grid[2] = 0;
    c->nnz = 0;
    c->mat_ready = 0;
    const int n = p->n;
    Plan pl;
    if (!carve_plan(c->plan, c->plan_bytes, n, c->capacity, pl)) return SC_ERR_INVALID;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (n == 0) {
        SC_HIP_TRY(hipMemsetAsync(pl.cptr, 0, sizeof(int), stream));
        SC_HIP_TRY(hipMemsetAsync(pl.inc_ptr, 0, sizeof(int), stream));
        SC_HIP_TRY(hipStreamSynchronize(stream));
        return SC_OK;
    }
    if (!p->pos || !p->axis || !p->radius || !p->half_len || !p->mob || !u_nc) return SC_ERR_INVALID;
    if (c->capacity > 0 && (!c->ci || !c->cj || !c->phi || !c->q || !c->frame))
        return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return SC_ERR_WORKSPACE;
    if (ws_bytes < contacts_ws_bytes(n, c->capacity)) return SC_ERR_WORKSPACE;

    const size_t nb = cell_budget(n);
    Carver cv{static_cast<char *>(ws), ws_bytes};
    int *flags = cv.take<int>(kFlagCount);
    unsigned long long *max_ext = cv.take<unsigned long long>(1);
    int *cell_of = cv.take<int>(n);
    int *members = cv.take<int>(n);
    int *cell_r = cv.take<int>(n);
    int *deg = cv.take<int>(n);
    int *fill = cv.take<int>(n);
    int *lane_cnt = cv.take<int>(static_cast<size_t>(kPairLanes) * n);
    double *prec = cv.take<double>(4 * static_cast<size_t>(n));
    double *hl = cv.take<double>(n);
    int *cell_start = cv.take<int>(nb + 1);
    int *cell_fill = cv.take<int>(nb + 1);
    const int sn = static_cast<int>((static_cast<size_t>(n) + 1 > nb + 1) ? n + 1 : nb + 1);
    int *scan_tmp = cv.take<int>(scan_tmp_ints(sn));
    int *stage = cv.take<int>(16);
    if (!cv.ok) return SC_ERR_WORKSPACE;

    Parts P{n, p->pos, p->axis, p->radius, p->half_len, p->mob};
    SC_HIP_TRY(hipMemsetAsync(flags, 0, kFlagCount * sizeof(int), stream));
    SC_HIP_TRY(hipMemsetAsync(max_ext, 0, sizeof(unsigned long long), stream));
    k_validate<<<grid_for(n), kBlock, 0, stream>>>(P, max_ext, flags);
    int hflags[kFlagCount];
    unsigned long long hext = 0;
    SC_HIP_TRY(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipMemcpyAsync(&hext, max_ext, sizeof(hext), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipStreamSynchronize(stream));
    if (hflags[kFlagBadInput]) return SC_ERR_NONFINITE;

    double ext;
    {
        long long bits = static_cast<long long>(hext);
        std::memcpy(&ext, &bits, sizeof(ext));
    }
    const double rmax = 2.0 * ext + delta;
    Grid g{};
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = box->lo[a];
        g.len[a] = box->len[a];
        if (box->periodic && box->len[a] < 2.0 * rmax) return SC_ERR_BOX;
        double m = std::floor(box->len[a] / rmax);
        g.nc[a] = m < 1.0 ? 1 : (m > 1024.0 ? 1024 : static_cast<int>(m));
    }
    // keep the grid within the workspace's cell budget (bigger cells stay correct)
    while (static_cast<size_t>(g.nc[0]) * g.nc[1] * g.nc[2] > nb) {
        int a = (g.nc[0] >= g.nc[1] && g.nc[0] >= g.nc[2]) ? 0 : (g.nc[1] >= g.nc[2] ? 1 : 2);
        g.nc[a] = g.nc[a] > 1 ? (g.nc[a] + 1) / 2 : 1;
    }
    const size_t ncell = static_cast<size_t>(g.nc[0]) * g.nc[1] * g.nc[2];
    for (int a = 0; a < 3; ++a) {
        g.side[a] = box->len[a] / g.nc[a];
        c->grid[a] = g.nc[a];
    }
    g.periodic = box->periodic ? 1 : 0;
    g.delta = delta;

    // bin particles and rank them in cell order
    SC_HIP_TRY(hipMemsetAsync(cell_start, 0, (ncell + 1) * sizeof(int), stream));
    SC_HIP_TRY(hipMemsetAsync(cell_fill, 0, ncell * sizeof(int), stream));
    k_bin<<<grid_for(n), kBlock, 0, stream>>>(P, g, cell_of, cell_start);
    scan_exclusive(cell_start, cell_start, static_cast<int>(ncell), scan_tmp, stream);
    k_scatter<<<grid_for(n), kBlock, 0, stream>>>(n, cell_of, cell_start, cell_fill, members);
    k_rank<<<grid_for(n), kBlock, 0, stream>>>(P, cell_of, cell_start, members, pl, prec, hl,
                                               cell_r);
    Ranked R{prec, hl, cell_r};

    // partners of higher rank, then offsets
    const int pair_blocks = grid_for(static_cast<long long>(n) * kPairLanes);
    k_count_pairs<<<pair_blocks, kBlock, 0, stream>>>(n, R, pl, g, cell_start, lane_cnt, flags);
    scan_exclusive(pl.cptr, pl.cptr, n, scan_tmp, stream);
    SC_HIP_TRY(hipMemcpyAsync(stage, pl.cptr + n, sizeof(int), hipMemcpyDeviceToDevice, stream));
    SC_HIP_TRY(hipMemcpyAsync(stage + 1, flags, kFlagCount * sizeof(int), hipMemcpyDeviceToDevice,
                              stream));
    int hstage[1 + kFlagCount];
    SC_HIP_TRY(hipMemcpyAsync(hstage, stage, sizeof(hstage), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipStreamSynchronize(stream));
    const int nc = hstage[0];
    c->count = nc;
    c->n_parallel = hstage[1 + kFlagParallel];
    c->n_zero_dist = hstage[1 + kFlagZero];
    c->n_borderline = hstage[1 + kFlagBorder];
    if (nc > c->capacity) return SC_ERR_CAPACITY;

    k_write_pairs<<<pair_blocks, kBlock, 0, stream>>>(n, R, pl, g, cell_start, lane_cnt);
    k_finish_pairs<<<grid_for(n), kBlock, 0, stream>>>(n, R, pl, g, c->ci, c->cj, c->phi,
                                                       c->frame);
    // incidence lists and signed column entries
    SC_HIP_TRY(hipMemsetAsync(deg, 0, n * sizeof(int), stream));
    SC_HIP_TRY(hipMemsetAsync(fill, 0, n * sizeof(int), stream));
    if (nc > 0) k_second_degree<<<grid_for(nc), kBlock, 0, stream>>>(nc, pl, deg);
    k_inc_counts<<<grid_for(n), kBlock, 0, stream>>>(n, pl, deg);
    scan_exclusive(pl.inc_ptr, pl.inc_ptr, n, scan_tmp, stream);
    unsigned long long *dsq = max_ext;  // the extent word is free again
    SC_HIP_TRY(hipMemsetAsync(dsq, 0, sizeof(unsigned long long), stream));
    if (nc > 0) {
        k_inc_fill<<<grid_for(nc), kBlock, 0, stream>>>(nc, pl, fill);
        k_inc_finish<<<grid_for(n), kBlock, 0, stream>>>(n, pl, c->frame);
        k_q<<<grid_for(nc), kBlock, 0, stream>>>(nc, c->ci, c->cj, c->phi, c->frame, u_nc, dt,
                                                 c->q, flags);
        k_deg_squares<<<grid_for(n), kBlock, 0, stream>>>(n, pl, dsq);
    }
    unsigned long long hdsq = 0;
    SC_HIP_TRY(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipMemcpyAsync(&hdsq, dsq, sizeof(hdsq), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipStreamSynchronize(stream));
    SC_HIP_TRY(hipGetLastError());
    c->nnz = nc > 0 ? static_cast<int64_t>(hdsq) - nc : 0;
    if (hflags[kFlagNonfiniteQ]) return SC_ERR_NONFINITE;
    return SC_OK;
}
