// sc_matrix_pass.hpp -- device side of the assembled-M solvers shared by the
// single-instance and batched persistent kernels: the workgroup's share of
// the slices, the LDS residency of M, the one-pass product and Algorithm 1
// on one part's rows.
#pragma once

#include "sc_chain.hpp"
#include "sc_common.hpp"
#include "sc_matrix.hpp"

namespace sc {

// Slices of part L of P (a workgroup of the grid, or a member of a team),
// balanced by nonzeros: part L owns slices [s0, s1) with s0 the first slice
// whose offset reaches L * nnz / P.
struct SliceChunk {
    int s0, s1, l0, l1;  // slices and the rows they cover
};

__device__ inline int first_slice_at(const MatView &M, long long target) {
    int lo = 0, hi = M.ns;  // smallest s with soff[s] >= target
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (M.soff[mid] < target) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ inline SliceChunk slice_chunk(const MatView &M, long long L, long long G) {
    __shared__ int bounds[2];
    const long long nnz = M.soff[M.ns];
    if (threadIdx.x == 0) bounds[0] = L == 0 ? 0 : first_slice_at(M, L * nnz / G);
    if (threadIdx.x == 1) bounds[1] = L == G - 1 ? M.ns : first_slice_at(M, (L + 1) * nnz / G);
    __syncthreads();
    SliceChunk c;
    c.s0 = bounds[0];
    c.s1 = bounds[1];
    c.l0 = min(c.s0 * kWave, M.nc);
    c.l1 = min(c.s1 * kWave, M.nc);
    __syncthreads();
    return c;
}

// Diagonal of row l (depth 0 holds every row of the slice in lane order).
__device__ inline double mat_diag(const MatView &M, int l) {
    return M.val[M.soff[l / kWave] + l % kWave];
}

// Part of M kept in LDS for the whole persistent solve. The workgroup's
// dynamic LDS is split evenly over its waves; each wave walks its slices in
// its fixed processing order and keeps a prefix of each slice's entries
// until its region is full, so the fill and every pass agree on which
// entries live in LDS without any table. The rest is read from global
// memory.
extern __shared__ double sc_lds_dyn[];

struct WaveCache {
    double *val;
    int32_t *col;
    int cap;  // entries in this wave's region
};

// Entries of the wave's slices, in the order the pass visits them.
template <int R, int BS>
__device__ __forceinline__ int wave_entries(const MatView &M, const SliceChunk &ch) {
    constexpr int NW = BS / kWave;
    int e = 0;
    for (int s = ch.s0 + threadIdx.x / kWave; s < ch.s1; s += NW * R)
        for (int r = 0; r < R; ++r) {
            const int sr = s + r * NW;
            if (sr < ch.s1) e += M.soff[sr + 1] - M.soff[sr];
        }
    return __builtin_amdgcn_readfirstlane(e);
}

// Splits the workgroup's `cap` entries of LDS over its waves in proportion
// to their entries, so that all waves leave about the same share in global
// memory.
template <int R, int BS>
__device__ WaveCache wave_cache(const MatView &M, const SliceChunk &ch, int cap) {
    constexpr int NW = BS / kWave;
    __shared__ int need[NW];
    const int wv = threadIdx.x / kWave;
    const int e = wave_entries<R, BS>(M, ch);
    if (threadIdx.x % kWave == 0) need[wv] = e;
    __syncthreads();
    long long tot = 0, before = 0;
    for (int w = 0; w < NW; ++w) {
        if (w == wv) before = tot;
        tot += need[w];
    }
    __syncthreads();
    auto share = [&](long long x) {
        return tot <= cap ? x : x * cap / (tot > 0 ? tot : 1);
    };
    const long long b0 = share(before), b1 = share(before + e);
    WaveCache w;
    w.val = sc_lds_dyn + b0;
    w.col = reinterpret_cast<int32_t *>(sc_lds_dyn + cap) + b0;
    w.cap = static_cast<int>(b1 - b0);
    return w;
}

// Calls f(r, first entry, entries, LDS offset, entries in LDS) for every
// slice of the wave in processing order (R slices per step, as the pass).
template <int R, int BS, class F>
__device__ __forceinline__ void walk_wave_slices(const MatView &M, const SliceChunk &ch,
                                                 int cap, int s, int &used, F f) {
    constexpr int NW = BS / kWave;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int sr = s + r * NW;
        int e0 = 0, ne = 0;
        if (sr < ch.s1) {
            e0 = __builtin_amdgcn_readfirstlane(M.soff[sr]);
            ne = __builtin_amdgcn_readfirstlane(M.soff[sr + 1]) - e0;
        }
        const int k = min(ne, cap - used);
        f(r, e0, ne, used, k);
        used += k;
    }
}

template <int R, int BS>
__device__ void fill_cache(const MatView &M, const SliceChunk &ch, const WaveCache &W) {
    constexpr int NW = BS / kWave;
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    int used = 0;
    for (int s = ch.s0 + wv; s < ch.s1 && used < W.cap; s += NW * R)
        walk_wave_slices<R, BS>(M, ch, W.cap, s, used, [&](int, int e0, int, int at, int k) {
            for (int x = lane; x < k; x += kWave) {
                W.val[at + x] = M.val[e0 + x];
                W.col[at + x] = M.col[e0 + x];
            }
        });
    __syncthreads();
}

// Slice metadata of a wave's first kMetaGroups groups of R slices: the
// lane's row length, each slice's first entry, entry count and width. They
// do not change during a solve, so the pass reads them from registers
// instead of starting every iteration with a dependent global load.
constexpr int kMetaGroups = 2;

template <int R>
struct WaveMeta {
    int n[kMetaGroups][R], e0[kMetaGroups][R], ne[kMetaGroups][R], wid[kMetaGroups][R];
};

template <int R, int BS>
__device__ __forceinline__ void slice_meta(const MatView &M, const SliceChunk &ch, int sr,
                                           int &n, int &e0, int &ne, int &wid) {
    const int lane = threadIdx.x % kWave;
    n = e0 = ne = wid = 0;
    if (sr < ch.s1) {
        const int l = sr * kWave + lane;
        n = l < M.nc ? M.len[l] : 0;
        e0 = __builtin_amdgcn_readfirstlane(M.soff[sr]);
        ne = __builtin_amdgcn_readfirstlane(M.soff[sr + 1]) - e0;
        wid = __builtin_amdgcn_readfirstlane(M.swid[sr]);
    }
}

template <int R, int BS>
__device__ WaveMeta<R> wave_meta(const MatView &M, const SliceChunk &ch) {
    constexpr int NW = BS / kWave;
    WaveMeta<R> m;
#pragma unroll
    for (int k = 0; k < kMetaGroups; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r)
            slice_meta<R, BS>(M, ch, ch.s0 + threadIdx.x / kWave + (k * R + r) * NW, m.n[k][r],
                              m.e0[k][r], m.ne[k][r], m.wid[k][r]);
    return m;
}

// One pass over the chunk's rows: acc_l = sum_k val_k x(col_k), summed in
// storage order (so a row's value does not depend on the launch shape).
// Each wave takes R slices at a time (one lane per row). Per batch of B
// depths it reads the columns, issues every gather, then reads the values
// and accumulates. The batch has no per-entry branch, so its gathers are in
// flight together: a lane without an entry at a depth gathers its own row
// and adds nothing. pre(l) loads the row's own inputs up front; ld(m) loads
// column m's record and tf(record) gives x(m); epi(l, acc, pre) finishes the
// row. A scheduling barrier keeps every gather of a batch ahead of the first
// use of any of them (left to itself the compiler may interleave each load
// with its transform and wait for it, one round trip per entry). LDS
// residency follows the walk of fill_cache. Values of M are read from LDS, or
// for entries past the wave's share with global loads issued after the
// gathers.
template <int R, int BS, int B = 8 / R, class P, class LD, class TF, class E>
__device__ __forceinline__ void spmv_pass(const MatView &M, const SliceChunk &ch,
                                          const WaveCache &W, const WaveMeta<R> &Mt, P pre,
                                          LD ld, TF tf, E epi) {
    // B: depths per batch (8 / R measured best for 16-byte records)
    constexpr int NW = BS / kWave;
    using Pre = decltype(pre(0));
    using Xr = decltype(ld(0));
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const unsigned long long below = (1ull << lane) - 1ull;
    int used = 0;
    int n[R], pos[R], e0[R], lds0[R], nlds[R], row[R], wid;
    Pre pv[R];
    double acc[R];
    int li[R][B];
    Xr xr[R][B];
    // row metadata of slice group grp (slices s + r NW)
    auto setup = [&](int s, int grp) {
        wid = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int sr = s + r * NW;
            int ne, w;
            if (grp < kMetaGroups) {
#pragma unroll
                for (int k = 0; k < kMetaGroups; ++k)
                    if (k == grp) {
                        n[r] = Mt.n[k][r];
                        e0[r] = Mt.e0[k][r];
                        ne = Mt.ne[k][r];
                        w = Mt.wid[k][r];
                    }
            } else {
                slice_meta<R, BS>(M, ch, sr, n[r], e0[r], ne, w);
            }
            lds0[r] = used;
            nlds[r] = min(ne, W.cap - used);
            used += nlds[r];
            wid = max(wid, w);
            const int l = sr * kWave + lane;
            row[r] = min(l, M.nc - 1);  // a valid row for lanes past the end
            pos[r] = e0[r];
            pv[r] = pre(row[r]);
            acc[r] = 0.0;
        }
    };
    // columns of depths t0 .. t0 + B - 1 and their gathers
    bool spill = false;
    auto load = [&](int t0) {
        int c[R][B];
        spill = false;
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const bool on = t0 + b < n[r];
                const unsigned long long bal = __ballot(on);
                const int at = pos[r] + __popcll(bal & below);
                pos[r] += __popcll(bal);
                const int o = at - e0[r];
                const bool in_lds = on && o < nlds[r];
                spill |= on && !in_lds;
                // LDS index (0 is always a valid slot) or, if spilled, -1 - global index
                li[r][b] = in_lds ? lds0[r] + o : (on ? -1 - at : 0);
                const int cl = W.col[in_lds ? lds0[r] + o : 0];
                c[r][b] = in_lds ? cl : row[r];
            }
        }
        spill = __any(spill);
        if (spill) {  // entries of M past the wave's LDS share
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int cg = ld_global(M.col + (li[r][b] < 0 ? -1 - li[r][b] : 0));
                    c[r][b] = li[r][b] < 0 ? cg : c[r][b];
                }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int b = 0; b < B; ++b) xr[r][b] = ld(c[r][b]);
        __builtin_amdgcn_sched_barrier(0);
    };
    // values (LDS reads; global loads, in flight together, where the batch
    // holds entries past the wave's LDS share) and the products
    auto consume = [&](int t0) {
        if (spill) {
            double vg[R][B];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int b = 0; b < B; ++b)
                    vg[r][b] = ld_global(M.val + (li[r][b] < 0 ? -1 - li[r][b] : 0));
#pragma unroll
            for (int r = 0; r < R; ++r) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int k = li[r][b];
                    const double vs = W.val[k < 0 ? 0 : k];
                    const double v = k < 0 ? vg[r][b] : vs;
                    const bool on = t0 + b < n[r];
                    acc[r] += on ? v * tf(xr[r][b]) : 0.0;
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const bool on = t0 + b < n[r];
                    acc[r] += on ? W.val[li[r][b]] * tf(xr[r][b]) : 0.0;
                }
            }
        }
    };
    auto finish = [&](int s) {
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (n[r] > 0) epi((s + r * NW) * kWave + lane, acc[r], pv[r]);
    };
    int grp = 0;
    for (int s = ch.s0 + wv; s < ch.s1; s += NW * R, ++grp) {
        setup(s, grp);
        for (int t0 = 0; t0 < wid; t0 += B) {
            load(t0);
            consume(t0);
        }
        finish(s);
    }
}

__device__ inline double project(double v) { return v < 0.0 ? 0.0 : v; }

struct Ident {
    __device__ double operator()(double x) const { return x; }
};

// With one barrier per iteration, a workgroup may write the partials of
// reduction r + 1 while a slower one still reads those of reduction r, so
// consecutive reductions use alternate halves of the partials buffer (a
// workgroup cannot get two reductions ahead: the barrier holds it).
__device__ inline double *part_buf(double *part, int r, int half = kPartHalf) {
    return part + (r & 1) * half;
}

// BBPGD state per contact: (gamma, g) interleaved so that a column costs one
// 16-byte gather.
struct alignas(16) GG {
    double gam, g;
};

__device__ __forceinline__ GG ld_gg(const GG *p) {
    const auto *q = gmem(p);
    return GG{q->gam, q->g};
}

// Algorithm 1 on the rows of one part (of `nparts`) of an assembled M: the
// part's slices `rc`, its LDS share `W`, its partial-sum slot `slot`, and a
// barrier over all parts (the grid, or a team of workgroups). x0 = gamma_0
// (nullptr: zero). Partials alternate between part and part + half. Writes
// gamma and g of its own rows; part 0 writes `ctrl`.
template <int R, int BS, class Bar, int B = 8 / R>
__device__ void bbpgd_rows(const MatView &Mv, const SliceChunk &rc, const WaveCache &W,
                           const double *q, const double *x0, double *gamma, double *g,
                           GG *zb0, GG *zb1, double *part, int half, int slot, int nparts,
                           Bar &bar,
                           double tol, int max_iter, int bb, SolveCtrl *ctrl) {
    const MatView &M = Mv;
    const WaveMeta<R> Mt = wave_meta<R, BS>(M, rc);
    GG *const z[2] = {zb0, zb1};
    const int l0 = rc.l0, l1 = rc.l1;
    double alpha = 0.0, res = 0.0, tot[4];
    int iters = 0, mvops = 0, status = SC_NOT_CONVERGED, ndegen = 0;
    bool ok;

    // g0 = M gamma0 + q
    {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        GG *z0 = z[0];
        spmv_pass<R, BS>(M, rc, W, Mt, [&](int l) { return GG{x0 ? x0[l] : 0.0, q[l]}; },
                         [&](int m) { return x0 ? ld_global(x0 + m) : 0.0; }, Ident{},
                         [&](int l, double v, GG pq) {
            const double gl = v + pq.g;
            const double gm = pq.gam;
            z0[l] = GG{gm, gl};
            const double mm = gm < gl ? gm : gl;
            acc[0] += mm * mm;
            acc[1] += gl * gl;
        });
        write_partial<4, BS>(part_buf(part, 0, half), acc, slot);
    }
    ok = bar.sync();
    grid_reduce<4, BS>(part_buf(part, 0, half), tot, nparts);
    mvops = 1;
    res = sqrt(tot[0]);
    const double g0g0 = tot[1];
    int last = 0;  // buffer holding the last iterate
    if (!ok) {
        status = SC_ERR_TIMEOUT;
    } else if (!isfinite(res)) {
        status = SC_ERR_NONFINITE;
    } else if (res < tol) {
        status = SC_OK;  // gamma0 already satisfies the tolerance
    } else {
        // initial step size alpha0 = g0^T g0 / g0^T M g0 (the diagonal leads each row)
        {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            const GG *z0 = z[0];
            spmv_pass<R, BS>(M, rc, W, Mt, [&](int l) { return GG{z0[l].g, mat_diag(M, l)}; },
                             [&](int m) { return ld_global(&z0[m].g); }, Ident{},
                             [&](int l, double v, GG pd) {
                                 acc[0] += pd.gam * v;
                                 acc[1] = fmax(acc[1], pd.g);
                             });
            write_partial<4, BS, 1>(part_buf(part, 1, half), acc, slot);
        }
        ok = bar.sync();
        grid_reduce<4, BS, 1>(part_buf(part, 1, half), tot, nparts);
        mvops = 2;
        if (tot[0] > 0.0 && isfinite(tot[0]) && isfinite(g0g0)) {
            alpha = g0g0 / tot[0];
        } else {
            alpha = tot[1] > 0.0 ? 1.0 / tot[1] : 1.0;
            ++ndegen;
        }
        if (!ok) status = SC_ERR_TIMEOUT;
        for (int j = 1; ok && j <= max_iter; ++j) {
            const GG *zc = z[(j - 1) & 1];
            GG *zn = z[j & 1];
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            // projected step and new gradient in one pass: gamma_j formed per column on the fly
            struct Own {
                GG z;
                double q;
            };
            spmv_pass<R, BS, B>(
                M, rc, W, Mt, [&](int l) { return Own{ld_gg(zc + l), ld_global(q + l)}; },
                [&](int m) { return ld_gg(zc + m); },
                [&](const GG &zm) { return project(zm.gam - alpha * zm.g); },
                [&](int l, double v, const Own &o) {
                    const GG zl = o.z;
                    const double gm = project(zl.gam - alpha * zl.g);
                    const double gl = v + o.q;
                    // streamed past L2: the next barrier's write-back has less to flush
                    __builtin_nontemporal_store(gm, &gmem(zn)[l].gam);
                    __builtin_nontemporal_store(gl, &gmem(zn)[l].g);
                    const double mm = gm < gl ? gm : gl;
                    const double s = gm - zl.gam, y = gl - zl.g;
                    acc[0] += mm * mm;
                    acc[1] += s * s;
                    acc[2] += s * y;
                    acc[3] += y * y;
                });
            write_partial<4, BS>(part_buf(part, j + 1, half), acc, slot);
            ok = bar.sync();
            grid_reduce<4, BS>(part_buf(part, j + 1, half), tot, nparts);
            iters = j;
            last = j & 1;
            ++mvops;
            res = sqrt(tot[0]);
            if (!ok) {
                status = SC_ERR_TIMEOUT;
                break;
            }
            if (!isfinite(res)) {
                status = SC_ERR_NONFINITE;
                break;
            }
            if (res < tol) {
                status = SC_OK;
                break;
            }
            const bool bb2 = (bb == 2) || (bb == 3 && (j % 2 == 0));
            const double num = bb2 ? tot[2] : tot[1];
            const double den = bb2 ? tot[3] : tot[2];
            if (den > 0.0 && num > 0.0 && isfinite(num) && isfinite(den))
                alpha = num / den;
            else
                ++ndegen;
        }
    }
    // each part wrote its own rows of the last iterate; copy them out
    const GG *zf = z[last];
    for (int l = l0 + threadIdx.x; l < l1; l += BS) {
        const GG zl = zf[l];
        gamma[l] = zl.gam;
        g[l] = zl.g;
    }
    if (slot == 0 && threadIdx.x == 0) {
        SolveCtrl &c = *ctrl;
        c.alpha = alpha;
        c.res = res;
        c.iters = iters;
        c.mvops = mvops;
        c.status = status;
        c.ndegen = ndegen;
    }
}

// CG state per contact: (r_{i-1}, w_{i-1} = A r_{i-1}, s_{i-2}) interleaved,
// so that forming r_i for a column costs one 32-byte gather.
struct alignas(32) RWS {
    double r, w, s, pad;
};

__device__ __forceinline__ RWS ld_rws(const RWS *p) {
    const auto *q = gmem(p);
    return RWS{q->r, q->w, q->s, 0.0};
}

// Chronopoulos-Gear CG on M_AA (z0.r holds the masked right-hand side,
// the other fields and p, x are zero on entry). Iteration i forms
// r_i = r_{i-1} - alpha (w_{i-1} + beta s_{i-2}) per column on the fly,
// w_i = A r_i per active row (inactive rows are all zero), the row's own
// updates of p, s and x, and the dot products (r_i, r_i), (w_i, r_i).
// Runs on the rows of one part (of `nparts`) with a barrier over all parts,
// as bbpgd_rows; part 0 writes `ctrl`.
template <int R, int BS, class Bar>
__device__ void cg_rows(const MatView &M, const SliceChunk &rc, const WaveCache &W,
                        const WaveMeta<R> &Mt, const double *gamma, RWS *z0buf, RWS *z1buf,
                        double *p, double *x, double *part, int half, int slot, int nparts,
                        Bar &bar, double tol, int max_iter, CgCtrl *ctrl) {
    RWS *const z[2] = {z0buf, z1buf};
    double tot[2];
    bool ok;
    {
        double acc[2] = {0.0, 0.0};
        const RWS *z0 = z[0];
        RWS *z1 = z[1];
        spmv_pass<R, BS>(M, rc, W, Mt,
                         [&](int l) { return GG{ld_global(&z0[l].r), ld_global(gamma + l)}; },
                         [&](int m) { return ld_global(&z0[m].r); }, Ident{},
                         [&](int l, double v, GG o) {
            const double rl = o.gam;
            const double wl = o.g > 0.0 ? v : 0.0;
            auto *zo = &gmem(z1)[l];
            zo->r = rl;
            zo->w = wl;
            zo->s = 0.0;
            zo->pad = 0.0;
            acc[0] += rl * rl;
            acc[1] += wl * rl;
        });
        write_partial<2, BS>(part_buf(part, 0, half), acc, slot);
    }
    ok = bar.sync();
    grid_reduce<2, BS>(part_buf(part, 0, half), tot, nparts);
    const double bnorm2 = tot[0];
    double gam_prev = tot[0], alpha = 0.0, beta = 0.0, res = bnorm2 > 0.0 ? 1.0 : 0.0;
    int iters = 0, status = SC_NOT_CONVERGED;
    if (!ok) {
        status = SC_ERR_TIMEOUT;
    } else if (!isfinite(tot[0]) || !isfinite(tot[1])) {
        status = SC_ERR_NONFINITE;
    } else if (bnorm2 == 0.0) {
        status = SC_OK;
    } else if (tot[1] > 0.0) {
        alpha = tot[0] / tot[1];
        for (int i = 1; i <= max_iter; ++i) {
            const RWS *zc = z[i & 1];
            RWS *zn = z[(i & 1) ^ 1];
            double acc[2] = {0.0, 0.0};
            struct Own {
                RWS z;
                double p, x, act;
            };
            spmv_pass<R, BS, R == 1 ? 4 : 8 / R>(  // 24-byte records: 4 in flight (measured)

                M, rc, W, Mt,
                [&](int l) {
                    return Own{ld_rws(zc + l), ld_global(p + l), ld_global(x + l),
                               ld_global(gamma + l)};
                },
                [&](int m) { return ld_rws(zc + m); },
                [&](const RWS &zm) { return zm.r - alpha * (zm.w + beta * zm.s); },
                [&](int l, double v, const Own &o) {
                    const RWS zl = o.z;
                    const double sl = zl.w + beta * zl.s;
                    const double pl = zl.r + beta * o.p;
                    gmem(x)[l] = o.x + alpha * pl;
                    gmem(p)[l] = pl;
                    const double rl = zl.r - alpha * sl;
                    const double wl = o.act > 0.0 ? v : 0.0;
                    __builtin_nontemporal_store(rl, &gmem(zn)[l].r);
                    __builtin_nontemporal_store(wl, &gmem(zn)[l].w);
                    __builtin_nontemporal_store(sl, &gmem(zn)[l].s);
                    acc[0] += rl * rl;
                    acc[1] += wl * rl;
                });
            write_partial<2, BS>(part_buf(part, i, half), acc, slot);
            ok = bar.sync();
            grid_reduce<2, BS>(part_buf(part, i, half), tot, nparts);
            iters = i;
            res = sqrt(tot[0] / bnorm2);
            if (!ok) {
                status = SC_ERR_TIMEOUT;
                break;
            }
            if (!isfinite(tot[0]) || !isfinite(tot[1])) {
                status = SC_ERR_NONFINITE;
                break;
            }
            if (tot[0] <= tol * tol * bnorm2) {
                status = SC_OK;
                break;
            }
            beta = tot[0] / gam_prev;
            const double den = tot[1] - beta * tot[0] / alpha;
            if (!(den > 0.0)) break;  // lost positive definiteness numerically
            alpha = tot[0] / den;
            gam_prev = tot[0];
        }
    }
    if (slot == 0 && threadIdx.x == 0) {
        ctrl->alpha = alpha;
        ctrl->res = res;
        ctrl->iters = iters;
        ctrl->status = status;
    }
}

}  // namespace sc
