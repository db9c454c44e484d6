// sc_matrix.hip -- assembled M = D^T Mob D and the one-barrier persistent
// solvers built on it (gfx950).
//
// With a block-diagonal mobility, M is sparse: contacts l and m interact
// only through a shared particle k, M_lm = a_lk^T Mob_k a_mk (a_lk the signed
// column entries of contact l on particle k), so row l has
// deg(ci) + deg(cj) - 1 entries. Forming it once turns each BBPGD iteration
// into a single contact-major pass: the projected step of Algorithm 1 (steps
// 8-9) is formed on the fly for every column, g = M gamma + q (step 10) and
// the sums of steps 11 and 14-15 are accumulated, then one grid barrier and
// a fixed-order reduction decide the next step. The adjoint's masked CG is
// laid out the same way. Rows are in solver order, so column gathers stay
// local.
//
// Storage: rows are cut into slices of 64 consecutive rows, one wave and one
// lane per row. Within a slice the entries are stored depth by depth (all
// first entries of the slice's rows, then all second entries, ...) and each
// depth holds only the rows that are that long, packed in lane order. A
// wave's load at one depth is therefore one contiguous run, no padding is
// stored, and the row order (and so gather locality) is untouched. The
// position of a lane's entry at depth t is the slice offset plus the entries
// of the shallower depths plus the number of lower lanes still active at t,
// all of which the wave derives from ballots of (t < len).
#include <climits>

#include "sc_chain.hpp"
#include "sc_common.hpp"
#include "sc_matrix.hpp"
#include "sc_plan.hpp"
#include "sc_sync.hpp"

namespace sc {

namespace {

__global__ void k_row_lengths(ChainView C, int32_t *len) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= C.nc) return;
    const int ri = C.cs[2 * l], rj = C.cs[2 * l + 1];
    len[l] = (C.inc_ptr[ri + 1] - C.inc_ptr[ri]) + (C.inc_ptr[rj + 1] - C.inc_ptr[rj]) - 1;
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
    return v;
}

// Entries and widest row of every slice (one wave per slice).
__global__ void k_slice_sums(int nc, int ns, const int32_t *len, int32_t *soff, int32_t *swid) {
    const int sl = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (sl >= ns) return;  // whole waves
    const int l = sl * kWave + threadIdx.x % kWave;
    const int v = l < nc ? len[l] : 0;
    const int tot = wave_sum_int(v), wid = wave_max_int(v);
    if (threadIdx.x % kWave == 0) {
        soff[sl] = tot;
        swid[sl] = wid;
    }
}

// Walks the entries of row l in storage order: the diagonal first, then the
// other contacts of ci in ci's incidence order, then those of cj in cj's
// incidence order. M_lm = b_mk^T (Mob_k a_lk) for the shared particle k.
struct RowWalk {
    int l, ends[2], side, e, e1, own;
    V3 u, w;

    // K a_lk for the particle of `sd`, positioned on its first non-own entry;
    // returns the own entry's value (the particle's share of the diagonal).
    __device__ double open(const ChainView &C, int sd) {
        side = sd;
        const int k = ends[sd];
        e = C.inc_ptr[k];
        e1 = C.inc_ptr[k + 1];
        own = e;
        for (int x = e; x < e1; ++x)
            if ((C.inc[x] >> 1) == l) own = x;
        const double *a = C.dpm + 6 * static_cast<long long>(own);
        plan_mobility(C.pdat + 8 * static_cast<long long>(k), v3(a[0], a[1], a[2]),
                      v3(a[3], a[4], a[5]), u, w);
        if (e == own) ++e;
        return value(C, own);
    }
    __device__ double value(const ChainView &C, int x) const {
        const double *b = C.dpm + 6 * static_cast<long long>(x);
        return b[0] * u.x + b[1] * u.y + b[2] * u.z + b[3] * w.x + b[4] * w.y + b[5] * w.z;
    }
    // the diagonal; leaves the walk on the first off-diagonal entry
    __device__ double start(const ChainView &C, int row) {
        l = row;
        ends[0] = C.cs[2 * row];
        ends[1] = C.cs[2 * row + 1];
        const double d1 = open(C, 1);
        const double d0 = open(C, 0);
        settle(C);
        return d0 + d1;
    }
    __device__ void settle(const ChainView &C) {
        if (e >= e1 && side == 0) open(C, 1);
    }
    __device__ void next(const ChainView &C) {
        ++e;
        if (e == own) ++e;
        settle(C);
    }
};

// One wave per slice writes its rows depth by depth (layout in the file
// header); lanes without an entry at a depth sit out that depth's ballot.
__global__ void k_assemble(ChainView C, int ns, const int32_t *len, const int32_t *soff,
                           const int32_t *swid, int32_t *col, double *val) {
    const int sl = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (sl >= ns) return;  // whole waves
    const int lane = threadIdx.x % kWave;
    const int l = sl * kWave + lane;
    const int n = l < C.nc ? len[l] : 0;
    const unsigned long long below = (1ull << lane) - 1ull;
    int pos = soff[sl];
    const int wid = swid[sl];
    RowWalk rw;
    double diag = 0.0;
    if (n > 0) diag = rw.start(C, l);
    for (int t = 0; t < wid; ++t) {
        const bool on = t < n;
        const unsigned long long bal = __ballot(on);
        if (on) {
            const int at = pos + __popcll(bal & below);
            if (t == 0) {
                col[at] = l;
                val[at] = diag;
            } else {
                col[at] = C.inc[rw.e] >> 1;
                val[at] = rw.value(C, rw.e);
                rw.next(C);
            }
        }
        pos += __popcll(bal);
    }
}

// Slices of the workgroup, balanced by nonzeros: logical workgroup L owns
// slices [s0, s1) with s0 the first slice whose offset reaches L * nnz / G.
struct SliceChunk {
    int s0, s1, l0, l1;  // slices and the rows they cover
};

__device__ __forceinline__ int first_slice_at(const MatView &M, long long target) {
    int lo = 0, hi = M.ns;  // smallest s with soff[s] >= target
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (M.soff[mid] < target) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ SliceChunk slice_chunk(const MatView &M) {
    __shared__ int bounds[2];
    const long long L = logical_block(), G = gridDim.x;
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
__device__ __forceinline__ double mat_diag(const MatView &M, int l) {
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

// One pass over the chunk's rows: acc_l = sum_k val_k x(col_k), summed in
// storage order (so a row's value does not depend on the launch shape).
// Each wave takes R slices at a time (one lane per row). Per batch of B
// depths it reads the columns, issues every gather, then reads the values
// and accumulates. The batch has no per-entry branch, so its gathers are in
// flight together: a lane without an entry at a depth gathers its own row
// and adds nothing. pre(l) loads the row's own inputs up front; epi(l, acc,
// pre) finishes the row.
template <int R, int BS, class P, class X, class E>
__device__ __forceinline__ void spmv_pass(const MatView &M, const SliceChunk &ch,
                                          const WaveCache &W, P pre, X xf, E epi) {
    constexpr int NW = BS / kWave;
    constexpr int B = 8 / R;  // depths per batch (measured best with 1024 threads)
    using Pre = decltype(pre(0));
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const unsigned long long below = (1ull << lane) - 1ull;
    int used = 0;
    for (int s = ch.s0 + wv; s < ch.s1; s += NW * R) {
        int n[R], pos[R], e0[R], lds0[R], nlds[R], row[R];
        Pre pv[R];
        double acc[R];
        int wid = 0;
        walk_wave_slices<R, BS>(M, ch, W.cap, s, used, [&](int r, int f, int, int at, int k) {
            e0[r] = f;
            lds0[r] = at;
            nlds[r] = k;
        });
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int sr = s + r * NW;
            const bool have = sr < ch.s1;
            const int l = sr * kWave + lane;
            row[r] = min(l, M.nc - 1);  // a valid row for lanes past the end
            n[r] = have && l < M.nc ? M.len[l] : 0;
            pos[r] = e0[r];
            wid = max(wid, have ? __builtin_amdgcn_readfirstlane(M.swid[sr]) : 0);
            pv[r] = pre(row[r]);
            acc[r] = 0.0;
        }
        for (int t0 = 0; t0 < wid; t0 += B) {
            int c[R][B], li[R][B];
            bool spill = false;
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
            if (__any(spill)) {
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int b = 0; b < B; ++b)
                        if (li[r][b] < 0) c[r][b] = M.col[-1 - li[r][b]];
            }
            double x[R][B];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int b = 0; b < B; ++b) x[r][b] = xf(c[r][b]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const int k = li[r][b];
                    const double v = k < 0 ? M.val[-1 - k] : W.val[k];
                    const bool on = t0 + b < n[r];
                    acc[r] += on ? v * x[r][b] : 0.0;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (n[r] > 0) epi((s + r * NW) * kWave + lane, acc[r], pv[r]);
    }
}

__device__ __forceinline__ double project(double v) { return v < 0.0 ? 0.0 : v; }

// BBPGD state per contact: (gamma, g) interleaved so that a column costs one
// 16-byte gather.
struct GG {
    double gam, g;
};

struct MatSolve {
    MatView M;
    const double *q;
    double *gamma;          // in: gamma_0; out: last iterate
    double *g;              // out: M gamma + q
    GG *z[2];               // iterate buffers
    double *part;
    GridSync *sync;
    SolveCtrl *ctrl;
    double tol;
    int max_iter, bb;
    int cache;              // LDS entries of the workgroup
};

template <int R, int BS>
__global__ void __launch_bounds__(BS) k_bbpgd_mat(MatSolve A) {
    GridBarrier bar;
    bar.init(A.sync);
    const SliceChunk rc = slice_chunk(A.M);
    const WaveCache W = wave_cache<R, BS>(A.M, rc, A.cache);
    fill_cache<R, BS>(A.M, rc, W);
    const int l0 = rc.l0, l1 = rc.l1;
    double alpha = 0.0, res = 0.0, tot[4];
    int iters = 0, mvops = 0, status = SC_NOT_CONVERGED, ndegen = 0;
    bool ok;

    // step 2: g0 = M gamma0 + q
    {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const double *x = A.gamma;
        GG *z0 = A.z[0];
        spmv_pass<R, BS>(A.M, rc, W, [&](int l) { return GG{x[l], A.q[l]}; },
                              [&](int m) { return x[m]; }, [&](int l, double v, GG pq) {
            const double gl = v + pq.g;
            const double gm = pq.gam;
            z0[l] = GG{gm, gl};
            const double mm = gm < gl ? gm : gl;
            acc[0] += mm * mm;
            acc[1] += gl * gl;
        });
        write_partial<4, BS>(A.part, acc);
    }
    ok = bar.sync();
    grid_reduce<4, BS>(A.part, tot);
    mvops = 1;
    res = sqrt(tot[0]);
    const double g0g0 = tot[1];
    int last = 0;  // buffer holding the last iterate
    if (!ok) {
        status = SC_ERR_TIMEOUT;
    } else if (!isfinite(res)) {
        status = SC_ERR_NONFINITE;
    } else if (res < A.tol) {
        status = SC_OK;  // steps 3-5
    } else {
        // step 6: alpha0 = g0^T g0 / g0^T M g0 (the diagonal leads each row)
        {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            const GG *z0 = A.z[0];
            spmv_pass<R, BS>(A.M, rc, W,
                                  [&](int l) { return GG{z0[l].g, mat_diag(A.M, l)}; },
                                  [&](int m) { return z0[m].g; },
                                  [&](int l, double v, GG pd) {
                                      acc[0] += pd.gam * v;
                                      acc[1] = fmax(acc[1], pd.g);
                                  });
            write_partial<4, BS, 1>(A.part, acc);
        }
        ok = bar.sync();
        grid_reduce<4, BS, 1>(A.part, tot);
        mvops = 2;
        if (tot[0] > 0.0 && isfinite(tot[0]) && isfinite(g0g0)) {
            alpha = g0g0 / tot[0];
        } else {
            alpha = tot[1] > 0.0 ? 1.0 / tot[1] : 1.0;
            ++ndegen;
        }
        if (!ok) status = SC_ERR_TIMEOUT;
        for (int j = 1; ok && j <= A.max_iter; ++j) {
            const GG *zc = A.z[(j - 1) & 1];
            GG *zn = A.z[j & 1];
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            // steps 8-10 in one pass: gamma_j formed per column on the fly
            struct Own {
                GG z;
                double q;
            };
            spmv_pass<R, BS>(
                A.M, rc, W, [&](int l) { return Own{zc[l], A.q[l]}; },
                [&](int m) {
                    const GG zm = zc[m];
                    return project(zm.gam - alpha * zm.g);
                },
                [&](int l, double v, const Own &o) {
                    const GG zl = o.z;
                    const double gm = project(zl.gam - alpha * zl.g);
                    const double gl = v + o.q;
                    zn[l] = GG{gm, gl};
                    const double mm = gm < gl ? gm : gl;
                    const double s = gm - zl.gam, y = gl - zl.g;
                    acc[0] += mm * mm;
                    acc[1] += s * s;
                    acc[2] += s * y;
                    acc[3] += y * y;
                });
            write_partial<4, BS>(A.part, acc);
            ok = bar.sync();
            grid_reduce<4, BS>(A.part, tot);
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
            if (res < A.tol) {
                status = SC_OK;
                break;
            }
            const bool bb2 = (A.bb == 2) || (A.bb == 3 && (j % 2 == 0));
            const double num = bb2 ? tot[2] : tot[1];
            const double den = bb2 ? tot[3] : tot[2];
            if (den > 0.0 && num > 0.0 && isfinite(num) && isfinite(den))
                alpha = num / den;
            else
                ++ndegen;
        }
    }
    // each workgroup wrote its own rows of the last iterate; copy them out
    const GG *zf = A.z[last];
    for (int l = l0 + threadIdx.x; l < l1; l += BS) {
        const GG zl = zf[l];
        A.gamma[l] = zl.gam;
        A.g[l] = zl.g;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        SolveCtrl &c = *A.ctrl;
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
struct RWS {
    double r, w, s, pad;
};

struct MatCg {
    MatView M;
    const double *gamma;
    RWS *z[2];
    double *p, *x;
    double *part;
    GridSync *sync;
    CgCtrl *ctrl;
    double tol;
    int max_iter;
    int cache;              // LDS entries of the workgroup
};

// Chronopoulos-Gear CG on M_AA (z[0].r holds the masked right-hand side,
// the other fields and p, x are zero on entry). Iteration i forms
// r_i = r_{i-1} - alpha (w_{i-1} + beta s_{i-2}) per column on the fly,
// w_i = A r_i per active row (inactive rows are all zero), the row's own
// updates of p, s and x, and the dot products (r_i, r_i), (w_i, r_i).
template <int R, int BS>
__global__ void __launch_bounds__(BS) k_cg_mat(MatCg A) {
    GridBarrier bar;
    bar.init(A.sync);
    const SliceChunk rc = slice_chunk(A.M);
    const WaveCache W = wave_cache<R, BS>(A.M, rc, A.cache);
    fill_cache<R, BS>(A.M, rc, W);
    double tot[2];
    bool ok;
    {
        double acc[2] = {0.0, 0.0};
        const RWS *z0 = A.z[0];
        RWS *z1 = A.z[1];
        spmv_pass<R, BS>(A.M, rc, W, [&](int l) { return GG{z0[l].r, A.gamma[l]}; },
                              [&](int m) { return z0[m].r; }, [&](int l, double v, GG o) {
            const double rl = o.gam;
            const double wl = o.g > 0.0 ? v : 0.0;
            z1[l] = RWS{rl, wl, 0.0, 0.0};
            acc[0] += rl * rl;
            acc[1] += wl * rl;
        });
        write_partial<2, BS>(A.part, acc);
    }
    ok = bar.sync();
    grid_reduce<2, BS>(A.part, tot);
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
        for (int i = 1; i <= A.max_iter; ++i) {
            const RWS *zc = A.z[i & 1];
            RWS *zn = A.z[(i & 1) ^ 1];
            double acc[2] = {0.0, 0.0};
            struct Own {
                RWS z;
                double p, x, act;
            };
            spmv_pass<R, BS>(
                A.M, rc, W, [&](int l) { return Own{zc[l], A.p[l], A.x[l], A.gamma[l]}; },
                [&](int m) {
                    const RWS zm = zc[m];
                    return zm.r - alpha * (zm.w + beta * zm.s);
                },
                [&](int l, double v, const Own &o) {
                    const RWS zl = o.z;
                    const double sl = zl.w + beta * zl.s;
                    const double pl = zl.r + beta * o.p;
                    A.x[l] = o.x + alpha * pl;
                    A.p[l] = pl;
                    const double rl = zl.r - alpha * sl;
                    const double wl = o.act > 0.0 ? v : 0.0;
                    zn[l] = RWS{rl, wl, sl, 0.0};
                    acc[0] += rl * rl;
                    acc[1] += wl * rl;
                });
            write_partial<2, BS>(A.part, acc);
            ok = bar.sync();
            grid_reduce<2, BS>(A.part, tot);
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
            if (tot[0] <= A.tol * A.tol * bnorm2) {
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
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.ctrl->alpha = alpha;
        A.ctrl->res = res;
        A.ctrl->iters = iters;
        A.ctrl->status = status;
    }
}

using BbMatKernel = void (*)(MatSolve);
using CgMatKernel = void (*)(MatCg);

template <int BS>
BbMatKernel bb_mat_bs(int spw) {
    switch (spw) {
    case 2: return k_bbpgd_mat<2, BS>;
    case 4: return k_bbpgd_mat<4, BS>;
    default: return k_bbpgd_mat<1, BS>;
    }
}

template <int BS>
CgMatKernel cg_mat_bs(int spw) {
    switch (spw) {
    case 2: return k_cg_mat<2, BS>;
    case 4: return k_cg_mat<4, BS>;
    default: return k_cg_mat<1, BS>;
    }
}

}  // namespace

size_t matrix_bytes(int32_t nc, int64_t nnz) {
    if (nc < 0 || nnz < 0 || nnz > INT_MAX) return 0;
    const size_t cc = static_cast<size_t>(nc), zz = static_cast<size_t>(nnz);
    const size_t ns = static_cast<size_t>(slices(nc));
    return align_up(cc * sizeof(int32_t), 256) + align_up((ns + 1) * sizeof(int32_t), 256) +
           align_up(ns * sizeof(int32_t), 256) + align_up(zz * sizeof(int32_t), 256) +
           align_up(zz * sizeof(double), 256) +
           align_up(static_cast<size_t>(scan_tmp_ints(slices(nc) + 1)) * sizeof(int32_t), 256) +
           256;
}

bool carve_matrix(void *base, size_t bytes, int32_t nc, int64_t nnz, MatBufs &m) {
    const size_t need = matrix_bytes(nc, nnz);
    if (!base || need == 0 || bytes < need || (reinterpret_cast<uintptr_t>(base) & 255) != 0)
        return false;
    Carver cv{static_cast<char *>(base), bytes};
    const int ns = slices(nc);
    m.ns = ns;
    m.len = cv.take<int32_t>(static_cast<size_t>(nc));
    m.soff = cv.take<int32_t>(static_cast<size_t>(ns) + 1);
    m.swid = cv.take<int32_t>(static_cast<size_t>(ns));
    m.col = cv.take<int32_t>(static_cast<size_t>(nnz));
    m.val = cv.take<double>(static_cast<size_t>(nnz));
    m.scan_tmp = cv.take<int32_t>(scan_tmp_ints(ns + 1));
    return cv.ok;
}

MatView mat_view(int32_t nc, const MatBufs &m) {
    return MatView{nc, m.ns, m.len, m.soff, m.swid, m.col, m.val};
}

namespace {

// Dynamic LDS for the matrix cache of a persistent kernel: everything the
// workgroup does not use statically, at 12 bytes per entry (value and
// column). `request`: 0 = as much as fits, < 0 = none, > 0 = at most that
// many entries per wave. *per_wave is the workgroup's entries over its waves.
hipError_t cache_shape(const void *fn, int block, int request, int *per_wave, size_t *dyn) {
    *per_wave = 0;
    *dyn = 16;  // the pass reads slot 0 unconditionally
    if (request < 0) return hipSuccess;
    int dev = 0, max_lds = 0;
    hipFuncAttributes fa;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess) e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    const int nw = block / kWave;
    const long long room = static_cast<long long>(max_lds) - static_cast<long long>(fa.sharedSizeBytes) - 256;
    long long per = room > 0 ? room / (12LL * nw) : 0;
    per -= per % 2;  // keeps the column block 8-byte aligned
    if (request > 0 && per > request) per = request - request % 2;
    if (per < 2) return hipSuccess;
    *per_wave = static_cast<int>(per);
    *dyn = static_cast<size_t>(per) * 12 * nw;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(*dyn));
}

}  // namespace

hipError_t launch_bbpgd_mat(const MatView &M, const double *q, double *gamma, double *g,
                            double *zbuf, double *part, GridSync *sync, SolveCtrl *ctrl,
                            double tol, int max_iter, int bb, int spw, int cache, int block,
                            int grid, hipStream_t s, int *grid_used, int *cache_used) {
    BbMatKernel kern = block == 256   ? bb_mat_bs<256>(spw)
                       : block == 512 ? bb_mat_bs<512>(spw)
                                      : bb_mat_bs<1024>(spw);
    const void *fn = reinterpret_cast<const void *>(kern);
    size_t dyn = 0;
    int per = 0;
    hipError_t e = cache_shape(fn, block, cache, &per, &dyn);
    if (e != hipSuccess) return e;
    *cache_used = per;
    const int G = persistent_grid(fn, block, grid, dyn);
    *grid_used = G;
    if (G < 1) return hipErrorInvalidConfiguration;
    MatSolve A;
    A.M = M;
    A.q = q;
    A.gamma = gamma;
    A.g = g;
    A.z[0] = reinterpret_cast<GG *>(zbuf);
    A.z[1] = reinterpret_cast<GG *>(zbuf) + M.nc;
    A.part = part;
    A.sync = sync;
    A.ctrl = ctrl;
    A.tol = tol;
    A.max_iter = max_iter;
    A.bb = bb;
    A.cache = per * (block / kWave);
    void *args[] = {&A};
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(block), args, dyn, s);
}

hipError_t launch_cg_mat(const MatView &M, const double *gamma, double *zbuf, double *p,
                         double *x, double *part, GridSync *sync, CgCtrl *ctrl, double tol,
                         int max_iter, int spw, int cache, int block, int grid, hipStream_t s,
                         int *grid_used, int *cache_used) {
    CgMatKernel kern = block == 256   ? cg_mat_bs<256>(spw)
                       : block == 512 ? cg_mat_bs<512>(spw)
                                      : cg_mat_bs<1024>(spw);
    const void *fn = reinterpret_cast<const void *>(kern);
    size_t dyn = 0;
    int per = 0;
    hipError_t e = cache_shape(fn, block, cache, &per, &dyn);
    if (e != hipSuccess) return e;
    *cache_used = per;
    const int G = persistent_grid(fn, block, grid, dyn);
    *grid_used = G;
    if (G < 1) return hipErrorInvalidConfiguration;
    MatCg A;
    A.M = M;
    A.gamma = gamma;
    A.z[0] = reinterpret_cast<RWS *>(zbuf);
    A.z[1] = reinterpret_cast<RWS *>(zbuf) + M.nc;
    A.p = p;
    A.x = x;
    A.part = part;
    A.sync = sync;
    A.ctrl = ctrl;
    A.tol = tol;
    A.max_iter = max_iter;
    A.cache = per * (block / kWave);
    void *args[] = {&A};
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(block), args, dyn, s);
}

}  // namespace sc

using namespace sc;

extern "C" size_t sc_matrix_bytes(int32_t count, int64_t nnz) {
    return matrix_bytes(count, nnz);
}

extern "C" int sc_assemble_matrix(const sc_particles *p, sc_contacts *c, void *stream) {
    if (!p || !c || p->n < 0 || c->count < 0 || c->count > c->capacity) return SC_ERR_INVALID;
    c->mat_ready = 0;
    Plan pl;
    if (!carve_plan(c->plan, c->plan_bytes, p->n, c->capacity, pl)) return SC_ERR_INVALID;
    MatBufs mb;
    if (!carve_matrix(c->mat, c->mat_bytes, c->count, c->nnz, mb)) return SC_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nc = c->count;
    if (nc > 0) {
        const ChainView C = chain_view(p, c, pl, nullptr);
        const int per = kBlock / kWave;  // slices per workgroup
        k_row_lengths<<<grid_for(nc), kBlock, 0, s>>>(C, mb.len);
        k_slice_sums<<<(mb.ns + per - 1) / per, kBlock, 0, s>>>(nc, mb.ns, mb.len, mb.soff,
                                                              mb.swid);
        scan_exclusive(mb.soff, mb.soff, mb.ns, mb.scan_tmp, s);
        k_assemble<<<(mb.ns + per - 1) / per, kBlock, 0, s>>>(C, mb.ns, mb.len, mb.soff, mb.swid,
                                                            mb.col, mb.val);
    } else {
        SC_HIP_TRY(hipMemsetAsync(mb.soff, 0, sizeof(int32_t), s));
    }
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    c->mat_ready = 1;
    return SC_OK;
}
