// sc_solve.hip -- BBPGD (Algorithm 1, section 3.3.1) as one persistent,
// cooperative kernel on gfx950, plus single-launch products.
//
// One iteration is two passes of the chain (sc_chain.hpp) separated by grid
// barriers (sc_sync.hpp):
//   pass A: gamma_j = max(0, gamma_{j-1} - alpha g_{j-1}) formed on the fly
//     for every incidence (the projected descent step; the owning incidence
//     stores it), and U = Mob D gamma_j;
//   pass B: g_j = D^T U + q (the new gradient) with the partial sums of
//     ||min(gamma_j, g_j)||^2 (Eq. mmapnorm), s^T s, s^T y and y^T y.
// After the second barrier every workgroup reduces all partials in the same
// fixed order and takes the same decision: stop, or the next BB step size.
// No floating-point atomics are used, so the iterates are
// bitwise reproducible for a given launch shape.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>

#include "sc_chain.hpp"
#include "sc_chain_lds.hpp"
#include "sc_common.hpp"
#include "sc_matrix.hpp"
#include "sc_matrix_pass.hpp"
#include "sc_plan.hpp"
#include "sc_sync.hpp"

namespace sc {

namespace {

using Ctrl = SolveCtrl;

struct SolveArgs {
    ChainView C;
    const double *q;
    double *gamma;         // in: gamma_0 (if warm); out: the last iterate
    double *g;             // out: M gamma + q
    GG *z[2];              // (gamma_j, g_j) records, alternating per iteration
    double *part;          // [G][4]
    GridSync *sync;
    Ctrl *ctrl;
    double tol;
    int max_iter, bb;
    int warm;
    int rank_cap;  // dynamic LDS of the chain: incidence ranges of up to rank_cap - 1 ranks
    int inc_cap;   //   and the codes and D columns of the workgroup's first inc_cap incidences
};

__device__ __forceinline__ double m_diag(const ChainView &C, int l) {
    // M_ll = D_l^T Mob D_l
    const int ri = C.cs[2 * l], rj = C.cs[2 * l + 1];
    const double *f = C.frame + 9 * static_cast<long long>(l);
    const V3 n = load3(f), ti = load3(f + 3), tj = load3(f + 6);
    V3 ui, wi, uj, wj;
    plan_mobility(C.pdat + 8 * static_cast<long long>(ri), n, ti, ui, wi);
    if (rj < 0) return dot(n, ui) + dot(ti, wi);  // wall contact
    plan_mobility(C.pdat + 8 * static_cast<long long>(rj), n, tj, uj, wj);
    return dot(n, ui) + dot(ti, wi) + dot(n, uj) + dot(tj, wj);
}

// Matrix-free BBPGD. The iterate lives in (gamma, g) records, one 16-byte
// record per contact, so that pass A forms every projected step
// gamma_j = max(0, gamma_{j-1} - alpha g_{j-1}) from one gather and stores
// nothing, and pass B, which evaluates the same expression for its own
// contacts (the same bits), writes each contact's new record in one
// coalesced store.
template <int LPP, int BS>
__global__ void __launch_bounds__(BS) k_bbpgd(SolveArgs A) {
    GridBarrier bar;
    bar.init(A.sync);
    const ChainView &C = A.C;
    int k0, k1, l0, l1;
    chunk(C.n, k0, k1);
    chunk(C.nc, l0, l1);
    const ChainLds L = chain_lds_fill(C, A.rank_cap, A.inc_cap, k0, k1);

    double alpha = 0.0, res = 0.0;
    int iters = 0, mvops = 0, status = SC_NOT_CONVERGED, ndegen = 0, last = 0;
    bool ok = true;
    const double *x0 = A.warm ? A.gamma : nullptr;

    // g0 = M gamma0 + q
    pass_a_lds<LPP, BS>(C, L, k0, k1, [&](int code, int) {
        return x0 ? ld_global(x0 + (code >> 1)) : 0.0;
    });
    ok = bar.sync();
    {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        GG *z0 = A.z[0];
        for (int l = l0 + threadIdx.x; l < l1; l += BS) {
            const double gl = dt_u(C, l) + A.q[l];
            const double gm = x0 ? x0[l] : 0.0;
            __builtin_nontemporal_store(gm, &gmem(z0)[l].gam);
            __builtin_nontemporal_store(gl, &gmem(z0)[l].g);
            const double m = gm < gl ? gm : gl;
            acc[0] += m * m;
            acc[1] += gl * gl;
        }
        write_partial<4, BS>(A.part, acc);
    }
    ok = ok && bar.sync();
    double tot[4];
    grid_reduce<4, BS>(A.part, tot);
    mvops = 1;
    res = sqrt(tot[0]);
    const double g0g0 = tot[1];
    if (!ok) {
        status = SC_ERR_TIMEOUT;
    } else if (!isfinite(res)) {
        status = SC_ERR_NONFINITE;
    } else if (res < A.tol) {
        status = SC_OK;  // gamma0 already satisfies the tolerance
    } else {
        // initial step size alpha0 = g0^T g0 / g0^T M g0
        const GG *z0 = A.z[0];
        pass_a_lds<LPP, BS>(C, L, k0, k1,
                            [&](int code, int) { return ld_gg(z0 + (code >> 1)).g; });
        ok = bar.sync();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int l = l0 + threadIdx.x; l < l1; l += BS) {
            acc[0] += z0[l].g * dt_u(C, l);
            acc[1] = fmax(acc[1], m_diag(C, l));
        }
        write_partial<4, BS, 1>(A.part, acc);
        ok = ok && bar.sync();
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
            // pass A: the projected step formed per incidence from one record
            pass_a_lds<LPP, BS>(C, L, k0, k1, [&](int code, int) {
                const GG zm = ld_gg(zc + (code >> 1));
                return project(zm.gam - alpha * zm.g);
            });
            ok = bar.sync();
            // pass B: new records, residual and BB sums
            double acc2[4] = {0.0, 0.0, 0.0, 0.0};
            for (int l = l0 + threadIdx.x; l < l1; l += BS) {
                const GG zl = ld_gg(zc + l);
                const double gm = project(zl.gam - alpha * zl.g);
                const double gl = dt_u(C, l) + A.q[l];
                __builtin_nontemporal_store(gm, &gmem(zn)[l].gam);
                __builtin_nontemporal_store(gl, &gmem(zn)[l].g);
                const double m = gm < gl ? gm : gl;
                const double s = gm - zl.gam;
                const double y = gl - zl.g;
                acc2[0] += m * m;
                acc2[1] += s * s;
                acc2[2] += s * y;
                acc2[3] += y * y;
            }
            write_partial<4, BS>(A.part, acc2);
            ok = ok && bar.sync();
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
    // every workgroup copies out its own contacts of the last iterate
    const GG *zf = A.z[last];
    for (int l = l0 + threadIdx.x; l < l1; l += BS) {
        const GG zl = zf[l];
        A.gamma[l] = zl.gam;
        A.g[l] = zl.g;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctrl &c = *A.ctrl;
        c.alpha = alpha;
        c.res = res;
        c.iters = iters;
        c.mvops = mvops;
        c.status = status;
        c.ndegen = ndegen;
    }
}

// Single-launch products on the solver layout.
template <int LPP>
__global__ void __launch_bounds__(kBlock)
k_mob_d(ChainView C, const double *x, const int *order, double *f_out, double *u_out) {
    // one logical chunk per workgroup over all ranks
    int k0, k1;
    chunk(C.n, k0, k1);
    pass_a<LPP, kBlock>(C, k0, k1, [&](int code, int) { return x[code >> 1]; });
    if (!f_out && !u_out) return;
    __syncthreads();
    // scatter to caller order; F is recomputed from U = Mob F by a second
    // gather only when requested
    for (int k = k0 + threadIdx.x; k < k1; k += kBlock) {
        const long long o = 6 * static_cast<long long>(order[k]);
        const double *Uk = C.U + 8 * static_cast<long long>(k);
        if (u_out)
            for (int a = 0; a < 6; ++a) u_out[o + a] = Uk[a];
        if (f_out) {
            double f[6] = {0, 0, 0, 0, 0, 0};
            for (int e = C.inc_ptr[k]; e < C.inc_ptr[k + 1]; ++e) {
                const double w = x[C.inc[e] >> 1];
                const double *d = C.dpm + 6 * static_cast<long long>(e);
                for (int a = 0; a < 6; ++a) f[a] += w * d[a];
            }
            for (int a = 0; a < 6; ++a) f_out[o + a] = f[a];
        }
    }
}

__global__ void k_dt(ChainView C, double *y) {
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < C.nc; l += gridDim.x * blockDim.x)
        y[l] = dt_u(C, l);
}

__global__ void k_count_active(int nc, const double *gamma, int *count) {
    int cnt = 0;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < nc; l += gridDim.x * blockDim.x)
        cnt += gamma[l] > 0.0;
    for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
    __shared__ int ws[kBlock / kWave];
    if (threadIdx.x % kWave == 0) ws[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kBlock / kWave; ++w) s += ws[w];
        if (s) atomicAdd(count, s);
    }
}

__global__ void k_mobility(int n, const double *axis, const double *mob, const double *f,
                           double *u) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    V3 uu, ww;
    const double *fk = f + 6 * static_cast<long long>(k);
    mobility_apply(load3(axis + 3 * k), mob + 4 * k, load3(fk), load3(fk + 3), uu, ww);
    store3(u + 6 * static_cast<long long>(k), uu);
    store3(u + 6 * static_cast<long long>(k) + 3, ww);
}

struct Timing {
    hipEvent_t t0 = nullptr, t1 = nullptr;
    bool ok = false;
};

thread_local Timing tl_timing;

Timing &timing() {
    Timing &tm = tl_timing;
    if (!tm.ok) {
        if (hipEventCreate(&tm.t0) != hipSuccess || hipEventCreate(&tm.t1) != hipSuccess)
            return tm;
        tm.ok = true;
    }
    return tm;
}

using BbKernel = void (*)(SolveArgs);

template <int BS>
BbKernel bb_kernel_bs(int lpp) {
    switch (lpp) {
    case 1: return k_bbpgd<1, BS>;
    case 2: return k_bbpgd<2, BS>;
    case 8: return k_bbpgd<8, BS>;
    default: return k_bbpgd<4, BS>;
    }
}

BbKernel bb_kernel(int lpp, int block) {
    return block == 256 ? bb_kernel_bs<256>(lpp)
                        : block == 512 ? bb_kernel_bs<512>(lpp) : bb_kernel_bs<1024>(lpp);
}

// Largest co-resident grid for a persistent kernel (cached per kernel and
// dynamic LDS size) and the number of CUs.
int max_coresident(const void *fn, int block, size_t dyn, int *cus) {
    static thread_local const void *last_fn = nullptr;
    static thread_local size_t last_dyn = 0;
    static thread_local int last = 0, last_cus = 0;
    if (fn != last_fn || dyn != last_dyn) {
        int per_cu = 0, dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipGetDeviceProperties(&prop, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, dyn) != hipSuccess)
            return 0;
        last_fn = fn;
        last_dyn = dyn;
        last = per_cu * prop.multiProcessorCount;
        last_cus = prop.multiProcessorCount;
    }
    *cus = last_cus;
    return last;
}

}  // namespace

bool thread_events(hipEvent_t *t0, hipEvent_t *t1) {
    Timing &tm = timing();
    if (!tm.ok) return false;
    *t0 = tm.t0;
    *t1 = tm.t1;
    return true;
}

// Destroys the calling thread's timing events (recreated on the next timed
// solve).
void release_solve_host() {
    Timing &tm = tl_timing;
    if (tm.t0) (void)hipEventDestroy(tm.t0);
    if (tm.t1) (void)hipEventDestroy(tm.t1);
    tm = Timing{};
}

// At most one workgroup per CU: with two 1024-thread workgroups per CU the
// occupancy query allowed the launch, yet the start-up barrier of one
// kernel variant timed out waiting for workgroups that never became
// resident, so larger grids are not used.
int persistent_grid(const void *fn, int block, int requested, size_t dyn) {
    int cus = 0;
    const int cap = max_coresident(fn, block, dyn, &cus);
    int g = requested > 0 ? requested : cus;
    if (g > cap) g = cap;
    if (g > cus) g = cus;
    if (g > kMaxReduceBlocks) g = kMaxReduceBlocks;
    if (g >= 8) g -= g % 8;
    return g < 1 ? 1 : g;
}

ChainView chain_view(const sc_particles *p, const sc_contacts *c, const Plan &pl, double *U) {
    return ChainView{p->n, c->count, pl.pdat, pl.inc_ptr, pl.inc, pl.dpm, pl.cs, c->frame, U};
}

void launch_mob_d(const ChainView &C, const double *x, const int *order, double *f_out,
                  double *u_out, hipStream_t s) {
    if (C.n <= 0) return;
    const int blocks = grid_for(C.n, kBlock / 4);
    k_mob_d<4><<<blocks, kBlock, 0, s>>>(C, x, order, f_out, u_out);
}

void launch_dt(const ChainView &C, double *y, hipStream_t s) {
    if (C.nc <= 0) return;
    int b = grid_for(C.nc);
    if (b > kMaxReduceBlocks) b = kMaxReduceBlocks;
    k_dt<<<b, kBlock, 0, s>>>(C, y);
}

size_t solve_ws_bytes(int32_t n, int32_t cap) {
    const size_t nn = static_cast<size_t>(n), cc = static_cast<size_t>(cap);
    size_t b = 0;
    b += align_up(4 * cc * sizeof(double), 256);          // second gamma/g buffers or (gamma, g) records
    b += align_up(8 * nn * sizeof(double), 256);          // U (rank order)
    b += align_up(2 * kPartHalf * sizeof(double), 256);
    b += align_up(sizeof(GridSync), 256);
    b += align_up(sizeof(Ctrl), 256);
    return b + 2048;
}

}  // namespace sc

using namespace sc;

namespace {

int check_common(const sc_particles *p, const sc_contacts *c, Plan &pl) {
    if (!p || !c || p->n < 0 || c->count < 0 || c->count > c->capacity) return SC_ERR_INVALID;
    if (!carve_plan(c->plan, c->plan_bytes, p->n, c->capacity, pl)) return SC_ERR_INVALID;
    if (c->count > 0 && (!c->ci || !c->cj || !c->frame || !c->q)) return SC_ERR_INVALID;
    return SC_OK;
}

bool ws_ok(void *ws, size_t ws_bytes, size_t need) {
    return ws && (reinterpret_cast<uintptr_t>(ws) & 255) == 0 && ws_bytes >= need;
}

}  // namespace

extern "C" int sc_apply_mobility(const sc_particles *p, const double *f, double *u,
                                 void *stream) {
    if (!p || p->n < 0) return SC_ERR_INVALID;
    if (p->n == 0) return SC_OK;
    if (!f || !u || !p->axis || !p->mob) return SC_ERR_INVALID;
    k_mobility<<<grid_for(p->n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
        p->n, p->axis, p->mob, f, u);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}

extern "C" int sc_mvop(const sc_particles *p, const sc_contacts *c, const double *x, double *y,
                       void *ws, size_t ws_bytes, void *stream) {
    Plan pl;
    int rc = check_common(p, c, pl);
    if (rc) return rc;
    if (c->count == 0) return SC_OK;
    if (!x || !y) return SC_ERR_INVALID;
    if (!ws_ok(ws, ws_bytes, solve_ws_bytes(p->n, c->capacity))) return SC_ERR_WORKSPACE;
    Carver cv{static_cast<char *>(ws), ws_bytes};
    cv.take<double>(4 * static_cast<size_t>(c->capacity));
    double *U = cv.take<double>(8 * static_cast<size_t>(p->n));
    if (!cv.ok) return SC_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const ChainView C = chain_view(p, c, pl, U);
    launch_mob_d(C, x, pl.order, nullptr, nullptr, s);
    launch_dt(C, y, s);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}

namespace {

// Checked arguments, carved workspace and launch choice of one solve.
struct Prepared {
    Plan pl;
    bool use_mat = false;
    MatBufs mb{};
    double *zbuf = nullptr, *U = nullptr, *part = nullptr;
    GridSync *sync = nullptr;
    Ctrl *ctrl = nullptr;
    int lpp = 4, spw = 1, block = 1024, G = 1, cache_used = 0;
    BbKernel kern = nullptr;
    SolveArgs A{};
};

// The solve's argument checks (everything but the workspace): the plan and
// the assembled matrix are carved, the product chosen. Host arithmetic only.
int check_args(const sc_particles *p, const sc_contacts *c, const sc_solve_opts *opts,
               const double *gamma, const double *g, Plan &pl, bool &use_mat, MatBufs &mb) {
    int rc = check_common(p, c, pl);
    if (rc) return rc;
    if (!opts) return SC_ERR_INVALID;
    if (!(opts->tol > 0.0) || opts->max_iter < 0 || opts->bb < 1 || opts->bb > 3 ||
        !lanes_ok(opts->lanes_per_particle) || !spw_ok(opts->slices_per_wave) ||
        opts->lds_entries_per_wave < -1 || opts->grid < 0 || opts->spin_limit < 0 ||
        !block_ok(opts->block) || opts->op < 0 ||
        opts->op > SC_OP_MATRIX || (opts->op == SC_OP_MATRIX && !c->mat_ready))
        return SC_ERR_INVALID;
    use_mat = opts->op == SC_OP_MATRIX || (opts->op == SC_OP_AUTO && c->mat_ready);
    if (use_mat && !carve_matrix(c->mat, c->mat_bytes, c->count, c->nnz, mb))
        return SC_ERR_INVALID;
    if (c->count > 0 && (!gamma || !g)) return SC_ERR_INVALID;
    return SC_OK;
}

int prepare(const sc_particles *p, const sc_contacts *c, const sc_solve_opts *opts,
            double *gamma, double *g, void *ws, size_t ws_bytes, Prepared &P) {
    int rc = check_args(p, c, opts, gamma, g, P.pl, P.use_mat, P.mb);
    if (rc) return rc;
    const int n = p->n;
    if (!ws_ok(ws, ws_bytes, solve_ws_bytes(n, c->capacity))) return SC_ERR_WORKSPACE;
    Carver cv{static_cast<char *>(ws), ws_bytes};
    P.zbuf = cv.take<double>(4 * static_cast<size_t>(c->capacity));
    P.U = cv.take<double>(8 * static_cast<size_t>(n));
    P.part = cv.take<double>(2 * kPartHalf);
    P.sync = cv.take<GridSync>(1);
    P.ctrl = cv.take<Ctrl>(1);
    if (!cv.ok) return SC_ERR_WORKSPACE;
    P.lpp = opts->lanes_per_particle ? opts->lanes_per_particle : 4;
    P.spw = opts->slices_per_wave ? opts->slices_per_wave : 1;
    P.block = opts->block ? opts->block : 1024;
    P.kern = bb_kernel(P.lpp, P.block);
    SolveArgs &A = P.A;
    A.C = chain_view(p, c, P.pl, P.U);
    A.q = c->q;
    A.gamma = gamma;
    A.g = g;
    A.z[0] = reinterpret_cast<GG *>(P.zbuf);
    A.z[1] = reinterpret_cast<GG *>(P.zbuf) + c->capacity;
    A.warm = opts->warm_start ? 1 : 0;
    A.part = P.part;
    A.sync = P.sync;
    A.ctrl = P.ctrl;
    A.tol = opts->tol;
    A.max_iter = opts->max_iter;
    A.bb = opts->bb;
    return SC_OK;
}

// The persistent solve kernel (assembled M or the chain) on `s`.
// Workgroups of the persistent assembled-M solve when the caller leaves the
// grid open. A product costs the latency of its dependent steps (column
// gathers, the grid barrier, the reduction), which grows with the number of
// workgroups, plus the work per workgroup, which shrinks with it. Measured on
// gfx950 the best count grows about as sqrt(nnz) / 5: 16 at 8,000 nonzeros,
// 32 at 30,000-100,000, 64-128 at 300,000, 128 at 650,000, every CU from
// about 1.5 million; up to 26% per product below a full grid on the small
// systems. A multiple of 8 (one per XCD), clamped to the CUs by
// persistent_grid.
int matrix_grid(long long nnz) {
    const long long k = std::llround(std::sqrt(static_cast<double>(nnz > 0 ? nnz : 0)) / 40.0);
    return static_cast<int>(8 * std::min(std::max(k, 1LL), 1LL << 20));
}

hipError_t launch_solver(Prepared &P, const sc_contacts *c, const sc_solve_opts *opts,
                         double *gamma, double *g, hipStream_t s) {
    if (P.use_mat)
        return launch_bbpgd_mat(mat_view(c->count, P.mb), c->q, gamma, g, P.zbuf, P.part,
                                P.sync, P.ctrl, opts->tol, opts->max_iter, opts->bb, P.spw,
                                opts->lds_entries_per_wave, P.block,
                                opts->grid > 0 ? opts->grid : matrix_grid(c->nnz), s, &P.G,
                                &P.cache_used);
    // pass A's static data in LDS (lds_entries_per_wave: -1 none, > 0 at most
    // that many incidences per wave)
    const int req = opts->lds_entries_per_wave;
    const size_t dyn = chain_lds_dyn(req);
    P.G = persistent_grid(reinterpret_cast<const void *>(P.kern), P.block, opts->grid, dyn);
    if (P.G < 1) return hipErrorInvalidConfiguration;
    const ChainLdsPlan lp = chain_lds_plan(P.A.C.n, c->count, P.G, P.block, req, dyn);
    P.A.rank_cap = lp.rank_cap;
    P.A.inc_cap = lp.inc_cap;
    P.cache_used = lp.per_wave;
    void *args[] = {&P.A};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(P.kern), dim3(P.G),
                                      dim3(P.block), args, dyn, s);
}

void fill_launch_stats(const Prepared &P, sc_stats *st) {
    st->grid = P.G;
    st->block = P.block;
    st->lanes_per_particle = P.use_mat ? 0 : P.lpp;
    st->slices_per_wave = P.use_mat ? P.spw : 0;
    st->lds_entries_per_wave = P.cache_used;
    st->op = P.use_mat ? SC_OP_MATRIX : SC_OP_CHAIN;
}

// ---- device-side bookkeeping of the non-synchronising solve ----

// Clears the barrier block and the control block (the spin limit set), and
// gamma_0 for a cold start: one launch in place of the memsets, so that the
// sequence can be captured into a graph.
__global__ void k_async_reset(double *gamma, int nc, int zero_gamma, unsigned *sync_words,
                              int n_sync_words, unsigned spin_limit, unsigned *ctrl_words,
                              int n_ctrl_words) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    const int lim = static_cast<int>(offsetof(GridSync, limit) / sizeof(unsigned));
    for (int w = t; w < n_sync_words; w += stride) sync_words[w] = w == lim ? spin_limit : 0u;
    for (int w = t; w < n_ctrl_words; w += stride) ctrl_words[w] = 0u;
    if (zero_gamma)
        for (int l = t; l < nc; l += stride) gamma[l] = 0.0;
}

__global__ void k_fill_zero(double *a, long long count) {
    for (long long k = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; k < count;
         k += static_cast<long long>(gridDim.x) * blockDim.x)
        a[k] = 0.0;
}

// sc_stats on the device from the control block (launch fields from the host).
__global__ void k_async_stats(const Ctrl *ctrl, const int *n_active, sc_stats launch,
                              sc_stats *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc_stats o = launch;
    if (ctrl) {
        o.status = ctrl->status;
        o.iters = ctrl->iters;
        o.mvops = ctrl->mvops;
        o.residual = ctrl->res;
        o.alpha = ctrl->alpha;
        o.n_degenerate = ctrl->ndegen;
        o.n_active = *n_active;
    }
    *st = o;
}

// Inside a stream capture the persistent kernel's node must carry the
// cooperative attribute (a captured launch does not keep it): the node just
// captured is the stream's only current dependency.
int mark_cooperative_if_captured(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SC_HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusActive) return SC_OK;
    const hipGraphNode_t *deps = nullptr;
    size_t nd = 0;
    SC_HIP_TRY(hipStreamGetCaptureInfo_v2(s, &cs, nullptr, nullptr, &deps, &nd));
    if (nd != 1 || !deps) return SC_ERR_HIP;
    hipGraphNodeType ty;
    SC_HIP_TRY(hipGraphNodeGetType(deps[0], &ty));
    if (ty != hipGraphNodeTypeKernel) return SC_ERR_HIP;
    hipKernelNodeAttrValue v{}, chk{};
    v.cooperative = 1;
    SC_HIP_TRY(hipGraphKernelNodeSetAttribute(deps[0], hipKernelNodeAttributeCooperative, &v));
    SC_HIP_TRY(hipGraphKernelNodeGetAttribute(deps[0], hipKernelNodeAttributeCooperative, &chk));
    return chk.cooperative == 1 ? SC_OK : SC_ERR_HIP;
}

}  // namespace

int sc::check_solve_args(const sc_particles *p, const sc_contacts *c,
                         const sc_solve_opts *opts, const double *gamma, const double *g,
                         const sc_stats *st) {
    if (!st) return SC_ERR_INVALID;
    Plan pl;
    bool use_mat = false;
    MatBufs mb{};
    return check_args(p, c, opts, gamma, g, pl, use_mat, mb);
}

// The body of sc_solve_lcp on a given workspace. `timed`: measure the
// persistent kernel with HIP events (created once per host thread); without
// it st->kernel_ms is 0 and no event is created.
int sc::solve_lcp_on(const sc_particles *p, const sc_contacts *c, const sc_solve_opts *opts,
                     double *gamma, double *g, double *f_c, double *u_c, sc_stats *st, void *ws,
                     size_t ws_bytes, void *stream_, bool timed) {
    if (!st) return SC_ERR_INVALID;
    Prepared P;
    int rc = prepare(p, c, opts, gamma, g, ws, ws_bytes, P);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    const int n = p->n, nc = c->count;
    *st = sc_stats{};

    if (nc == 0) {
        // no constraints: the zero force solves the (empty) LCP after one product
        if (f_c) SC_HIP_TRY(hipMemsetAsync(f_c, 0, 6 * sizeof(double) * n, s));
        if (u_c) SC_HIP_TRY(hipMemsetAsync(u_c, 0, 6 * sizeof(double) * n, s));
        SC_HIP_TRY(hipStreamSynchronize(s));
        st->status = SC_OK;
        st->mvops = 1;
        return SC_OK;
    }
    Timing *tm = nullptr;
    if (timed) {
        tm = &timing();
        if (!tm->ok) return SC_ERR_HIP;
    }
    if (!opts->warm_start) SC_HIP_TRY(hipMemsetAsync(gamma, 0, sizeof(double) * nc, s));
    SC_HIP_TRY(hipMemsetAsync(P.sync, 0, sizeof(GridSync), s));
    if (opts->spin_limit > 0)
        SC_HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(&P.sync->limit[0]),
                                     opts->spin_limit, 1, s));
    SC_HIP_TRY(hipMemsetAsync(P.ctrl, 0, sizeof(Ctrl), s));
    if (tm) SC_HIP_TRY(hipEventRecord(tm->t0, s));
    SC_HIP_TRY(launch_solver(P, c, opts, gamma, g, s));
    if (tm) SC_HIP_TRY(hipEventRecord(tm->t1, s));
    // the active count into the control block (zeroed above), the outputs,
    // then one copy and one synchronisation
    int b = grid_for(nc);
    if (b > kMaxReduceBlocks) b = kMaxReduceBlocks;
    k_count_active<<<b, kBlock, 0, s>>>(nc, gamma, &P.ctrl->n_active);
    if (f_c || u_c) launch_mob_d(P.A.C, gamma, P.pl.order, f_c, u_c, s);
    Ctrl hc;
    SC_HIP_TRY(hipMemcpyAsync(&hc, P.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    float kernel_ms = 0.0f;
    if (tm) SC_HIP_TRY(hipEventElapsedTime(&kernel_ms, tm->t0, tm->t1));
    st->status = hc.status;
    st->iters = hc.iters;
    st->mvops = hc.mvops;
    st->n_active = hc.n_active;
    st->residual = hc.res;
    st->alpha = hc.alpha;
    st->n_degenerate = hc.ndegen;
    st->kernel_ms = kernel_ms;
    fill_launch_stats(P, st);
    return hc.status;
}

extern "C" int sc_solve_lcp(const sc_particles *p, const sc_contacts *c,
                            const sc_solve_opts *opts, double *gamma, double *g, double *f_c,
                            double *u_c, sc_stats *st, void *ws, size_t ws_bytes,
                            void *stream) {
    return solve_lcp_on(p, c, opts, gamma, g, f_c, u_c, st, ws, ws_bytes, stream, true);
}

extern "C" int sc_solve_lcp_async(const sc_particles *p, const sc_contacts *c,
                                  const sc_solve_opts *opts, double *gamma, double *g,
                                  double *f_c, double *u_c, sc_stats *st_dev, void *ws,
                                  size_t ws_bytes, void *stream_) {
    if (!st_dev) return SC_ERR_INVALID;
    Prepared P;
    int rc = prepare(p, c, opts, gamma, g, ws, ws_bytes, P);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    const int n = p->n, nc = c->count;
    sc_stats launch{};
    if (nc == 0) {
        const long long m = 6LL * n;
        if (f_c && m) k_fill_zero<<<grid_for(m), kBlock, 0, s>>>(f_c, m);
        if (u_c && m) k_fill_zero<<<grid_for(m), kBlock, 0, s>>>(u_c, m);
        launch.status = SC_OK;
        launch.mvops = 1;
        k_async_stats<<<1, 64, 0, s>>>(nullptr, nullptr, launch, st_dev);
        SC_HIP_TRY(hipGetLastError());
        return SC_OK;
    }
    const int nsync = static_cast<int>(sizeof(GridSync) / sizeof(unsigned));
    const int nctrl = static_cast<int>(sizeof(Ctrl) / sizeof(unsigned));
    int rb = grid_for(nc);
    if (rb > kMaxReduceBlocks) rb = kMaxReduceBlocks;
    k_async_reset<<<rb, kBlock, 0, s>>>(gamma, nc, opts->warm_start ? 0 : 1,
                                        reinterpret_cast<unsigned *>(P.sync), nsync,
                                        static_cast<unsigned>(opts->spin_limit),
                                        reinterpret_cast<unsigned *>(P.ctrl), nctrl);
    SC_HIP_TRY(hipGetLastError());
    SC_HIP_TRY(launch_solver(P, c, opts, gamma, g, s));
    rc = mark_cooperative_if_captured(s);
    if (rc != SC_OK) return rc;
    k_count_active<<<rb, kBlock, 0, s>>>(nc, gamma, &P.ctrl->n_active);
    if (f_c || u_c) launch_mob_d(P.A.C, gamma, P.pl.order, f_c, u_c, s);
    fill_launch_stats(P, &launch);
    k_async_stats<<<1, 64, 0, s>>>(P.ctrl, &P.ctrl->n_active, launch, st_dev);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}
