// sc_batch.hip -- many independent collision LCPs (each with its own
// assembled M) solved by Algorithm 1 in one persistent launch (gfx950).
//
// The grid (one workgroup per CU) splits into teams of workgroups that share
// one XCD, so a team barrier stays inside one L2 and needs no write-back.
// Team leaders take instances from a work queue ordered by nonzeros, largest
// first (greedy list scheduling); every member then runs Algorithm 1 on its
// nnz-balanced share of the instance's slices, with the instance's M partly
// resident in LDS, exactly as the single-instance solver does over the whole
// grid. Either every instance gets the same team size, or each queue
// position k has a size class t_k (a power of two that grows with the
// instance's nonzeros, non-increasing along the queue): teams start as large
// as the classes allow and, when the instance a team takes belongs to a
// smaller class, halve until they fit it, the lower half keeping the
// instance and the upper half going back to the queue. So the largest
// instances, which set the critical path, get many workgroups and the many
// small ones few. An instance's arithmetic depends only on its team size, not
// on which team takes it, so results are reproducible.
// With the adjoint enabled, the team then differentiates the instance's
// converged solution (the implicit adjoint on its active set, not in the
// paper): F_c = D gamma and U_c, the masked right-hand side, the CG on M_AA
// (same layout as the solve), dL/dq, V_w = Mob D w, the per-contact
// geometric derivatives and their per-particle sums, with team barriers
// between the steps. A reset kernel (no memset) precedes the persistent
// kernel, so the pair can be captured in a HIP graph and replayed. A batch
// in build mode first builds every instance's contacts and M on the device
// (sc_batch_build.hip); a finalize kernel then writes each instance's row
// and slice counts into its descriptor and orders the queue, so that build,
// solves and adjoints are one graph.
#include <algorithm>
#include <climits>
#include <numeric>
#include <vector>

#include "sc_adjoint_dev.hpp"
#include "sc_batch_build.hpp"
#include "sc_chain.hpp"
#include "sc_common.hpp"
#include "sc_matrix.hpp"
#include "sc_matrix_pass.hpp"
#include "sc_plan.hpp"
#include "sc_sync.hpp"

namespace sc {

namespace {

constexpr int kMaxTeam = 32;            // workgroups of one XCD (256 CUs / 8)
constexpr int kTeamPartHalf = 4 * kMaxTeam;
constexpr int kXcdCount = 8;             // XCDs of the device the grid spans
constexpr long long kTuneTarget0 = 4096;  // autotuner: nonzeros per workgroup 4096 * 2^i
constexpr int kTunePolicies = 12;         // 6 size-class targets, 6 single team sizes

struct BatchDesc {
    MatView M;
    const double *q;
    double *gamma, *g;
    GG *z0, *z1;
    // adjoint
    ChainView C;            // C.U holds U_c = Mob D gamma (rank order)
    Plan pl;
    PBox box;
    const int *ci, *cj;
    const double *pos, *axis, *half_len, *u_nc, *dLdg;
    double inv_dt;
    double *dq, *dpos;
    double *F;              // [n][6] D gamma, caller order
    double *Vw;             // [n][8] Mob D w, rank order
    double *grad;           // [nc][3]
    double *p, *x;          // [nc]
    RWS *r0, *r1;           // [nc] each
};

struct alignas(256) BatchCtl {
    unsigned next[32];              // work queue head
    unsigned err[32];               // timeout flag
    unsigned init[32];              // start-up arrivals
    unsigned xslot[kMaxXcc][32];    // workgroups per XCD (slot counters)
};

struct BatchArgs {
    const BatchDesc *items;
    const int *order;       // queue position -> instance, by nonzeros, descending
    const int *tcls;        // queue position -> team size of that instance
    SolveCtrl *ctrl;        // [count], per instance
    BatchCtl *ctl;
    TeamSync *tsync;        // [team-tree nodes]
    double *part;           // [team-tree nodes][2 * kTeamPartHalf]
    int count, team, warm, cache;  // team: the initial team size
    double tol;
    int max_iter, bb;
    int adjoint, adj_max_iter;  // adjoint: 0 none, 1 dL/dF = D gamma (+ dL/dgamma), 2 dL/dgamma
    double adj_tol;
    CgCtrl *cgctrl;             // [count]
};

// Team size of an instance with `nnz` nonzeros: the smallest power of two
// t with t * target >= nnz, within [1, tmax]; tmax when target <= 0 (one
// size for every instance).
__device__ int team_class(long long nnz, long long target, int tmax) {
    if (target <= 0) return tmax;
    const long long need = (nnz + target - 1) / target;
    int t = 1;
    while (t < tmax && t < need) t <<= 1;
    return t;
}

// Clears the queue, barrier counters and per-instance results (an instance
// no team reached keeps SC_ERR_TIMEOUT), and sets the team size of every
// queue position for both launches from its nonzeros (qnnz).
__global__ void k_batch_reset(BatchCtl *ctl, TeamSync *ts, int nnodes, SolveCtrl *ctrl,
                              CgCtrl *cg, int count, const long long *qnnz, int *tcls,
                              long long target_f, int tmax_f, long long target_a, int tmax_a) {
    unsigned *c = reinterpret_cast<unsigned *>(ctl);  // one block per stage
    for (int k = threadIdx.x; k < static_cast<int>(2 * sizeof(BatchCtl) / 4); k += blockDim.x)
        c[k] = 0u;
    unsigned *t = reinterpret_cast<unsigned *>(ts);
    const long long nt = 2LL * nnodes * (sizeof(TeamSync) / 4);  // one set per stage
    for (long long k = threadIdx.x; k < nt; k += blockDim.x) t[k] = 0u;
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        tcls[k] = team_class(qnnz[k], target_f, tmax_f);
        tcls[count + k] = team_class(qnnz[k], target_a, tmax_a);
    }
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        ctrl[k] = SolveCtrl{};
        ctrl[k].status = SC_ERR_TIMEOUT;
        if (cg) {
            cg[k] = CgCtrl{};
            cg[k].status = SC_ERR_TIMEOUT;
        }
    }
}

// After a build: each instance's row and slice counts into its descriptor
// (none for an instance whose build failed) and the work order by nonzeros,
// largest first, ties by index (the host's order for prebuilt batches).
__global__ void k_batch_finalize(BatchDesc *items, const BuildOut *out, int *order,
                                 long long *qnnz, int count) {
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        const bool ok = out[k].status == SC_OK;
        BatchDesc &d = items[k];
        d.M.nc = ok ? out[k].nc : 0;
        d.M.ns = ok ? out[k].ns : 0;
        d.C.nc = d.M.nc;
    }
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        const long long nk = out[k].status == SC_OK ? out[k].nnz : 0;
        int r = 0;
        for (int j = 0; j < count; ++j) {
            const long long nj = out[j].status == SC_OK ? out[j].nnz : 0;
            r += nj > nk || (nj == nk && j < k);
        }
        order[r] = k;
        qnnz[r] = nk;
    }
}

// The adjoint steps of one instance on a team (member `member` of t): the
// member's share of particles [k0, k1), its rows of the solve's chunk.
template <int R, int BS>
__device__ void adjoint_rows(const BatchArgs &A, const BatchDesc &D, const SliceChunk &ch,
                             const WaveCache &W, double *part, int member, int t, TeamBarrier &tb,
                             int item) {
    const int n = D.C.n;
    const int k0 = static_cast<int>(static_cast<long long>(member) * n / t);
    const int k1 = static_cast<int>(static_cast<long long>(member + 1) * n / t);
    const bool fc = A.adjoint == 1;
    bool ok = tb.sync();  // every gamma of the instance is final
    for (int k = k0 + threadIdx.x; k < k1; k += BS)
        mob_d_one(D.C, k, D.gamma, D.pl.order, fc ? D.F : nullptr, D.C.U);
    ok = tb.sync() && ok;
    for (int l = ch.l0 + threadIdx.x; l < ch.l1; l += BS) {
        D.r0[l] = RWS{cg_rhs_one(l, D.ci, D.cj, D.C.frame, D.gamma, D.dLdg, fc ? D.F : nullptr),
                      0.0, 0.0, 0.0};
        D.p[l] = 0.0;
        D.x[l] = 0.0;
    }
    ok = tb.sync() && ok;
    const WaveMeta<R> Mt = wave_meta<R, BS>(D.M, ch);
    cg_rows<R, BS>(D.M, ch, W, Mt, D.gamma, D.r0, D.r1, D.p, D.x, part, kTeamPartHalf, member, t,
                   tb, A.adj_tol, ok ? A.adj_max_iter : 0, A.cgctrl + item);
    for (int l = ch.l0 + threadIdx.x; l < ch.l1; l += BS)
        D.dq[l] = D.gamma[l] > 0.0 ? -D.x[l] : 0.0;
    for (int k = k0 + threadIdx.x; k < k1; k += BS)
        mob_d_one(D.C, k, D.x, D.pl.order, nullptr, D.Vw);
    tb.sync();
    for (int l = ch.l0 + threadIdx.x; l < ch.l1; l += BS) {
        const V3 gv = contact_grad_one(l, D.ci, D.cj, D.pl.cs, D.pos, D.axis, D.half_len, D.box,
                                       D.gamma, D.x, fc ? D.F : nullptr, D.Vw, D.u_nc, D.C.U,
                                       D.inv_dt);
        double *go = D.grad + 3 * static_cast<long long>(l);
        go[0] = gv.x;
        go[1] = gv.y;
        go[2] = gv.z;
    }
    tb.sync();
    for (int k = k0 + threadIdx.x; k < k1; k += BS) gather_pos_one(k, D.pl, D.grad, D.dpos);
}

// STAGE 0 solves every instance, STAGE 1 (a second launch, so that each
// kernel keeps its own register budget) runs the adjoint of every solution.
template <int R, int BS, int STAGE>
__global__ void __launch_bounds__(BS) k_bbpgd_batch(BatchArgs A) {
    __shared__ int sh[4];
    BatchCtl *ctl = A.ctl;
    int t = A.team;
    // team formation: slot of this workgroup within its XCD, then teams of t
    // consecutive slots in each XCD (workgroups left over sit out)
    if (threadIdx.x == 0) {
        const unsigned x = xcc_id();
        const unsigned slot = __hip_atomic_fetch_add(&ctl->xslot[x][0], 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&ctl->init[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const bool good = spin_reach(&ctl->init[0], gridDim.x, &ctl->err[0]);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        int base = 0;
        for (unsigned k = 0; k < x; ++k) base += static_cast<int>(ld_relaxed(&ctl->xslot[k][0])) / t;
        const int mine = static_cast<int>(ld_relaxed(&ctl->xslot[x][0])) / t;
        const int s = static_cast<int>(slot);
        sh[0] = good && s < mine * t ? base + s / t : -1;  // team
        sh[1] = s % t;                                     // member
    }
    __syncthreads();
    const int team0 = sh[0];
    int member = sh[1];
    __syncthreads();
    if (team0 < 0) return;
    // A team is a node of its initial team's binary tree (heap numbering:
    // 1 is the initial team, 2v and 2v + 1 the halves of v), so every
    // sub-team has a barrier and partial sums of its own.
    int node = 1;
    auto node_id = [&]() { return team0 * 2 * A.team + node; };
    TeamBarrier tb{A.tsync + node_id(), &ctl->err[0], static_cast<unsigned>(t), 0u};
    double *part = A.part + static_cast<long long>(node_id()) * 2 * kTeamPartHalf;
    for (;;) {
        if (member == 0 && threadIdx.x == 0) {
            const unsigned k =
                __hip_atomic_fetch_add(&ctl->next[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh[2] = static_cast<int>(k);
            if (t > 1)
                __hip_atomic_store(&tb.s->item[0], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const bool ok = tb.sync();
        if (threadIdx.x == 0 && t > 1) sh[2] = static_cast<int>(ld_relaxed(&tb.s->item[0]));
        __syncthreads();
        const int k = sh[2];
        __syncthreads();
        if (!ok || k >= A.count) break;
        // halve down to the instance's team size: the lower half keeps it,
        // the upper half (a team of its own) goes back to the queue
        const int tk = min(A.tcls[k], t);
        bool handed_on = false;
        while (t > tk) {
            const int half = t >> 1;
            const bool upper = member >= half;
            node = 2 * node + (upper ? 1 : 0);
            member -= upper ? half : 0;
            t = half;
            tb = TeamBarrier{A.tsync + node_id(), &ctl->err[0], static_cast<unsigned>(t), 0u};
            part = A.part + static_cast<long long>(node_id()) * 2 * kTeamPartHalf;
            if (upper) {
                handed_on = true;
                break;
            }
        }
        if (handed_on) continue;
        const int item = A.order[k];
        const BatchDesc D = A.items[item];
        const SliceChunk ch = slice_chunk(D.M, member, t);
        const WaveCache W = wave_cache<R, BS>(D.M, ch, A.cache);
        fill_cache<R, BS>(D.M, ch, W);
        // 4 gathers in flight per wave: the team logic leaves fewer registers
        constexpr int B = R == 1 ? 4 : 8 / R;
        if constexpr (STAGE == 0)
            bbpgd_rows<R, BS, TeamBarrier, B>(D.M, ch, W, D.q, A.warm ? D.gamma : nullptr, D.gamma,
                                              D.g, D.z0, D.z1, part, kTeamPartHalf, member, t, tb,
                                              A.tol, A.max_iter, A.bb, A.ctrl + item);
        else
            adjoint_rows<R, BS>(A, D, ch, W, part, member, t, tb, item);
    }
}

using BatchKernel = void (*)(BatchArgs);

template <int STAGE>
BatchKernel batch_kernel(int block) {
    switch (block) {
    case 256: return k_bbpgd_batch<1, 256, STAGE>;
    case 512: return k_bbpgd_batch<1, 512, STAGE>;
    default: return k_bbpgd_batch<1, 1024, STAGE>;
    }
}

// Dynamic LDS for the matrix cache (as for the single-instance solver).
hipError_t batch_cache(const void *fn, int block, int *per_block, size_t *dyn) {
    int dev = 0, max_lds = 0;
    hipFuncAttributes fa;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess) e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    const int nw = block / kWave;
    long long per = (static_cast<long long>(max_lds) - static_cast<long long>(fa.sharedSizeBytes) - 256) /
                    (12LL * nw);
    per -= per % 2;
    if (per < 2) per = 0;
    *per_block = static_cast<int>(per) * nw;
    *dyn = per > 0 ? static_cast<size_t>(per) * 12 * nw : 16;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(*dyn));
}

bool team_ok(int t) {
    return t == 0 || t == 1 || t == 2 || t == 4 || t == 8 || t == 16 || t == 32;
}

// rows an instance's solve buffers hold: its contacts, or in build mode its
// capacity
size_t rows(const sc_contacts &c, bool build) {
    const int r = build ? c.capacity : c.count;
    return static_cast<size_t>(r > 0 ? r : 1);
}
size_t z_doubles(const sc_contacts &c, bool build) { return 4 * rows(c, build); }
// adjoint scratch per instance: F [n][6], U_c and V_w [n][8] each,
// grad [nc][3], p, x [nc], two record arrays [nc][4]
size_t adj_doubles(const sc_batch_item &it, bool build) {
    const size_t n = static_cast<size_t>(it.p.n > 0 ? it.p.n : 1);
    return 22 * n + 13 * rows(it.c, build) + 8 * 256;
}

}  // namespace

}  // namespace sc

using namespace sc;

struct sc_batch {
    int count = 0;
    std::vector<int32_t> counts;       // rows per instance
    BatchArgs args{};
    int nnodes = 0;                    // team-tree nodes per launch (2 per workgroup)
    int team = 1, block = 1024, grid = 0;
    int block_adj = 512, cache_adj = 0;  // the adjoint launch's block and LDS entries
    size_t dyn_adj = 0;
    int team_adj = 1;                  // team size of the adjoint launch
    long long target = 0, target_adj = 0;  // nonzeros per workgroup of the size
                                           // classes (0: `team` for every instance)
    int tmax = kMaxTeam;               // initial team size with size classes: the
                                       // workgroups of one XCD, at most 32
    long long *qnnz = nullptr;         // [count] nonzeros per queue position
    int *tcls = nullptr;               // [2][count] team size per queue position
    size_t dyn = 0;
    const void *fn = nullptr, *fn_adj = nullptr;
    bool build = false;
    BatchBuild bld;                    // build mode: tables and scratch
    std::vector<BuildInst> bhost;
    BatchDesc *descs = nullptr;        // device copies the finalize kernel updates
    int *order = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float tune_ms[kTunePolicies] = {};      // autotuner: build + forward per policy
    float tune_adj_ms[kTunePolicies] = {};  // autotuner: adjoint launch per policy
};

namespace {

size_t batch_ws_bytes(int32_t count, const sc_batch_item *items, int nnodes, bool adj,
                      bool build) {
    const size_t nd = static_cast<size_t>(std::max(count, 1));
    size_t b = 0;
    b += align_up(sizeof(CgCtrl) * nd, 256);
    if (adj)
        for (int32_t k = 0; k < count; ++k)
            b += 8 * 256 + sizeof(double) * adj_doubles(items[k], build);
    b += align_up(2 * sizeof(BatchCtl), 256);
    b += align_up(2 * sizeof(TeamSync) * static_cast<size_t>(nnodes), 256);
    b += align_up(sizeof(double) * 2 * kTeamPartHalf * static_cast<size_t>(nnodes), 256);
    b += align_up(sizeof(long long) * nd, 256);
    b += align_up(2 * sizeof(int) * nd, 256);
    b += align_up(sizeof(BatchDesc) * nd, 256);
    b += align_up(sizeof(int) * nd, 256);
    b += align_up(sizeof(SolveCtrl) * nd, 256);
    for (int32_t k = 0; k < count; ++k)
        b += align_up(sizeof(double) * z_doubles(items[k].c, build), 256);
    if (build) b += batch_build_bytes(count, items);
    return b + 256;
}

// `mid` (optional) is recorded between the forward and the adjoint launch.
int enqueue(sc_batch *b, hipStream_t s, hipEvent_t mid = nullptr) {
    if (b->build) {
        const int rc = batch_build_enqueue(b->bld, s);
        if (rc != SC_OK) return rc;
        k_batch_finalize<<<1, 1024, 0, s>>>(b->descs, b->bld.out, b->order, b->qnnz, b->count);
    }
    const int t0 = b->target > 0 ? b->tmax : b->team;
    const int t0a = b->target_adj > 0 ? b->tmax : b->team_adj;
    k_batch_reset<<<1, 256, 0, s>>>(b->args.ctl, b->args.tsync, b->nnodes, b->args.ctrl,
                                     b->args.adjoint ? b->args.cgctrl : nullptr, b->count,
                                     b->qnnz, b->tcls, b->target, t0, b->target_adj, t0a);
    BatchArgs a = b->args;
    a.team = t0;
    a.tcls = b->tcls;
    void *args[] = {&a};
    SC_HIP_TRY(hipLaunchCooperativeKernel(b->fn, dim3(b->grid), dim3(b->block), args, b->dyn, s));
    if (mid) SC_HIP_TRY(hipEventRecord(mid, s));
    if (b->args.adjoint) {
        BatchArgs c = a;
        c.cache = b->cache_adj;
        c.team = t0a;
        c.tcls = b->tcls + b->count;
        c.ctl = b->args.ctl + 1;
        c.tsync = b->args.tsync + b->nnodes;
        void *cargs[] = {&c};
        SC_HIP_TRY(hipLaunchCooperativeKernel(b->fn_adj, dim3(b->grid), dim3(b->block_adj),
                                              cargs, b->dyn_adj, s));
    }
    return SC_OK;
}

}  // namespace

extern "C" size_t sc_batch_workspace_bytes(int32_t count, const sc_batch_item *items,
                                           const sc_batch_opts *opts) {
    if (count < 0 || (count > 0 && !items) || !opts) return 0;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 1024;
    return batch_ws_bytes(count, items, 2 * std::max(cus, 1), opts->adjoint != 0,
                          opts->build != 0);
}

extern "C" int sc_batch_create(int32_t count, const sc_batch_item *items, const sc_batch_opts *opts,
                               void *ws, size_t ws_bytes, void *stream, sc_batch **out) {
    if (!out || !opts || count < 0 || (count > 0 && !items)) return SC_ERR_INVALID;
    *out = nullptr;
    if (!(opts->tol > 0.0) || opts->max_iter < 0 || opts->bb < 1 || opts->bb > 3 ||
        !team_ok(opts->team) || !team_ok(opts->adjoint_team) || opts->nnz_per_workgroup < 0 ||
        opts->adjoint_nnz_per_workgroup < 0 || (opts->team > 0 && opts->nnz_per_workgroup > 0) ||
        (opts->adjoint_team > 0 && opts->adjoint_nnz_per_workgroup > 0) ||
        !block_ok(opts->block) || !block_ok(opts->adjoint_block) || opts->adjoint < 0 || opts->adjoint > 2 ||
        (opts->adjoint && (!(opts->adjoint_tol > 0.0) || opts->adjoint_max_iter < 0)) ||
        opts->build < 0 || opts->build > 1)
        return SC_ERR_INVALID;
    const bool adj = opts->adjoint != 0;
    const bool build = opts->build != 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<BatchDesc> descs(static_cast<size_t>(count));
    std::vector<long long> nnz(static_cast<size_t>(count));
    for (int32_t k = 0; k < count; ++k) {
        const sc_contacts &c = items[k].c;
        const int rows_k = build ? c.capacity : c.count;
        if (build ? (c.capacity < 0 || c.nnz < 0)
                  : (c.count < 0 || c.count > c.capacity || !c.mat_ready))
            return SC_ERR_INVALID;
        if (!c.q || (rows_k > 0 && (!items[k].gamma || !items[k].g))) return SC_ERR_INVALID;
        MatBufs mb{};
        if (!carve_matrix(c.mat, c.mat_bytes, rows_k, c.nnz, mb)) return SC_ERR_INVALID;
        descs[k].M = mat_view(build ? 0 : c.count, mb);
        if (adj) {
            const sc_batch_item &it = items[k];
            Plan pl;
            if (it.p.n < 0 || !carve_plan(c.plan, c.plan_bytes, it.p.n, c.capacity, pl) ||
                !(it.dt > 0.0) ||
                (it.p.n > 0 && (!it.u_nc || !it.dL_dpos || !it.p.pos || !it.p.axis ||
                                !it.p.half_len)) ||
                (rows_k > 0 && (!it.dL_dq || !c.ci || !c.cj || !c.frame)))
                return SC_ERR_INVALID;
            BatchDesc &d = descs[k];
            d.pl = pl;
            d.C = ChainView{it.p.n, build ? 0 : c.count, pl.pdat, pl.inc_ptr, pl.inc, pl.dpm,
                            pl.cs, c.frame, nullptr};
            d.box = PBox{{it.box.len[0], it.box.len[1], it.box.len[2]}, it.box.periodic ? 1 : 0};
            d.ci = c.ci;
            d.cj = c.cj;
            d.pos = it.p.pos;
            d.axis = it.p.axis;
            d.half_len = it.p.half_len;
            d.u_nc = it.u_nc;
            d.dLdg = it.dL_dgamma;
            d.inv_dt = 1.0 / it.dt;
            d.dq = it.dL_dq;
            d.dpos = it.dL_dpos;
        }
        descs[k].q = c.q;
        descs[k].gamma = items[k].gamma;
        descs[k].g = items[k].g;
        nnz[k] = c.nnz;
    }
    auto *b = new sc_batch;
    b->count = count;
    b->build = build;
    b->block = opts->block ? opts->block : 1024;
    // the adjoint's state does not fit 1024 threads' registers (it spills),
    // so its launch defaults to 512
    b->block_adj = opts->adjoint_block ? opts->adjoint_block : 512;
    b->fn = reinterpret_cast<const void *>(batch_kernel<0>(b->block));
    b->fn_adj = reinterpret_cast<const void *>(batch_kernel<1>(b->block_adj));
    int per_block = 0;
    if (batch_cache(b->fn, b->block, &per_block, &b->dyn) != hipSuccess ||
        batch_cache(b->fn_adj, b->block_adj, &b->cache_adj, &b->dyn_adj) != hipSuccess) {
        delete b;
        return SC_ERR_HIP;
    }
    // both stages use the smaller LDS share, so that one walk serves both
    b->grid = std::min(persistent_grid(b->fn, b->block, 0, b->dyn),
                       persistent_grid(b->fn_adj, b->block_adj, 0, b->dyn_adj));
    b->nnodes = 2 * b->grid;
    // size classes start from teams of one XCD's workgroups (a power of two)
    while (b->tmax > 1 && b->tmax * kXcdCount > b->grid) b->tmax >>= 1;
    if (b->grid < 1) {
        delete b;
        return SC_ERR_HIP;
    }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 ||
        ws_bytes < batch_ws_bytes(count, items, b->nnodes, adj, build)) {
        delete b;
        return SC_ERR_WORKSPACE;
    }
    Carver cv{static_cast<char *>(ws), ws_bytes};
    BatchArgs &a = b->args;
    a.ctl = cv.take<BatchCtl>(2);
    a.tsync = cv.take<TeamSync>(2 * static_cast<size_t>(b->nnodes));
    a.part = cv.take<double>(2 * kTeamPartHalf * static_cast<size_t>(b->nnodes));
    b->qnnz = cv.take<long long>(static_cast<size_t>(std::max(count, 1)));
    b->tcls = cv.take<int>(2 * static_cast<size_t>(std::max(count, 1)));
    BatchDesc *d_descs = cv.take<BatchDesc>(static_cast<size_t>(std::max(count, 1)));
    int *d_order = cv.take<int>(static_cast<size_t>(std::max(count, 1)));
    a.ctrl = cv.take<SolveCtrl>(static_cast<size_t>(std::max(count, 1)));
    a.cgctrl = cv.take<CgCtrl>(static_cast<size_t>(std::max(count, 1)));
    for (int32_t k = 0; k < count; ++k) {
        GG *z = reinterpret_cast<GG *>(cv.take<double>(z_doubles(items[k].c, build)));
        descs[k].z0 = z;
        descs[k].z1 = z + rows(items[k].c, build);
        b->counts.push_back(items[k].c.count);
        if (adj) {
            const size_t n = static_cast<size_t>(std::max(items[k].p.n, 1));
            const size_t nc = rows(items[k].c, build);
            BatchDesc &d = descs[k];
            d.F = cv.take<double>(6 * n);
            d.C.U = cv.take<double>(8 * n);
            d.Vw = cv.take<double>(8 * n);
            d.grad = cv.take<double>(3 * nc);
            d.p = cv.take<double>(nc);
            d.x = cv.take<double>(nc);
            d.r0 = reinterpret_cast<RWS *>(cv.take<double>(4 * nc));
            d.r1 = reinterpret_cast<RWS *>(cv.take<double>(4 * nc));
        }
    }
    if (!cv.ok) {
        delete b;
        return SC_ERR_WORKSPACE;
    }
    if (build) {
        const int rc = batch_build_plan(count, items, cv, s, b->bld, b->bhost);
        if (rc != SC_OK) {
            delete b;
            return rc == SC_ERR_INVALID && !cv.ok ? SC_ERR_WORKSPACE : rc;
        }
    }
    b->descs = d_descs;
    b->order = d_order;
    std::vector<int> order(static_cast<size_t>(count));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nnz[x] > nnz[y]; });
    std::vector<long long> qnnz(static_cast<size_t>(count));
    for (int32_t r = 0; r < count; ++r) qnnz[r] = nnz[order[r]];
    a.items = d_descs;
    a.order = d_order;
    a.count = count;
    a.warm = opts->warm_start ? 1 : 0;
    a.cache = per_block;
    a.tol = opts->tol;
    a.max_iter = opts->max_iter;
    a.bb = opts->bb;
    a.adjoint = opts->adjoint;
    a.adj_tol = opts->adjoint_tol;
    a.adj_max_iter = opts->adjoint_max_iter;
    if (count > 0) {
        if (hipMemcpyAsync(d_descs, descs.data(), sizeof(BatchDesc) * count, hipMemcpyHostToDevice,
                           s) != hipSuccess ||
            hipMemcpyAsync(d_order, order.data(), sizeof(int) * count, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(b->qnnz, qnnz.data(), sizeof(long long) * count,
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            delete b;
            return SC_ERR_HIP;
        }
    }
    // the forward's policy: one team size, size classes, or tuned classes
    b->team = opts->team > 0 ? opts->team : b->tmax;
    b->target = opts->team > 0 ? 0 : opts->nnz_per_workgroup;
    const bool tune = opts->team == 0 && opts->nnz_per_workgroup == 0;
    // the adjoint's: its own if given, else the forward's (tuned with it)
    const bool adj_own = opts->adjoint_team > 0 || opts->adjoint_nnz_per_workgroup > 0;
    b->team_adj = opts->adjoint_team > 0 ? opts->adjoint_team : adj_own ? b->tmax : b->team;
    b->target_adj = opts->adjoint_team > 0 ? 0 : adj_own ? opts->adjoint_nnz_per_workgroup
                                                         : b->target;
    if (tune) {
        // autotuner: solve the batch once per policy (size classes for
        // 4096 * 2^i nonzeros per workgroup, then one team size 1, 2, ..., 32),
        // the forward and adjoint launches timed apart, and keep the fastest
        // policy of each launch. Team sizes above one XCD's workgroups cannot
        // form and are skipped.
        hipEvent_t e[3] = {nullptr, nullptr, nullptr};
        int rc = SC_OK;
        for (auto &ev : e)
            if (rc == SC_OK && hipEventCreate(&ev) != hipSuccess) rc = SC_ERR_HIP;
        auto cfg_team = [&](int i) { return i < 6 ? b->tmax : 1 << (i - 6); };
        auto cfg_target = [&](int i) { return i < 6 ? kTuneTarget0 << i : 0LL; };
        int pf = -1, pa = -1;
        for (int i = 0; i < kTunePolicies && rc == SC_OK; ++i) {
            if (cfg_team(i) > b->tmax) continue;
            b->team = cfg_team(i);
            b->target = cfg_target(i);
            if (!adj_own) {
                b->team_adj = b->team;
                b->target_adj = b->target;
            }
            rc = hipEventRecord(e[0], s) == hipSuccess ? enqueue(b, s, e[1]) : SC_ERR_HIP;
            if (rc == SC_OK && (hipEventRecord(e[2], s) != hipSuccess ||
                                hipEventSynchronize(e[2]) != hipSuccess ||
                                hipEventElapsedTime(&b->tune_ms[i], e[0], e[1]) != hipSuccess ||
                                hipEventElapsedTime(&b->tune_adj_ms[i], e[1], e[2]) != hipSuccess))
                rc = SC_ERR_HIP;
            if (pf < 0 || b->tune_ms[i] < b->tune_ms[pf]) pf = i;
            if (pa < 0 || b->tune_adj_ms[i] < b->tune_adj_ms[pa]) pa = i;
        }
        if (rc == SC_OK && pf < 0) rc = SC_ERR_HIP;
        if (rc == SC_OK) {
            b->team = cfg_team(pf);
            b->target = cfg_target(pf);
            if (!adj_own) {
                b->team_adj = adj ? cfg_team(pa) : b->team;
                b->target_adj = adj ? cfg_target(pa) : b->target;
            }
        }
        for (auto &ev : e)
            if (ev) (void)hipEventDestroy(ev);
        if (rc != SC_OK) {
            delete b;
            return rc;
        }
    }
    *out = b;
    return SC_OK;
}

extern "C" int sc_batch_solve(sc_batch *b, void *stream) {
    if (!b) return SC_ERR_INVALID;
    if (b->count == 0) return SC_OK;
    return enqueue(b, static_cast<hipStream_t>(stream));
}

namespace {

// Captures reset + persistent kernel on a private stream (the caller's may be
// the legacy default stream, which cannot be captured), marks the persistent
// kernel's node cooperative and instantiates the graph.
int build_graph(sc_batch *b) {
    hipStream_t cs = nullptr;
    SC_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    int rc = SC_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = SC_ERR_HIP;
    } else {
        rc = enqueue(b, cs);
        if (hipStreamEndCapture(cs, &g) != hipSuccess || !g) rc = SC_ERR_HIP;
    }
    (void)hipStreamDestroy(cs);
    if (rc != SC_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    size_t nn = 0;
    std::vector<hipGraphNode_t> nodes;
    int marked = 0;
    if (hipGraphGetNodes(g, nullptr, &nn) == hipSuccess) {
        nodes.resize(nn);
        if (hipGraphGetNodes(g, nodes.data(), &nn) != hipSuccess) nn = 0;
    }
    for (size_t i = 0; i < nn && rc == SC_OK; ++i) {
        hipGraphNodeType ty;
        hipKernelNodeParams kp{};
        if (hipGraphNodeGetType(nodes[i], &ty) != hipSuccess) rc = SC_ERR_HIP;
        if (rc != SC_OK || ty != hipGraphNodeTypeKernel) continue;
        if (hipGraphKernelNodeGetParams(nodes[i], &kp) != hipSuccess) rc = SC_ERR_HIP;
        if (rc != SC_OK || (kp.func != b->fn && kp.func != b->fn_adj)) continue;
        hipKernelNodeAttrValue v{}, chk{};
        v.cooperative = 1;
        if (hipGraphKernelNodeSetAttribute(nodes[i], hipKernelNodeAttributeCooperative, &v) !=
                hipSuccess ||
            hipGraphKernelNodeGetAttribute(nodes[i], hipKernelNodeAttributeCooperative, &chk) !=
                hipSuccess ||
            chk.cooperative != 1)
            rc = SC_ERR_HIP;
        ++marked;
    }
    if (rc == SC_OK && marked != (b->args.adjoint ? 2 : 1)) rc = SC_ERR_HIP;
    if (rc == SC_OK && hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        b->exec = nullptr;
        rc = SC_ERR_HIP;
    }
    if (rc != SC_OK) {
        (void)hipGraphDestroy(g);
        return rc;
    }
    b->graph = g;
    return SC_OK;
}

}  // namespace

extern "C" int sc_batch_graph_launch(sc_batch *b, void *stream) {
    if (!b) return SC_ERR_INVALID;
    if (b->count == 0) return SC_OK;
    if (!b->exec) {
        const int rc = build_graph(b);
        if (rc != SC_OK) return rc;
    }
    SC_HIP_TRY(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
    return SC_OK;
}

extern "C" int sc_batch_stats(const sc_batch *b, sc_stats *stats, sc_stats *adj,
                              sc_batch_info *info, void *stream) {
    if (!b || (b->count > 0 && !stats)) return SC_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (info) {
        info->team = b->team;
        info->block = b->block;
        info->grid = b->grid;
        info->lds_entries_per_wave = b->args.cache / (b->block / kWave);
        info->adjoint_block = b->block_adj;
        for (int i = 0; i < kTunePolicies; ++i) info->tune_ms[i] = b->tune_ms[i];
        info->team_adjoint = b->team_adj;
        for (int i = 0; i < kTunePolicies; ++i) info->tune_adjoint_ms[i] = b->tune_adj_ms[i];
        info->nnz_per_workgroup = static_cast<int32_t>(b->target);
        info->adjoint_nnz_per_workgroup = static_cast<int32_t>(b->target_adj);
    }
    if (b->count == 0) return SC_OK;
    std::vector<SolveCtrl> h(static_cast<size_t>(b->count));
    SC_HIP_TRY(hipMemcpyAsync(h.data(), b->args.ctrl, sizeof(SolveCtrl) * b->count,
                              hipMemcpyDeviceToHost, s));
    // team size per instance: the class of its queue position (capped by the
    // initial team size, as the kernel does)
    std::vector<int> cls(2 * static_cast<size_t>(b->count)), ord(static_cast<size_t>(b->count));
    SC_HIP_TRY(hipMemcpyAsync(cls.data(), b->tcls, sizeof(int) * 2 * b->count,
                              hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipMemcpyAsync(ord.data(), b->order, sizeof(int) * b->count,
                              hipMemcpyDeviceToHost, s));
    std::vector<CgCtrl> hc(static_cast<size_t>(b->count));
    if (adj && b->args.adjoint)
        SC_HIP_TRY(hipMemcpyAsync(hc.data(), b->args.cgctrl, sizeof(CgCtrl) * b->count,
                                  hipMemcpyDeviceToHost, s));
    std::vector<BuildOut> ho(static_cast<size_t>(b->build ? b->count : 0));
    if (b->build)
        SC_HIP_TRY(hipMemcpyAsync(ho.data(), b->bld.out, sizeof(BuildOut) * b->count,
                                  hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    std::vector<int> tf(static_cast<size_t>(b->count)), ta(static_cast<size_t>(b->count));
    const int t0 = b->target > 0 ? b->tmax : b->team;
    const int t0a = b->target_adj > 0 ? b->tmax : b->team_adj;
    for (int r = 0; r < b->count; ++r) {
        if (ord[r] < 0 || ord[r] >= b->count) return SC_ERR_HIP;
        tf[ord[r]] = std::min(cls[r], t0);
        ta[ord[r]] = std::min(cls[b->count + r], t0a);
    }
    // an instance whose build failed reports the build's status
    for (int k = 0; k < static_cast<int>(ho.size()); ++k)
        if (ho[k].status != SC_OK) {
            h[k] = SolveCtrl{};
            h[k].status = ho[k].status;
            hc[k] = CgCtrl{};
            hc[k].status = ho[k].status;
        }
    if (adj) {
        for (int k = 0; k < b->count; ++k) {
            adj[k] = sc_stats{};
            adj[k].status = b->args.adjoint ? hc[k].status : SC_OK;
            adj[k].iters = hc[k].iters;
            adj[k].mvops = hc[k].iters + 1;
            adj[k].residual = hc[k].res;
            adj[k].alpha = hc[k].alpha;
            adj[k].grid = ta[k];
            adj[k].block = b->block_adj;
            adj[k].lds_entries_per_wave = b->cache_adj / (b->block_adj / kWave);
            adj[k].op = SC_OP_MATRIX;
            adj[k].n_active = -1;
        }
    }
    for (int k = 0; k < b->count; ++k) {
        sc_stats &st = stats[k];
        st = sc_stats{};
        st.status = h[k].status;
        st.iters = h[k].iters;
        st.mvops = h[k].mvops;
        st.residual = h[k].res;
        st.alpha = h[k].alpha;
        st.n_degenerate = h[k].ndegen;
        st.grid = tf[k];
        st.block = b->block;
        st.op = SC_OP_MATRIX;
        st.slices_per_wave = 1;
        st.lds_entries_per_wave = b->args.cache / (b->block / kWave);
        st.n_active = -1;
    }
    return SC_OK;
}

extern "C" int sc_batch_contacts(const sc_batch *b, int32_t *count, int64_t *nnz,
                                 int32_t *status, void *stream) {
    if (!b || !b->build) return SC_ERR_INVALID;
    if (b->count == 0) return SC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<BuildOut> ho(static_cast<size_t>(b->count));
    SC_HIP_TRY(hipMemcpyAsync(ho.data(), b->bld.out, sizeof(BuildOut) * b->count,
                              hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < b->count; ++k) {
        if (count) count[k] = ho[k].nc;
        if (nnz) nnz[k] = ho[k].nnz;
        if (status) status[k] = ho[k].status;
    }
    return SC_OK;
}

extern "C" void sc_batch_destroy(sc_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
}
