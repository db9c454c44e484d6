// sc_adjoint.hip -- implicit adjoint of the converged LCP on gfx950.
//
// Not in the paper: differentiating the LCP of LCP LCPdef on its active set
// A = {gamma > 0} (section 3.2) gives M_AA gamma_A = -q_A, hence for a loss
// L(gamma, F_c = D gamma), with b = dL/dgamma + D^T dL/dF_c,
//   M_AA w_A = b_A,  w_I = 0,  dL/dq = -w,
// and for a change of the centres (orientations, mobility and U_nc fixed)
//   dL = sum_l dD_l^T [gamma_l (dL/dF - V_w) - w_l (U_nc + U_c)] - sum_l w_l dPhi_l/dt
// with U_c = Mob D gamma and V_w = Mob D w.
//
// The masked system is solved by conjugate gradients in the single-reduction
// form of Chronopoulos and Gear (one product and one fused pair of dot
// products per iteration) inside one persistent kernel laid out like the
// BBPGD iteration: pass A applies the previous iteration's vector updates on
// the fly and forms U = Mob D r, pass B forms w = A r and both dot products.
// The geometric derivatives are then formed per contact and gathered per
// particle (no floating-point atomics).
#include <cmath>
#include <vector>

#include "sc_chain.hpp"
#include "sc_chain_lds.hpp"
#include "sc_common.hpp"
#include "sc_geometry.hpp"
#include "sc_matrix.hpp"
#include "sc_plan.hpp"
#include "sc_sync.hpp"
#include "sc_adjoint_dev.hpp"

namespace sc {

namespace {

struct CgArgs {
    ChainView C;
    const double *gamma;  // active set: gamma > 0
    double *r[2], *s[2], *p, *x, *w;
    double *part;         // [G][2]
    GridSync *sync;
    CgCtrl *ctrl;
    double tol;
    int max_iter;
    int rank_cap, inc_cap;  // pass A's static data in LDS (sc_chain_lds.hpp)
};

template <int LPP, int BS>
__global__ void __launch_bounds__(BS) k_cg(CgArgs A) {
    GridBarrier bar;
    bar.init(A.sync);
    const ChainView &C = A.C;
    int k0, k1, l0, l1;
    chunk(C.n, k0, k1);
    chunk(C.nc, l0, l1);
    const ChainLds L = chain_lds_fill(C, A.rank_cap, A.inc_cap, k0, k1);
    bool ok;
    double tot[2];

    // first product: w = A r0 and the dot products (r0, r0), (w, r0)
    pass_a_lds<LPP, BS>(C, L, k0, k1, [&](int code, int) { return A.r[0][code >> 1]; });
    ok = bar.sync();
    {
        double acc[2] = {0.0, 0.0};
        for (int l = l0 + threadIdx.x; l < l1; l += BS) {
            const double wl = A.gamma[l] > 0.0 ? dt_u(C, l) : 0.0;
            A.w[l] = wl;
            const double rl = A.r[0][l];
            acc[0] += rl * rl;
            acc[1] += wl * rl;
        }
        write_partial<2, BS>(A.part, acc);
    }
    ok = ok && bar.sync();
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
    } else if (!(tot[1] > 0.0)) {
        status = SC_NOT_CONVERGED;  // M_AA not positive on r0
    } else {
        alpha = tot[0] / tot[1];
        for (int i = 1; i <= A.max_iter; ++i) {
            const int cur = (i - 1) & 1, nxt = i & 1;
            const double *rc = A.r[cur], *sc_ = A.s[cur];
            double *rn_out = A.r[nxt], *sn_out = A.s[nxt];
            // p <- r + beta p, s <- w + beta s, x <- x + alpha p, r <- r - alpha s
            pass_a_lds<LPP, BS>(C, L, k0, k1, [&](int code, int) {
                const int l = code >> 1;
                const double sl = A.w[l] + beta * sc_[l];
                const double rn = rc[l] - alpha * sl;
                if (code & 1) {
                    const double pl = rc[l] + beta * A.p[l];
                    A.x[l] = A.x[l] + alpha * pl;
                    A.p[l] = pl;
                    sn_out[l] = sl;
                    rn_out[l] = rn;
                }
                return rn;
            });
            ok = bar.sync();
            double acc[2] = {0.0, 0.0};
            for (int l = l0 + threadIdx.x; l < l1; l += BS) {
                const double wl = A.gamma[l] > 0.0 ? dt_u(C, l) : 0.0;
                A.w[l] = wl;
                const double rl = rn_out[l];
                acc[0] += rl * rl;
                acc[1] += wl * rl;
            }
            write_partial<2, BS>(A.part, acc);
            ok = ok && bar.sync();
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

// r0 = mask(b) with b = dL/dgamma + D^T dL/dF (dL/dF in caller order),
// written with a stride (1 for a plain vector, 4 into (r, w, s, pad)
// records); the active set is counted on the way.
__global__ void k_cg_rhs(int nc, const int *ci, const int *cj, const double *frame,
                         const double *gamma, const double *dLdg, const double *dLdF, double *r,
                         int stride, int *n_active) {
    int cnt = 0;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < nc; l += gridDim.x * blockDim.x) {
        const bool act = gamma[l] > 0.0;
        r[static_cast<long long>(l) * stride] = cg_rhs_one(l, ci, cj, frame, gamma, dLdg, dLdF);
        cnt += act;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
    __shared__ int ws[kBlock / kWave];
    if (threadIdx.x % kWave == 0) ws[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int k = 0; k < kBlock / kWave; ++k) s += ws[k];
        if (s) atomicAdd(n_active, s);
    }
}

__global__ void k_contact_grad(int nc, const int *__restrict__ ci, const int *__restrict__ cj,
                               const int *__restrict__ cs, const double *__restrict__ pos,
                               const double *__restrict__ axis,
                               const double *__restrict__ half_len, PBox box,
                               const double *__restrict__ gamma, const double *__restrict__ w,
                               const double *__restrict__ dLdF, const double *__restrict__ Vw,
                               const double *__restrict__ Unc, const double *__restrict__ Uc,
                               double inv_dt, double *__restrict__ grad) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    const V3 g = contact_grad_one(l, ci, cj, cs, pos, axis, half_len, box, gamma, w, dLdF, Vw,
                                  Unc, Uc, inv_dt);
    double *gout = grad + 3 * static_cast<long long>(l);
    gout[0] = g.x;
    gout[1] = g.y;
    gout[2] = g.z;
}

// dL/dc_k = sum over k's contacts of -grad (k is ci) or +grad (k is cj),
// gathered per rank and written at the caller index.
__global__ void k_gather_pos(int n, Plan pl, const double *__restrict__ grad,
                             double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    gather_pos_one(k, pl, grad, out);
}

__global__ void k_neg_masked(int nc, const double *gamma, const double *x, double *out) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nc) out[l] = gamma[l] > 0.0 ? -x[l] : 0.0;
}

using CgKernel = void (*)(CgArgs);

template <int BS>
CgKernel cg_kernel_bs(int lpp) {
    switch (lpp) {
    case 1: return k_cg<1, BS>;
    case 2: return k_cg<2, BS>;
    case 8: return k_cg<8, BS>;
    default: return k_cg<4, BS>;
    }
}

CgKernel cg_kernel(int lpp, int block) {
    return block == 256 ? cg_kernel_bs<256>(lpp)
                        : block == 512 ? cg_kernel_bs<512>(lpp) : cg_kernel_bs<1024>(lpp);
}

// The adjoint's (and the polish's) workspace, carved in one order.
struct CgBufs {
    double *zrec, *r0, *r1, *s0, *s1, *wv, *pv, *x, *grad, *U, *Vw, *Uc, *part;
    GridSync *sync;
    CgCtrl *ctrl;
};

bool carve_cg(void *ws, size_t ws_bytes, int n, long long cap, CgBufs &B) {
    Carver cv{static_cast<char *>(ws), ws_bytes};
    // one contiguous block: the chain CG's vectors r0 r1 s0 s1 w, or the
    // matrix CG's two arrays of (r, w, s, pad) records
    B.zrec = cv.take<double>(8 * cap);
    B.r0 = B.zrec;
    B.r1 = B.zrec + cap;
    B.s0 = B.zrec + 2 * cap;
    B.s1 = B.zrec + 3 * cap;
    B.wv = B.zrec + 4 * cap;
    B.pv = cv.take<double>(cap);
    B.x = cv.take<double>(cap);
    B.grad = cv.take<double>(3 * cap);
    B.U = cv.take<double>(8 * static_cast<size_t>(n));
    B.Vw = cv.take<double>(8 * static_cast<size_t>(n));
    B.Uc = cv.take<double>(8 * static_cast<size_t>(n));
    B.part = cv.take<double>(2 * kPartHalf);
    B.sync = cv.take<GridSync>(1);
    B.ctrl = cv.take<CgCtrl>(1);
    return cv.ok;
}

bool cg_opts_ok(const sc_adjoint_opts *o, const sc_contacts *c) {
    return o->tol > 0.0 && o->max_iter >= 0 && lanes_ok(o->lanes_per_particle) &&
           spw_ok(o->slices_per_wave) && o->lds_entries_per_wave >= -1 && o->grid >= 0 &&
           block_ok(o->block) && o->op >= 0 && o->op <= SC_OP_MATRIX &&
           !(o->op == SC_OP_MATRIX && !c->mat_ready);
}

// The launch a masked CG used.
struct CgRun {
    bool use_mat = false;
    int lpp = 4, spw = 1, block = 1024, G = 1, cache_used = 0;
};

// Enqueues M_AA x_A = b_A by conjugate gradients into B.x (x = 0 off A),
// with A = {mask > 0} and b = dLdg + D^T dLdF (either may be null), timed
// by e0/e1 around the persistent kernel; ctrl->n_active counts A.
hipError_t enqueue_masked_cg(const sc_particles *p, const sc_contacts *c, const Plan &pl,
                             const double *mask, const double *dLdg, const double *dLdF,
                             const sc_adjoint_opts *opts, const CgBufs &B, CgRun &R,
                             hipEvent_t e0, hipEvent_t e1, hipStream_t s) {
    const int nc = c->count;
    R.use_mat = opts->op == SC_OP_MATRIX || (opts->op == SC_OP_AUTO && c->mat_ready);
    R.lpp = opts->lanes_per_particle ? opts->lanes_per_particle : 4;
    R.spw = opts->slices_per_wave ? opts->slices_per_wave : 1;
    R.block = opts->block ? opts->block : 1024;
    MatBufs mb{};
    if (R.use_mat && !carve_matrix(c->mat, c->mat_bytes, nc, c->nnz, mb))
        return hipErrorInvalidValue;
    CgKernel kern = cg_kernel(R.lpp, R.block);
    const size_t dyn = chain_lds_dyn(opts->lds_entries_per_wave);
    R.G = R.use_mat ? 1
                    : persistent_grid(reinterpret_cast<const void *>(kern), R.block, opts->grid,
                                      dyn);
    if (R.G < 1) return hipErrorInvalidConfiguration;
    hipError_t e;
    if ((e = hipMemsetAsync(B.ctrl, 0, sizeof(CgCtrl), s)) != hipSuccess ||
        (e = hipMemsetAsync(B.sync, 0, sizeof(GridSync), s)) != hipSuccess ||
        (e = hipMemsetAsync(B.s0, 0, sizeof(double) * nc, s)) != hipSuccess ||
        (e = hipMemsetAsync(B.pv, 0, sizeof(double) * nc, s)) != hipSuccess ||
        (e = hipMemsetAsync(B.x, 0, sizeof(double) * nc, s)) != hipSuccess)
        return e;
    if (R.use_mat && (e = hipMemsetAsync(B.zrec, 0, sizeof(double) * 4 * nc, s)) != hipSuccess)
        return e;
    int nb = grid_for(nc);
    if (nb > kMaxReduceBlocks) nb = kMaxReduceBlocks;
    k_cg_rhs<<<nb, kBlock, 0, s>>>(nc, c->ci, c->cj, c->frame, mask, dLdg, dLdF, B.r0,
                                   R.use_mat ? 4 : 1, &B.ctrl->n_active);
    if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
    if (R.use_mat) {
        e = launch_cg_mat(mat_view(nc, mb), mask, B.zrec, B.pv, B.x, B.part, B.sync, B.ctrl,
                          opts->tol, opts->max_iter, R.spw, opts->lds_entries_per_wave, R.block,
                          opts->grid, s, &R.G, &R.cache_used);
    } else {
        CgArgs A;
        A.C = chain_view(p, c, pl, B.U);
        A.gamma = mask;
        A.r[0] = B.r0;
        A.r[1] = B.r1;
        A.s[0] = B.s0;
        A.s[1] = B.s1;
        A.p = B.pv;
        A.x = B.x;
        A.w = B.wv;
        A.part = B.part;
        A.sync = B.sync;
        A.ctrl = B.ctrl;
        A.tol = opts->tol;
        A.max_iter = opts->max_iter;
        const ChainLdsPlan lp = chain_lds_plan(p->n, nc, R.G, R.block,
                                               opts->lds_entries_per_wave, dyn);
        A.rank_cap = lp.rank_cap;
        A.inc_cap = lp.inc_cap;
        R.cache_used = lp.per_wave;
        void *args[] = {&A};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(R.G),
                                       dim3(R.block), args, dyn, s);
    }
    if (e != hipSuccess) return e;
    return hipEventRecord(e1, s);
}

// --------------------------------------------------- active-set polish
//
// mask = 1 on A = {gamma > 0}, else 0.
__global__ void k_polish_mask(int nc, const double *gamma, double *mask) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nc) mask[l] = gamma[l] > 0.0 ? 1.0 : 0.0;
}

// gamma_A = -x_A (x solves M_AA x_A = q_A), 0 off A
__global__ void k_polish_gamma(int nc, const double *mask, const double *x, double *gam) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nc) gam[l] = mask[l] > 0.0 ? -x[l] : 0.0;
}

// g = y + q with y = M gamma (from the two-pass product)
__global__ void k_add_q(int nc, const double *q, double *y) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nc) y[l] += q[l];
}

// Violators of the candidate (gamma, g) on A: gamma_l < 0 in A (leaves A),
// g_l < 0 off A (joins A); the mask is moved to the next active set in
// place, the violators counted, and each block's sum of min(gamma, g)^2
// written to part[block] (summed in block order on the host). Grid-stride,
// so a fixed number of blocks covers any count.
__global__ void k_polish_check(int nc, double *mask, const double *gam, const double *g,
                               int *nviol, double *part) {
    __shared__ double red[kBlock];
    double m2 = 0.0;
    int v = 0;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < nc; l += gridDim.x * blockDim.x) {
        const bool act = mask[l] > 0.0;
        const bool leave = act && gam[l] < 0.0, join = !act && g[l] < 0.0;
        v += leave || join;
        if (leave || join) mask[l] = act ? 0.0 : 1.0;
        const double mm = gam[l] < g[l] ? gam[l] : g[l];
        m2 += mm * mm;
    }
    red[threadIdx.x] = m2;
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (threadIdx.x % kWave == 0 && v) atomicAdd(nviol, v);
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

size_t adjoint_ws_bytes(int32_t n, int32_t cap) {
    const size_t nn = static_cast<size_t>(n), cc = static_cast<size_t>(cap);
    size_t b = 0;
    b += align_up(8 * cc * sizeof(double), 256);        // CG vectors or (r, w, s) records
    b += 2 * align_up(cc * sizeof(double), 256);        // p, x
    b += align_up(3 * cc * sizeof(double), 256);        // grad
    b += 3 * align_up(8 * nn * sizeof(double), 256);    // U, Vw, Uc (rank order)
    b += align_up(2 * kPartHalf * sizeof(double), 256);
    b += align_up(sizeof(GridSync), 256);
    b += align_up(sizeof(CgCtrl), 256);
    return b + 2048;
}

}  // namespace sc

using namespace sc;

extern "C" int sc_solve_lcp_adjoint(const sc_particles *p, const sc_box *box,
                                    const sc_contacts *c, const double *u_nc, double dt,
                                    const double *gamma, const double *dL_dgamma,
                                    const double *dL_df, double *dL_dq, double *dL_dpos,
                                    const sc_adjoint_opts *opts, sc_stats *st, void *ws,
                                    size_t ws_bytes, void *stream_) {
    if (!p || !box || !c || !opts || !st || p->n < 0 || c->count < 0 ||
        c->count > c->capacity)
        return SC_ERR_INVALID;
    if (!(dt > 0.0) || !cg_opts_ok(opts, c)) return SC_ERR_INVALID;
    *st = sc_stats{};
    const int n = p->n, nc = c->count;
    Plan pl;
    if (!carve_plan(c->plan, c->plan_bytes, n, c->capacity, pl)) return SC_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    if (n > 0 && (!dL_dpos || !p->pos || !p->axis || !p->half_len || !p->mob || !u_nc))
        return SC_ERR_INVALID;
    if (nc > 0 && (!gamma || !dL_dq || !c->ci || !c->cj || !c->frame)) return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 ||
        ws_bytes < adjoint_ws_bytes(n, c->capacity))
        return SC_ERR_WORKSPACE;
    if (nc == 0) {
        if (n > 0) SC_HIP_TRY(hipMemsetAsync(dL_dpos, 0, 3 * sizeof(double) * n, s));
        SC_HIP_TRY(hipStreamSynchronize(s));
        st->status = SC_OK;
        return SC_OK;
    }
    CgBufs B;
    if (!carve_cg(ws, ws_bytes, n, c->capacity, B)) return SC_ERR_WORKSPACE;
    double *x = B.x, *grad = B.grad, *Vw = B.Vw, *Uc = B.Uc;
    CgCtrl *ctrl = B.ctrl;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!thread_events(&e0, &e1)) return SC_ERR_HIP;
    CgRun R;
    SC_HIP_TRY(enqueue_masked_cg(p, c, pl, gamma, dL_dgamma, dL_df, opts, B, R, e0, e1, s));
    // dL/dq = -w on A; V_w = Mob D w; U_c = Mob D gamma; geometric terms
    k_neg_masked<<<grid_for(nc), kBlock, 0, s>>>(nc, gamma, x, dL_dq);
    ChainView Cv = chain_view(p, c, pl, Vw), Cc = chain_view(p, c, pl, Uc);
    launch_mob_d(Cv, x, pl.order, nullptr, nullptr, s);
    launch_mob_d(Cc, gamma, pl.order, nullptr, nullptr, s);
    PBox pb{{box->len[0], box->len[1], box->len[2]}, box->periodic ? 1 : 0};
    k_contact_grad<<<grid_for(nc), kBlock, 0, s>>>(nc, c->ci, c->cj, pl.cs, p->pos, p->axis,
                                                   p->half_len, pb, gamma, x, dL_df, Vw, u_nc,
                                                   Uc, 1.0 / dt, grad);
    k_gather_pos<<<grid_for(n), kBlock, 0, s>>>(n, pl, grad, dL_dpos);
    CgCtrl hc;
    SC_HIP_TRY(hipMemcpyAsync(&hc, ctrl, sizeof(CgCtrl), hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    float cg_ms = 0.0f;
    SC_HIP_TRY(hipEventElapsedTime(&cg_ms, e0, e1));
    st->kernel_ms = cg_ms;
    st->status = hc.status;
    st->iters = hc.iters;
    st->mvops = hc.iters + 1;
    st->n_active = hc.n_active;
    st->residual = hc.res;
    st->alpha = hc.alpha;
    st->grid = R.G;
    st->block = R.block;
    st->lanes_per_particle = R.use_mat ? 0 : R.lpp;
    st->slices_per_wave = R.use_mat ? R.spw : 0;
    st->lds_entries_per_wave = R.cache_used;
    st->op = R.use_mat ? SC_OP_MATRIX : SC_OP_CHAIN;
    return hc.status;
}

extern "C" int sc_polish_lcp(const sc_particles *p, const sc_contacts *c, double *gamma,
                             double *g, double *f_c, double *u_c, const sc_adjoint_opts *opts,
                             int32_t max_pass, sc_stats *st, void *ws, size_t ws_bytes,
                             void *stream_) {
    if (!p || !c || !opts || !st || p->n < 0 || c->count < 0 || c->count > c->capacity ||
        max_pass < 0 || !cg_opts_ok(opts, c))
        return SC_ERR_INVALID;
    const int n = p->n, nc = c->count;
    Plan pl;
    if (!carve_plan(c->plan, c->plan_bytes, n, c->capacity, pl)) return SC_ERR_INVALID;
    if (nc > 0 && (!gamma || !g || !c->ci || !c->cj || !c->frame || !c->q))
        return SC_ERR_INVALID;
    if (n > 0 && !p->mob) return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 ||
        ws_bytes < adjoint_ws_bytes(n, c->capacity))
        return SC_ERR_WORKSPACE;
    *st = sc_stats{};
    hipStream_t s = static_cast<hipStream_t>(stream_);
    if (nc == 0) {
        if (f_c && n > 0) SC_HIP_TRY(hipMemsetAsync(f_c, 0, 6 * sizeof(double) * n, s));
        if (u_c && n > 0) SC_HIP_TRY(hipMemsetAsync(u_c, 0, 6 * sizeof(double) * n, s));
        SC_HIP_TRY(hipStreamSynchronize(s));
        st->status = SC_OK;
        return SC_OK;
    }
    CgBufs B;
    if (!carve_cg(ws, ws_bytes, n, c->capacity, B)) return SC_ERR_WORKSPACE;
    const long long cap = c->capacity;
    double *gnew = B.grad, *mask = B.grad + cap, *ynew = B.grad + 2 * cap;
    int *nviol = &B.ctrl->pad;  // the CG leaves this word alone
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!thread_events(&e0, &e1)) return SC_ERR_HIP;
    const ChainView C = chain_view(p, c, pl, B.U);
    const int nb = grid_for(nc);
    const int nr = nb < kMaxReduceBlocks ? nb : kMaxReduceBlocks;  // blocks of the check
    std::vector<double> hp(static_cast<size_t>(nr));
    const int passes_max = max_pass ? max_pass : 20;
    k_polish_mask<<<nb, kBlock, 0, s>>>(nc, gamma, mask);
    CgRun R;
    int passes = 0, iters = 0, status = SC_NOT_CONVERGED;
    float ms_total = 0.0f;
    double res2 = 0.0;
    for (; passes < passes_max;) {
        SC_HIP_TRY(enqueue_masked_cg(p, c, pl, mask, c->q, nullptr, opts, B, R, e0, e1, s));
        k_polish_gamma<<<nb, kBlock, 0, s>>>(nc, mask, B.x, gnew);
        launch_mob_d(C, gnew, pl.order, nullptr, nullptr, s);
        launch_dt(C, ynew, s);
        k_add_q<<<nb, kBlock, 0, s>>>(nc, c->q, ynew);
        SC_HIP_TRY(hipMemsetAsync(nviol, 0, sizeof(int), s));
        k_polish_check<<<nr, kBlock, 0, s>>>(nc, mask, gnew, ynew, nviol, B.part);
        CgCtrl hc;
        SC_HIP_TRY(hipMemcpyAsync(&hc, B.ctrl, sizeof(CgCtrl), hipMemcpyDeviceToHost, s));
        SC_HIP_TRY(hipMemcpyAsync(hp.data(), B.part, sizeof(double) * nr, hipMemcpyDeviceToHost,
                                  s));
        SC_HIP_TRY(hipStreamSynchronize(s));
        SC_HIP_TRY(hipGetLastError());
        float ms = 0.0f;
        SC_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        ms_total += ms;
        ++passes;
        iters += hc.iters;
        if (hc.status != SC_OK) {  // the active block's solve did not converge (or failed)
            status = hc.status;
            break;
        }
        if (hc.pad == 0) {  // no violator: the candidate solves the LCP on its active set
            res2 = 0.0;
            for (int b = 0; b < nr; ++b) res2 += hp[b];
            st->n_active = hc.n_active;
            status = SC_OK;
            break;
        }
    }
    if (status == SC_OK) {
        SC_HIP_TRY(hipMemcpyAsync(gamma, gnew, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
        SC_HIP_TRY(hipMemcpyAsync(g, ynew, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
    } else {
        // not settled: keep the input, and give g = M gamma + q for it
        launch_mob_d(C, gamma, pl.order, nullptr, nullptr, s);
        launch_dt(C, g, s);
        k_add_q<<<nb, kBlock, 0, s>>>(nc, c->q, g);
        k_polish_mask<<<nb, kBlock, 0, s>>>(nc, gamma, mask);
        SC_HIP_TRY(hipMemsetAsync(nviol, 0, sizeof(int), s));
        k_polish_check<<<nr, kBlock, 0, s>>>(nc, mask, gamma, g, nviol, B.part);
        SC_HIP_TRY(hipMemcpyAsync(hp.data(), B.part, sizeof(double) * nr, hipMemcpyDeviceToHost,
                                  s));
        SC_HIP_TRY(hipStreamSynchronize(s));
        res2 = 0.0;
        for (int b = 0; b < nr; ++b) res2 += hp[b];
    }
    if (f_c || u_c) launch_mob_d(C, gamma, pl.order, f_c, u_c, s);
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    st->status = status;
    st->iters = iters;
    st->mvops = passes;
    st->residual = std::sqrt(res2);
    st->kernel_ms = ms_total;
    st->grid = R.G;
    st->block = R.block;
    st->lanes_per_particle = R.use_mat ? 0 : R.lpp;
    st->slices_per_wave = R.use_mat ? R.spw : 0;
    st->lds_entries_per_wave = R.cache_used;
    st->op = R.use_mat ? SC_OP_MATRIX : SC_OP_CHAIN;
    return status;
}
