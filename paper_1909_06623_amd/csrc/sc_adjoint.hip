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
#include "sc_chain.hpp"
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
};

template <int LPP, int BS>
__global__ void __launch_bounds__(BS) k_cg(CgArgs A) {
    GridBarrier bar;
    bar.init(A.sync);
    const ChainView &C = A.C;
    int k0, k1, l0, l1;
    chunk(C.n, k0, k1);
    chunk(C.nc, l0, l1);
    bool ok;
    double tot[2];

    // first product: w = A r0 and the dot products (r0, r0), (w, r0)
    pass_a<LPP, BS>(C, k0, k1, [&](int code, int) { return A.r[0][code >> 1]; });
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
            pass_a<LPP, BS>(C, k0, k1, [&](int code, int) {
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
    if (!(dt > 0.0) || !(opts->tol > 0.0) || opts->max_iter < 0 ||
        !lanes_ok(opts->lanes_per_particle) || !spw_ok(opts->slices_per_wave) ||
        opts->lds_entries_per_wave < -1 || opts->grid < 0 ||
        !block_ok(opts->block) || opts->op < 0 ||
        opts->op > SC_OP_MATRIX || (opts->op == SC_OP_MATRIX && !c->mat_ready))
        return SC_ERR_INVALID;
    *st = sc_stats{};
    const int n = p->n, nc = c->count;
    const bool use_mat = opts->op == SC_OP_MATRIX || (opts->op == SC_OP_AUTO && c->mat_ready);
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
    const long long cap = c->capacity;
    Carver cv{static_cast<char *>(ws), ws_bytes};
    // one contiguous block: the chain CG's vectors r0 r1 s0 s1 w, or the
    // matrix CG's two arrays of (r, w, s, pad) records
    double *zrec = cv.take<double>(8 * cap);
    double *r0 = zrec, *r1 = zrec + cap, *s0 = zrec + 2 * cap, *s1 = zrec + 3 * cap;
    double *wv = zrec + 4 * cap;
    double *pv = cv.take<double>(cap), *x = cv.take<double>(cap);
    double *grad = cv.take<double>(3 * cap);
    double *U = cv.take<double>(8 * static_cast<size_t>(n));
    double *Vw = cv.take<double>(8 * static_cast<size_t>(n));
    double *Uc = cv.take<double>(8 * static_cast<size_t>(n));
    double *part = cv.take<double>(2 * kPartHalf);
    GridSync *sync = cv.take<GridSync>(1);
    CgCtrl *ctrl = cv.take<CgCtrl>(1);
    if (!cv.ok) return SC_ERR_WORKSPACE;

    const int lpp = opts->lanes_per_particle ? opts->lanes_per_particle : 4;
    const int spw = opts->slices_per_wave ? opts->slices_per_wave : 1;
    int cache_used = 0;
    const int block = opts->block ? opts->block : 1024;
    MatBufs mb{};
    if (use_mat && !carve_matrix(c->mat, c->mat_bytes, nc, c->nnz, mb)) return SC_ERR_INVALID;
    CgKernel kern = cg_kernel(lpp, block);
    int G = use_mat ? 1 : persistent_grid(reinterpret_cast<const void *>(kern), block, opts->grid);
    if (G < 1) return SC_ERR_HIP;

    SC_HIP_TRY(hipMemsetAsync(ctrl, 0, sizeof(CgCtrl), s));
    SC_HIP_TRY(hipMemsetAsync(sync, 0, sizeof(GridSync), s));
    SC_HIP_TRY(hipMemsetAsync(s0, 0, sizeof(double) * nc, s));
    SC_HIP_TRY(hipMemsetAsync(pv, 0, sizeof(double) * nc, s));
    SC_HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * nc, s));
    int nb = grid_for(nc);
    if (nb > kMaxReduceBlocks) nb = kMaxReduceBlocks;
    if (use_mat) SC_HIP_TRY(hipMemsetAsync(zrec, 0, sizeof(double) * 4 * nc, s));
    k_cg_rhs<<<nb, kBlock, 0, s>>>(nc, c->ci, c->cj, c->frame, gamma, dL_dgamma, dL_df, r0,
                                   use_mat ? 4 : 1, &ctrl->n_active);
    CgArgs A;
    A.C = chain_view(p, c, pl, U);
    A.gamma = gamma;
    A.r[0] = r0;
    A.r[1] = r1;
    A.s[0] = s0;
    A.s[1] = s1;
    A.p = pv;
    A.x = x;
    A.w = wv;
    A.part = part;
    A.sync = sync;
    A.ctrl = ctrl;
    A.tol = opts->tol;
    A.max_iter = opts->max_iter;
    void *args[] = {&A};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!thread_events(&e0, &e1)) return SC_ERR_HIP;
    SC_HIP_TRY(hipEventRecord(e0, s));
    if (use_mat) {
        SC_HIP_TRY(launch_cg_mat(mat_view(nc, mb), gamma, zrec, pv, x, part, sync, ctrl,
                                 opts->tol, opts->max_iter, spw, opts->lds_entries_per_wave,
                                 block, opts->grid, s, &G, &cache_used));
    } else {
        SC_HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kern), dim3(G),
                                              dim3(block), args, 0, s));
    }
    SC_HIP_TRY(hipEventRecord(e1, s));
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
    st->grid = G;
    st->block = block;
    st->lanes_per_particle = use_mat ? 0 : lpp;
    st->slices_per_wave = use_mat ? spw : 0;
    st->lds_entries_per_wave = cache_used;
    st->op = use_mat ? SC_OP_MATRIX : SC_OP_CHAIN;
    return hc.status;
}
