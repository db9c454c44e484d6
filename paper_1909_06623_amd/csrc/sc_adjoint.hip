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
// products per iteration), laid out exactly like the BBPGD iteration:
// a particle-major gather pass that also applies the previous iteration's
// vector updates on the fly, and a contact-major pass that forms A r and both
// dot products; the last workgroup picks alpha and beta. The geometric
// derivatives of each contact are then formed per contact and gathered per
// particle (no floating-point atomics).
#include "sc_common.hpp"
#include "sc_geometry.hpp"

namespace sc {

namespace {

struct CgCtrl {
    double alpha, beta, gam_prev, bnorm2, tol, res;
    int iters, done, status, max_iter;
    unsigned ticket;
    int n_active;
    int pad[2];
};

__global__ void k_cg_init(CgCtrl *c, double tol, int max_iter) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        CgCtrl z{};
        z.tol = tol;
        z.max_iter = max_iter;
        *c = z;
    }
}

// r0 = mask(b), b = dL/dgamma + D^T dL/dF; p = s = x = 0; count |A|.
__global__ void k_cg_rhs(int nc, const double *gamma, const double *dLdg, const double *dtf,
                         double *r, double *p, double *s, double *x, CgCtrl *c) {
    int cnt = 0;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < nc; l += gridDim.x * blockDim.x) {
        const bool act = gamma[l] > 0.0;
        double b = 0.0;
        if (dLdg) b += dLdg[l];
        if (dtf) b += dtf[l];
        r[l] = act ? b : 0.0;
        p[l] = 0.0;
        s[l] = 0.0;
        x[l] = 0.0;
        cnt += act;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
    if (threadIdx.x % kWave == 0 && cnt) atomicAdd(&c->n_active, cnt);
}

// Particle-major pass of CG iteration i >= 1: with (alpha, beta) of step
// i-1, per active contact
//   p <- r + beta p,  s <- w + beta s_old,  x <- x + alpha p,  r_new = r - alpha s
// (p, x updated in place by the i-side thread; s and r written to the next
// buffers), then U = Mob D r_new. FIRST: U = Mob D r (no update).
template <bool FIRST>
__global__ void __launch_bounds__(kBlock)
k_cg_a(int n, const double *__restrict__ axis, const double *__restrict__ mob,
       const int *__restrict__ i_ptr, const int *__restrict__ j_ptr,
       const int *__restrict__ j_list, const double *__restrict__ frame, long long cap,
       const double *__restrict__ r_cur, const double *__restrict__ s_cur,
       const double *__restrict__ wv, double *__restrict__ p, double *__restrict__ x,
       double *__restrict__ r_nxt, double *__restrict__ s_nxt, double *__restrict__ U,
       const CgCtrl *__restrict__ c) {
    if (c->done) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double alpha = c->alpha, beta = c->beta;
    V3 f = v3(0.0, 0.0, 0.0), t = v3(0.0, 0.0, 0.0);
    const int a0 = i_ptr[k], a1 = i_ptr[k + 1];
    for (int l = a0; l < a1; ++l) {
        double rn;
        if (FIRST) {
            rn = r_cur[l];
        } else {
            const double pl = r_cur[l] + beta * p[l];
            const double sl = wv[l] + beta * s_cur[l];
            x[l] = x[l] + alpha * pl;
            p[l] = pl;
            s_nxt[l] = sl;
            rn = r_cur[l] - alpha * sl;
            r_nxt[l] = rn;
        }
        f = f - rn * frame3(frame, cap, 0, l);
        t = t - rn * frame3(frame, cap, 3, l);
    }
    const int b0 = j_ptr[k], b1 = j_ptr[k + 1];
    for (int m = b0; m < b1; ++m) {
        const int l = j_list[m];
        const double rn =
            FIRST ? r_cur[l] : r_cur[l] - alpha * (wv[l] + beta * s_cur[l]);
        f = f + rn * frame3(frame, cap, 0, l);
        t = t + rn * frame3(frame, cap, 6, l);
    }
    V3 u, om;
    mobility_apply(load3(axis + 3 * k), mob + 4 * k, f, t, u, om);
    double *Uk = U + 6 * static_cast<long long>(k);
    store3(Uk, u);
    store3(Uk + 3, om);
}

// Contact-major pass: w = mask(D^T U) = A r, and the dot products r.r, w.r.
// The last workgroup forms beta_i = gamma_i / gamma_{i-1} and
// alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}).
template <bool FIRST>
__global__ void __launch_bounds__(kBlock)
k_cg_b(int nc, const int *__restrict__ ci, const int *__restrict__ cj,
       const double *__restrict__ frame, long long cap, const double *__restrict__ U,
       const double *__restrict__ gamma, const double *__restrict__ r, double *__restrict__ wv,
       double *__restrict__ partials, CgCtrl *c) {
    __shared__ double lds[2][kBlock / kWave];
    __shared__ int last;
    if (c->done) return;
    double acc[2] = {0.0, 0.0};
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < nc; l += gridDim.x * blockDim.x) {
        double w = 0.0;
        if (gamma[l] > 0.0) {
            const V3 n = frame3(frame, cap, 0, l), ti = frame3(frame, cap, 3, l),
                     tj = frame3(frame, cap, 6, l);
            const double *Ui = U + 6 * static_cast<long long>(ci[l]);
            const double *Uj = U + 6 * static_cast<long long>(cj[l]);
            w = -dot(n, load3(Ui)) - dot(ti, load3(Ui + 3)) + dot(n, load3(Uj)) +
                dot(tj, load3(Uj + 3));
        }
        wv[l] = w;
        const double rl = r[l];
        acc[0] += rl * rl;
        acc[1] += w * rl;
    }
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    acc[0] = wave_sum(acc[0]);
    acc[1] = wave_sum(acc[1]);
    if (lane == 0) {
        lds[0][wid] = acc[0];
        lds[1][wid] = acc[1];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            s0 += lds[0][w];
            s1 += lds[1][w];
        }
        __hip_atomic_store(partials + 2 * blockIdx.x, s0, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(partials + 2 * blockIdx.x + 1, s1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        const unsigned t =
            __hip_atomic_fetch_add(&c->ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;
    acc[0] = acc[1] = 0.0;
    for (int b = threadIdx.x; b < static_cast<int>(gridDim.x); b += blockDim.x) {
        acc[0] += __hip_atomic_load(partials + 2 * b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        acc[1] +=
            __hip_atomic_load(partials + 2 * b + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    acc[0] = wave_sum(acc[0]);
    acc[1] = wave_sum(acc[1]);
    __syncthreads();
    if (lane == 0) {
        lds[0][wid] = acc[0];
        lds[1][wid] = acc[1];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double gam = 0.0, del = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) {
        gam += lds[0][w];
        del += lds[1][w];
    }
    CgCtrl &C = *c;
    C.ticket = 0;
    if (FIRST) C.bnorm2 = gam;
    C.res = C.bnorm2 > 0.0 ? sqrt(gam / C.bnorm2) : 0.0;
    if (!isfinite(gam) || !isfinite(del)) {
        C.status = SC_ERR_NONFINITE;
        C.done = 1;
        return;
    }
    if (gam <= C.tol * C.tol * C.bnorm2 || C.bnorm2 == 0.0) {
        C.status = SC_OK;
        C.done = 1;
        return;
    }
    if (!FIRST) C.iters += 1;
    if (C.iters >= C.max_iter) {
        C.status = SC_NOT_CONVERGED;
        C.done = 1;
        return;
    }
    const double beta = FIRST ? 0.0 : gam / C.gam_prev;
    const double den = FIRST ? del : del - beta * gam / C.alpha;
    if (!(den > 0.0)) {  // M_AA lost positive definiteness numerically
        C.status = SC_NOT_CONVERGED;
        C.done = 1;
        return;
    }
    C.beta = beta;
    C.alpha = gam / den;
    C.gam_prev = gam;
}

// Per-contact derivative of J_l(r) = D_l(r)^T [E_i; E_j] - (w_l/dt) Phi_l(r)
// with respect to r = c_j - c_i (orientations fixed), where
// E_k = gamma_l (dL/dF_k - V_w,k) - w_l (U_nc,k + U_c,k). The closest-point
// parameters s, t move with r only while strictly inside their segment:
// both free -> implicit differentiation of the 2x2 stationarity conditions;
// one free -> its 1-D projection; both clamped (or a sphere) -> fixed.
__global__ void k_contact_grad(int nc, const int *__restrict__ ci, const int *__restrict__ cj,
                               const double *__restrict__ pos, const double *__restrict__ axis,
                               const double *__restrict__ half_len, PBox box,
                               const double *__restrict__ gamma, const double *__restrict__ w,
                               const double *__restrict__ dLdF, const double *__restrict__ Vw,
                               const double *__restrict__ Unc, const double *__restrict__ Uc,
                               double inv_dt, double *__restrict__ grad, long long cap) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    const double gl = gamma[l], wl = w[l];
    if (gl == 0.0 && wl == 0.0) {
        grad[l] = grad[cap + l] = grad[2 * cap + l] = 0.0;
        return;
    }
    const int i = ci[l], j = cj[l];
    const V3 pi = load3(axis + 3 * i), pj = load3(axis + 3 * j);
    const double hi = half_len[i], hj = half_len[j];
    const V3 r = min_image(load3(pos + 3 * i), load3(pos + 3 * j), box);
    double s, t;
    closest_st(r, pi, hi, pj, hj, s, t);
    const bool s_free = hi > 0.0 && s > -hi && s < hi;
    const bool t_free = hj > 0.0 && t > -hj && t < hj;
    V3 ds = v3(0.0, 0.0, 0.0), dt = v3(0.0, 0.0, 0.0);
    if (s_free && t_free) {
        const double b = dot(pi, pj), den = 1.0 - b * b;
        ds = (1.0 / den) * (pi - b * pj);
        dt = (1.0 / den) * (b * pi - pj);
    } else if (t_free) {
        dt = -1.0 * pj;
    } else if (s_free) {
        ds = pi;
    }
    const V3 d = r + t * pj - s * pi;
    const double rho = sqrt(dot(d, d));
    const V3 n = (1.0 / rho) * d;
    // E_i, E_j (6-vectors as force and torque parts)
    V3 EiF, EiT, EjF, EjT;
    {
        const long long oi = 6 * static_cast<long long>(i), oj = 6 * static_cast<long long>(j);
        V3 fi = dLdF ? load3(dLdF + oi) : v3(0, 0, 0), ti = dLdF ? load3(dLdF + oi + 3) : v3(0, 0, 0);
        V3 fj = dLdF ? load3(dLdF + oj) : v3(0, 0, 0), tj = dLdF ? load3(dLdF + oj + 3) : v3(0, 0, 0);
        EiF = gl * (fi - load3(Vw + oi)) - wl * (load3(Unc + oi) + load3(Uc + oi));
        EiT = gl * (ti - load3(Vw + oi + 3)) - wl * (load3(Unc + oi + 3) + load3(Uc + oi + 3));
        EjF = gl * (fj - load3(Vw + oj)) - wl * (load3(Unc + oj) + load3(Uc + oj));
        EjT = gl * (tj - load3(Vw + oj + 3)) - wl * (load3(Unc + oj + 3) + load3(Uc + oj + 3));
    }
    // J_d = dd/dr = I + p_j dt^T - p_i ds^T, so J_d^T u = u + dt (p_j.u) - ds (p_i.u);
    // dn/dr = (I - n n^T) J_d / rho.
    auto JdT = [&](V3 u) { return u + dot(pj, u) * dt - dot(pi, u) * ds; };
    auto JnT = [&](V3 v) { return (1.0 / rho) * JdT(v - dot(n, v) * n); };
    const V3 vn = (EjF - EiF) - s * cross(EiT, pi) + t * cross(EjT, pj);
    const V3 g = JnT(vn) - dot(cross(pi, n), EiT) * ds + dot(cross(pj, n), EjT) * dt -
                 (wl * inv_dt) * JdT(n);
    grad[l] = g.x;
    grad[cap + l] = g.y;
    grad[2 * cap + l] = g.z;
}

// dL/dc_k = sum over contacts with j == k of grad - sum over those with i == k.
__global__ void k_gather_pos(int n, const int *__restrict__ i_ptr, const int *__restrict__ j_ptr,
                             const int *__restrict__ j_list, const double *__restrict__ grad,
                             long long cap, double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int l = i_ptr[k]; l < i_ptr[k + 1]; ++l) {
        gx -= grad[l];
        gy -= grad[cap + l];
        gz -= grad[2 * cap + l];
    }
    for (int m = j_ptr[k]; m < j_ptr[k + 1]; ++m) {
        const int l = j_list[m];
        gx += grad[l];
        gy += grad[cap + l];
        gz += grad[2 * cap + l];
    }
    out[3 * static_cast<long long>(k) + 0] = gx;
    out[3 * static_cast<long long>(k) + 1] = gy;
    out[3 * static_cast<long long>(k) + 2] = gz;
}

__global__ void k_neg_masked(int nc, const double *gamma, const double *x, double *out) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nc) out[l] = gamma[l] > 0.0 ? -x[l] : 0.0;
}

int cg_blocks(int nc) {
    int b = grid_for(nc);
    return b > kMaxReduceBlocks ? kMaxReduceBlocks : b;
}

}  // namespace

size_t adjoint_ws_bytes(int32_t n, int32_t cap) {
    const size_t nn = static_cast<size_t>(n), cc = static_cast<size_t>(cap);
    size_t b = 0;
    b += 8 * align_up(cc * sizeof(double), 256);        // r[2], s[2], p, x, w, dtf
    b += align_up(3 * cc * sizeof(double), 256);        // grad
    b += 3 * align_up(6 * nn * sizeof(double), 256);    // U, Vw, Uc
    b += align_up(2 * kMaxReduceBlocks * sizeof(double), 256);
    b += align_up(sizeof(CgCtrl), 256);
    return b + 1024;
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
    if (!(dt > 0.0) || !(opts->tol > 0.0) || opts->max_iter < 0) return SC_ERR_INVALID;
    *st = sc_stats{};
    const int n = p->n, nc = c->count;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    if (n > 0 && (!dL_dpos || !p->pos || !p->axis || !p->half_len || !p->mob || !u_nc))
        return SC_ERR_INVALID;
    if (nc > 0 && (!gamma || !dL_dq || !c->ci || !c->cj || !c->frame || !c->i_ptr ||
                   !c->j_ptr || !c->j_list))
        return SC_ERR_INVALID;
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
    double *r[2] = {cv.take<double>(cap), cv.take<double>(cap)};
    double *sv[2] = {cv.take<double>(cap), cv.take<double>(cap)};
    double *pv = cv.take<double>(cap);
    double *x = cv.take<double>(cap);
    double *wv = cv.take<double>(cap);
    double *dtf = cv.take<double>(cap);
    double *grad = cv.take<double>(3 * cap);
    double *U = cv.take<double>(6 * static_cast<size_t>(n));
    double *Vw = cv.take<double>(6 * static_cast<size_t>(n));
    double *Uc = cv.take<double>(6 * static_cast<size_t>(n));
    double *partials = cv.take<double>(2 * kMaxReduceBlocks);
    CgCtrl *ctrl = cv.take<CgCtrl>(1);
    if (!cv.ok) return SC_ERR_WORKSPACE;

    const int nb = cg_blocks(nc);
    k_cg_init<<<1, 1, 0, s>>>(ctrl, opts->tol, opts->max_iter);
    if (dL_df) launch_DT(nc, c->ci, c->cj, c->frame, cap, dL_df, dtf, s);
    k_cg_rhs<<<nb, kBlock, 0, s>>>(nc, gamma, dL_dgamma, dL_df ? dtf : nullptr, r[0], pv,
                                   sv[0], x, ctrl);
    k_cg_a<true><<<grid_for(n), kBlock, 0, s>>>(n, p->axis, p->mob, c->i_ptr, c->j_ptr,
                                                c->j_list, c->frame, cap, r[0], sv[0], wv, pv,
                                                x, r[1], sv[1], U, ctrl);
    k_cg_b<true><<<nb, kBlock, 0, s>>>(nc, c->ci, c->cj, c->frame, cap, U, gamma, r[0], wv,
                                       partials, ctrl);
    // CG iterations in chunks, polled one chunk behind through a host copy
    const int chunk = 16;
    int it = 0;
    int done_host = 0;
    while (it < opts->max_iter && !done_host) {
        const int upto = it + chunk < opts->max_iter ? it + chunk : opts->max_iter;
        for (int i = it + 1; i <= upto; ++i) {
            const int cur = (i - 1) & 1, nxt = i & 1;
            k_cg_a<false><<<grid_for(n), kBlock, 0, s>>>(n, p->axis, p->mob, c->i_ptr,
                                                         c->j_ptr, c->j_list, c->frame, cap,
                                                         r[cur], sv[cur], wv, pv, x, r[nxt],
                                                         sv[nxt], U, ctrl);
            k_cg_b<false><<<nb, kBlock, 0, s>>>(nc, c->ci, c->cj, c->frame, cap, U, gamma,
                                                r[nxt], wv, partials, ctrl);
        }
        it = upto;
        SC_HIP_TRY(hipMemcpyAsync(&done_host, &ctrl->done, sizeof(int), hipMemcpyDeviceToHost, s));
        SC_HIP_TRY(hipStreamSynchronize(s));
    }
    CgCtrl hc;
    SC_HIP_TRY(hipMemcpyAsync(&hc, ctrl, sizeof(CgCtrl), hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    if (!hc.done) hc.status = SC_NOT_CONVERGED;

    // dL/dq = -w on A; V_w = Mob D w; U_c = Mob D gamma; geometric terms
    k_neg_masked<<<grid_for(nc), kBlock, 0, s>>>(nc, gamma, x, dL_dq);
    launch_mob_D(n, p->axis, p->mob, c->i_ptr, c->j_ptr, c->j_list, c->frame, cap, x, Vw,
                 nullptr, s);
    launch_mob_D(n, p->axis, p->mob, c->i_ptr, c->j_ptr, c->j_list, c->frame, cap, gamma, Uc,
                 nullptr, s);
    PBox pb{{box->len[0], box->len[1], box->len[2]}, box->periodic ? 1 : 0};
    k_contact_grad<<<grid_for(nc), kBlock, 0, s>>>(nc, c->ci, c->cj, p->pos, p->axis,
                                                   p->half_len, pb, gamma, x, dL_df, Vw, u_nc,
                                                   Uc, 1.0 / dt, grad, cap);
    k_gather_pos<<<grid_for(n), kBlock, 0, s>>>(n, c->i_ptr, c->j_ptr, c->j_list, grad, cap,
                                                dL_dpos);
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    st->status = hc.status;
    st->iters = hc.iters;
    st->mvops = hc.iters + 1;
    st->n_active = hc.n_active;
    st->residual = hc.res;
    st->alpha = hc.alpha;
    return hc.status;
}
