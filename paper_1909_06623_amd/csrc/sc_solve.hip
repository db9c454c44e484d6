// sc_solve.hip -- matrix-free M x = D^T Mob D x and the BBPGD solve
// (Algorithm 1, section 3.3.1) on gfx950.
//
// One product is two gather passes (no floating-point atomics, so results
// are bitwise reproducible run to run):
//   phase A, one thread per particle k: F_k = sum over k's contacts of
//     -/+ (n_l, tau_l) w_l, then U_k = Mob_k F_k. In the descent pass the
//     weight is the projected step w_l = max(0, gamma_l - alpha g_l) and the
//     i-side thread stores it as the new iterate (Algorithm 1 steps 8-9).
//   phase B, grid-stride over contacts: (D^T U)_l = -n.U_i - tau_i.W_i +
//     n.U_j + tau_j.W_j, g_l = that + q_l, and the partial sums of
//     ||min(gamma, g)||^2, s^T s, s^T y, y^T y. The last workgroup to finish
//     reduces the partials in a fixed order and updates the solver state
//     (residual test, BB step of step 15) in device memory.
// The host enqueues iterations in chunks and polls a pinned "done" flag one
// chunk behind, so the GPU never waits for the host between iterations.
#include <mutex>

#include "sc_common.hpp"

namespace sc {

namespace {

struct Ctrl {
    double alpha;      // step size for the next descent step
    double res;        // ||min(gamma, g)||_2 of the latest iterate
    double g0g0;       // g_0^T g_0 (numerator of alpha_0)
    double tol;
    int iters;         // descent steps completed
    int mvops;
    int status;
    int done;
    unsigned ticket;   // last-workgroup election counter
    int ndegen;
    int max_iter;
    int bb;
    int n_active;
    int pad[3];
};

enum PhaseB { kG0 = 0, kMG0 = 1, kIter = 2, kPlain = 3 };

__global__ void k_init_ctrl(Ctrl *ctrl, double tol, int max_iter, int bb) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        Ctrl c{};
        c.tol = tol;
        c.max_iter = max_iter;
        c.bb = bb;
        *ctrl = c;
    }
}

// Projection of Algorithm 1 step 9 (negative components set to zero);
// written so that a NaN propagates instead of being clamped away.
__device__ __forceinline__ double project(double v) { return v < 0.0 ? 0.0 : v; }

// STEP == false: U = Mob D x. STEP == true: U = Mob D gamma_new with
// gamma_new = max(0, x - alpha g) computed on the fly and stored by the
// i-side thread into gam_next.
template <bool STEP>
__global__ void __launch_bounds__(kBlock)
k_phase_a(int n, const double *__restrict__ axis, const double *__restrict__ mob,
          const int *__restrict__ i_ptr, const int *__restrict__ j_ptr,
          const int *__restrict__ j_list, const double *__restrict__ frame, long long cap,
          const double *__restrict__ x, const double *__restrict__ g_cur,
          double *__restrict__ gam_next, double *__restrict__ U, double *__restrict__ F_out,
          const Ctrl *__restrict__ ctrl) {
    if (ctrl && ctrl->done) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double alpha = STEP ? ctrl->alpha : 0.0;
    V3 f = v3(0.0, 0.0, 0.0), t = v3(0.0, 0.0, 0.0);
    const int a0 = i_ptr[k], a1 = i_ptr[k + 1];
    for (int l = a0; l < a1; ++l) {
        double w;
        if (STEP) {
            w = project(x[l] - alpha * g_cur[l]);
            gam_next[l] = w;
        } else {
            w = x[l];
        }
        f = f - w * frame3(frame, cap, 0, l);
        t = t - w * frame3(frame, cap, 3, l);
    }
    const int b0 = j_ptr[k], b1 = j_ptr[k + 1];
    for (int m = b0; m < b1; ++m) {
        const int l = j_list[m];
        const double w = STEP ? project(x[l] - alpha * g_cur[l]) : x[l];
        f = f + w * frame3(frame, cap, 0, l);
        t = t + w * frame3(frame, cap, 6, l);
    }
    V3 u, om;
    mobility_apply(load3(axis + 3 * k), mob + 4 * k, f, t, u, om);
    double *Uk = U + 6 * static_cast<long long>(k);
    store3(Uk, u);
    store3(Uk + 3, om);
    if (F_out) {
        double *Fk = F_out + 6 * static_cast<long long>(k);
        store3(Fk, f);
        store3(Fk + 3, t);
    }
}

__device__ __forceinline__ double m_diag(V3 n, V3 ti, V3 tj, const double *axis,
                                         const double *mob, int i, int j) {
    V3 ui, wi, uj, wj;
    mobility_apply(load3(axis + 3 * i), mob + 4 * i, n, ti, ui, wi);
    mobility_apply(load3(axis + 3 * j), mob + 4 * j, n, tj, uj, wj);
    return dot(n, ui) + dot(ti, wi) + dot(n, uj) + dot(tj, wj);
}

template <int MODE>
__global__ void __launch_bounds__(kBlock)
k_phase_b(int nc, const int *__restrict__ ci, const int *__restrict__ cj,
          const double *__restrict__ frame, long long cap, const double *__restrict__ q,
          const double *__restrict__ U, const double *__restrict__ axis,
          const double *__restrict__ mob, const double *__restrict__ gam_new,
          const double *__restrict__ gam_old, const double *__restrict__ g_old,
          double *__restrict__ g_new, double *__restrict__ partials, Ctrl *ctrl) {
    __shared__ double lds[4][kBlock / kWave];
    __shared__ int last;
    if (MODE != kPlain && ctrl->done) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int stride = gridDim.x * blockDim.x;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < nc; l += stride) {
        const V3 n = frame3(frame, cap, 0, l), ti = frame3(frame, cap, 3, l),
                 tj = frame3(frame, cap, 6, l);
        const int i = ci[l], j = cj[l];
        const double *Ui = U + 6 * static_cast<long long>(i);
        const double *Uj = U + 6 * static_cast<long long>(j);
        const double v = -dot(n, load3(Ui)) - dot(ti, load3(Ui + 3)) + dot(n, load3(Uj)) +
                         dot(tj, load3(Uj + 3));
        if (MODE == kPlain) {
            g_new[l] = v;
        } else if (MODE == kG0) {
            const double gl = v + q[l];
            g_new[l] = gl;
            const double gm = gam_new[l];
            const double m = gm < gl ? gm : gl;
            acc[0] += m * m;
            acc[1] += gl * gl;
        } else if (MODE == kMG0) {
            acc[0] += g_old[l] * v;
            acc[1] = fmax(acc[1], m_diag(n, ti, tj, axis, mob, i, j));
        } else {
            const double gl = v + q[l];
            g_new[l] = gl;
            const double gm = gam_new[l];
            const double m = gm < gl ? gm : gl;
            const double s = gm - gam_old[l];
            const double y = gl - g_old[l];
            acc[0] += m * m;
            acc[1] += s * s;
            acc[2] += s * y;
            acc[3] += y * y;
        }
    }
    if (MODE == kPlain) return;

    // workgroup partials (the max of kMG0 travels in slot 1 as a max)
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        acc[k] = (MODE == kMG0 && k == 1) ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0)
        for (int k = 0; k < 4; ++k) lds[k][wid] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double out[4];
        for (int k = 0; k < 4; ++k) {
            double s = lds[k][0];
            for (int w = 1; w < kBlock / kWave; ++w)
                s = (MODE == kMG0 && k == 1) ? fmax(s, lds[k][w]) : s + lds[k][w];
            out[k] = s;
        }
        for (int k = 0; k < 4; ++k)
            __hip_atomic_store(partials + 4 * blockIdx.x + k, out[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        const unsigned t = __hip_atomic_fetch_add(&ctrl->ticket, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!last) return;

    // last workgroup: reduce gridDim.x partials in a fixed order
    for (int k = 0; k < 4; ++k) {
        double s = (MODE == kMG0 && k == 1) ? 0.0 : 0.0;
        for (int b = threadIdx.x; b < static_cast<int>(gridDim.x); b += blockDim.x) {
            const double v = __hip_atomic_load(partials + 4 * b + k, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
            s = (MODE == kMG0 && k == 1) ? fmax(s, v) : s + v;
        }
        acc[k] = s;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        acc[k] = (MODE == kMG0 && k == 1) ? wave_max(acc[k]) : wave_sum(acc[k]);
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < 4; ++k) lds[k][wid] = acc[k];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double tot[4];
    for (int k = 0; k < 4; ++k) {
        double s = lds[k][0];
        for (int w = 1; w < kBlock / kWave; ++w)
            s = (MODE == kMG0 && k == 1) ? fmax(s, lds[k][w]) : s + lds[k][w];
        tot[k] = s;
    }
    Ctrl &c = *ctrl;
    c.ticket = 0;
    if (MODE == kG0) {
        // Algorithm 1 steps 2-5
        c.mvops = 1;
        c.res = sqrt(tot[0]);
        c.g0g0 = tot[1];
        if (!isfinite(c.res)) {
            c.status = SC_ERR_NONFINITE;
            c.done = 1;
        } else if (c.res < c.tol) {
            c.status = SC_OK;
            c.done = 1;
        }
    } else if (MODE == kMG0) {
        // step 6: alpha_0 = g0^T g0 / g0^T M g0
        c.mvops = 2;
        const double den = tot[0];
        if (den > 0.0 && isfinite(den) && isfinite(c.g0g0)) {
            c.alpha = c.g0g0 / den;
        } else {
            c.alpha = tot[1] > 0.0 ? 1.0 / tot[1] : 1.0;
            c.ndegen += 1;
        }
        c.status = SC_NOT_CONVERGED;
        if (c.max_iter <= 0) c.done = 1;
    } else {
        // steps 10-15 after the descent step j
        const int j = c.iters + 1;
        c.iters = j;
        c.mvops += 1;
        c.res = sqrt(tot[0]);
        if (!isfinite(c.res)) {
            c.status = SC_ERR_NONFINITE;
            c.done = 1;
        } else if (c.res < c.tol) {
            c.status = SC_OK;
            c.done = 1;
        } else {
            const bool bb2 = (c.bb == 2) || (c.bb == 3 && (j % 2 == 0));
            const double num = bb2 ? tot[2] : tot[1];
            const double den = bb2 ? tot[3] : tot[2];
            if (den > 0.0 && num > 0.0 && isfinite(num) && isfinite(den))
                c.alpha = num / den;
            else
                c.ndegen += 1;
            if (j >= c.max_iter) c.done = 1;
        }
    }
}

__global__ void k_count_active(int nc, const double *gamma, Ctrl *ctrl) {
    int cnt = 0;
    for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < nc; l += gridDim.x * blockDim.x)
        cnt += gamma[l] > 0.0;
    for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
    if (threadIdx.x % kWave == 0 && cnt) atomicAdd(&ctrl->n_active, cnt);
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

// Pinned host words used to poll the device "done" flag without stalling
// the stream (allocated once per process).
struct PollSlots {
    int *words = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t t0 = nullptr, t1 = nullptr;  // timing of the iteration loop
    bool ok = false;
};

PollSlots &poll_slots() {
    thread_local PollSlots ps;
    if (!ps.ok) {
        if (hipHostMalloc(reinterpret_cast<void **>(&ps.words), 2 * sizeof(int),
                          hipHostMallocDefault) != hipSuccess)
            return ps;
        if (hipEventCreateWithFlags(&ps.ev[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ps.ev[1], hipEventDisableTiming) != hipSuccess ||
            hipEventCreate(&ps.t0) != hipSuccess || hipEventCreate(&ps.t1) != hipSuccess)
            return ps;
        ps.ok = true;
    }
    return ps;
}

int reduce_blocks(int nc) {
    int b = grid_for(nc);
    return b > kMaxReduceBlocks ? kMaxReduceBlocks : b;
}

}  // namespace

void launch_mob_D(int n, const double *axis, const double *mob, const int *i_ptr,
                  const int *j_ptr, const int *j_list, const double *frame, long long cap,
                  const double *x, double *U, double *F, hipStream_t s) {
    if (n <= 0) return;
    k_phase_a<false><<<grid_for(n), kBlock, 0, s>>>(n, axis, mob, i_ptr, j_ptr, j_list, frame,
                                                    cap, x, nullptr, nullptr, U, F, nullptr);
}

void launch_DT(int nc, const int *ci, const int *cj, const double *frame, long long cap,
               const double *U, double *y, hipStream_t s) {
    if (nc <= 0) return;
    k_phase_b<kPlain><<<reduce_blocks(nc), kBlock, 0, s>>>(nc, ci, cj, frame, cap, nullptr, U,
                                                           nullptr, nullptr, nullptr, nullptr,
                                                           nullptr, y, nullptr, nullptr);
}

size_t solve_ws_bytes(int32_t n, int32_t cap) {
    const size_t nn = static_cast<size_t>(n), cc = static_cast<size_t>(cap);
    size_t b = 0;
    b += 2 * align_up(cc * sizeof(double), 256);          // second gamma, g buffers
    b += align_up(6 * nn * sizeof(double), 256);          // U
    b += align_up(4 * kMaxReduceBlocks * sizeof(double), 256);
    b += align_up(sizeof(Ctrl), 256);
    return b + 1024;
}

}  // namespace sc

using namespace sc;

namespace {

struct Chain {
    int n, nc;
    long long cap;
    const double *axis, *mob, *frame, *q;
    const int *ci, *cj, *i_ptr, *j_ptr, *j_list;
    double *U, *partials;
    Ctrl *ctrl;
    hipStream_t s;

    void phase_a(const double *x, double *F_out, double *Uout = nullptr) const {
        k_phase_a<false><<<grid_for(n), kBlock, 0, s>>>(n, axis, mob, i_ptr, j_ptr, j_list,
                                                        frame, cap, x, nullptr, nullptr,
                                                        Uout ? Uout : U, F_out, nullptr);
    }
    void phase_a_step(const double *gam, const double *g, double *gam_next) const {
        k_phase_a<true><<<grid_for(n), kBlock, 0, s>>>(n, axis, mob, i_ptr, j_ptr, j_list,
                                                       frame, cap, gam, g, gam_next, U,
                                                       nullptr, ctrl);
    }
    template <int MODE>
    void phase_b(const double *gam_new, const double *gam_old, const double *g_old,
                 double *g_new, const double *Uin = nullptr) const {
        k_phase_b<MODE><<<reduce_blocks(nc), kBlock, 0, s>>>(
            nc, ci, cj, frame, cap, q, Uin ? Uin : U, axis, mob, gam_new, gam_old, g_old,
            g_new, partials, ctrl);
    }
};

int check_common(const sc_particles *p, const sc_contacts *c) {
    if (!p || !c || p->n < 0 || c->count < 0 || c->count > c->capacity) return SC_ERR_INVALID;
    if (p->n > 0 && (!p->axis || !p->mob)) return SC_ERR_INVALID;
    if (c->count > 0 && (!c->ci || !c->cj || !c->frame || !c->q || !c->i_ptr || !c->j_ptr ||
                         !c->j_list))
        return SC_ERR_INVALID;
    return SC_OK;
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
    int rc = check_common(p, c);
    if (rc) return rc;
    if (c->count == 0) return SC_OK;
    if (!x || !y) return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 ||
        ws_bytes < solve_ws_bytes(p->n, c->capacity))
        return SC_ERR_WORKSPACE;
    Carver cv{static_cast<char *>(ws), ws_bytes};
    cv.take<double>(c->capacity);
    cv.take<double>(c->capacity);
    double *U = cv.take<double>(6 * static_cast<size_t>(p->n));
    if (!cv.ok) return SC_ERR_WORKSPACE;
    Chain ch{p->n, c->count, c->capacity, p->axis, p->mob, c->frame, c->q, c->ci, c->cj,
             c->i_ptr, c->j_ptr, c->j_list, U, nullptr, nullptr,
             static_cast<hipStream_t>(stream)};
    ch.phase_a(x, nullptr);
    ch.phase_b<kPlain>(nullptr, nullptr, nullptr, y);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}

extern "C" int sc_solve_lcp(const sc_particles *p, const sc_contacts *c,
                            const sc_solve_opts *opts, double *gamma, double *g, double *f_c,
                            double *u_c, sc_stats *st, void *ws, size_t ws_bytes,
                            void *stream_) {
    int rc = check_common(p, c);
    if (rc) return rc;
    if (!opts || !st) return SC_ERR_INVALID;
    if (!(opts->tol > 0.0) || opts->max_iter < 0 || opts->bb < 1 || opts->bb > 3)
        return SC_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    const int n = p->n, nc = c->count;
    *st = sc_stats{};
    if (nc > 0 && (!gamma || !g)) return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 ||
        ws_bytes < solve_ws_bytes(n, c->capacity))
        return SC_ERR_WORKSPACE;
    Carver cv{static_cast<char *>(ws), ws_bytes};
    double *gam1 = cv.take<double>(c->capacity);
    double *g1 = cv.take<double>(c->capacity);
    double *U = cv.take<double>(6 * static_cast<size_t>(n));
    double *partials = cv.take<double>(4 * kMaxReduceBlocks);
    Ctrl *ctrl = cv.take<Ctrl>(1);
    if (!cv.ok) return SC_ERR_WORKSPACE;

    if (nc == 0) {
        // no constraints: the zero force solves the (empty) LCP after one product
        if (f_c) SC_HIP_TRY(hipMemsetAsync(f_c, 0, 6 * sizeof(double) * n, s));
        if (u_c) SC_HIP_TRY(hipMemsetAsync(u_c, 0, 6 * sizeof(double) * n, s));
        SC_HIP_TRY(hipStreamSynchronize(s));
        st->status = SC_OK;
        st->mvops = 1;
        return SC_OK;
    }
    PollSlots &ps = poll_slots();
    if (!ps.ok) return SC_ERR_HIP;

    Chain ch{n, nc, c->capacity, p->axis, p->mob, c->frame, c->q, c->ci, c->cj,
             c->i_ptr, c->j_ptr, c->j_list, U, partials, ctrl, s};
    double *G[2] = {gamma, gam1};
    double *Gg[2] = {g, g1};

    k_init_ctrl<<<1, 1, 0, s>>>(ctrl, opts->tol, opts->max_iter, opts->bb);
    if (!opts->warm_start) SC_HIP_TRY(hipMemsetAsync(gamma, 0, sizeof(double) * nc, s));
    // steps 2-6
    ch.phase_a(G[0], nullptr);
    ch.phase_b<kG0>(G[0], nullptr, nullptr, Gg[0]);
    k_phase_a<false><<<grid_for(n), kBlock, 0, s>>>(n, p->axis, p->mob, c->i_ptr, c->j_ptr,
                                                    c->j_list, c->frame, c->capacity, Gg[0],
                                                    nullptr, nullptr, U, nullptr, ctrl);
    ch.phase_b<kMG0>(nullptr, nullptr, Gg[0], nullptr);

    // steps 7-16, enqueued in chunks; poll one chunk behind
    const int chunk = opts->check_every > 0 ? opts->check_every : 16;
    int enqueued = 0, slot = 0, pending = 0;
    bool stop = false;
    ps.words[0] = ps.words[1] = 0;
    SC_HIP_TRY(hipEventRecord(ps.t0, s));
    while (!stop) {
        if (enqueued < opts->max_iter) {
            const int upto = enqueued + chunk < opts->max_iter ? enqueued + chunk : opts->max_iter;
            for (int j = enqueued + 1; j <= upto; ++j) {
                const int cur = (j - 1) & 1, nxt = j & 1;
                ch.phase_a_step(G[cur], Gg[cur], G[nxt]);
                ch.phase_b<kIter>(G[nxt], G[cur], Gg[cur], Gg[nxt]);
            }
            enqueued = upto;
            SC_HIP_TRY(hipMemcpyAsync(ps.words + slot, &ctrl->done, sizeof(int),
                                      hipMemcpyDeviceToHost, s));
            SC_HIP_TRY(hipEventRecord(ps.ev[slot], s));
            ++pending;
            slot ^= 1;
        } else {
            stop = true;
        }
        if (pending == 2 || stop) {
            // wait for the older chunk (the one in `slot` after the flip)
            if (pending > 0) {
                SC_HIP_TRY(hipEventSynchronize(ps.ev[slot]));
                --pending;
                if (ps.words[slot]) stop = true;
            }
        }
    }
    SC_HIP_TRY(hipEventRecord(ps.t1, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    float loop_ms = 0.0f;
    SC_HIP_TRY(hipEventElapsedTime(&loop_ms, ps.t0, ps.t1));
    Ctrl hc;
    SC_HIP_TRY(hipMemcpy(&hc, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
    // the last iterate lives in buffer (iters & 1)
    if (hc.iters & 1) {
        SC_HIP_TRY(hipMemcpyAsync(gamma, gam1, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
        SC_HIP_TRY(hipMemcpyAsync(g, g1, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
    }
    k_count_active<<<reduce_blocks(nc), kBlock, 0, s>>>(nc, gamma, ctrl);
    if (f_c || u_c) ch.phase_a(gamma, f_c, u_c);
    int nact = 0;
    SC_HIP_TRY(hipMemcpyAsync(&nact, &ctrl->n_active, sizeof(int), hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    st->status = hc.status;
    st->iters = hc.iters;
    st->mvops = hc.mvops;
    st->n_active = nact;
    st->residual = hc.res;
    st->alpha = hc.alpha;
    st->n_degenerate = hc.ndegen;
    st->loop_ms = loop_ms;
    return hc.status;
}
