// sc_mobsolve.hip -- BBPGD (Algorithm 1, section 3.3.1) behind a general
// mobility, and the Rotne-Prager-Yamakawa mobility of spheres.
//
// Section 2 defines the mobility as a dense SPD map from forces and torques to
// velocities, and in section 3.3 each product M x = D^T Mob D x is one
// mobility problem for the force D x. Here the mobility is a caller-supplied
// function (sc_mobility_fn) that enqueues u = Mob f on the solver's stream, so
// one iteration is a sequence of launches:
//
//   scatter: gamma_j = max(0, gamma_{j-1} - alpha g_{j-1}) formed on the fly
//            for every incidence (the owning incidence stores it) and
//            F = D gamma_j per particle, in caller order;
//   mobility: U = Mob F (the callback);
//   gather:  g_j = D^T U + q per contact, with block partials of
//            ||min(gamma_j, g_j)||^2, s^T s, s^T y, y^T y and |{gamma_j > 0}|;
//   finish:  one workgroup folds the partials in a fixed order and decides:
//            stop, or the next BB step size.
//
// The iteration index and the decision live on the device (MsCtrl), so the
// host enqueues iterations in chunks without waiting; once the finish kernel
// has set `done`, the remaining launches of the chunk return at once (the
// callback still runs on stale data, and its results are ignored). The host
// polls `done` one chunk behind, through pinned memory, so the GPU always has
// the next chunk queued.
//
// RPY (Zuk, Wajnryb, Mizerski and Szymczak, J. Fluid Mech. 2014, unequal
// radii with the overlap forms): translations couple pairwise, each sphere's
// rotation has its single-sphere mobility 1/(8 pi mu a^3), and rotations do
// not couple (this keeps Mob SPD). The pair sum is an O(n^2) tiled N-body
// kernel on the FP64 vector units: 64 targets per workgroup (one per lane,
// the four waves sharing out the sources), sources staged through LDS, the
// source range split over a second grid dimension so that small systems
// still fill the chip; wave and split partial sums are added in a fixed
// order, so the result is deterministic.
#include <cmath>

#include "sc_adjoint_dev.hpp"
#include "sc_common.hpp"
#include "sc_plan.hpp"
#include "sc_sync.hpp"

namespace sc {

namespace {

struct MsCtrl {
    double alpha, res;
    int iters;      // descent steps taken
    int mvops;      // products M x evaluated before the decision to stop
    int status;     // SC_OK, SC_NOT_CONVERGED, SC_ERR_NONFINITE
    int ndegen;
    int done;       // set once the solve has stopped
    int n_active;
    int final_buf;  // buffer (0/1) holding the last iterate
    int pad;
};

constexpr int kMsLanes = 4;     // lanes sharing one particle's incidence list
constexpr int kNV = 5;          // partial sums per gather block

struct MsView {
    int n, nc;
    const int *order;       // rank -> caller index
    const int *inc_ptr;     // [n+1] by rank
    const int *inc;         // incidence codes 2 l + owner
    const double *dpm;      // [2 cap][6] signed column entries
    const int *ci, *cj;     // caller indices (cj < 0: wall)
    const int *cs;          // [nc][2] ranks
    const double *pdat;     // [n][8] per rank
    const double *frame;    // [nc][9]
    const double *q;
};

__device__ __forceinline__ double project(double v) { return v < 0.0 ? 0.0 : v; }

// F = D w per particle (caller order). STEP: w_l = max(0, gc_l - alpha ggc_l),
// stored by the owning incidence into gn; otherwise w = x.
template <bool STEP>
__global__ void __launch_bounds__(kBlock)
k_ms_scatter(MsView V, const double *x, const double *gc, const double *ggc, double *gn,
             const MsCtrl *ctrl, double *f) {
    if (STEP && ctrl->done) return;
    const double alpha = STEP ? ctrl->alpha : 0.0;
    const int k = (blockIdx.x * kBlock + threadIdx.x) / kMsLanes;
    const int lane = threadIdx.x % kMsLanes;
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (k < V.n) {
        const int e1 = V.inc_ptr[k + 1];
        for (int e = V.inc_ptr[k] + lane; e < e1; e += kMsLanes) {
            const int code = V.inc[e];
            const int m = code >> 1;
            double w;
            if (STEP) {
                w = project(gc[m] - alpha * ggc[m]);
                if (code & 1) gn[m] = w;
            } else {
                w = x[m];
            }
            const double *d = V.dpm + 6 * static_cast<long long>(e);
#pragma unroll
            for (int c = 0; c < 6; ++c) a[c] += w * d[c];
        }
    }
#pragma unroll
    for (int off = kMsLanes / 2; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 6; ++c) a[c] += __shfl_xor(a[c], off, kWave);
    if (k < V.n && lane == 0) {
        double *fk = f + 6 * static_cast<long long>(V.order[k]);
#pragma unroll
        for (int c = 0; c < 6; ++c) fk[c] = a[c];
    }
}

// (D^T u)_l with u in caller order.
__device__ __forceinline__ double dt_u_caller(const MsView &V, const double *u, int l) {
    const double *fr = V.frame + 9 * static_cast<long long>(l);
    const double *ui = u + 6 * static_cast<long long>(V.ci[l]);
    const double vi = -(fr[0] * ui[0] + fr[1] * ui[1] + fr[2] * ui[2]) -
                      (fr[3] * ui[3] + fr[4] * ui[4] + fr[5] * ui[5]);
    const int j = V.cj[l];
    if (j < 0) return vi;  // wall contact: the particle's side only
    const double *uj = u + 6 * static_cast<long long>(j);
    return vi + (fr[0] * uj[0] + fr[1] * uj[1] + fr[2] * uj[2]) +
           (fr[6] * uj[3] + fr[7] * uj[4] + fr[8] * uj[5]);
}

// D_l^T Mob_self D_l from the particles' own (dry) mobility blocks.
__device__ __forceinline__ double self_diag(const MsView &V, int l) {
    const double *fr = V.frame + 9 * static_cast<long long>(l);
    const V3 nn = load3(fr);
    V3 u, w;
    plan_mobility(V.pdat + 8 * static_cast<long long>(V.cs[2 * l]), nn, load3(fr + 3), u, w);
    double d = dot(nn, u) + dot(load3(fr + 3), w);
    const int rj = V.cs[2 * l + 1];
    if (rj >= 0) {
        plan_mobility(V.pdat + 8 * static_cast<long long>(rj), nn, load3(fr + 6), u, w);
        d += dot(nn, u) + dot(load3(fr + 6), w);
    }
    return d;
}

enum { kG0 = 0, kAlpha0 = 1, kIter = 2 };

// Block partials of one gather, written to part[blockIdx.x][0..kNV).
__device__ __forceinline__ void ms_partials(double (&v)[kNV], double *part, bool max4) {
    __shared__ double red[kNV][kBlock / kWave];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < kNV; ++c) v[c] = (max4 && c == 4) ? wave_max(v[c]) : wave_sum(v[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < kNV; ++c) red[c][wid] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < kNV; ++c) {
            double s = red[c][0];
            for (int w = 1; w < kBlock / kWave; ++w)
                s = (max4 && c == 4) ? fmax(s, red[c][w]) : s + red[c][w];
            part[static_cast<long long>(blockIdx.x) * kNV + c] = s;
        }
    }
}

// kG0: out = D^T u + q for gamma = gam; partials (res2, -, -, -, active).
// kAlpha0: t = D^T u for x = g (= ggc); partials (g.g, g.t, -, -, max self diag).
// kIter: out = D^T u + q for gamma_j = gam (gamma_{j-1} = gc, g_{j-1} = ggc);
//        partials (res2, ss, sy, yy, active).
template <int MODE>
__global__ void __launch_bounds__(kBlock)
k_ms_gather(MsView V, const double *u, const double *gam, const double *gc, const double *ggc,
            double *out, const MsCtrl *ctrl, double *part) {
    if (MODE != kG0 && ctrl->done) return;
    double v[kNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l = blockIdx.x * kBlock + threadIdx.x; l < V.nc; l += gridDim.x * kBlock) {
        const double du = dt_u_caller(V, u, l);
        if (MODE == kAlpha0) {
            const double gl = ggc[l];
            v[0] += gl * gl;
            v[1] += gl * du;
            v[4] = fmax(v[4], self_diag(V, l));
        } else {
            const double gn = du + V.q[l];
            out[l] = gn;
            const double gm = gam[l];
            const double m = gm < gn ? gm : gn;
            v[0] += m * m;
            v[4] += gm > 0.0 ? 1.0 : 0.0;
            if (MODE == kIter) {
                const double s = gm - gc[l], y = gn - ggc[l];
                v[1] += s * s;
                v[2] += s * y;
                v[3] += y * y;
            }
        }
    }
    ms_partials(v, part, MODE == kAlpha0);
}

// One workgroup: fold the gather partials in a fixed order, then decide.
template <int MODE>
__global__ void __launch_bounds__(kBlock)
k_ms_finish(const double *part, int nparts, MsCtrl *ctrl, double tol, int max_iter, int bb) {
    if (MODE != kG0 && ctrl->done) return;
    __shared__ double tot[kNV];
    const int lane = threadIdx.x % kWave, c = threadIdx.x / kWave;
    // waves 0-3 fold values 0-3, then wave 0 folds value 4
    for (int pass = 0; pass < 2; ++pass) {
        const int k = pass == 0 ? c : 4;
        if (pass == 1 && c != 0) break;
        if (k < kNV) {
            const bool mx = MODE == kAlpha0 && k == 4;
            double x = 0.0;   // the self diagonal is >= 0
            for (int b = lane; b < nparts; b += kWave) {
                const double y = part[static_cast<long long>(b) * kNV + k];
                x = mx ? fmax(x, y) : x + y;
            }
            x = mx ? wave_max(x) : wave_sum(x);
            if (lane == 0) tot[k] = x;
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    MsCtrl C = *ctrl;
    if (MODE == kG0) {
        C.mvops = 1;
        C.iters = 0;
        C.res = sqrt(tot[0]);
        C.n_active = static_cast<int>(tot[4]);
        C.final_buf = 0;
        if (!std::isfinite(C.res)) {
            C.status = SC_ERR_NONFINITE;
            C.done = 1;
        } else if (C.res < tol) {
            C.status = SC_OK;
            C.done = 1;
        } else {
            C.status = SC_NOT_CONVERGED;
        }
    } else if (MODE == kAlpha0) {
        C.mvops = 2;
        const double num = tot[0], den = tot[1];
        if (den > 0.0 && std::isfinite(den) && std::isfinite(num)) {
            C.alpha = num / den;
        } else {
            C.alpha = tot[4] > 0.0 ? 1.0 / tot[4] : 1.0;
            C.ndegen += 1;
        }
        if (max_iter == 0) C.done = 1;
    } else {
        const int j = C.iters + 1;
        C.mvops += 1;
        C.iters = j;
        C.final_buf = j & 1;
        C.res = sqrt(tot[0]);
        C.n_active = static_cast<int>(tot[4]);
        if (!std::isfinite(C.res)) {
            C.status = SC_ERR_NONFINITE;
            C.done = 1;
        } else if (C.res < tol) {
            C.status = SC_OK;
            C.done = 1;
        } else {
            const bool bb2 = bb == 2 || (bb == 3 && (j % 2 == 0));
            const double num = bb2 ? tot[2] : tot[1];
            const double den = bb2 ? tot[3] : tot[2];
            if (den > 0.0 && num > 0.0 && std::isfinite(num) && std::isfinite(den))
                C.alpha = num / den;
            else
                C.ndegen += 1;
            if (j >= max_iter) C.done = 1;
        }
    }
    *ctrl = C;
}

// ---------------------------------------------------------- adjoint CG
//
// The masked system M_AA w_A = b_A of the implicit adjoint (not in the paper;
// the derivation is the dry solver's, which holds for any symmetric
// mobility) by conjugate gradients, one mobility call per iteration:
//   scatter: p = r + beta p_prev per incidence (owner stores), F = D p;
//   mobility: U = Mob F;
//   gather: t = mask(D^T U), partial p.t;   finish: alpha = rr / p.t;
//   update: x += alpha p, r -= alpha t, partial r.r;   finish: beta, stop.

struct CgMobCtrl {
    double alpha, beta, rr, rr0, res;
    int iters, status, done, n_active;
};

__global__ void __launch_bounds__(kBlock)
k_am_rhs(MsView V, const double *gamma, const double *dLdg, const double *dLdF, double *r,
         double *x, double *p0, double *part) {
    double v[kNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l = blockIdx.x * kBlock + threadIdx.x; l < V.nc; l += gridDim.x * kBlock) {
        const double b = cg_rhs_one(l, V.ci, V.cj, V.frame, gamma, dLdg, dLdF);
        r[l] = b;
        x[l] = 0.0;
        p0[l] = 0.0;
        v[0] += b * b;
        v[4] += gamma[l] > 0.0 ? 1.0 : 0.0;
    }
    ms_partials(v, part, false);
}

__global__ void __launch_bounds__(kBlock)
k_am_scatter(MsView V, const double *r, const double *pc, double *pn, const CgMobCtrl *ctrl,
             double *f) {
    if (ctrl->done) return;
    const double beta = ctrl->beta;
    const int k = (blockIdx.x * kBlock + threadIdx.x) / kMsLanes;
    const int lane = threadIdx.x % kMsLanes;
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (k < V.n) {
        const int e1 = V.inc_ptr[k + 1];
        for (int e = V.inc_ptr[k] + lane; e < e1; e += kMsLanes) {
            const int code = V.inc[e];
            const int m = code >> 1;
            const double w = r[m] + beta * pc[m];
            if (code & 1) pn[m] = w;
            const double *d = V.dpm + 6 * static_cast<long long>(e);
#pragma unroll
            for (int c = 0; c < 6; ++c) a[c] += w * d[c];
        }
    }
#pragma unroll
    for (int off = kMsLanes / 2; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 6; ++c) a[c] += __shfl_xor(a[c], off, kWave);
    if (k < V.n && lane == 0) {
        double *fk = f + 6 * static_cast<long long>(V.order[k]);
#pragma unroll
        for (int c = 0; c < 6; ++c) fk[c] = a[c];
    }
}

__global__ void __launch_bounds__(kBlock)
k_am_gather(MsView V, const double *u, const double *gamma, const double *p, double *tv,
            const CgMobCtrl *ctrl, double *part) {
    if (ctrl->done) return;
    double v[kNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l = blockIdx.x * kBlock + threadIdx.x; l < V.nc; l += gridDim.x * kBlock) {
        const double tl = gamma[l] > 0.0 ? dt_u_caller(V, u, l) : 0.0;
        tv[l] = tl;
        v[0] += p[l] * tl;
    }
    ms_partials(v, part, false);
}

__global__ void __launch_bounds__(kBlock)
k_am_update(int nc, const double *p, const double *tv, double *x, double *r,
            const CgMobCtrl *ctrl, double *part) {
    if (ctrl->done) return;
    const double alpha = ctrl->alpha;
    double v[kNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l = blockIdx.x * kBlock + threadIdx.x; l < nc; l += gridDim.x * kBlock) {
        x[l] = x[l] + alpha * p[l];
        const double rl = r[l] - alpha * tv[l];
        r[l] = rl;
        v[0] += rl * rl;
    }
    ms_partials(v, part, false);
}

// STAGE 0: rr0 after the right-hand side; 1: alpha; 2: beta and the stop test.
template <int STAGE>
__global__ void __launch_bounds__(kBlock)
k_am_finish(const double *part, int nparts, CgMobCtrl *ctrl, double tol, int max_iter) {
    if (STAGE != 0 && ctrl->done) return;
    __shared__ double tot[2];
    const int lane = threadIdx.x % kWave, c = threadIdx.x / kWave;
    if (c < 2) {
        const int k = c == 0 ? 0 : 4;
        double x = 0.0;
        for (int b = lane; b < nparts; b += kWave) x += part[static_cast<long long>(b) * kNV + k];
        x = wave_sum(x);
        if (lane == 0) tot[c] = x;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    CgMobCtrl C = *ctrl;
    if (STAGE == 0) {
        C.rr = C.rr0 = tot[0];
        C.beta = 0.0;
        C.res = tot[0] > 0.0 ? 1.0 : 0.0;
        C.n_active = static_cast<int>(tot[1]);
        if (!std::isfinite(tot[0])) {
            C.status = SC_ERR_NONFINITE;
            C.done = 1;
        } else if (tot[0] == 0.0) {
            C.status = SC_OK;
            C.done = 1;
        } else {
            C.status = SC_NOT_CONVERGED;
            if (max_iter == 0) C.done = 1;
        }
    } else if (STAGE == 1) {
        const double pt = tot[0];
        if (!std::isfinite(pt)) {
            C.status = SC_ERR_NONFINITE;
            C.done = 1;
        } else if (!(pt > 0.0)) {
            C.done = 1;   // M_AA not positive on p (numerically)
        } else {
            C.alpha = C.rr / pt;
        }
    } else {
        const double rr = tot[0];
        C.iters += 1;
        C.res = sqrt(rr / C.rr0);
        if (!std::isfinite(rr)) {
            C.status = SC_ERR_NONFINITE;
            C.done = 1;
        } else if (rr <= tol * tol * C.rr0) {
            C.status = SC_OK;
            C.done = 1;
        } else {
            C.beta = rr / C.rr;
            C.rr = rr;
            if (C.iters >= max_iter) C.done = 1;
        }
    }
    *ctrl = C;
}

__global__ void k_am_post(int nc, const double *gamma, const double *x, double *dLdq) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nc) dLdq[l] = gamma[l] > 0.0 ? -x[l] : 0.0;
}

// Caller-order [n][6] -> rank-order [n][8] (the layout of the geometric
// gradient's velocity reads).
__global__ void k_am_rank8(int n, const int *order, const double *src, double *dst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double *s = src + 6 * static_cast<long long>(order[k]);
    double *d = dst + 8 * static_cast<long long>(k);
    for (int c = 0; c < 6; ++c) d[c] = s[c];
    d[6] = 0.0;
    d[7] = 0.0;
}

__global__ void k_am_contact_grad(int nc, const int *ci, const int *cj, const int *cs,
                                  const double *pos, const double *axis, const double *half_len,
                                  PBox box, const double *gamma, const double *w,
                                  const double *dLdF, const double *Vw8, const double *Unc,
                                  const double *Uc8, double inv_dt, double *grad) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    const V3 g = contact_grad_one(l, ci, cj, cs, pos, axis, half_len, box, gamma, w, dLdF, Vw8,
                                  Unc, Uc8, inv_dt);
    double *o = grad + 3 * static_cast<long long>(l);
    o[0] = g.x;
    o[1] = g.y;
    o[2] = g.z;
}

__global__ void k_am_gather_pos(int n, Plan pl, const double *grad, double *out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) gather_pos_one(k, pl, grad, out);
}

// a += b (elementwise, m entries)
__global__ void k_am_add(long long m, double *a, const double *b) {
    const long long k = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < m) a[k] += b[k];
}

// a -= b (elementwise, m entries)
__global__ void k_am_sub(long long m, double *a, const double *b) {
    const long long k = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < m) a[k] -= b[k];
}

// ------------------------------------------------------------------ RPY

constexpr int kRpyBlock = 256;
constexpr int kRpyTargets = kWave;   // targets per workgroup
constexpr int kRpyMinSources = 64;   // smallest source range of one split
constexpr int kRpyMaxSplits = 64;    // bounds the partial sums (64 x n x 3 doubles)
// Workgroups per launch the splits aim at: measured on MI355X (256 CUs), about
// 16k short workgroups keep every CU busy to the end of the launch better than
// one round of long ones (20000 spheres: 0.53 ms against 0.66 ms at 4k).
constexpr int kRpyTargetBlocks = 16384;

struct RpyConst {
    double k8;      // 1 / (8 pi mu)
    double k6;      // 1 / (6 pi mu)
};

// 1/sqrt(x) for x > 0: the hardware estimate y (relative error below 2^-24,
// measured on 2^20 arguments from 1e-6 to 1e8) refined by one third-order
// step of the binomial series of (1 - e)^(-1/2), e = 1 - x y^2:
// y (1 + e/2 + 3 e^2 / 8), whose truncation error (about 5/16 e^3) is far
// below rounding; five operations against seven for two Newton steps.
__device__ __forceinline__ double rsqrt_refined(double x) {
#pragma clang fp contract(fast)
    const double y = __builtin_amdgcn_rsq(x);
    const double e = 1.0 - (x * y) * y;
    return y + (y * e) * (0.5 + 0.375 * e);
}

// acc += RPY(x_i - x_j; a_i, a_j) F_j / (8 pi mu) (translational coupling),
// with (fx, fy, fz) = F_j / (8 pi mu): the callers scale each source's force
// once when they load it, which takes a product out of every pair. The self
// pair (same index) adds nothing. Separated pairs take the first branch; the
// overlap forms and the self pair share the rare second one, whose
// 1 / (6 pi mu) prefactors become 4/3 relative to 1 / (8 pi mu).
__device__ __forceinline__ void rpy_pair(double dx, double dy, double dz, double ai, double aj,
                                         double fx, double fy, double fz, bool self, double &ux,
                                         double &uy, double &uz) {
    // The library is built without floating-point contraction (the contact
    // geometry rounds exactly as written); this sum, checked against the
    // oracle to a tolerance, lets the compiler fuse multiply-adds.
#pragma clang fp contract(fast)
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double sa = ai + aj;
    double A, B;   // U = A F + B (d.F) d, d unnormalised, F scaled as above
    if (r2 > sa * sa) {
        const double ri = rsqrt_refined(r2);
        const double ri2 = ri * ri;
        const double s2 = (ai * ai + aj * aj) * ri2;
        A = ri * (1.0 + s2 * (1.0 / 3.0));
        B = ri * (1.0 - s2) * ri2;
    } else {
        const double da = ai - aj;
        if (self) {
            A = 0.0;
            B = 0.0;
        } else if (r2 > da * da) {
            const double r = sqrt(r2);
            const double pre = (4.0 / 3.0) / (ai * aj);
            const double dd = da * da;
            const double t = dd + 3.0 * r2;
            const double r3 = r2 * r;
            A = pre * (16.0 * r3 * sa - t * t) / (32.0 * r3);
            const double w = dd - r2;
            B = pre * 3.0 * w * w / (32.0 * r3) / r2;
        } else {
            A = (4.0 / 3.0) / (ai > aj ? ai : aj);
            B = 0.0;
        }
    }
    const double dF = dx * fx + dy * fy + dz * fz;
    const double bd = B * dF;
    // two fused multiply-adds per component into the running sum
    ux += A * fx;
    ux += bd * dx;
    uy += A * fy;
    uy += bd * dy;
    uz += A * fz;
    uz += bd * dz;
}

// Workgroup: 64 targets (one per lane) and 4 waves; the waves take every
// fourth source of each LDS tile, and their sums are added in wave order.
// A source is three 16-byte pairs and one double in LDS, so a pair reads it
// with four LDS loads instead of seven (the LDS pipe is shared by the four
// SIMDs of the CU).
__global__ void __launch_bounds__(kRpyBlock)
k_rpy_pairs(int n, const double *__restrict__ pos, const double *__restrict__ rad,
            const double *__restrict__ f, RpyConst K, int splits, double *__restrict__ part) {
    constexpr int NW = kRpyBlock / kWave;
    __shared__ double2 sxy[kRpyBlock], sza[kRpyBlock], sfxy[kRpyBlock];
    __shared__ double sfz[kRpyBlock];
    __shared__ double red[3][kRpyBlock];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int i = blockIdx.x * kRpyTargets + lane;
    const int s = blockIdx.y;
    const int j0 = static_cast<int>(static_cast<long long>(s) * n / splits);
    const int j1 = static_cast<int>(static_cast<long long>(s + 1) * n / splits);
    const bool live = i < n;
    const double xi = live ? pos[3 * i] : 0.0, yi = live ? pos[3 * i + 1] : 0.0,
                 zi = live ? pos[3 * i + 2] : 0.0, ai = live ? rad[i] : 1.0;
    double ux = 0.0, uy = 0.0, uz = 0.0;
    for (int t = j0; t < j1; t += kRpyBlock) {
        const int cnt = j1 - t < kRpyBlock ? j1 - t : kRpyBlock;
        __syncthreads();
        if (threadIdx.x < cnt) {
            const int j = t + threadIdx.x;
            sxy[threadIdx.x] = make_double2(pos[3 * j], pos[3 * j + 1]);
            sza[threadIdx.x] = make_double2(pos[3 * j + 2], rad[j]);
            sfxy[threadIdx.x] = make_double2(K.k8 * f[6 * static_cast<long long>(j)],
                                             K.k8 * f[6 * static_cast<long long>(j) + 1]);
            sfz[threadIdx.x] = K.k8 * f[6 * static_cast<long long>(j) + 2];
        }
        __syncthreads();
        const int me = i - t;   // this target's own index within the tile, if there
#pragma unroll 2
        for (int m = w; m < cnt; m += NW) {
            const double2 p = sxy[m], q = sza[m], fq = sfxy[m];
            rpy_pair(xi - p.x, yi - p.y, zi - q.x, ai, q.y, fq.x, fq.y, sfz[m], m == me, ux, uy,
                     uz);
        }
    }
    red[0][threadIdx.x] = ux;
    red[1][threadIdx.x] = uy;
    red[2][threadIdx.x] = uz;
    __syncthreads();
    if (w == 0 && live) {
        double v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double acc = red[c][lane];
            for (int q = 1; q < NW; ++q) acc += red[c][q * kWave + lane];
            v[c] = acc;
        }
        double *p = part + 3 * (static_cast<long long>(s) * n + i);
        p[0] = v[0];
        p[1] = v[1];
        p[2] = v[2];
    }
}

// u = self terms + the splits' sums (in split order); one thread per
// (sphere, component), so the split loads of a wave are independent.
__global__ void k_rpy_finish(int n, const double *rad, const double *f, RpyConst K, int splits,
                             const double *part, double *u) {
    const long long k = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= 6LL * n) return;
    const int i = static_cast<int>(k / 6), c = static_cast<int>(k % 6);
    const double a = rad[i];
    const double fi = f[k];
    if (c >= 3) {
        u[k] = 0.75 * K.k6 / (a * a * a) * fi;   // 1/(8 pi mu a^3)
        return;
    }
    double acc = K.k6 / a * fi;                  // 1/(6 pi mu a)
    const double *p = part + 3LL * i + c;
    const long long stride = 3LL * n;
#pragma unroll 8
    for (int s = 0; s < splits; ++s) acc += p[s * stride];
    u[k] = acc;
}

// Gradient of s(d) = a_k^T M(d) f_j + a_j^T M(d) f_k in d = c_k - c_j, with
// M = A(r) I + Bt(r) d d^T per branch (A, Bt and their r-derivatives), added
// to (gx, gy, gz); the self pair and one sphere inside the other add nothing.
__device__ __forceinline__ void rpy_grad_pair(const RpyConst &K, double dx, double dy, double dz,
                                              double ai, double aj, const double (&ak)[3],
                                              const double (&fk)[3], double ajx, double ajy,
                                              double ajz, double fjx, double fjy, double fjz,
                                              bool self, double &gx, double &gy, double &gz) {
#pragma clang fp contract(fast)
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double sa = ai + aj;
    double dA, Bt, dB, ri;
    if (r2 > sa * sa) {
        ri = rsqrt_refined(r2);
        const double ri2 = ri * ri;
        const double S = ai * ai + aj * aj;
        dA = K.k8 * ri2 * (-1.0 - S * ri2);
        Bt = K.k8 * ri2 * ri * (1.0 - S * ri2);
        dB = K.k8 * ri2 * ri2 * (-3.0 + 5.0 * S * ri2);
    } else {
        const double da = ai - aj;
        const double d2 = da * da;
        if (self || !(r2 > d2)) return;
        const double r = sqrt(r2);
        ri = 1.0 / r;
        const double pre = K.k6 / (ai * aj) * (3.0 / 32.0);
        const double T = d2 + 3.0 * r2;
        const double ri4 = ri * ri * ri * ri;
        const double w = d2 - r2;
        dA = -pre * T * (r2 - d2) * ri4;
        Bt = pre * w * w * ri4 * ri;
        dB = pre * w * (r2 - 5.0 * d2) * ri4 * ri * ri;
    }
    const double P = ak[0] * fjx + ak[1] * fjy + ak[2] * fjz + ajx * fk[0] + ajy * fk[1] +
                     ajz * fk[2];
    const double akd = ak[0] * dx + ak[1] * dy + ak[2] * dz;
    const double ajd = ajx * dx + ajy * dy + ajz * dz;
    const double fkd = fk[0] * dx + fk[1] * dy + fk[2] * dz;
    const double fjd = fjx * dx + fjy * dy + fjz * dz;
    const double Q = akd * fjd + ajd * fkd;
    const double cd = (dA * P + dB * Q) * ri;
    gx += cd * dx + Bt * (fjd * ak[0] + akd * fjx + fkd * ajx + ajd * fk[0]);
    gy += cd * dy + Bt * (fjd * ak[1] + akd * fjy + fkd * ajy + ajd * fk[1]);
    gz += cd * dz + Bt * (fjd * ak[2] + akd * fjz + fkd * ajz + ajd * fk[2]);
}

// g_k = sum_j of the pair gradients, laid out like k_rpy_pairs (64 targets
// per workgroup, the waves sharing each LDS tile of sources, source splits
// over the second grid dimension, fixed-order sums).
__global__ void __launch_bounds__(kRpyBlock)
k_rpy_grad_pairs(int n, const double *__restrict__ pos, const double *__restrict__ rad,
                 const double *__restrict__ a, const double *__restrict__ f, RpyConst K,
                 int splits, double *__restrict__ part) {
    constexpr int NW = kRpyBlock / kWave;
    __shared__ double sx[kRpyBlock], sy[kRpyBlock], sz[kRpyBlock], sr[kRpyBlock];
    __shared__ double sa[3][kRpyBlock], sf[3][kRpyBlock];
    __shared__ double red[3][kRpyBlock];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int i = blockIdx.x * kRpyTargets + lane;
    const int s = blockIdx.y;
    const int j0 = static_cast<int>(static_cast<long long>(s) * n / splits);
    const int j1 = static_cast<int>(static_cast<long long>(s + 1) * n / splits);
    const bool live = i < n;
    const double xi = live ? pos[3 * i] : 0.0, yi = live ? pos[3 * i + 1] : 0.0,
                 zi = live ? pos[3 * i + 2] : 0.0, ai = live ? rad[i] : 1.0;
    double ak[3], fk[3];
    for (int c = 0; c < 3; ++c) {
        ak[c] = live ? a[6 * static_cast<long long>(i) + c] : 0.0;
        fk[c] = live ? f[6 * static_cast<long long>(i) + c] : 0.0;
    }
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int t = j0; t < j1; t += kRpyBlock) {
        const int cnt = j1 - t < kRpyBlock ? j1 - t : kRpyBlock;
        __syncthreads();
        if (threadIdx.x < cnt) {
            const int j = t + threadIdx.x;
            sx[threadIdx.x] = pos[3 * j];
            sy[threadIdx.x] = pos[3 * j + 1];
            sz[threadIdx.x] = pos[3 * j + 2];
            sr[threadIdx.x] = rad[j];
            for (int c = 0; c < 3; ++c) {
                sa[c][threadIdx.x] = a[6 * static_cast<long long>(j) + c];
                sf[c][threadIdx.x] = f[6 * static_cast<long long>(j) + c];
            }
        }
        __syncthreads();
        const int me = i - t;
        for (int m = w; m < cnt; m += NW)
            rpy_grad_pair(K, xi - sx[m], yi - sy[m], zi - sz[m], ai, sr[m], ak, fk, sa[0][m],
                          sa[1][m], sa[2][m], sf[0][m], sf[1][m], sf[2][m], m == me, gx, gy, gz);
    }
    red[0][threadIdx.x] = gx;
    red[1][threadIdx.x] = gy;
    red[2][threadIdx.x] = gz;
    __syncthreads();
    if (w == 0 && live) {
        double *p = part + 3 * (static_cast<long long>(s) * n + i);
        for (int c = 0; c < 3; ++c) {
            double acc = red[c][lane];
            for (int q = 1; q < NW; ++q) acc += red[c][q * kWave + lane];
            p[c] = acc;
        }
    }
}

// g = sum of the splits' partial gradients, in split order.
__global__ void k_rpy_grad_finish(int n, int splits, const double *part, double *g) {
    const long long k = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= 3LL * n) return;
    double acc = 0.0;
    const long long stride = 3LL * n;
#pragma unroll 8
    for (int s = 0; s < splits; ++s) acc += part[k + s * stride];
    g[k] = acc;
}

int rpy_splits(int n) {
    const int bx = grid_for(n, kRpyTargets);
    int s = (kRpyTargetBlocks + bx - 1) / bx;
    const long long smax = (static_cast<long long>(n) + kRpyMinSources - 1) / kRpyMinSources;
    if (s > smax) s = static_cast<int>(smax);
    if (s > kRpyMaxSplits) s = kRpyMaxSplits;
    return s < 1 ? 1 : s;
}

// ------------------------------------------------- persistent RPY solve
//
// Algorithm 1 with the RPY mobility in one cooperative launch (one 1024-thread
// workgroup per CU), for systems small enough that launch gaps would
// dominate the callback path. One iteration is two phases separated by grid
// barriers. Pairs: the RPY sum in units of 64 targets x one source split (the
// 16 waves of a workgroup take every 16th source of each LDS tile; partial
// sums per split); each unit forms F = D gamma_j of its sources itself, with
// gamma_j = max(0, gamma_{j-1} - alpha g_{j-1}) taken per incidence from the
// previous iterate, and the units of the first target block store F for the
// self terms. Gather: gamma_j per contact (stored), U from the self terms and
// the splits' partial sums, g = D^T U + q and the iteration's partial sums.
// A fixed-order grid reduction follows, after which every workgroup takes
// the same decision. All sums are in fixed orders, so the iterates are
// reproducible for a given grid.

constexpr int kPB = 1024;                 // threads per workgroup
constexpr int kPW = kPB / kWave;          // waves per workgroup
constexpr int kPLanes = 4;                // threads forming one source's F
constexpr int kPTile = kPB / kPLanes;     // sources per LDS tile

struct RpyPersArgs {
    MsView V;
    const double *pos, *rad;
    RpyConst K;
    int splits;
    double *F;            // [n][6] caller order
    double *part;         // [splits][n][3]
    double *gam[2], *gg[2];
    double *red;          // [grid][kNV]
    GridSync *sync;
    MsCtrl *ctrl;
    double tol;
    int max_iter, bb;
};

// What the pair phase multiplies by D: x itself, or (step) the projected
// step max(0, gc - alpha ggc). A runtime flag, so that the pair phase and
// its LDS tiles exist once in the kernel.
struct PWeights {
    const double *x, *gc, *ggc;
    double alpha;
    bool step;
};

// Source of rank k for the pair sum: centre, radius and the force part of
// F_k = sum over its incidences of w_m D-column entries. kPLanes adjacent
// threads take every kPLanes-th incidence and add their sums in a fixed
// butterfly, so all of them must call this together; lane 0 stores the whole
// F_k (force and torque) when `store`.
__device__ __forceinline__ void p_source(const RpyPersArgs &A, const PWeights &Wt, int k,
                                         int lane, bool store, double (&v)[7]) {
    const MsView &V = A.V;
    const int j = V.order[k];
    v[0] = A.pos[3 * j];
    v[1] = A.pos[3 * j + 1];
    v[2] = A.pos[3 * j + 2];
    v[3] = A.rad[j];
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int e1 = V.inc_ptr[k + 1];
    for (int e = V.inc_ptr[k] + lane; e < e1; e += kPLanes) {
        const int m = V.inc[e] >> 1;
        const double w = Wt.step ? project(Wt.gc[m] - Wt.alpha * Wt.ggc[m]) : Wt.x[m];
        const double *d = V.dpm + 6 * static_cast<long long>(e);
#pragma unroll
        for (int c = 0; c < 6; ++c) a[c] += w * d[c];
    }
#pragma unroll
    for (int off = kPLanes / 2; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 6; ++c) a[c] += __shfl_xor(a[c], off, kWave);
    v[4] = a[0];
    v[5] = a[1];
    v[6] = a[2];
    if (store && lane == 0) {
        double *fj = A.F + 6 * static_cast<long long>(j);
#pragma unroll
        for (int c = 0; c < 6; ++c) fj[c] = a[c];
    }
}

// The RPY pair sum: units (64-target block, source split), dealt to the
// workgroups in logical order; part[s][i] = sum over split s of the pairs.
// Splits are ranges of ranks (sources in the contact plan's order).
__device__ void p_pairs(const RpyPersArgs &A, const PWeights &Wt) {
    __shared__ double sx[kPTile], sy[kPTile], sz[kPTile], sa[kPTile];
    __shared__ double sfx[kPTile], sfy[kPTile], sfz[kPTile];
    __shared__ int sj[kPTile];
    __shared__ double red3[3][kPB];
    const int n = A.V.n, S = A.splits;
    const int bx = (n + kRpyTargets - 1) / kRpyTargets;
    const int units = bx * S;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int src = threadIdx.x / kPLanes, sl = threadIdx.x % kPLanes;
    for (int u = logical_block(); u < units; u += gridDim.x) {
        const int tx = u % bx, s = u / bx;
        const bool store = tx == 0;
        const int i = tx * kRpyTargets + lane;
        const int k0 = static_cast<int>(static_cast<long long>(s) * n / S);
        const int k1 = static_cast<int>(static_cast<long long>(s + 1) * n / S);
        const bool live = i < n;
        const double xi = live ? A.pos[3 * i] : 0.0, yi = live ? A.pos[3 * i + 1] : 0.0,
                     zi = live ? A.pos[3 * i + 2] : 0.0, ai = live ? A.rad[i] : 1.0;
        double ux = 0.0, uy = 0.0, uz = 0.0;
        // the next tile's sources are formed in registers while the current
        // tile is summed
        double nv[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int nj = -1;
        if (k0 + src < k1) {   // the same for the kPLanes threads of a source
            p_source(A, Wt, k0 + src, sl, store, nv);
            nj = A.V.order[k0 + src];
        }
        for (int t = k0; t < k1; t += kPTile) {
            const int cnt = k1 - t < kPTile ? k1 - t : kPTile;
            __syncthreads();
            if (sl == 0 && src < cnt) {
                sx[src] = nv[0];
                sy[src] = nv[1];
                sz[src] = nv[2];
                sa[src] = nv[3];
                sfx[src] = A.K.k8 * nv[4];
                sfy[src] = A.K.k8 * nv[5];
                sfz[src] = A.K.k8 * nv[6];
                sj[src] = nj;
            }
            __syncthreads();
            const int tn = t + kPTile;
            if (tn + src < k1) {
                p_source(A, Wt, tn + src, sl, store, nv);
                nj = A.V.order[tn + src];
            }
            for (int m = w; m < cnt; m += kPW)
                rpy_pair(xi - sx[m], yi - sy[m], zi - sz[m], ai, sa[m], sfx[m], sfy[m],
                         sfz[m], sj[m] == i, ux, uy, uz);
        }
        red3[0][threadIdx.x] = ux;
        red3[1][threadIdx.x] = uy;
        red3[2][threadIdx.x] = uz;
        __syncthreads();
        if (w == 0 && live) {
            double *pp = A.part + 3 * (static_cast<long long>(s) * n + i);
            for (int c = 0; c < 3; ++c) {
                double acc = red3[c][lane];
                for (int q = 1; q < kPW; ++q) acc += red3[c][q * kWave + lane];
                pp[c] = acc;
            }
        }
        __syncthreads();
    }
}

// U of particle i: the self terms plus the splits' sums, in split order.
// The split loads go out in groups of kPGroup before any is added, so a
// contact waits about S / kPGroup memory latencies instead of 3 S.
constexpr int kPGroup = 4;
__device__ __forceinline__ void p_velocity(const RpyPersArgs &A, int i, double (&u)[6]) {
    const double a = A.rad[i];
    const double *fi = A.F + 6 * static_cast<long long>(i);
    const double st = A.K.k6 / a, sr = 0.75 * A.K.k6 / (a * a * a);
    const long long stride = 3LL * A.V.n;
    const double *pp = A.part + 3LL * i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        u[c] = st * fi[c];
        u[3 + c] = sr * fi[3 + c];
    }
    const int S = A.splits;
    int s = 0;
    for (; s + kPGroup <= S; s += kPGroup) {
        double t[kPGroup][3];
#pragma unroll
        for (int k = 0; k < kPGroup; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) t[k][c] = pp[(s + k) * stride + c];
#pragma unroll
        for (int k = 0; k < kPGroup; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) u[c] += t[k][c];
    }
    for (; s < S; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) u[c] += pp[s * stride + c];
}

// D_l^T U for contact l with U formed from the partial sums.
__device__ __forceinline__ double p_dt_u(const RpyPersArgs &A, int l) {
    const MsView &V = A.V;
    const double *fr = V.frame + 9 * static_cast<long long>(l);
    double ui[6];
    p_velocity(A, V.ci[l], ui);
    const double vi = -(fr[0] * ui[0] + fr[1] * ui[1] + fr[2] * ui[2]) -
                      (fr[3] * ui[3] + fr[4] * ui[4] + fr[5] * ui[5]);
    const int j = V.cj[l];
    if (j < 0) return vi;
    double uj[6];
    p_velocity(A, j, uj);
    return vi + (fr[0] * uj[0] + fr[1] * uj[1] + fr[2] * uj[2]) +
           (fr[6] * uj[3] + fr[7] * uj[4] + fr[8] * uj[5]);
}

// The gather over this workgroup's contacts; modes as k_ms_gather. kIter
// forms gamma_j = max(0, gc - alpha ggc) per contact and stores it in gn.
// Partials go to A.red through write_partial (slot = logical workgroup).
template <int MODE>
__device__ void p_gather(const RpyPersArgs &A, const double *gam, const double *gc,
                         const double *ggc, double alpha, double *gn, double *out) {
    const MsView &V = A.V;
    int l0, l1;
    chunk(V.nc, l0, l1);
    double v[kNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int l = l0 + threadIdx.x; l < l1; l += kPB) {
        const double du = p_dt_u(A, l);
        if (MODE == kAlpha0) {
            const double gl = ggc[l];
            v[0] += gl * gl;
            v[1] += gl * du;
            v[4] = fmax(v[4], self_diag(V, l));
        } else {
            double gm;
            if (MODE == kIter) {
                gm = project(gc[l] - alpha * ggc[l]);
                gn[l] = gm;
            } else {
                gm = gam[l];
            }
            const double gnew = du + V.q[l];
            out[l] = gnew;
            const double m = gm < gnew ? gm : gnew;
            v[0] += m * m;
            v[4] += gm > 0.0 ? 1.0 : 0.0;
            if (MODE == kIter) {
                const double sd = gm - gc[l], y = gnew - ggc[l];
                v[1] += sd * sd;
                v[2] += sd * y;
                v[3] += y * y;
            }
        }
    }
    write_partial<kNV, kPB, MODE == kAlpha0 ? 4 : -1>(A.red, v);
}

__global__ void __launch_bounds__(kPB) k_bbpgd_rpy(RpyPersArgs A) {
    GridBarrier bar;
    bar.init(A.sync);
    double tot[kNV];
    double alpha = 0.0, res = 0.0;
    int status = SC_NOT_CONVERGED, iters = 0, mvops = 0, ndegen = 0, n_active = 0, last = 0;
    // g0 = M gamma0 + q
    p_pairs(A, PWeights{A.gam[0], nullptr, nullptr, 0.0, false});
    bool ok = bar.sync();
    p_gather<kG0>(A, A.gam[0], nullptr, nullptr, 0.0, nullptr, A.gg[0]);
    ok = ok && bar.sync();
    grid_reduce<kNV, kPB>(A.red, tot);
    mvops = 1;
    res = sqrt(tot[0]);
    n_active = static_cast<int>(tot[4]);
    if (!ok) {
        status = SC_ERR_TIMEOUT;
    } else if (!isfinite(res)) {
        status = SC_ERR_NONFINITE;
    } else if (res < A.tol) {
        status = SC_OK;
    } else {
        // alpha0 = g0^T g0 / g0^T M g0 (fallback: 1 / max self diagonal)
        p_pairs(A, PWeights{A.gg[0], nullptr, nullptr, 0.0, false});
        ok = bar.sync();
        p_gather<kAlpha0>(A, nullptr, nullptr, A.gg[0], 0.0, nullptr, nullptr);
        ok = ok && bar.sync();
        grid_reduce<kNV, kPB, 4>(A.red, tot);
        mvops = 2;
        if (tot[1] > 0.0 && isfinite(tot[1]) && isfinite(tot[0])) {
            alpha = tot[0] / tot[1];
        } else {
            alpha = tot[4] > 0.0 ? 1.0 / tot[4] : 1.0;
            ++ndegen;
        }
        if (!ok) status = SC_ERR_TIMEOUT;
        for (int j = 1; ok && j <= A.max_iter; ++j) {
            const int cur = (j - 1) & 1, nxt = j & 1;
            // both phases read gamma_{j-1}, g_{j-1} (buffers cur); the gather
            // stores gamma_j, g_j (buffers nxt), which nothing reads before
            // the barrier that ends this iteration
            p_pairs(A, PWeights{nullptr, A.gam[cur], A.gg[cur], alpha, true});
            ok = bar.sync();
            p_gather<kIter>(A, nullptr, A.gam[cur], A.gg[cur], alpha, A.gam[nxt], A.gg[nxt]);
            ok = ok && bar.sync();
            grid_reduce<kNV, kPB>(A.red, tot);
            iters = j;
            last = nxt;
            ++mvops;
            res = sqrt(tot[0]);
            n_active = static_cast<int>(tot[4]);
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
            const bool bb2 = A.bb == 2 || (A.bb == 3 && (j % 2 == 0));
            const double num = bb2 ? tot[2] : tot[1];
            const double den = bb2 ? tot[3] : tot[2];
            if (den > 0.0 && num > 0.0 && isfinite(num) && isfinite(den))
                alpha = num / den;
            else
                ++ndegen;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        MsCtrl C;
        C.alpha = alpha;
        C.res = res;
        C.iters = iters;
        C.mvops = mvops;
        C.status = status;
        C.ndegen = ndegen;
        C.done = 1;
        C.n_active = n_active;
        C.final_buf = last;
        C.pad = 0;
        *A.ctrl = C;
    }
}

// Source splits of the persistent pair phase: about one (target block,
// split) unit per workgroup, so that each workgroup loads and reduces once
// per product and U sums few partials (measured faster than two or four
// units per workgroup up to 2000 spheres); never more than rpy_splits(n),
// whose partial sums the sc_rpy workspace holds.
int rpy_pers_splits(int n, int grid) {
    const int bx = grid_for(n, kRpyTargets);
    int s = (grid + bx - 1) / bx;
    const int smax = rpy_splits(n);
    if (s > smax) s = smax;
    return s < 1 ? 1 : s;
}

size_t rpy_pers_ws_bytes(int32_t n, int32_t cap) {
    const size_t nn = static_cast<size_t>(n), cc = static_cast<size_t>(cap);
    size_t b = 0;
    b += 2 * align_up(cc * sizeof(double), 256);       // second gamma / g buffers
    b += align_up(6 * nn * sizeof(double), 256);       // F
    b += align_up(kNV * kMaxReduceBlocks * sizeof(double), 256);
    b += align_up(sizeof(GridSync), 256);
    b += align_up(sizeof(MsCtrl), 256);
    return b + 1024;
}

// ------------------------------------------------------------------ host

// Host copies of a control block, one per chunk parity, in pinned memory
// (allocated once per host thread, kept for the life of the process).
constexpr size_t kPinnedSlot = 128;
static_assert(sizeof(MsCtrl) <= kPinnedSlot && sizeof(CgMobCtrl) <= kPinnedSlot, "pinned slot");

thread_local char *tl_pinned = nullptr;

char *pinned_slots() {
    char *&p = tl_pinned;
    if (!p && hipHostMalloc(reinterpret_cast<void **>(&p), 2 * kPinnedSlot,
                            hipHostMallocDefault) != hipSuccess)
        p = nullptr;
    return p;
}

struct Events {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};  // t0, t1, chunk parity 0, 1
    bool ok = true;
    Events() {
        for (int k = 0; k < 4; ++k)
            if (hipEventCreateWithFlags(&e[k], k < 2 ? hipEventDefault : hipEventDisableTiming) !=
                hipSuccess) {
                e[k] = nullptr;
                ok = false;
            }
    }
    ~Events() {
        for (auto ev : e)
            if (ev) (void)hipEventDestroy(ev);
    }
};

size_t am_ws_bytes(int32_t n, int32_t cap) {
    const size_t nn = static_cast<size_t>(n), cc = static_cast<size_t>(cap);
    size_t b = 0;
    b += 5 * align_up(cc * sizeof(double), 256);       // r, t, x, p (two buffers)
    b += align_up(3 * cc * sizeof(double), 256);       // per-contact gradient
    b += 7 * align_up(6 * nn * sizeof(double), 256);   // F, U, F_w, V_w, F_c, U_c, F_tot
    b += 2 * align_up(8 * nn * sizeof(double), 256);   // V_w, U_c in rank order
    b += align_up(3 * nn * sizeof(double), 256);       // mobility gradient
    b += align_up(kNV * kMaxReduceBlocks * sizeof(double), 256);
    b += align_up(sizeof(CgMobCtrl), 256);
    return b + 2048;
}

size_t ms_ws_bytes(int32_t n, int32_t cap) {
    const size_t nn = static_cast<size_t>(n), cc = static_cast<size_t>(cap);
    size_t b = 0;
    b += 2 * align_up(cc * sizeof(double), 256);       // second gamma / g buffers
    b += 2 * align_up(6 * nn * sizeof(double), 256);   // F, U (caller order)
    b += align_up(kNV * kMaxReduceBlocks * sizeof(double), 256);
    b += align_up(sizeof(MsCtrl), 256);
    return b + 1024;
}

}  // namespace

// Frees the calling thread's pinned control-block slots (allocated again on
// the next solve that needs them).
void release_mob_host() {
    if (tl_pinned) (void)hipHostFree(tl_pinned);
    tl_pinned = nullptr;
}

}  // namespace sc

using namespace sc;

extern "C" size_t sc_rpy_work_bytes(int32_t n) {
    if (n <= 0) return 256;
    return align_up(3 * sizeof(double) * static_cast<size_t>(rpy_splits(n)) * n, 256) + 256;
}

extern "C" int sc_rpy_apply(void *ctx, int32_t n, const double *f, double *u, void *stream) {
    const sc_rpy *R = static_cast<const sc_rpy *>(ctx);
    if (!R || n < 0 || n != R->n || !(R->mu > 0.0) || !std::isfinite(R->mu)) return SC_ERR_INVALID;
    if (n == 0) return SC_OK;
    if (!R->pos || !R->radius || !f || !u) return SC_ERR_INVALID;
    if (!R->work || (reinterpret_cast<uintptr_t>(R->work) & 255) != 0 ||
        R->work_bytes < sc_rpy_work_bytes(n))
        return SC_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int splits = rpy_splits(n);
    const RpyConst K{1.0 / (8.0 * M_PI * R->mu), 1.0 / (6.0 * M_PI * R->mu)};
    double *part = static_cast<double *>(R->work);
    const dim3 grid(grid_for(n, kRpyTargets), splits);
    k_rpy_pairs<<<grid, kRpyBlock, 0, s>>>(n, R->pos, R->radius, f, K, splits, part);
    k_rpy_finish<<<grid_for(6LL * n), kBlock, 0, s>>>(n, R->radius, f, K, splits, part, u);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}

extern "C" int sc_rpy_grad(void *ctx, int32_t n, const double *a, const double *f, double *g,
                           void *stream) {
    const sc_rpy *R = static_cast<const sc_rpy *>(ctx);
    if (!R || n < 0 || n != R->n || !(R->mu > 0.0) || !std::isfinite(R->mu)) return SC_ERR_INVALID;
    if (n == 0) return SC_OK;
    if (!R->pos || !R->radius || !a || !f || !g) return SC_ERR_INVALID;
    if (!R->work || (reinterpret_cast<uintptr_t>(R->work) & 255) != 0 ||
        R->work_bytes < sc_rpy_work_bytes(n))
        return SC_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int splits = rpy_splits(n);
    const RpyConst K{1.0 / (8.0 * M_PI * R->mu), 1.0 / (6.0 * M_PI * R->mu)};
    double *part = static_cast<double *>(R->work);
    const dim3 grid(grid_for(n, kRpyTargets), splits);
    k_rpy_grad_pairs<<<grid, kRpyBlock, 0, s>>>(n, R->pos, R->radius, a, f, K, splits, part);
    k_rpy_grad_finish<<<grid_for(3LL * n), kBlock, 0, s>>>(n, splits, part, g);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}

extern "C" int sc_dry_apply(void *ctx, int32_t n, const double *f, double *u, void *stream) {
    const sc_particles *p = static_cast<const sc_particles *>(ctx);
    if (!p || n != p->n) return SC_ERR_INVALID;
    return sc_apply_mobility(p, f, u, stream);
}

extern "C" size_t sc_solve_mob_work_bytes(int32_t n, int32_t capacity) {
    if (n < 0 || capacity < 0) return 0;
    return ms_ws_bytes(n, capacity);
}

extern "C" int sc_solve_lcp_mob(const sc_particles *p, const sc_contacts *c,
                                const sc_solve_opts *opts, sc_mobility_fn mob, void *mob_ctx,
                                int32_t check_every, double *gamma, double *g, double *f_c,
                                double *u_c, sc_stats *st, void *ws, size_t ws_bytes,
                                void *stream_) {
    if (!p || !c || !opts || !st || !mob || p->n < 0 || c->count < 0 || c->count > c->capacity)
        return SC_ERR_INVALID;
    if (!(opts->tol > 0.0) || opts->max_iter < 0 || opts->bb < 1 || opts->bb > 3 ||
        check_every < 0 || check_every > 4096)
        return SC_ERR_INVALID;
    Plan pl;
    if (!carve_plan(c->plan, c->plan_bytes, p->n, c->capacity, pl)) return SC_ERR_INVALID;
    const int n = p->n, nc = c->count;
    if (nc > 0 && (!c->ci || !c->cj || !c->frame || !c->q || !gamma || !g)) return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 ||
        ws_bytes < ms_ws_bytes(n, c->capacity))
        return SC_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    *st = sc_stats{};
    Carver cv{static_cast<char *>(ws), ws_bytes};
    double *gam1 = cv.take<double>(static_cast<size_t>(c->capacity));
    double *g1 = cv.take<double>(static_cast<size_t>(c->capacity));
    double *F = cv.take<double>(6 * static_cast<size_t>(n));
    double *U = cv.take<double>(6 * static_cast<size_t>(n));
    double *part = cv.take<double>(kNV * static_cast<size_t>(kMaxReduceBlocks));
    MsCtrl *ctrl = cv.take<MsCtrl>(1);
    if (!cv.ok) return SC_ERR_WORKSPACE;

    if (nc == 0) {
        // no constraints: the zero force; U_c = Mob 0 = 0
        if (f_c) SC_HIP_TRY(hipMemsetAsync(f_c, 0, 6 * sizeof(double) * n, s));
        if (u_c) SC_HIP_TRY(hipMemsetAsync(u_c, 0, 6 * sizeof(double) * n, s));
        SC_HIP_TRY(hipStreamSynchronize(s));
        st->status = SC_OK;
        st->mvops = 1;
        return SC_OK;
    }
    char *slots = pinned_slots();
    Events ev;
    if (!slots || !ev.ok) return SC_ERR_HIP;
    MsCtrl *hc0 = reinterpret_cast<MsCtrl *>(slots);
    MsCtrl *hc1 = reinterpret_cast<MsCtrl *>(slots + kPinnedSlot);
    MsCtrl *hctrl[2] = {hc0, hc1};
    hipEvent_t t0 = ev.e[0], t1 = ev.e[1];

    const MsView V{n, nc, pl.order, pl.inc_ptr, pl.inc, pl.dpm, c->ci, c->cj, pl.cs, pl.pdat,
                   c->frame, c->q};
    double *gam[2] = {gamma, gam1};
    double *gg[2] = {g, g1};
    const int sb = grid_for(static_cast<long long>(n) * kMsLanes);
    int gb = grid_for(nc);
    if (gb > kMaxReduceBlocks) gb = kMaxReduceBlocks;
    const double tol = opts->tol;
    const int max_iter = opts->max_iter, bb = opts->bb;
    const int K = check_every > 0 ? check_every : 4;

    if (!opts->warm_start) SC_HIP_TRY(hipMemsetAsync(gamma, 0, sizeof(double) * nc, s));
    SC_HIP_TRY(hipMemsetAsync(ctrl, 0, sizeof(MsCtrl), s));
    SC_HIP_TRY(hipEventRecord(t0, s));
    int rc = SC_OK;
    // g0 = M gamma0 + q
    k_ms_scatter<false><<<sb, kBlock, 0, s>>>(V, gamma, nullptr, nullptr, nullptr, ctrl, F);
    rc = mob(mob_ctx, n, F, U, s);
    if (rc) return rc;
    k_ms_gather<kG0><<<gb, kBlock, 0, s>>>(V, U, gamma, nullptr, nullptr, g, ctrl, part);
    k_ms_finish<kG0><<<1, kBlock, 0, s>>>(part, gb, ctrl, tol, max_iter, bb);
    // alpha0 = g0^T g0 / g0^T M g0 (skipped on the device once done)
    k_ms_scatter<false><<<sb, kBlock, 0, s>>>(V, g, nullptr, nullptr, nullptr, ctrl, F);
    rc = mob(mob_ctx, n, F, U, s);
    if (rc) return rc;
    k_ms_gather<kAlpha0><<<gb, kBlock, 0, s>>>(V, U, nullptr, nullptr, g, nullptr, ctrl, part);
    k_ms_finish<kAlpha0><<<1, kBlock, 0, s>>>(part, gb, ctrl, tol, max_iter, bb);
    SC_HIP_TRY(hipGetLastError());
    // a gamma0 that already meets the tolerance needs no iteration: wait once
    SC_HIP_TRY(hipMemcpyAsync(hctrl[1], ctrl, sizeof(MsCtrl), hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipEventRecord(ev.e[3], s));
    SC_HIP_TRY(hipEventSynchronize(ev.e[3]));
    bool stop = hctrl[1]->done != 0;

    // iterations in chunks of K; `done` is read one chunk behind, so the
    // GPU always has the next chunk queued
    int chunk = 0;
    for (int j0 = 1; j0 <= max_iter && !stop; j0 += K, ++chunk) {
        const int j1 = j0 + K - 1 < max_iter ? j0 + K - 1 : max_iter;
        for (int j = j0; j <= j1; ++j) {
            const int cur = (j - 1) & 1, nxt = j & 1;
            k_ms_scatter<true><<<sb, kBlock, 0, s>>>(V, nullptr, gam[cur], gg[cur], gam[nxt],
                                                     ctrl, F);
            rc = mob(mob_ctx, n, F, U, s);
            if (rc) return rc;
            k_ms_gather<kIter><<<gb, kBlock, 0, s>>>(V, U, gam[nxt], gam[cur], gg[cur],
                                                     gg[nxt], ctrl, part);
            k_ms_finish<kIter><<<1, kBlock, 0, s>>>(part, gb, ctrl, tol, max_iter, bb);
        }
        SC_HIP_TRY(hipGetLastError());
        const int slot = chunk & 1;
        SC_HIP_TRY(hipMemcpyAsync(hctrl[slot], ctrl, sizeof(MsCtrl), hipMemcpyDeviceToHost, s));
        SC_HIP_TRY(hipEventRecord(ev.e[2 + slot], s));
        if (chunk > 0) {
            SC_HIP_TRY(hipEventSynchronize(ev.e[2 + (slot ^ 1)]));
            if (hctrl[slot ^ 1]->done) stop = true;
        }
    }
    SC_HIP_TRY(hipEventRecord(t1, s));
    MsCtrl hc;
    SC_HIP_TRY(hipMemcpyAsync(&hc, ctrl, sizeof(MsCtrl), hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.0f;
    SC_HIP_TRY(hipEventElapsedTime(&ms, t0, t1));
    if (hc.final_buf == 1) {
        SC_HIP_TRY(hipMemcpyAsync(gamma, gam1, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
        SC_HIP_TRY(hipMemcpyAsync(g, g1, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
    }
    if (f_c || u_c) {
        double *fo = f_c ? f_c : F;
        k_ms_scatter<false><<<sb, kBlock, 0, s>>>(V, gamma, nullptr, nullptr, nullptr, ctrl, fo);
        SC_HIP_TRY(hipGetLastError());
        if (u_c) {
            rc = mob(mob_ctx, n, fo, u_c, s);
            if (rc) return rc;
        }
    }
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    st->status = hc.status;
    st->iters = hc.iters;
    st->mvops = hc.mvops;
    st->n_active = hc.n_active;
    st->residual = hc.res;
    st->alpha = hc.alpha;
    st->n_degenerate = hc.ndegen;
    st->kernel_ms = ms;
    st->grid = gb;
    st->block = kBlock;
    st->lanes_per_particle = kMsLanes;
    st->op = SC_OP_CALLBACK;
    return hc.status;
}

extern "C" size_t sc_adjoint_mob_work_bytes(int32_t n, int32_t capacity) {
    if (n < 0 || capacity < 0) return 0;
    return am_ws_bytes(n, capacity);
}

extern "C" int sc_solve_lcp_adjoint_mob(const sc_particles *p, const sc_box *box,
                                        const sc_contacts *c, const double *u_nc,
                                        const double *f_ext, double dt, const double *gamma,
                                        const double *dL_dgamma, const double *dL_df,
                                        sc_mobility_fn mob, void *mob_ctx,
                                        sc_mobility_grad_fn mob_grad, void *mob_grad_ctx,
                                        const sc_adjoint_opts *opts, int32_t check_every,
                                        double *dL_dq, double *dL_dpos, sc_stats *st, void *ws,
                                        size_t ws_bytes, void *stream_) {
    if (!p || !box || !c || !opts || !st || !mob || p->n < 0 || c->count < 0 ||
        c->count > c->capacity)
        return SC_ERR_INVALID;
    if (!(dt > 0.0) || !std::isfinite(dt) || !(opts->tol > 0.0) || opts->max_iter < 0 ||
        check_every < 0 || check_every > 4096)
        return SC_ERR_INVALID;
    Plan pl;
    if (!carve_plan(c->plan, c->plan_bytes, p->n, c->capacity, pl)) return SC_ERR_INVALID;
    const int n = p->n, nc = c->count;
    if (n > 0 && (!dL_dpos || !p->pos || !p->axis || !p->half_len || !p->mob || !u_nc ||
                  (mob_grad && !f_ext)))
        return SC_ERR_INVALID;
    if (nc > 0 && (!gamma || !dL_dq || !c->ci || !c->cj || !c->frame)) return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 ||
        ws_bytes < am_ws_bytes(n, c->capacity))
        return SC_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    *st = sc_stats{};
    if (nc == 0) {
        // no constraints: gamma and w are empty, every term vanishes
        if (n > 0) SC_HIP_TRY(hipMemsetAsync(dL_dpos, 0, 3 * sizeof(double) * n, s));
        SC_HIP_TRY(hipStreamSynchronize(s));
        st->status = SC_OK;
        return SC_OK;
    }
    const size_t cap = static_cast<size_t>(c->capacity), nn = static_cast<size_t>(n);
    Carver cv{static_cast<char *>(ws), ws_bytes};
    double *r = cv.take<double>(cap), *tv = cv.take<double>(cap), *x = cv.take<double>(cap);
    double *pv[2] = {cv.take<double>(cap), cv.take<double>(cap)};
    double *grad = cv.take<double>(3 * cap);
    double *F = cv.take<double>(6 * nn), *U = cv.take<double>(6 * nn);
    double *Fw = cv.take<double>(6 * nn), *Vw = cv.take<double>(6 * nn);
    double *Fc = cv.take<double>(6 * nn), *Uc = cv.take<double>(6 * nn);
    double *Ftot = cv.take<double>(6 * nn);
    double *Vw8 = cv.take<double>(8 * nn), *Uc8 = cv.take<double>(8 * nn);
    double *gm = cv.take<double>(3 * nn);
    double *part = cv.take<double>(kNV * static_cast<size_t>(kMaxReduceBlocks));
    CgMobCtrl *ctrl = cv.take<CgMobCtrl>(1);
    if (!cv.ok) return SC_ERR_WORKSPACE;
    char *slots = pinned_slots();
    Events ev;
    if (!slots || !ev.ok) return SC_ERR_HIP;
    CgMobCtrl *hctrl[2] = {reinterpret_cast<CgMobCtrl *>(slots),
                           reinterpret_cast<CgMobCtrl *>(slots + kPinnedSlot)};

    const MsView V{n, nc, pl.order, pl.inc_ptr, pl.inc, pl.dpm, c->ci, c->cj, pl.cs, pl.pdat,
                   c->frame, c->q};
    const int sb = grid_for(static_cast<long long>(n) * kMsLanes);
    int gb = grid_for(nc);
    if (gb > kMaxReduceBlocks) gb = kMaxReduceBlocks;
    const double tol = opts->tol;
    const int max_iter = opts->max_iter;
    const int K = check_every > 0 ? check_every : 4;
    int rc = SC_OK;

    SC_HIP_TRY(hipMemsetAsync(ctrl, 0, sizeof(CgMobCtrl), s));
    SC_HIP_TRY(hipEventRecord(ev.e[0], s));
    k_am_rhs<<<gb, kBlock, 0, s>>>(V, gamma, dL_dgamma, dL_df, r, x, pv[0], part);
    k_am_finish<0><<<1, kBlock, 0, s>>>(part, gb, ctrl, tol, max_iter);
    SC_HIP_TRY(hipGetLastError());
    SC_HIP_TRY(hipMemcpyAsync(hctrl[1], ctrl, sizeof(CgMobCtrl), hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipEventRecord(ev.e[3], s));
    SC_HIP_TRY(hipEventSynchronize(ev.e[3]));
    bool stop = hctrl[1]->done != 0;
    int chunk = 0;
    for (int i0 = 1; i0 <= max_iter && !stop; i0 += K, ++chunk) {
        const int i1 = i0 + K - 1 < max_iter ? i0 + K - 1 : max_iter;
        for (int i = i0; i <= i1; ++i) {
            const int cur = (i - 1) & 1, nxt = i & 1;
            k_am_scatter<<<sb, kBlock, 0, s>>>(V, r, pv[cur], pv[nxt], ctrl, F);
            rc = mob(mob_ctx, n, F, U, s);
            if (rc) return rc;
            k_am_gather<<<gb, kBlock, 0, s>>>(V, U, gamma, pv[nxt], tv, ctrl, part);
            k_am_finish<1><<<1, kBlock, 0, s>>>(part, gb, ctrl, tol, max_iter);
            k_am_update<<<gb, kBlock, 0, s>>>(nc, pv[nxt], tv, x, r, ctrl, part);
            k_am_finish<2><<<1, kBlock, 0, s>>>(part, gb, ctrl, tol, max_iter);
        }
        SC_HIP_TRY(hipGetLastError());
        const int slot = chunk & 1;
        SC_HIP_TRY(hipMemcpyAsync(hctrl[slot], ctrl, sizeof(CgMobCtrl), hipMemcpyDeviceToHost, s));
        SC_HIP_TRY(hipEventRecord(ev.e[2 + slot], s));
        if (chunk > 0) {
            SC_HIP_TRY(hipEventSynchronize(ev.e[2 + (slot ^ 1)]));
            if (hctrl[slot ^ 1]->done) stop = true;
        }
    }
    SC_HIP_TRY(hipEventRecord(ev.e[1], s));
    // dL/dq = -w on A; F_w = D w, V_w = Mob F_w; F_c = D gamma, U_c = Mob F_c
    k_am_post<<<grid_for(nc), kBlock, 0, s>>>(nc, gamma, x, dL_dq);
    k_ms_scatter<false><<<sb, kBlock, 0, s>>>(V, x, nullptr, nullptr, nullptr, nullptr, Fw);
    rc = mob(mob_ctx, n, Fw, Vw, s);
    if (rc) return rc;
    k_ms_scatter<false><<<sb, kBlock, 0, s>>>(V, gamma, nullptr, nullptr, nullptr, nullptr, Fc);
    rc = mob(mob_ctx, n, Fc, Uc, s);
    if (rc) return rc;
    // the per-contact geometric part, with the velocities of this mobility
    k_am_rank8<<<grid_for(n), kBlock, 0, s>>>(n, pl.order, Vw, Vw8);
    k_am_rank8<<<grid_for(n), kBlock, 0, s>>>(n, pl.order, Uc, Uc8);
    const PBox pb{{box->len[0], box->len[1], box->len[2]}, box->periodic ? 1 : 0};
    k_am_contact_grad<<<grid_for(nc), kBlock, 0, s>>>(nc, c->ci, c->cj, pl.cs, p->pos, p->axis,
                                                      p->half_len, pb, gamma, x, dL_df, Vw8, u_nc,
                                                      Uc8, 1.0 / dt, grad);
    k_am_gather_pos<<<grid_for(n), kBlock, 0, s>>>(n, pl, grad, dL_dpos);
    // the mobility's own dependence on the centres: -d/dc [F_w^T Mob(c) (F_c + F_ext)]
    if (mob_grad) {
        SC_HIP_TRY(hipMemcpyAsync(Ftot, Fc, 6 * sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
        k_am_add<<<grid_for(6LL * n), kBlock, 0, s>>>(6LL * n, Ftot, f_ext);
        rc = mob_grad(mob_grad_ctx, n, Fw, Ftot, gm, s);
        if (rc) return rc;
        k_am_sub<<<grid_for(3LL * n), kBlock, 0, s>>>(3LL * n, dL_dpos, gm);
    }
    SC_HIP_TRY(hipGetLastError());
    CgMobCtrl hc;
    SC_HIP_TRY(hipMemcpyAsync(&hc, ctrl, sizeof(CgMobCtrl), hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.0f;
    SC_HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
    st->status = hc.status;
    st->iters = hc.iters;
    st->mvops = hc.iters;
    st->n_active = hc.n_active;
    st->residual = hc.res;
    st->alpha = hc.alpha;
    st->kernel_ms = ms;
    st->grid = gb;
    st->block = kBlock;
    st->lanes_per_particle = kMsLanes;
    st->op = SC_OP_CALLBACK;
    return hc.status;
}

extern "C" size_t sc_solve_rpy_work_bytes(int32_t n, int32_t capacity) {
    if (n < 0 || capacity < 0) return 0;
    return rpy_pers_ws_bytes(n, capacity);
}

extern "C" int sc_solve_lcp_rpy(const sc_particles *p, const sc_contacts *c, const sc_rpy *R,
                                const sc_solve_opts *opts, double *gamma, double *g,
                                double *f_c, double *u_c, sc_stats *st, void *ws,
                                size_t ws_bytes, void *stream_) {
    if (!p || !c || !R || !opts || !st || p->n < 0 || c->count < 0 || c->count > c->capacity)
        return SC_ERR_INVALID;
    if (!(opts->tol > 0.0) || opts->max_iter < 0 || opts->bb < 1 || opts->bb > 3 ||
        opts->grid < 0 || opts->spin_limit < 0)
        return SC_ERR_INVALID;
    if (R->n != p->n || !(R->mu > 0.0) || !std::isfinite(R->mu)) return SC_ERR_INVALID;
    Plan pl;
    if (!carve_plan(c->plan, c->plan_bytes, p->n, c->capacity, pl)) return SC_ERR_INVALID;
    const int n = p->n, nc = c->count;
    if (nc > 0 && (!c->ci || !c->cj || !c->frame || !c->q || !gamma || !g)) return SC_ERR_INVALID;
    if (n > 0 && (!R->pos || !R->radius)) return SC_ERR_INVALID;
    if (n > 0 && (!R->work || (reinterpret_cast<uintptr_t>(R->work) & 255) != 0 ||
                  R->work_bytes < sc_rpy_work_bytes(n)))
        return SC_ERR_WORKSPACE;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0 ||
        ws_bytes < rpy_pers_ws_bytes(n, c->capacity))
        return SC_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream_);
    *st = sc_stats{};
    Carver cv{static_cast<char *>(ws), ws_bytes};
    double *gam1 = cv.take<double>(static_cast<size_t>(c->capacity));
    double *g1 = cv.take<double>(static_cast<size_t>(c->capacity));
    double *F = cv.take<double>(6 * static_cast<size_t>(n));
    double *red = cv.take<double>(kNV * static_cast<size_t>(kMaxReduceBlocks));
    GridSync *sync = cv.take<GridSync>(1);
    MsCtrl *ctrl = cv.take<MsCtrl>(1);
    if (!cv.ok) return SC_ERR_WORKSPACE;
    if (nc == 0) {
        if (f_c) SC_HIP_TRY(hipMemsetAsync(f_c, 0, 6 * sizeof(double) * n, s));
        if (u_c) SC_HIP_TRY(hipMemsetAsync(u_c, 0, 6 * sizeof(double) * n, s));
        SC_HIP_TRY(hipStreamSynchronize(s));
        st->status = SC_OK;
        st->mvops = 1;
        return SC_OK;
    }
    Events ev;
    if (!ev.ok) return SC_ERR_HIP;
    const int G = persistent_grid(reinterpret_cast<const void *>(k_bbpgd_rpy), kPB, opts->grid);
    if (G < 1) return SC_ERR_HIP;
    RpyPersArgs A;
    A.V = MsView{n, nc, pl.order, pl.inc_ptr, pl.inc, pl.dpm, c->ci, c->cj, pl.cs, pl.pdat,
                 c->frame, c->q};
    A.pos = R->pos;
    A.rad = R->radius;
    A.K = RpyConst{1.0 / (8.0 * M_PI * R->mu), 1.0 / (6.0 * M_PI * R->mu)};
    A.splits = rpy_pers_splits(n, G);
    A.F = F;
    A.part = static_cast<double *>(R->work);
    A.gam[0] = gamma;
    A.gam[1] = gam1;
    A.gg[0] = g;
    A.gg[1] = g1;
    A.red = red;
    A.sync = sync;
    A.ctrl = ctrl;
    A.tol = opts->tol;
    A.max_iter = opts->max_iter;
    A.bb = opts->bb;
    if (!opts->warm_start) SC_HIP_TRY(hipMemsetAsync(gamma, 0, sizeof(double) * nc, s));
    SC_HIP_TRY(hipMemsetAsync(sync, 0, sizeof(GridSync), s));
    if (opts->spin_limit > 0)
        SC_HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(&sync->limit[0]),
                                     opts->spin_limit, 1, s));
    SC_HIP_TRY(hipMemsetAsync(ctrl, 0, sizeof(MsCtrl), s));
    void *args[] = {&A};
    SC_HIP_TRY(hipEventRecord(ev.e[0], s));
    SC_HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_bbpgd_rpy), dim3(G),
                                          dim3(kPB), args, 0, s));
    SC_HIP_TRY(hipEventRecord(ev.e[1], s));
    MsCtrl hc;
    SC_HIP_TRY(hipMemcpyAsync(&hc, ctrl, sizeof(MsCtrl), hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    float ms = 0.0f;
    SC_HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
    if (hc.final_buf == 1) {
        SC_HIP_TRY(hipMemcpyAsync(gamma, gam1, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
        SC_HIP_TRY(hipMemcpyAsync(g, g1, sizeof(double) * nc, hipMemcpyDeviceToDevice, s));
    }
    if (f_c || u_c) {
        double *fo = f_c ? f_c : F;
        const int sb = grid_for(static_cast<long long>(n) * kMsLanes);
        k_ms_scatter<false><<<sb, kBlock, 0, s>>>(A.V, gamma, nullptr, nullptr, nullptr, nullptr,
                                                  fo);
        SC_HIP_TRY(hipGetLastError());
        if (u_c) {
            const int rc = sc_rpy_apply(const_cast<sc_rpy *>(R), n, fo, u_c, s);
            if (rc) return rc;
        }
    }
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    st->status = hc.status;
    st->iters = hc.iters;
    st->mvops = hc.mvops;
    st->n_active = hc.n_active;
    st->residual = hc.res;
    st->alpha = hc.alpha;
    st->n_degenerate = hc.ndegen;
    st->kernel_ms = ms;
    st->grid = G;
    st->block = kPB;
    st->lanes_per_particle = kPLanes;   // threads forming one source's F in the pair phase
    st->op = SC_OP_RPY;
    return hc.status;
}
