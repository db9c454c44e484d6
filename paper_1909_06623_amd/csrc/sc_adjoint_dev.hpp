// sc_adjoint_dev.hpp -- per-contact and per-particle steps of the implicit
// adjoint (not in the paper; the derivation is in sc_adjoint.hip's header),
// shared by the single-instance kernels and the batched persistent kernel.
#pragma once

#include "sc_chain.hpp"
#include "sc_common.hpp"
#include "sc_geometry.hpp"
#include "sc_plan.hpp"

namespace sc {

// Right-hand side of the masked adjoint system for contact l:
// b_l = dL/dgamma_l + (D^T dL/dF)_l on the active set, 0 elsewhere.
// dLdF is [n][6] in caller order (ci, cj are caller indices).
__device__ inline double cg_rhs_one(int l, const int *ci, const int *cj, const double *frame,
                                   const double *gamma, const double *dLdg, const double *dLdF) {
    const bool act = gamma[l] > 0.0;
    double b = dLdg ? dLdg[l] : 0.0;
    if (dLdF) {
        const double *f = frame + 9 * static_cast<long long>(l);
        const double *ui = dLdF + 6 * static_cast<long long>(ci[l]);
        double v = -dot(load3(f), load3(ui)) - dot(load3(f + 3), load3(ui + 3));
        if (cj[l] >= 0) {
            const double *uj = dLdF + 6 * static_cast<long long>(cj[l]);
            v = v + dot(load3(f), load3(uj)) + dot(load3(f + 6), load3(uj + 3));
        }
        b += v;
    }
    return act ? b : 0.0;
}

// Per-contact derivative of J_l(r) = D_l(r)^T [E_i; E_j] - (w_l/dt) Phi_l(r)
// with respect to r = c_j - c_i (orientations fixed), where
// E_k = gamma_l (dL/dF_k - V_w,k) - w_l (U_nc,k + U_c,k). The closest-point
// parameters s, t move with r only while strictly inside their segment:
// both free -> implicit differentiation of the 2x2 stationarity conditions;
// one free -> its 1-D projection; both clamped (or a sphere) -> fixed.
__device__ __noinline__ V3 contact_grad_one(int l, const int *__restrict__ ci, const int *__restrict__ cj,
                                     const int *__restrict__ cs, const double *__restrict__ pos,
                                     const double *__restrict__ axis,
                                     const double *__restrict__ half_len, const PBox &box,
                                     const double *__restrict__ gamma, const double *__restrict__ w,
                                     const double *__restrict__ dLdF, const double *__restrict__ Vw,
                                     const double *__restrict__ Unc, const double *__restrict__ Uc,
                                     double inv_dt) {
    const double gl = gamma[l], wl = w[l];
    if (gl == 0.0 && wl == 0.0) return v3(0.0, 0.0, 0.0);
    const int i = ci[l], j = cj[l];
    if (j < 0) {
        // a plane wall: n and tau_i do not move with c_i and dPhi/dc_i is the
        // face's inward normal m, so dJ/dc_i = -(w_l/dt) m; the gather puts
        // -grad on particle i
        const int face = -1 - j, a = face >> 1;
        const double m = (face & 1) ? -1.0 : 1.0;
        const double gv = wl * inv_dt * m;
        return v3(a == 0 ? gv : 0.0, a == 1 ? gv : 0.0, a == 2 ? gv : 0.0);
    }
    const long long ri = cs[2 * l], rj = cs[2 * l + 1];
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
    const long long oi = 6 * static_cast<long long>(i), oj = 6 * static_cast<long long>(j);
    const V3 zero = v3(0.0, 0.0, 0.0);
    const V3 fi = dLdF ? load3(dLdF + oi) : zero, tqi = dLdF ? load3(dLdF + oi + 3) : zero;
    const V3 fj = dLdF ? load3(dLdF + oj) : zero, tqj = dLdF ? load3(dLdF + oj + 3) : zero;
    const double *Vi = Vw + 8 * ri, *Vj = Vw + 8 * rj, *Ci = Uc + 8 * ri, *Cj = Uc + 8 * rj;
    const V3 EiF = gl * (fi - load3(Vi)) - wl * (load3(Unc + oi) + load3(Ci));
    const V3 EiT = gl * (tqi - load3(Vi + 3)) - wl * (load3(Unc + oi + 3) + load3(Ci + 3));
    const V3 EjF = gl * (fj - load3(Vj)) - wl * (load3(Unc + oj) + load3(Cj));
    const V3 EjT = gl * (tqj - load3(Vj + 3)) - wl * (load3(Unc + oj + 3) + load3(Cj + 3));
    // J_d = dd/dr = I + p_j dt^T - p_i ds^T, so J_d^T u = u + dt (p_j.u) - ds (p_i.u);
    // dn/dr = (I - n n^T) J_d / rho.
    auto JdT = [&](V3 u) { return u + dot(pj, u) * dt - dot(pi, u) * ds; };
    auto JnT = [&](V3 v) { return (1.0 / rho) * JdT(v - dot(n, v) * n); };
    const V3 vn = (EjF - EiF) - s * cross(EiT, pi) + t * cross(EjT, pj);
    const V3 g = JnT(vn) - dot(cross(pi, n), EiT) * ds + dot(cross(pj, n), EjT) * dt -
                 (wl * inv_dt) * JdT(n);
    return g;
}

// dL/dc_k = sum over k's contacts of -grad (k is ci) or +grad (k is cj),
// gathered for rank k and written at its caller index.
__device__ inline void gather_pos_one(int k, const Plan &pl, const double *__restrict__ grad,
                                      double *__restrict__ out) {
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int e = pl.inc_ptr[k]; e < pl.inc_ptr[k + 1]; ++e) {
        const long long l = pl.inc[e] >> 1;
        const double sg = pl.cs[2 * l] == k ? -1.0 : 1.0;
        gx += sg * grad[3 * l + 0];
        gy += sg * grad[3 * l + 1];
        gz += sg * grad[3 * l + 2];
    }
    const long long o = 3 * static_cast<long long>(pl.order[k]);
    out[o + 0] = gx;
    out[o + 1] = gy;
    out[o + 2] = gz;
}

// F = D x and U = Mob F for rank k (signed D columns of its incidences);
// F in caller order [n][6] if f_out, U in rank order [n][8].
__device__ inline void mob_d_one(const ChainView &C, int k, const double *x, const int *order,
                                 double *f_out, double *U) {
    double f[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = C.inc_ptr[k]; e < C.inc_ptr[k + 1]; ++e) {
        const double w = x[C.inc[e] >> 1];
        const double *d = C.dpm + 6 * static_cast<long long>(e);
        for (int a = 0; a < 6; ++a) f[a] += w * d[a];
    }
    V3 u, wv;
    plan_mobility(C.pdat + 8 * static_cast<long long>(k), v3(f[0], f[1], f[2]),
                  v3(f[3], f[4], f[5]), u, wv);
    double *Uk = U + 8 * static_cast<long long>(k);
    Uk[0] = u.x; Uk[1] = u.y; Uk[2] = u.z;
    Uk[3] = wv.x; Uk[4] = wv.y; Uk[5] = wv.z;
    if (f_out) {
        const long long o = 6 * static_cast<long long>(order[k]);
        for (int a = 0; a < 6; ++a) f_out[o + a] = f[a];
    }
}

}  // namespace sc
