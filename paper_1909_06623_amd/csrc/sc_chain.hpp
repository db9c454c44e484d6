// sc_chain.hpp -- the two passes of one product M x = D^T Mob D x on the
// solver layout, written as device building blocks for persistent kernels.
//
//   pass A (particle-major): for each rank k, F_k = sum over its incidences of
//     w_l * (signed column entries), then U_k = Mob_k F_k. LPP lanes share a
//     particle's incidence list and combine their partial sums with a fixed
//     butterfly; the weight functor may also store per-contact updates.
//   pass B (contact-major): v_l = D_l^T U for each contact of the block's
//     range; a functor consumes v_l and accumulates up to four sums.
//
// Work is split in contiguous chunks per logical workgroup, and logical
// workgroups are numbered so that each XCD owns one contiguous range
// (hardware workgroups are dealt to the XCDs round-robin).
#pragma once

#include "sc_common.hpp"
#include "sc_plan.hpp"

namespace sc {

// Results of a persistent solve, written by workgroup 0.
struct SolveCtrl {
    double alpha, res;
    int iters, mvops, status, ndegen;
    int n_active, pad[3];
};

struct CgCtrl {
    double alpha, res;
    int iters, status, n_active, pad;
};

struct ChainView {
    int n, nc;
    const double *pdat;    // [n][8]
    const int *inc_ptr;    // [n+1]
    const int *inc;        // [2 nc]
    const double *dpm;     // [2 nc][6]
    const int *cs;         // [nc][2]
    const double *frame;   // [nc][9]
    double *U;             // [n][8] rank order: U xyz, W xyz, 2 pad
};

__device__ __forceinline__ int logical_block() {
    const int G = gridDim.x, b = blockIdx.x;
    return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
}

__device__ __forceinline__ void chunk(int units, int &u0, int &u1) {
    const long long L = logical_block(), G = gridDim.x;
    u0 = static_cast<int>(L * units / G);
    u1 = static_cast<int>((L + 1) * units / G);
}

// Pass A over ranks [k0, k1). weight(code, e) returns w for incidence e
// (contact code >> 1; code & 1 marks the owning incidence).
template <int LPP, int BS, class W>
__device__ __forceinline__ void pass_a(const ChainView &C, int k0, int k1, W weight) {
    constexpr int PER = BS / LPP;
    const int sub = threadIdx.x / LPP, lane = threadIdx.x % LPP;
    for (int base = k0; base < k1; base += PER) {
        const int k = base + sub;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0;
        if (k < k1) {
            const int e1 = C.inc_ptr[k + 1];
            for (int e = C.inc_ptr[k] + lane; e < e1; e += LPP) {
                const double w = weight(C.inc[e], e);
                const double *d = C.dpm + 6 * static_cast<long long>(e);
                a0 += w * d[0];
                a1 += w * d[1];
                a2 += w * d[2];
                a3 += w * d[3];
                a4 += w * d[4];
                a5 += w * d[5];
            }
        }
#pragma unroll
        for (int off = LPP / 2; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off, kWave);
            a1 += __shfl_xor(a1, off, kWave);
            a2 += __shfl_xor(a2, off, kWave);
            a3 += __shfl_xor(a3, off, kWave);
            a4 += __shfl_xor(a4, off, kWave);
            a5 += __shfl_xor(a5, off, kWave);
        }
        if (k < k1 && lane == 0) {
            V3 u, w;
            plan_mobility(C.pdat + 8 * static_cast<long long>(k), v3(a0, a1, a2), v3(a3, a4, a5),
                          u, w);
            double *Uk = C.U + 8 * static_cast<long long>(k);
            Uk[0] = u.x; Uk[1] = u.y; Uk[2] = u.z;
            Uk[3] = w.x; Uk[4] = w.y; Uk[5] = w.z;
        }
    }
}

// (D^T U)_l for contact l.
__device__ __forceinline__ double dt_u(const ChainView &C, int l) {
    const int ri = C.cs[2 * l], rj = C.cs[2 * l + 1];
    const double *f = C.frame + 9 * static_cast<long long>(l);
    const double *Ui = C.U + 8 * static_cast<long long>(ri);
    const double vi = -(f[0] * Ui[0] + f[1] * Ui[1] + f[2] * Ui[2]) -
                      (f[3] * Ui[3] + f[4] * Ui[4] + f[5] * Ui[5]);
    if (rj < 0) return vi;  // wall contact: the particle's side only
    const double *Uj = C.U + 8 * static_cast<long long>(rj);
    return vi + (f[0] * Uj[0] + f[1] * Uj[1] + f[2] * Uj[2]) +
           (f[6] * Uj[3] + f[7] * Uj[4] + f[8] * Uj[5]);
}

// Grid-wide reductions, in two halves around a grid barrier. Slot MAXSLOT
// (if >= 0) is a maximum, the others are sums; every order is fixed, so all
// workgroups compute bitwise identical totals and take identical decisions.

// Before the barrier: the workgroup's NV partials (wave butterflies, then
// one wave over the per-wave results) go to part[slot * NV + k]; the slot is
// the logical workgroup unless given.
template <int NV, int BS, int MAXSLOT = -1>
__device__ __forceinline__ void write_partial(double *part, double (&acc)[NV], int slot = -1) {
    constexpr int NW = BS / kWave;
    __shared__ double red[NV][NW];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = (k == MAXSLOT) ? wave_max(acc[k]) : wave_sum(acc[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k][wid] = acc[k];
    }
    __syncthreads();
    if (wid == 0) {
        const int L = slot >= 0 ? slot : logical_block();
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double x = lane < NW ? red[k][lane] : (k == MAXSLOT ? -HUGE_VAL : 0.0);
            x = (k == MAXSLOT) ? wave_max(x) : wave_sum(x);
            if (lane == 0) part[L * NV + k] = x;
        }
    }
}

// After the barrier: wave k folds value k of all G partials (lane-strided,
// then a butterfly) and the totals reach every thread through LDS. G is the
// grid size unless given.
template <int NV, int BS, int MAXSLOT = -1>
__device__ __forceinline__ void grid_reduce(const double *part, double (&tot)[NV], int nparts = -1) {
    static_assert(BS / kWave >= NV, "one wave per reduced value");
    __shared__ double out[NV];
    const int lane = threadIdx.x % kWave, k = threadIdx.x / kWave;
    const int G = nparts >= 0 ? nparts : static_cast<int>(gridDim.x);
    if (k < NV) {
        const bool mx = k == MAXSLOT;
        double x = mx ? -HUGE_VAL : 0.0;
        for (int L = lane; L < G; L += kWave) {
            const double y = part[L * NV + k];
            x = mx ? fmax(x, y) : x + y;
        }
        x = mx ? wave_max(x) : wave_sum(x);
        if (lane == 0) out[k] = x;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) tot[j] = out[j];
}

// Host helpers defined in sc_solve.hip.
ChainView chain_view(const sc_particles *p, const sc_contacts *c, const Plan &pl, double *U);
// U (rank order, into C.U) = Mob D x; optionally F = D x and U scattered to
// caller order ([n][6] each).
void launch_mob_d(const ChainView &C, const double *x, const int *order, double *f_out,
                  double *u_out, hipStream_t s);
// y = D^T C.U
void launch_dt(const ChainView &C, double *y, hipStream_t s);
// Grid size for a persistent kernel of `block` threads and `dyn` bytes of
// dynamic LDS: the request (0 = one workgroup per CU) clamped to one
// workgroup per CU and to what is co-resident, a multiple of 8 when possible.
int persistent_grid(const void *fn, int block, int requested, size_t dyn = 0);
// Valid tuning options (0 = default).
inline bool lanes_ok(int v) { return v == 0 || v == 1 || v == 2 || v == 4 || v == 8; }
inline bool spw_ok(int v) { return v == 0 || v == 1 || v == 2 || v == 4; }
inline bool block_ok(int v) { return v == 0 || v == 256 || v == 512 || v == 1024; }

}  // namespace sc
