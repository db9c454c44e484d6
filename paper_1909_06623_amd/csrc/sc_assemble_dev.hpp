// sc_assemble_dev.hpp -- assembly of M = D^T Mob D (LCP LCPdef) in the
// sliced depth-major layout of sc_matrix.hpp: per-row lengths, per-slice
// sums and the entries of one slice, shared by the single-suspension
// assembly and the batched build.
//
// With a block-diagonal mobility, contacts l and m interact only through a
// shared particle k, M_lm = a_lk^T Mob_k a_mk (a_lk the signed column entries
// of contact l on particle k), so row l has deg(ci) + deg(cj) - 1 entries.
#pragma once

#include "sc_chain.hpp"
#include "sc_common.hpp"
#include "sc_plan.hpp"

namespace sc {

// Row l lists the contacts of its particles: deg(ci) + deg(cj) - 1 entries
// (the contact itself once), deg(ci) for a wall contact (no second rank).
__device__ __forceinline__ int row_length(const ChainView &C, int l) {
    const int ri = C.cs[2 * l], rj = C.cs[2 * l + 1];
    const int di = C.inc_ptr[ri + 1] - C.inc_ptr[ri];
    return rj < 0 ? di : di + (C.inc_ptr[rj + 1] - C.inc_ptr[rj]) - 1;
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

// Entries and widest row of slice sl (called by all lanes of one wave).
__device__ __forceinline__ void slice_sums(int sl, int nc, const int32_t *len, int32_t *soff,
                                           int32_t *swid) {
    const int l = sl * kWave + threadIdx.x % kWave;
    const int v = l < nc ? len[l] : 0;
    const int tot = wave_sum_int(v), wid = wave_max_int(v);
    if (threadIdx.x % kWave == 0) {
        soff[sl] = tot;
        swid[sl] = wid;
    }
}

// Walks the entries of row l in storage order: the diagonal first, then the
// other contacts of its lower-ranked particle in that particle's incidence
// order, then those of the other particle. M_lm = b_mk^T (Mob_k a_lk) for the
// shared particle k.
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
    // the diagonal; leaves the walk on the first off-diagonal entry (a wall
    // contact's row has its particle's side only)
    __device__ double start(const ChainView &C, int row) {
        l = row;
        if (C.cs[2 * row + 1] < 0) {
            ends[0] = C.cs[2 * row];
            ends[1] = -1;
            const double d0 = open(C, 0);
            settle(C);
            return d0;
        }
        // the lower-ranked particle first: consecutive rows share it (rows are
        // grouped by it), so their entries line up depth by depth and the
        // lanes of one gather touch the same records
        const int a = C.cs[2 * row], b = C.cs[2 * row + 1];
        ends[0] = a < b ? a : b;
        ends[1] = a < b ? b : a;
        const double d1 = open(C, 1);
        const double d0 = open(C, 0);
        settle(C);
        return d0 + d1;
    }
    __device__ void settle(const ChainView &C) {
        if (e >= e1 && side == 0 && ends[1] >= 0) open(C, 1);
    }
    __device__ void next(const ChainView &C) {
        ++e;
        if (e == own) ++e;
        settle(C);
    }
};

// One wave writes slice sl's rows depth by depth; lanes without an entry at
// a depth sit out that depth's ballot.
__device__ __forceinline__ void assemble_slice(const ChainView &C, int sl, const int32_t *len,
                                               const int32_t *soff, const int32_t *swid,
                                               int32_t *col, double *val) {
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

}  // namespace sc
