// sc_plan.hpp -- the solver-side layout that sc_build_contacts writes into the
// caller's plan buffer and that the solve and adjoint read.
//
// Particles are ranked in cell order (cells row-major over the search grid,
// ties by caller index), so neighbouring ranks are neighbours in space and
// every gather of the solve stays local. Contacts are stored grouped by the
// rank of their lower-ranked particle, partners by increasing rank.
#pragma once

#include "sc_common.hpp"

namespace sc {

struct Plan {
    int32_t *order;    // [n] rank -> caller index
    int32_t *rank;     // [n] caller index -> rank
    double *pdat;      // [n][8] per rank: axis x y z, 0, a_par, a_perp, b_par, b_perp
    int32_t *cptr;     // [n+1] contacts whose lower rank is k: [cptr[k], cptr[k+1])
    int32_t *inc_ptr;  // [n+1] incidences of rank k: [inc_ptr[k], inc_ptr[k+1])
    int32_t *inc;      // [2 cap] incidence code 2 l + owner (owner stores gamma_l)
    double *dpm;       // [2 cap][6] signed column entries (-/+)(n_l, tau_l,side)
    int32_t *cs;       // [cap][2] ranks of (ci, cj)
};

inline size_t plan_bytes(int32_t n, int32_t cap) {
    const size_t nn = static_cast<size_t>(n), cc = static_cast<size_t>(cap);
    size_t b = 0;
    b += 2 * align_up(nn * sizeof(int32_t), 256);
    b += align_up(8 * nn * sizeof(double), 256);
    b += 2 * align_up((nn + 1) * sizeof(int32_t), 256);
    b += align_up(2 * cc * sizeof(int32_t), 256);
    b += align_up(12 * cc * sizeof(double), 256);
    b += align_up(2 * cc * sizeof(int32_t), 256);
    return b + 256;
}

inline bool carve_plan(void *base, size_t bytes, int32_t n, int32_t cap, Plan &p) {
    if (!base || (reinterpret_cast<uintptr_t>(base) & 255) != 0 || bytes < plan_bytes(n, cap))
        return false;
    Carver cv{static_cast<char *>(base), bytes};
    p.order = cv.take<int32_t>(n);
    p.rank = cv.take<int32_t>(n);
    p.pdat = cv.take<double>(8 * static_cast<size_t>(n));
    p.cptr = cv.take<int32_t>(static_cast<size_t>(n) + 1);
    p.inc_ptr = cv.take<int32_t>(static_cast<size_t>(n) + 1);
    p.inc = cv.take<int32_t>(2 * static_cast<size_t>(cap));
    p.dpm = cv.take<double>(12 * static_cast<size_t>(cap));
    p.cs = cv.take<int32_t>(2 * static_cast<size_t>(cap));
    return cv.ok;
}

// Dry mobility from a plan record: U = a_perp F + (a_par - a_perp)(p.F) p, W likewise.
__device__ __forceinline__ void plan_mobility(const double *rec, V3 f, V3 t, V3 &u, V3 &w) {
    const V3 p = v3(rec[0], rec[1], rec[2]);
    const double a_par = rec[4], a_perp = rec[5], b_par = rec[6], b_perp = rec[7];
    u = a_perp * f + ((a_par - a_perp) * dot(p, f)) * p;
    w = b_perp * t + ((b_par - b_perp) * dot(p, t)) * p;
}

}  // namespace sc
