// sc_contacts.hip -- close-pair detection and LCP assembly on gfx950.
//
// Builds the set A(C, delta) = {(i, j), i < j : Phi_ij <= delta} of section
// 3.2 with a uniform cell list (section 5.2 names cell lists as the standard
// near-neighbour method), the contact frames that define the columns of D
// (Eq. Dmatdef; their entries follow from Eq. Dtranspose) and
// q = Phi/dt + D^T U_nc (LCP LCPdef), plus the solver layout (sc_plan.hpp).
//
// Pipeline (stream-ordered; two host synchronisations: the interaction range
// sizes the grid, and the pair count is checked against capacity):
//   validate + max extent -> bin -> scan -> scatter -> rank particles in
//   cell order (ties by caller index) -> count partners of higher rank ->
//   scan -> write contacts (partners sorted by rank) -> incidence lists and
//   signed column entries -> q.
// Every decision is a pure function of the inputs, so the contact list and
// its order are independent of thread scheduling.
#include <cmath>
#include <cstring>

#include "sc_build_dev.hpp"
#include "sc_common.hpp"
#include "sc_geometry.hpp"
#include "sc_plan.hpp"

namespace sc {

namespace {

__global__ void k_validate(Parts P, unsigned long long *max_ext, int *flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    if (particle_bad(P, k)) {
        atomicOr(flags + kFlagBadInput, 1);
        return;
    }
    // non-negative doubles order like their bit patterns
    const double e = P.radius[k] + P.half_len[k];
    atomicMax(max_ext, static_cast<unsigned long long>(__double_as_longlong(e)));
}

__global__ void k_bin(Parts P, Grid g, int *cell_of, int *cell_count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    const int c = particle_cell(P, k, g, 0);
    cell_of[k] = c;
    atomicAdd(cell_count + c, 1);
}

__global__ void k_scatter(int n, const int *cell_of, const int *cell_start, int *cell_fill,
                          int *members) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int c = cell_of[k];
    members[cell_start[c] + atomicAdd(cell_fill + c, 1)] = k;
}

__global__ void k_rank(Parts P, const int *cell_of, const int *cell_start, const int *members,
                       Plan pl, double *prec, double *hl, int *cell_r) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    rank_particle(P, k, 0, 0, cell_of, cell_start, members, pl, prec, hl, cell_r);
}

// Count pass: kPairLanes consecutive threads per rank; per-lane counts go to
// lane_cnt, the rank's total to cptr.
__global__ void k_count_pairs(int n, Ranked R, Plan pl, Grid g, const int *cell_start,
                              int *lane_cnt, int *slots, int *flags) {
    const long long gid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int t = static_cast<int>(gid / kPairLanes), lane = static_cast<int>(gid % kPairLanes);
    if (t >= n) return;  // whole groups of kPairLanes leave together
    count_partners(t, lane, R, pl, g, cell_start, 0, lane_cnt + gid, slots + kLaneSlots * gid,
                   flags);
}

__global__ void k_write_pairs(int n, Ranked R, Plan pl, Grid g, const int *cell_start,
                              const int *lane_cnt, const int *slots) {
    const long long gid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int t = static_cast<int>(gid / kPairLanes), lane = static_cast<int>(gid % kPairLanes);
    if (t >= n) return;
    write_partners(t, lane, R, pl, g, cell_start, 0, lane_cnt + (gid - lane),
                   slots + kLaneSlots * gid);
}

__global__ void k_finish_pairs(int n, Ranked R, Plan pl, Grid g, int *ci, int *cj, double *phi,
                               double *frame) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    finish_partners(t, R, pl, g, ci, cj, phi, frame);
}

__global__ void k_second_degree(int nc, Plan pl, int *deg) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    count_second(l, pl, deg);
}

__global__ void k_inc_counts(int n, Plan pl, const int *deg) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    incidence_count(k, pl, deg);
}

__global__ void k_inc_fill(int nc, Plan pl, int *fill) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    incidence_fill(l, pl, fill);
}

__global__ void k_inc_finish(int n, Plan pl, const double *frame) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    incidence_finish(k, pl, frame);
}

// Nonzeros of M = D^T Mob D: contact rows l have deg(ci) + deg(cj) - 1
// entries, so the total is sum_k deg(k)^2 - n_c.
__global__ void k_deg_squares(int n, Plan pl, unsigned long long *sum) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long d2 = 0;
    if (k < n) {
        const unsigned long long d = pl.inc_ptr[k + 1] - pl.inc_ptr[k];
        d2 = d * d;
    }
    for (int off = kWave / 2; off > 0; off >>= 1)
        d2 += __shfl_xor(d2, off, kWave);
    __shared__ unsigned long long ws[kBlock / kWave];
    if (threadIdx.x % kWave == 0) ws[threadIdx.x / kWave] = d2;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += ws[w];
        if (t) atomicAdd(sum, t);
    }
}

__global__ void k_q(int nc, const int *ci, const int *cj, const double *phi,
                    const double *frame, const double *u_nc, double dt, double *q, int *flags) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    const double ql = contact_q(l, ci, cj, phi, frame, u_nc, dt);
    q[l] = ql;
    if (!isfinite(ql)) atomicOr(flags + kFlagNonfiniteQ, 1);
}

}  // namespace

size_t contacts_ws_bytes(int32_t n, int32_t cap) {
    (void)cap;
    const size_t nn = static_cast<size_t>(n), nb = cell_budget(n);
    size_t b = 0;
    b += align_up(kFlagCount * sizeof(int), 256) + 256;     // flags, max extent
    b += 5 * align_up(nn * sizeof(int), 256);                // cell_of, members, cell_r, deg, fill
    b += align_up(kPairLanes * nn * sizeof(int), 256);       // per-lane pair counts
    b += align_up(kLaneSlots * kPairLanes * nn * sizeof(int), 256);  // per-lane partners
    b += align_up(4 * nn * sizeof(double), 256);             // ranked centre + radius
    b += align_up(nn * sizeof(double), 256);                 // ranked half length
    b += 2 * align_up((nb + 1) * sizeof(int), 256);          // cell_start, cell_fill
    const size_t sn = (nn + 1 > nb + 1 ? nn + 1 : nb + 1);
    b += align_up(static_cast<size_t>(scan_tmp_ints(static_cast<int>(sn))) * sizeof(int), 256);
    b += 256;                                                // host-read staging
    return b + 2048;
}

}  // namespace sc

using namespace sc;

extern "C" size_t sc_plan_bytes(int32_t n, int32_t capacity) {
    if (n < 0 || capacity < 0) return 0;
    return plan_bytes(n, capacity);
}

extern "C" int sc_build_contacts(const sc_particles *p, const sc_box *box, double delta,
                                 const double *u_nc, double dt, sc_contacts *c, void *ws,
                                 size_t ws_bytes, void *stream_) {
    if (!p || !box || !c || p->n < 0 || c->capacity < 0) return SC_ERR_INVALID;
    if (!(delta >= 0.0) || !std::isfinite(delta) || !(dt > 0.0) || !std::isfinite(dt))
        return SC_ERR_INVALID;
    for (int a = 0; a < 3; ++a)
        if (!(box->len[a] > 0.0) || !std::isfinite(box->len[a]) || !std::isfinite(box->lo[a]))
            return SC_ERR_INVALID;
    if (box->walls < 0 || box->walls > 63 || (box->periodic && box->walls)) return SC_ERR_INVALID;
    c->count = 0;
    c->n_parallel = c->n_zero_dist = c->n_borderline = 0;
    c->grid[0] = c->grid[1] = c->grid[2] = 0;
    c->nnz = 0;
    c->mat_ready = 0;
    const int n = p->n;
    Plan pl;
    if (!carve_plan(c->plan, c->plan_bytes, n, c->capacity, pl)) return SC_ERR_INVALID;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (n == 0) {
        SC_HIP_TRY(hipMemsetAsync(pl.cptr, 0, sizeof(int), stream));
        SC_HIP_TRY(hipMemsetAsync(pl.inc_ptr, 0, sizeof(int), stream));
        SC_HIP_TRY(hipStreamSynchronize(stream));
        return SC_OK;
    }
    if (!p->pos || !p->axis || !p->radius || !p->half_len || !p->mob || !u_nc) return SC_ERR_INVALID;
    if (c->capacity > 0 && (!c->ci || !c->cj || !c->phi || !c->q || !c->frame))
        return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return SC_ERR_WORKSPACE;
    if (ws_bytes < contacts_ws_bytes(n, c->capacity)) return SC_ERR_WORKSPACE;

    const size_t nb = cell_budget(n);
    Carver cv{static_cast<char *>(ws), ws_bytes};
    int *flags = cv.take<int>(kFlagCount);
    unsigned long long *max_ext = cv.take<unsigned long long>(1);
    int *cell_of = cv.take<int>(n);
    int *members = cv.take<int>(n);
    int *cell_r = cv.take<int>(n);
    int *deg = cv.take<int>(n);
    int *fill = cv.take<int>(n);
    int *lane_cnt = cv.take<int>(static_cast<size_t>(kPairLanes) * n);
    int *slots = cv.take<int>(static_cast<size_t>(kLaneSlots) * kPairLanes * n);
    double *prec = cv.take<double>(4 * static_cast<size_t>(n));
    double *hl = cv.take<double>(n);
    int *cell_start = cv.take<int>(nb + 1);
    int *cell_fill = cv.take<int>(nb + 1);
    const int sn = static_cast<int>((static_cast<size_t>(n) + 1 > nb + 1) ? n + 1 : nb + 1);
    int *scan_tmp = cv.take<int>(scan_tmp_ints(sn));
    int *stage = cv.take<int>(16);
    if (!cv.ok) return SC_ERR_WORKSPACE;

    Parts P{n, p->pos, p->axis, p->radius, p->half_len, p->mob};
    SC_HIP_TRY(hipMemsetAsync(flags, 0, kFlagCount * sizeof(int), stream));
    SC_HIP_TRY(hipMemsetAsync(max_ext, 0, sizeof(unsigned long long), stream));
    k_validate<<<grid_for(n), kBlock, 0, stream>>>(P, max_ext, flags);
    int hflags[kFlagCount];
    unsigned long long hext = 0;
    SC_HIP_TRY(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipMemcpyAsync(&hext, max_ext, sizeof(hext), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipStreamSynchronize(stream));
    if (hflags[kFlagBadInput]) return SC_ERR_NONFINITE;

    double ext;
    {
        long long bits = static_cast<long long>(hext);
        std::memcpy(&ext, &bits, sizeof(ext));
    }
    const double rmax = 2.0 * ext + delta;
    Grid g;
    if (!make_grid(*box, n, delta, rmax, nb, g)) return SC_ERR_BOX;
    const size_t ncell = static_cast<size_t>(g.nc[0]) * g.nc[1] * g.nc[2];
    for (int a = 0; a < 3; ++a) c->grid[a] = g.nc[a];

    // bin particles and rank them in cell order
    SC_HIP_TRY(hipMemsetAsync(cell_start, 0, (ncell + 1) * sizeof(int), stream));
    SC_HIP_TRY(hipMemsetAsync(cell_fill, 0, ncell * sizeof(int), stream));
    k_bin<<<grid_for(n), kBlock, 0, stream>>>(P, g, cell_of, cell_start);
    scan_exclusive(cell_start, cell_start, static_cast<int>(ncell), scan_tmp, stream);
    k_scatter<<<grid_for(n), kBlock, 0, stream>>>(n, cell_of, cell_start, cell_fill, members);
    k_rank<<<grid_for(n), kBlock, 0, stream>>>(P, cell_of, cell_start, members, pl, prec, hl,
                                               cell_r);
    Ranked R{prec, hl, cell_r};

    // partners of higher rank, then offsets
    const int pair_blocks = grid_for(static_cast<long long>(n) * kPairLanes);
    k_count_pairs<<<pair_blocks, kBlock, 0, stream>>>(n, R, pl, g, cell_start, lane_cnt, slots,
                                                      flags);
    scan_exclusive(pl.cptr, pl.cptr, n, scan_tmp, stream);
    SC_HIP_TRY(hipMemcpyAsync(stage, pl.cptr + n, sizeof(int), hipMemcpyDeviceToDevice, stream));
    SC_HIP_TRY(hipMemcpyAsync(stage + 1, flags, kFlagCount * sizeof(int), hipMemcpyDeviceToDevice,
                              stream));
    int hstage[1 + kFlagCount];
    SC_HIP_TRY(hipMemcpyAsync(hstage, stage, sizeof(hstage), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipStreamSynchronize(stream));
    const int nc = hstage[0];
    c->count = nc;
    c->n_parallel = hstage[1 + kFlagParallel];
    c->n_zero_dist = hstage[1 + kFlagZero];
    c->n_borderline = hstage[1 + kFlagBorder];
    if (nc > c->capacity) return SC_ERR_CAPACITY;

    k_write_pairs<<<pair_blocks, kBlock, 0, stream>>>(n, R, pl, g, cell_start, lane_cnt, slots);
    k_finish_pairs<<<grid_for(n), kBlock, 0, stream>>>(n, R, pl, g, c->ci, c->cj, c->phi,
                                                       c->frame);
    // incidence lists and signed column entries
    SC_HIP_TRY(hipMemsetAsync(deg, 0, n * sizeof(int), stream));
    SC_HIP_TRY(hipMemsetAsync(fill, 0, n * sizeof(int), stream));
    if (nc > 0) k_second_degree<<<grid_for(nc), kBlock, 0, stream>>>(nc, pl, deg);
    k_inc_counts<<<grid_for(n), kBlock, 0, stream>>>(n, pl, deg);
    scan_exclusive(pl.inc_ptr, pl.inc_ptr, n, scan_tmp, stream);
    unsigned long long *dsq = max_ext;  // the extent word is free again
    SC_HIP_TRY(hipMemsetAsync(dsq, 0, sizeof(unsigned long long), stream));
    if (nc > 0) {
        k_inc_fill<<<grid_for(nc), kBlock, 0, stream>>>(nc, pl, fill);
        k_inc_finish<<<grid_for(n), kBlock, 0, stream>>>(n, pl, c->frame);
        k_q<<<grid_for(nc), kBlock, 0, stream>>>(nc, c->ci, c->cj, c->phi, c->frame, u_nc, dt,
                                                 c->q, flags);
        k_deg_squares<<<grid_for(n), kBlock, 0, stream>>>(n, pl, dsq);
    }
    unsigned long long hdsq = 0;
    SC_HIP_TRY(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipMemcpyAsync(&hdsq, dsq, sizeof(hdsq), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipStreamSynchronize(stream));
    SC_HIP_TRY(hipGetLastError());
    // rows: deg(i) + deg(j) - 1 for a pair, deg(i) for a wall contact
    c->nnz = nc > 0 ? static_cast<int64_t>(hdsq) - (nc - hflags[kFlagWalls]) : 0;
    if (hflags[kFlagNonfiniteQ]) return SC_ERR_NONFINITE;
    return SC_OK;
}
