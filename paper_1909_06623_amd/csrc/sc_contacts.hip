// sc_contacts.hip -- close-pair detection and LCP assembly on gfx950.
//
// Builds the set A(C, delta) = {(i, j), i < j : Phi_ij <= delta} of section
// 3.2 with a uniform cell list (section 5.2 names cell lists as the standard
// near-neighbour method), the contact frames that define the columns of D
// (Eq. Dmatdef; their entries follow from Eq. Dtranspose), the particle-major
// incidence used by the gather form of D gamma, and q = Phi/dt + D^T U_nc
// (LCP LCPdef).
//
// Pipeline (all stream-ordered, two host synchronisations: the interaction
// range sizes the grid, and the pair count is checked against capacity):
//   validate + max extent -> bin -> scan -> scatter -> count pairs -> scan
//   -> write pairs (sorted by j per i) -> j-side incidence -> q.
// Every per-pair decision is a pure function of the pair, so the contact
// list is independent of thread scheduling; within-cell member order does
// not matter because each i sorts its partners.
#include <cmath>
#include <cstring>

#include "sc_common.hpp"
#include "sc_geometry.hpp"

namespace sc {

namespace {

enum Flag {
    kFlagBadInput = 0,   // non-finite or out-of-range particle data
    kFlagParallel = 1,   // pairs resolved by the parallel-axes rule
    kFlagZero = 2,       // coincident cores
    kFlagBorder = 3,     // |Phi - delta| < 1e-12
    kFlagNonfiniteQ = 4, // q not finite (bad u_nc)
    kFlagCount = 8,
};

struct Grid {
    double lo[3], len[3], side[3];
    int nc[3];
    int periodic;
    double delta;
    __host__ __device__ PBox box() const { return PBox{{len[0], len[1], len[2]}, periodic}; }
};

struct Parts {
    int n;
    const double *pos, *axis, *radius, *half_len, *mob;
};

// ----------------------------------------------------------- cell list

__device__ __forceinline__ int cell_axis(double x, int a, const Grid &g) {
    double u = x - g.lo[a];
    if (g.periodic) u = u - g.len[a] * floor(u / g.len[a]);
    int c = static_cast<int>(floor(u / g.side[a]));
    return c < 0 ? 0 : (c >= g.nc[a] ? g.nc[a] - 1 : c);
}

// Distinct neighbour coordinates of cell coordinate c along axis a.
__device__ __forceinline__ int neighbours(int c, int a, const Grid &g, int out[3]) {
    int k = 0;
    for (int d = -1; d <= 1; ++d) {
        int x = c + d;
        if (g.periodic) {
            x = (x + g.nc[a]) % g.nc[a];
        } else if (x < 0 || x >= g.nc[a]) {
            continue;
        }
        bool dup = false;
        for (int e = 0; e < k; ++e) dup |= (out[e] == x);
        if (!dup) out[k++] = x;
    }
    return k;
}

__global__ void k_validate(Parts P, unsigned long long *max_ext, int *flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    bool bad = false;
    for (int a = 0; a < 3; ++a) bad |= !isfinite(P.pos[3 * k + a]) || !isfinite(P.axis[3 * k + a]);
    const double R = P.radius[k], h = P.half_len[k];
    bad |= !(R > 0.0) || !isfinite(R) || !(h >= 0.0) || !isfinite(h);
    for (int a = 0; a < 4; ++a) bad |= !(P.mob[4 * k + a] > 0.0) || !isfinite(P.mob[4 * k + a]);
    if (h > 0.0) {
        const V3 p = load3(P.axis + 3 * k);
        bad |= fabs(dot(p, p) - 1.0) > 1e-10;
    }
    if (bad) {
        atomicOr(flags + kFlagBadInput, 1);
        return;
    }
    // non-negative doubles order like their bit patterns
    const double e = R + h;
    atomicMax(max_ext, static_cast<unsigned long long>(__double_as_longlong(e)));
}

__global__ void k_bin(Parts P, Grid g, int *cell_of, int *cell_count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n) return;
    const int cx = cell_axis(P.pos[3 * k + 0], 0, g);
    const int cy = cell_axis(P.pos[3 * k + 1], 1, g);
    const int cz = cell_axis(P.pos[3 * k + 2], 2, g);
    const int c = (cz * g.nc[1] + cy) * g.nc[0] + cx;
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

// Visit every partner j > i of particle i (threads walk particles in cell
// order, so neighbouring lanes scan the same cells) whose pair has
// Phi <= delta, calling fn(j, geo).
template <class Fn>
__device__ __forceinline__ void for_close_partners(int i, const Parts &P, const Grid &g,
                                                   const int *cell_of, const int *cell_start,
                                                   const int *members, Fn fn) {
    const V3 ci = load3(P.pos + 3 * i), pi = load3(P.axis + 3 * i);
    const double Ri = P.radius[i], hi = P.half_len[i];
    const int c = cell_of[i];
    const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
    int nx[3], ny[3], nz[3];
    const int kx = neighbours(cx, 0, g, nx), ky = neighbours(cy, 1, g, ny),
              kz = neighbours(cz, 2, g, nz);
    for (int az = 0; az < kz; ++az)
        for (int ay = 0; ay < ky; ++ay)
            for (int ax = 0; ax < kx; ++ax) {
                const int cc = (nz[az] * g.nc[1] + ny[ay]) * g.nc[0] + nx[ax];
                const int end = cell_start[cc + 1];
                for (int m = cell_start[cc]; m < end; ++m) {
                    const int j = members[m];
                    if (j <= i) continue;
                    const V3 r = min_image(ci, load3(P.pos + 3 * j), g.box());
                    const double Rj = P.radius[j], hj = P.half_len[j];
                    // the core distance is at least |r| - hi - hj
                    const double reach = hi + hj + Ri + Rj + g.delta;
                    if (dot(r, r) > reach * reach * (1.0 + 1e-9)) continue;
                    const PairGeo G = pair_geo(r, pi, Ri, hi, load3(P.axis + 3 * j), Rj, hj);
                    if (G.phi <= g.delta) fn(j, G);
                }
            }
}

__global__ void k_count_pairs(Parts P, Grid g, const int *cell_of, const int *cell_start,
                              const int *members, int *count, int *flags) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.n) return;
    const int i = members[t];
    int cnt = 0, npar = 0, nzero = 0, nborder = 0;
    for_close_partners(i, P, g, cell_of, cell_start, members, [&](int, const PairGeo &G) {
        ++cnt;
        npar += G.flags & 1;
        nzero += (G.flags >> 1) & 1;
        nborder += fabs(G.phi - g.delta) < 1e-12;
    });
    count[i] = cnt;
    if (npar) atomicAdd(flags + kFlagParallel, npar);
    if (nzero) atomicAdd(flags + kFlagZero, nzero);
    if (nborder) atomicAdd(flags + kFlagBorder, nborder);
}

__global__ void k_write_pairs(Parts P, Grid g, const int *cell_of, const int *cell_start,
                              const int *members, const int *i_ptr, int *ci, int *cj,
                              double *phi, double *frame, long long cap) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.n) return;
    const int i = members[t];
    const int base = i_ptr[i], lim = i_ptr[i + 1] - base;
    int k = 0;
    // the count pass used the same pure predicate, so k ends at lim; the
    // bound only guards the segment
    for_close_partners(i, P, g, cell_of, cell_start, members, [&](int j, const PairGeo &) {
        if (k < lim) cj[base + k] = j;
        ++k;
    });
    if (k > lim) k = lim;
    // canonical order: partners of i by increasing j (segments are short)
    for (int a = 1; a < k; ++a) {
        const int v = cj[base + a];
        int b = a - 1;
        while (b >= 0 && cj[base + b] > v) {
            cj[base + b + 1] = cj[base + b];
            --b;
        }
        cj[base + b + 1] = v;
    }
    const V3 c_i = load3(P.pos + 3 * i), pi = load3(P.axis + 3 * i);
    const double Ri = P.radius[i], hi = P.half_len[i];
    for (int a = 0; a < k; ++a) {
        const long long l = base + a;
        const int j = cj[l];
        const V3 pj = load3(P.axis + 3 * j);
        const PairGeo G = pair_geo(min_image(c_i, load3(P.pos + 3 * j), g.box()), pi, Ri, hi, pj,
                                   P.radius[j], P.half_len[j]);
        ci[l] = i;
        phi[l] = G.phi;
        // moment arms of the contact points: tau_i = (s p_i) x n, tau_j = (t p_j) x n
        const V3 ti = cross(G.s * pi, G.n), tj = cross(G.t * pj, G.n);
        frame[0 * cap + l] = G.n.x;
        frame[1 * cap + l] = G.n.y;
        frame[2 * cap + l] = G.n.z;
        frame[3 * cap + l] = ti.x;
        frame[4 * cap + l] = ti.y;
        frame[5 * cap + l] = ti.z;
        frame[6 * cap + l] = tj.x;
        frame[7 * cap + l] = tj.y;
        frame[8 * cap + l] = tj.z;
    }
}

__global__ void k_j_degree(int nc, const int *cj, int *deg) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nc) atomicAdd(deg + cj[l], 1);
}

__global__ void k_j_fill(int nc, const int *cj, const int *j_ptr, int *fill, int *j_list) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    const int j = cj[l];
    j_list[j_ptr[j] + atomicAdd(fill + j, 1)] = l;
}

__global__ void k_j_sort(int n, const int *j_ptr, int *j_list) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int b0 = j_ptr[k], b1 = j_ptr[k + 1];
    for (int a = b0 + 1; a < b1; ++a) {
        const int v = j_list[a];
        int b = a - 1;
        while (b >= b0 && j_list[b] > v) {
            j_list[b + 1] = j_list[b];
            --b;
        }
        j_list[b + 1] = v;
    }
}

// q_l = Phi_l / dt + D_l^T U_nc (LCP LCPdef, scaled by 1/dt).
__global__ void k_q(int nc, const int *ci, const int *cj, const double *phi,
                    const double *frame, long long cap, const double *u_nc, double dt,
                    double *q, int *flags) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nc) return;
    const V3 n = frame3(frame, cap, 0, l), ti = frame3(frame, cap, 3, l),
             tj = frame3(frame, cap, 6, l);
    const double *ui = u_nc + 6 * static_cast<long long>(ci[l]);
    const double *uj = u_nc + 6 * static_cast<long long>(cj[l]);
    const double v = -dot(n, load3(ui)) - dot(ti, load3(ui + 3)) + dot(n, load3(uj)) +
                     dot(tj, load3(uj + 3));
    const double ql = phi[l] / dt + v;
    q[l] = ql;
    if (!isfinite(ql)) atomicOr(flags + kFlagNonfiniteQ, 1);
}

}  // namespace

size_t cell_budget(int32_t n) { return 2 * static_cast<size_t>(n) + 64; }

size_t contacts_ws_bytes(int32_t n, int32_t cap) {
    (void)cap;
    const size_t nn = static_cast<size_t>(n), nb = cell_budget(n);
    size_t b = 0;
    b += align_up(kFlagCount * sizeof(int), 256) + 256;     // flags
    b += 256;                                                // max extent
    b += 3 * align_up(nn * sizeof(int), 256);                // cell_of, members, j fill
    b += 2 * align_up((nb + 1) * sizeof(int), 256);          // cell_start, cell_fill
    const size_t sn = (nn + 1 > nb + 1 ? nn + 1 : nb + 1);
    b += align_up(static_cast<size_t>(scan_tmp_ints(static_cast<int>(sn))) * sizeof(int), 256);
    b += 256;                                                // host-read staging
    return b + 1024;
}

}  // namespace sc

using namespace sc;

extern "C" int sc_build_contacts(const sc_particles *p, const sc_box *box, double delta,
                                 const double *u_nc, double dt, sc_contacts *c, void *ws,
                                 size_t ws_bytes, void *stream_) {
    if (!p || !box || !c || p->n < 0 || c->capacity < 0) return SC_ERR_INVALID;
    if (!(delta >= 0.0) || !std::isfinite(delta) || !(dt > 0.0) || !std::isfinite(dt))
        return SC_ERR_INVALID;
    for (int a = 0; a < 3; ++a)
        if (!(box->len[a] > 0.0) || !std::isfinite(box->len[a]) || !std::isfinite(box->lo[a]))
            return SC_ERR_INVALID;
    c->count = 0;
    c->n_parallel = c->n_zero_dist = c->n_borderline = 0;
    c->grid[0] = c->grid[1] = c->grid[2] = 0;
    const int n = p->n;
    if (!c->i_ptr || !c->j_ptr) return SC_ERR_INVALID;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (n == 0) {
        SC_HIP_TRY(hipMemsetAsync(c->i_ptr, 0, sizeof(int), stream));
        SC_HIP_TRY(hipMemsetAsync(c->j_ptr, 0, sizeof(int), stream));
        SC_HIP_TRY(hipStreamSynchronize(stream));
        return SC_OK;
    }
    if (!p->pos || !p->axis || !p->radius || !p->half_len || !p->mob || !u_nc) return SC_ERR_INVALID;
    if (c->capacity > 0 && (!c->ci || !c->cj || !c->phi || !c->q || !c->frame || !c->j_list))
        return SC_ERR_INVALID;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return SC_ERR_WORKSPACE;
    if (ws_bytes < contacts_ws_bytes(n, c->capacity)) return SC_ERR_WORKSPACE;

    const size_t nb = cell_budget(n);
    Carver cv{static_cast<char *>(ws), ws_bytes};
    int *flags = cv.take<int>(kFlagCount);
    unsigned long long *max_ext = cv.take<unsigned long long>(1);
    int *cell_of = cv.take<int>(n);
    int *members = cv.take<int>(n);
    int *jfill = cv.take<int>(n);
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
    Grid g{};
    size_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = box->lo[a];
        g.len[a] = box->len[a];
        if (box->periodic && box->len[a] < 2.0 * rmax) return SC_ERR_BOX;
        double m = std::floor(box->len[a] / rmax);
        g.nc[a] = m < 1.0 ? 1 : (m > 1024.0 ? 1024 : static_cast<int>(m));
    }
    // keep the grid within the workspace's cell budget (bigger cells stay correct)
    while (static_cast<size_t>(g.nc[0]) * g.nc[1] * g.nc[2] > nb) {
        int a = (g.nc[0] >= g.nc[1] && g.nc[0] >= g.nc[2]) ? 0 : (g.nc[1] >= g.nc[2] ? 1 : 2);
        g.nc[a] = g.nc[a] > 1 ? (g.nc[a] + 1) / 2 : 1;
    }
    ncell = static_cast<size_t>(g.nc[0]) * g.nc[1] * g.nc[2];
    for (int a = 0; a < 3; ++a) {
        g.side[a] = box->len[a] / g.nc[a];
        c->grid[a] = g.nc[a];
    }
    g.periodic = box->periodic ? 1 : 0;
    g.delta = delta;

    // bin particles, then sort them by cell (order within a cell is free)
    SC_HIP_TRY(hipMemsetAsync(cell_start, 0, (ncell + 1) * sizeof(int), stream));
    SC_HIP_TRY(hipMemsetAsync(cell_fill, 0, ncell * sizeof(int), stream));
    k_bin<<<grid_for(n), kBlock, 0, stream>>>(P, g, cell_of, cell_start);
    scan_exclusive(cell_start, cell_start, static_cast<int>(ncell), scan_tmp, stream);
    k_scatter<<<grid_for(n), kBlock, 0, stream>>>(n, cell_of, cell_start, cell_fill, members);

    // count close partners per i, then offsets
    k_count_pairs<<<grid_for(n), kBlock, 0, stream>>>(P, g, cell_of, cell_start, members,
                                                      c->i_ptr, flags);
    scan_exclusive(c->i_ptr, c->i_ptr, n, scan_tmp, stream);
    SC_HIP_TRY(hipMemcpyAsync(stage, c->i_ptr + n, sizeof(int), hipMemcpyDeviceToDevice, stream));
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

    const long long cap = c->capacity;
    k_write_pairs<<<grid_for(n), kBlock, 0, stream>>>(P, g, cell_of, cell_start, members,
                                                      c->i_ptr, c->ci, c->cj, c->phi, c->frame,
                                                      cap);
    // j-side incidence: contacts l with cj[l] == k, ascending
    SC_HIP_TRY(hipMemsetAsync(c->j_ptr, 0, (n + 1) * sizeof(int), stream));
    SC_HIP_TRY(hipMemsetAsync(jfill, 0, n * sizeof(int), stream));
    if (nc > 0) {
        k_j_degree<<<grid_for(nc), kBlock, 0, stream>>>(nc, c->cj, c->j_ptr);
    }
    scan_exclusive(c->j_ptr, c->j_ptr, n, scan_tmp, stream);
    if (nc > 0) {
        k_j_fill<<<grid_for(nc), kBlock, 0, stream>>>(nc, c->cj, c->j_ptr, jfill, c->j_list);
        k_j_sort<<<grid_for(n), kBlock, 0, stream>>>(n, c->j_ptr, c->j_list);
        k_q<<<grid_for(nc), kBlock, 0, stream>>>(nc, c->ci, c->cj, c->phi, c->frame, cap, u_nc,
                                                 dt, c->q, flags);
    }
    SC_HIP_TRY(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, stream));
    SC_HIP_TRY(hipStreamSynchronize(stream));
    SC_HIP_TRY(hipGetLastError());
    if (hflags[kFlagNonfiniteQ]) return SC_ERR_NONFINITE;
    return SC_OK;
}
