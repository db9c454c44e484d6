// sc_batch_build.hip -- the build of every suspension of a batch (close pairs
// of section 3.2 with a cell list, contact frames for Eq. Dmatdef and
// Eq. Dtranspose, q of LCP LCPdef, incidence lists and the assembled M) as
// one sequence of launches over the whole batch, on gfx950.
//
// Each launch covers one shared index space (particles and ranks, cells,
// contact slots or matrix slices); a thread finds its suspension by binary
// search in that space's offsets and runs the same per-item step as the
// single-suspension build (sc_build_dev.hpp, sc_assemble_dev.hpp) on the
// suspension's own buffers, so the contacts and M of a suspension equal those
// of its own build bit for bit. Counts stay on the device: a suspension whose
// data are bad, whose particles outgrew the planned search grid or whose
// contacts or nonzeros exceed its capacity gets an error status and is
// skipped by every later step; the others are unaffected.
#include <algorithm>
#include <cstring>

#include "sc_assemble_dev.hpp"
#include "sc_batch_build.hpp"
#include "sc_build_dev.hpp"
#include "sc_common.hpp"

namespace sc {

namespace {

// The suspension owning index x of a space whose offsets are base[0..count]
// (base[0] = 0, non-decreasing): the k with base[k] <= x < base[k + 1].
__device__ __forceinline__ int owner(const int *base, int count, int x) {
    int lo = 0, hi = count;  // base[lo] <= x < base[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool input_bad(const BuildOut &o) {
    return o.flags[kFlagBadInput] != 0 || o.flags[kFlagExtent] != 0;
}

__device__ __forceinline__ Ranked ranked_of(const BatchBuild &B, const BuildInst &I) {
    return Ranked{B.prec + 4 * static_cast<long long>(I.pbase), B.hl + I.pbase,
                  B.cell_r + I.pbase};
}

__device__ __forceinline__ ChainView chain_of(const BuildInst &I, int nc) {
    return ChainView{I.P.n, nc, I.pl.pdat, I.pl.inc_ptr, I.pl.inc, I.pl.dpm, I.pl.cs, I.frame,
                     nullptr};
}

// Clears the per-call state: cell counters, degree and fill cursors, outputs.
__global__ void kb_reset(BatchBuild B) {
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    const long long i0 = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (long long i = i0; i <= B.C; i += stride) {
        B.cell_start[i] = 0;
        if (i < B.C) B.cell_fill[i] = 0;
    }
    for (long long i = i0; i < B.N; i += stride) {
        B.deg[i] = 0;
        B.fill[i] = 0;
    }
    for (long long i = i0; i < B.count; i += stride) B.out[i] = BuildOut{};
}

// Particle checks; when planning (ext_bits set) also the largest R + h.
__global__ void kb_validate(BatchBuild B, int planning) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.N) return;
    const int k = owner(B.pbase, B.count, x);
    const BuildInst &I = B.inst[k];
    const int i = x - I.pbase;
    if (particle_bad(I.P, i)) {
        atomicOr(B.out[k].flags + kFlagBadInput, 1);
        return;
    }
    const double e = I.P.radius[i] + I.P.half_len[i];
    if (planning)
        atomicMax(B.ext_bits + k, static_cast<unsigned long long>(__double_as_longlong(e)));
    else if (e > I.ext)
        atomicOr(B.out[k].flags + kFlagExtent, 1);
}

// Every particle is binned, also those of a suspension with bad data (all
// into its first cell), so that suspension k's ranks are exactly
// [pbase_k, pbase_k + n_k) of the shared rank space.
__global__ void kb_bin(BatchBuild B) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.N) return;
    const int k = owner(B.pbase, B.count, x);
    const BuildInst &I = B.inst[k];
    const int c = B.out[k].flags[kFlagBadInput] ? I.cbase
                                                : particle_cell(I.P, x - I.pbase, I.g, I.cbase);
    B.cell_of[x] = c;
    atomicAdd(B.cell_start + c, 1);
}

__global__ void kb_scatter(BatchBuild B) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.N) return;
    const int c = B.cell_of[x];
    B.members[B.cell_start[c] + atomicAdd(B.cell_fill + c, 1)] = x;
}

__global__ void kb_rank(BatchBuild B) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.N) return;
    const int k = owner(B.pbase, B.count, x);
    if (input_bad(B.out[k])) return;
    const BuildInst &I = B.inst[k];
    rank_particle(I.P, x - I.pbase, I.pbase, I.cbase, B.cell_of, B.cell_start, B.members, I.pl,
                  B.prec, B.hl, B.cell_r);
}

// kPairLanes consecutive threads per rank; all lanes of a rank belong to the
// same suspension and leave together.
__global__ void kb_count_pairs(BatchBuild B) {
    const long long gid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int x = static_cast<int>(gid / kPairLanes), lane = static_cast<int>(gid % kPairLanes);
    if (x >= B.N) return;
    const int k = owner(B.pbase, B.count, x);
    if (input_bad(B.out[k])) return;
    const BuildInst &I = B.inst[k];
    count_partners(x - I.pbase, lane, ranked_of(B, I), I.pl, I.g, B.cell_start + I.cbase,
                   I.pbase, B.lane_cnt + gid, B.slots + kLaneSlots * gid, B.out[k].flags);
}

// After the scan of the per-rank counts: the contact count and the status.
__global__ void kb_after_count(BatchBuild B) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B.count) return;
    const BuildInst &I = B.inst[k];
    BuildOut &o = B.out[k];
    if (o.flags[kFlagBadInput]) {
        o.status = SC_ERR_NONFINITE;
    } else if (o.flags[kFlagExtent]) {
        o.status = SC_ERR_BOX;
    } else {
        const int nc = I.pl.cptr[I.P.n];
        o.nc = nc;
        o.ns = (nc + kWave - 1) / kWave;
        if (nc > I.cap) o.status = SC_ERR_CAPACITY;
    }
}

__global__ void kb_write_pairs(BatchBuild B) {
    const long long gid = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int x = static_cast<int>(gid / kPairLanes), lane = static_cast<int>(gid % kPairLanes);
    if (x >= B.N) return;
    const int k = owner(B.pbase, B.count, x);
    if (B.out[k].status != SC_OK) return;
    const BuildInst &I = B.inst[k];
    write_partners(x - I.pbase, lane, ranked_of(B, I), I.pl, I.g, B.cell_start + I.cbase,
                   I.pbase, B.lane_cnt + (gid - lane), B.slots + kLaneSlots * gid);
}

__global__ void kb_finish_pairs(BatchBuild B) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.N) return;
    const int k = owner(B.pbase, B.count, x);
    if (B.out[k].status != SC_OK) return;
    const BuildInst &I = B.inst[k];
    finish_partners(x - I.pbase, ranked_of(B, I), I.pl, I.g, I.ci, I.cj, I.phi, I.frame);
}

__global__ void kb_second_degree(BatchBuild B) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.L) return;
    const int k = owner(B.lbase, B.count, x);
    const BuildOut &o = B.out[k];
    const BuildInst &I = B.inst[k];
    const int l = x - I.lbase;
    if (o.status != SC_OK || l >= o.nc) return;
    count_second(l, I.pl, B.deg + I.pbase);
}

__global__ void kb_inc_counts(BatchBuild B) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.N) return;
    const int k = owner(B.pbase, B.count, x);
    if (B.out[k].status != SC_OK) return;
    const BuildInst &I = B.inst[k];
    incidence_count(x - I.pbase, I.pl, B.deg + I.pbase);
}

__global__ void kb_inc_fill(BatchBuild B) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.L) return;
    const int k = owner(B.lbase, B.count, x);
    const BuildOut &o = B.out[k];
    const BuildInst &I = B.inst[k];
    const int l = x - I.lbase;
    if (o.status != SC_OK || l >= o.nc) return;
    incidence_fill(l, I.pl, B.fill + I.pbase);
}

__global__ void kb_inc_finish(BatchBuild B) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.N) return;
    const int k = owner(B.pbase, B.count, x);
    if (B.out[k].status != SC_OK) return;
    const BuildInst &I = B.inst[k];
    incidence_finish(x - I.pbase, I.pl, I.frame);
}

// q and the row lengths of M, per contact slot.
__global__ void kb_q_rows(BatchBuild B) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= B.L) return;
    const int k = owner(B.lbase, B.count, x);
    BuildOut &o = B.out[k];
    const BuildInst &I = B.inst[k];
    const int l = x - I.lbase;
    if (o.status != SC_OK || l >= o.nc) return;
    const double ql = contact_q(l, I.ci, I.cj, I.phi, I.frame, I.u_nc, I.dt);
    I.q[l] = ql;
    if (!isfinite(ql)) atomicOr(o.flags + kFlagNonfiniteQ, 1);
    I.mb.len[l] = row_length(chain_of(I, o.nc), l);
}

// One wave per slice slot.
__global__ void kb_slice_sums(BatchBuild B) {
    const int x = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (x >= B.S) return;  // whole waves
    const int k = owner(B.sbase, B.count, x);
    const BuildOut &o = B.out[k];
    const BuildInst &I = B.inst[k];
    const int sl = x - I.sbase;
    if (o.status != SC_OK || sl >= o.ns) return;
    slice_sums(sl, o.nc, I.mb.len, I.mb.soff, I.mb.swid);
}

// After the scan of the slice sums: nonzeros against capacity, q finite.
__global__ void kb_after_matrix(BatchBuild B) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= B.count) return;
    const BuildInst &I = B.inst[k];
    BuildOut &o = B.out[k];
    if (o.status != SC_OK) return;
    o.nnz = I.mb.soff[o.ns];
    if (o.flags[kFlagNonfiniteQ])
        o.status = SC_ERR_NONFINITE;
    else if (o.nnz > I.nnz_cap)
        o.status = SC_ERR_CAPACITY;
}

__global__ void kb_assemble(BatchBuild B) {
    const int x = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (x >= B.S) return;  // whole waves
    const int k = owner(B.sbase, B.count, x);
    const BuildOut &o = B.out[k];
    const BuildInst &I = B.inst[k];
    const int sl = x - I.sbase;
    if (o.status != SC_OK || sl >= o.ns) return;
    assemble_slice(chain_of(I, o.nc), sl, I.mb.len, I.mb.soff, I.mb.swid, I.mb.col, I.mb.val);
}

// Exclusive scans, one workgroup per suspension: which = 0 the per-rank
// contact counts, 1 the incidence counts, 2 the slice sums of M. A skipped
// suspension keeps a zero total.
__global__ void __launch_bounds__(1024) kb_seg_scan(BatchBuild B, int which) {
    const int k = blockIdx.x;
    const BuildInst &I = B.inst[k];
    const BuildOut &o = B.out[k];
    int *p;
    int len;
    if (which == 0) {
        p = I.pl.cptr;
        len = input_bad(o) ? 0 : I.P.n;
    } else if (which == 1) {
        p = I.pl.inc_ptr;
        len = o.status != SC_OK ? 0 : I.P.n;
    } else {
        p = I.mb.soff;
        len = o.status != SC_OK ? 0 : o.ns;
    }
    __shared__ int wsum[1024 / kWave + 1];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    int carry = 0;
    for (int base = 0; base < len; base += blockDim.x) {
        const int idx = base + threadIdx.x;
        const int v = idx < len ? p[idx] : 0;
        int incl = v;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int t = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += t;
        }
        if (lane == kWave - 1) wsum[wid] = incl;
        __syncthreads();
        if (wid == 0) {
            const int nw = blockDim.x / kWave;
            const int t = lane < nw ? wsum[lane] : 0;
            int ti = t;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int u = __shfl_up(ti, off, kWave);
                if (lane >= off) ti += u;
            }
            if (lane < nw) wsum[lane] = ti - t;
            if (lane == nw - 1) wsum[nw] = ti;
        }
        __syncthreads();
        if (idx < len) p[idx] = carry + wsum[wid] + incl - v;
        carry += wsum[blockDim.x / kWave];
        __syncthreads();
    }
    if (threadIdx.x == 0) p[len] = carry;
}

inline int blocks_for(long long items) {
    return static_cast<int>(std::max<long long>(1, (items + kBlock - 1) / kBlock));
}

}  // namespace

size_t batch_build_bytes(int32_t count, const sc_batch_item *items) {
    size_t n = 0, cells = 0;
    for (int32_t k = 0; k < count; ++k) {
        n += static_cast<size_t>(std::max(items[k].p.n, 0));
        cells += cell_budget(std::max(items[k].p.n, 0));
    }
    const size_t nd = static_cast<size_t>(std::max(count, 1));
    size_t b = 0;
    b += align_up(sizeof(BuildInst) * nd, 256) + align_up(sizeof(BuildOut) * nd, 256);
    b += 3 * align_up(sizeof(int) * (nd + 1), 256) + align_up(sizeof(unsigned long long) * nd, 256);
    const size_t nn = std::max<size_t>(n, 1);
    b += 6 * align_up(sizeof(int) * nn, 256);                  // cell_of .. fill, spare
    b += align_up(sizeof(int) * kPairLanes * nn, 256);         // per-lane pair counts
    b += align_up(sizeof(int) * kLaneSlots * kPairLanes * nn, 256);  // per-lane partners
    b += align_up(sizeof(double) * 4 * nn, 256) + align_up(sizeof(double) * nn, 256);
    b += 2 * align_up(sizeof(int) * (cells + 1), 256);
    b += align_up(sizeof(int) * scan_tmp_ints(static_cast<int>(cells + 1)), 256);
    return b + 256;
}

int batch_build_plan(int32_t count, const sc_batch_item *items, Carver &cv, hipStream_t s,
                     BatchBuild &b, std::vector<BuildInst> &host) {
    host.assign(static_cast<size_t>(count), BuildInst{});
    std::vector<int> pbase(static_cast<size_t>(count) + 1, 0), lbase(pbase), sbase(pbase);
    size_t cells_budget = 0;
    for (int32_t k = 0; k < count; ++k) {
        const sc_batch_item &it = items[k];
        const sc_contacts &c = it.c;
        BuildInst &I = host[k];
        const int n = it.p.n;
        if (n < 0 || c.capacity < 0 || c.nnz < 0 || !(it.dt > 0.0) || !(it.delta >= 0.0) ||
            !std::isfinite(it.delta))
            return SC_ERR_INVALID;
        for (int a = 0; a < 3; ++a)
            if (!(it.box.len[a] > 0.0) || !std::isfinite(it.box.len[a]) ||
                !std::isfinite(it.box.lo[a]))
                return SC_ERR_INVALID;
        if (it.box.walls < 0 || it.box.walls > 63 || (it.box.periodic && it.box.walls))
            return SC_ERR_INVALID;
        if (n > 0 && (!it.p.pos || !it.p.axis || !it.p.radius || !it.p.half_len || !it.p.mob ||
                      !it.u_nc))
            return SC_ERR_INVALID;
        if (c.capacity > 0 && (!c.ci || !c.cj || !c.phi || !c.q || !c.frame))
            return SC_ERR_INVALID;
        if (!carve_plan(c.plan, c.plan_bytes, n, c.capacity, I.pl)) return SC_ERR_INVALID;
        if (!carve_matrix(c.mat, c.mat_bytes, c.capacity, c.nnz, I.mb)) return SC_ERR_INVALID;
        I.P = Parts{n, it.p.pos, it.p.axis, it.p.radius, it.p.half_len, it.p.mob};
        I.u_nc = it.u_nc;
        I.dt = it.dt;
        I.ci = c.ci;
        I.cj = c.cj;
        I.phi = c.phi;
        I.q = c.q;
        I.frame = c.frame;
        I.cap = c.capacity;
        I.nnz_cap = c.nnz;
        I.pbase = pbase[k];
        I.lbase = lbase[k];
        I.sbase = sbase[k];
        pbase[k + 1] = pbase[k] + n;
        lbase[k + 1] = lbase[k] + c.capacity;
        sbase[k + 1] = sbase[k] + slices(c.capacity);
        cells_budget += cell_budget(n);
    }
    b.count = count;
    b.N = pbase[count];
    b.L = lbase[count];
    b.S = sbase[count];
    const size_t nd = static_cast<size_t>(std::max(count, 1));
    const size_t n = static_cast<size_t>(std::max(b.N, 1));
    b.inst = cv.take<BuildInst>(nd);
    b.out = cv.take<BuildOut>(nd);
    b.pbase = cv.take<int>(nd + 1);
    b.lbase = cv.take<int>(nd + 1);
    b.sbase = cv.take<int>(nd + 1);
    b.ext_bits = cv.take<unsigned long long>(nd);
    b.cell_of = cv.take<int>(n);
    b.members = cv.take<int>(n);
    b.cell_r = cv.take<int>(n);
    b.deg = cv.take<int>(n);
    b.fill = cv.take<int>(n);
    cv.take<int>(n);  // spare (keeps the layout of batch_build_bytes)
    b.lane_cnt = cv.take<int>(kPairLanes * n);
    b.slots = cv.take<int>(static_cast<size_t>(kLaneSlots) * kPairLanes * n);
    b.prec = cv.take<double>(4 * n);
    b.hl = cv.take<double>(n);
    b.cell_start = cv.take<int>(cells_budget + 1);
    b.cell_fill = cv.take<int>(cells_budget + 1);
    b.scan_tmp = cv.take<int>(scan_tmp_ints(static_cast<int>(cells_budget + 1)));
    if (!cv.ok) return SC_ERR_INVALID;
    if (count == 0) return SC_OK;

    // extents: upload the tables with provisional grids, measure, then fix
    // the grids and cell offsets
    b.C = 0;
    SC_HIP_TRY(hipMemcpyAsync(b.inst, host.data(), sizeof(BuildInst) * count,
                              hipMemcpyHostToDevice, s));
    SC_HIP_TRY(hipMemcpyAsync(b.pbase, pbase.data(), sizeof(int) * (count + 1),
                              hipMemcpyHostToDevice, s));
    SC_HIP_TRY(hipMemcpyAsync(b.lbase, lbase.data(), sizeof(int) * (count + 1),
                              hipMemcpyHostToDevice, s));
    SC_HIP_TRY(hipMemcpyAsync(b.sbase, sbase.data(), sizeof(int) * (count + 1),
                              hipMemcpyHostToDevice, s));
    kb_reset<<<blocks_for(std::max(b.N, count)), kBlock, 0, s>>>(b);
    SC_HIP_TRY(hipMemsetAsync(b.ext_bits, 0, sizeof(unsigned long long) * count, s));
    if (b.N > 0) kb_validate<<<blocks_for(b.N), kBlock, 0, s>>>(b, 1);
    std::vector<unsigned long long> ext(static_cast<size_t>(count));
    std::vector<BuildOut> out(static_cast<size_t>(count));
    SC_HIP_TRY(hipMemcpyAsync(ext.data(), b.ext_bits, sizeof(unsigned long long) * count,
                              hipMemcpyDeviceToHost, s));
    SC_HIP_TRY(hipMemcpyAsync(out.data(), b.out, sizeof(BuildOut) * count, hipMemcpyDeviceToHost,
                              s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    int cbase = 0;
    for (int32_t k = 0; k < count; ++k) {
        if (out[k].flags[kFlagBadInput]) return SC_ERR_NONFINITE;
        BuildInst &I = host[k];
        double e = 0.0;
        const long long bits = static_cast<long long>(ext[k]);
        std::memcpy(&e, &bits, sizeof(e));
        I.ext = e;
        I.cbase = cbase;
        if (I.P.n == 0) {
            I.ncell = 0;
            continue;
        }
        if (!make_grid(items[k].box, I.P.n, items[k].delta, 2.0 * e + items[k].delta,
                       cell_budget(I.P.n), I.g))
            return SC_ERR_BOX;
        I.ncell = I.g.nc[0] * I.g.nc[1] * I.g.nc[2];
        cbase += I.ncell;
    }
    b.C = cbase;
    SC_HIP_TRY(hipMemcpyAsync(b.inst, host.data(), sizeof(BuildInst) * count,
                              hipMemcpyHostToDevice, s));
    SC_HIP_TRY(hipStreamSynchronize(s));
    return SC_OK;
}

int batch_build_enqueue(const BatchBuild &b, hipStream_t s) {
    if (b.count == 0) return SC_OK;
    const int wave_blocks = std::max(1, (b.S + kBlock / kWave - 1) / (kBlock / kWave));
    kb_reset<<<blocks_for(std::max<long long>(std::max(b.N, b.C + 1), b.count)), kBlock, 0, s>>>(b);
    if (b.N > 0) {
        kb_validate<<<blocks_for(b.N), kBlock, 0, s>>>(b, 0);
        kb_bin<<<blocks_for(b.N), kBlock, 0, s>>>(b);
    }
    if (b.C > 0) scan_exclusive(b.cell_start, b.cell_start, b.C, b.scan_tmp, s);
    if (b.N > 0) {
        kb_scatter<<<blocks_for(b.N), kBlock, 0, s>>>(b);
        kb_rank<<<blocks_for(b.N), kBlock, 0, s>>>(b);
        kb_count_pairs<<<blocks_for(static_cast<long long>(b.N) * kPairLanes), kBlock, 0, s>>>(b);
    }
    kb_seg_scan<<<b.count, 1024, 0, s>>>(b, 0);
    kb_after_count<<<blocks_for(b.count), kBlock, 0, s>>>(b);
    if (b.N > 0) {
        kb_write_pairs<<<blocks_for(static_cast<long long>(b.N) * kPairLanes), kBlock, 0, s>>>(b);
        kb_finish_pairs<<<blocks_for(b.N), kBlock, 0, s>>>(b);
    }
    if (b.L > 0) kb_second_degree<<<blocks_for(b.L), kBlock, 0, s>>>(b);
    if (b.N > 0) kb_inc_counts<<<blocks_for(b.N), kBlock, 0, s>>>(b);
    kb_seg_scan<<<b.count, 1024, 0, s>>>(b, 1);
    if (b.L > 0) kb_inc_fill<<<blocks_for(b.L), kBlock, 0, s>>>(b);
    if (b.N > 0) kb_inc_finish<<<blocks_for(b.N), kBlock, 0, s>>>(b);
    if (b.L > 0) kb_q_rows<<<blocks_for(b.L), kBlock, 0, s>>>(b);
    if (b.S > 0) kb_slice_sums<<<wave_blocks, kBlock, 0, s>>>(b);
    kb_seg_scan<<<b.count, 1024, 0, s>>>(b, 2);
    kb_after_matrix<<<blocks_for(b.count), kBlock, 0, s>>>(b);
    if (b.S > 0) kb_assemble<<<wave_blocks, kBlock, 0, s>>>(b);
    SC_HIP_TRY(hipGetLastError());
    return SC_OK;
}

}  // namespace sc
