// sc_matrix.hip -- assembled M = D^T Mob D and the one-barrier persistent
// solvers built on it (gfx950).
//
// With a block-diagonal mobility, M is sparse: contacts l and m interact
// only through a shared particle k, M_lm = a_lk^T Mob_k a_mk (a_lk the signed
// column entries of contact l on particle k), so row l has
// deg(ci) + deg(cj) - 1 entries. Forming it once turns each BBPGD iteration
// into a single contact-major pass: the projected descent step of Algorithm
// 1 is formed on the fly for every column, g = M gamma + q and the sums of
// the stopping test and the BB step size are accumulated, then one grid barrier and
// a fixed-order reduction decide the next step. The adjoint's masked CG is
// laid out the same way. Rows are in solver order, so column gathers stay
// local.
//
// Storage: rows are cut into slices of 64 consecutive rows, one wave and one
// lane per row. Within a slice the entries are stored depth by depth (all
// first entries of the slice's rows, then all second entries, ...) and each
// depth holds only the rows that are that long, packed in lane order. A
// wave's load at one depth is therefore one contiguous run, no padding is
// stored, and the row order (and so gather locality) is untouched. The
// position of a lane's entry at depth t is the slice offset plus the entries
// of the shallower depths plus the number of lower lanes still active at t,
// all of which the wave derives from ballots of (t < len).
#include <climits>

#include "sc_assemble_dev.hpp"
#include "sc_chain.hpp"
#include "sc_common.hpp"
#include "sc_matrix.hpp"
#include "sc_matrix_pass.hpp"
#include "sc_plan.hpp"
#include "sc_sync.hpp"

namespace sc {

namespace {

__global__ void k_row_lengths(ChainView C, int32_t *len) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= C.nc) return;
    len[l] = row_length(C, l);
}

// Entries and widest row of every slice (one wave per slice).
__global__ void k_slice_sums(int nc, int ns, const int32_t *len, int32_t *soff, int32_t *swid) {
    const int sl = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (sl >= ns) return;  // whole waves
    slice_sums(sl, nc, len, soff, swid);
}

// One wave per slice writes its rows (layout in the file header).
__global__ void k_assemble(ChainView C, int ns, const int32_t *len, const int32_t *soff,
                           const int32_t *swid, int32_t *col, double *val) {
    const int sl = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (sl >= ns) return;  // whole waves
    assemble_slice(C, sl, len, soff, swid, col, val);
}

struct MatSolve {
    MatView M;
    const double *q;
    double *gamma;          // in: gamma_0; out: last iterate
    double *g;              // out: M gamma + q
    GG *z[2];               // iterate buffers
    double *part;
    GridSync *sync;
    SolveCtrl *ctrl;
    double tol;
    int max_iter, bb;
    int cache;              // LDS entries of the workgroup
};

template <int R, int BS>
__global__ void __launch_bounds__(BS) k_bbpgd_mat(MatSolve A) {
    GridBarrier bar;
    bar.init(A.sync);
    const int L = logical_block();
    const SliceChunk rc = slice_chunk(A.M, L, gridDim.x);
    const WaveCache W = wave_cache<R, BS>(A.M, rc, A.cache);
    fill_cache<R, BS>(A.M, rc, W);
    // 6 gathers in flight per wave (one slice per wave): measured best here
    constexpr int B = R == 1 ? 6 : 8 / R;
    bbpgd_rows<R, BS, GridBarrier, B>(A.M, rc, W, A.q, A.gamma, A.gamma, A.g, A.z[0], A.z[1],
                                      A.part, kPartHalf, L, gridDim.x, bar, A.tol, A.max_iter,
                                      A.bb, A.ctrl);
}

struct MatCg {
    MatView M;
    const double *gamma;
    RWS *z[2];
    double *p, *x;
    double *part;
    GridSync *sync;
    CgCtrl *ctrl;
    double tol;
    int max_iter;
    int cache;              // LDS entries of the workgroup
};

template <int R, int BS>
__global__ void __launch_bounds__(BS) k_cg_mat(MatCg A) {
    GridBarrier bar;
    bar.init(A.sync);
    const int L = logical_block();
    const SliceChunk rc = slice_chunk(A.M, L, gridDim.x);
    const WaveCache W = wave_cache<R, BS>(A.M, rc, A.cache);
    fill_cache<R, BS>(A.M, rc, W);
    const WaveMeta<R> Mt = wave_meta<R, BS>(A.M, rc);
    cg_rows<R, BS>(A.M, rc, W, Mt, A.gamma, A.z[0], A.z[1], A.p, A.x, A.part, kPartHalf, L,
                   gridDim.x, bar, A.tol, A.max_iter, A.ctrl);
}

using BbMatKernel = void (*)(MatSolve);
using CgMatKernel = void (*)(MatCg);

template <int BS>
BbMatKernel bb_mat_bs(int spw) {
    switch (spw) {
    case 2: return k_bbpgd_mat<2, BS>;
    case 4: return k_bbpgd_mat<4, BS>;
    default: return k_bbpgd_mat<1, BS>;
    }
}

template <int BS>
CgMatKernel cg_mat_bs(int spw) {
    switch (spw) {
    case 2: return k_cg_mat<2, BS>;
    case 4: return k_cg_mat<4, BS>;
    default: return k_cg_mat<1, BS>;
    }
}

}  // namespace

size_t matrix_bytes(int32_t nc, int64_t nnz) {
    if (nc < 0 || nnz < 0 || nnz > INT_MAX) return 0;
    const size_t cc = static_cast<size_t>(nc), zz = static_cast<size_t>(nnz);
    const size_t ns = static_cast<size_t>(slices(nc));
    return align_up(cc * sizeof(int32_t), 256) + align_up((ns + 1) * sizeof(int32_t), 256) +
           align_up(ns * sizeof(int32_t), 256) + align_up(zz * sizeof(int32_t), 256) +
           align_up(zz * sizeof(double), 256) +
           align_up(static_cast<size_t>(scan_tmp_ints(slices(nc) + 1)) * sizeof(int32_t), 256) +
           256;
}

bool carve_matrix(void *base, size_t bytes, int32_t nc, int64_t nnz, MatBufs &m) {
    const size_t need = matrix_bytes(nc, nnz);
    if (!base || need == 0 || bytes < need || (reinterpret_cast<uintptr_t>(base) & 255) != 0)
        return false;
    Carver cv{static_cast<char *>(base), bytes};
    const int ns = slices(nc);
    m.ns = ns;
    m.len = cv.take<int32_t>(static_cast<size_t>(nc));
    m.soff = cv.take<int32_t>(static_cast<size_t>(ns) + 1);
    m.swid = cv.take<int32_t>(static_cast<size_t>(ns));
    m.col = cv.take<int32_t>(static_cast<size_t>(nnz));
    m.val = cv.take<double>(static_cast<size_t>(nnz));
    m.scan_tmp = cv.take<int32_t>(scan_tmp_ints(ns + 1));
    return cv.ok;
}

MatView mat_view(int32_t nc, const MatBufs &m) {
    return MatView{nc, m.ns, m.len, m.soff, m.swid, m.col, m.val};
}

namespace {

// Dynamic LDS for the matrix cache of a persistent kernel: everything the
// workgroup does not use statically, at 12 bytes per entry (value and
// column). `request`: 0 = as much as fits, < 0 = none, > 0 = at most that
// many entries per wave. *per_wave is the workgroup's entries over its waves.
hipError_t cache_shape(const void *fn, int block, int request, int *per_wave, size_t *dyn) {
    *per_wave = 0;
    *dyn = 16;  // the pass reads slot 0 unconditionally
    if (request < 0) return hipSuccess;
    int dev = 0, max_lds = 0;
    hipFuncAttributes fa;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e == hipSuccess) e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    const int nw = block / kWave;
    const long long room = static_cast<long long>(max_lds) - static_cast<long long>(fa.sharedSizeBytes) - 256;
    long long per = room > 0 ? room / (12LL * nw) : 0;
    per -= per % 2;  // keeps the column block 8-byte aligned
    if (request > 0 && per > request) per = request - request % 2;
    if (per < 2) return hipSuccess;
    *per_wave = static_cast<int>(per);
    *dyn = static_cast<size_t>(per) * 12 * nw;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(*dyn));
}

}  // namespace

hipError_t launch_bbpgd_mat(const MatView &M, const double *q, double *gamma, double *g,
                            double *zbuf, double *part, GridSync *sync, SolveCtrl *ctrl,
                            double tol, int max_iter, int bb, int spw, int cache, int block,
                            int grid, hipStream_t s, int *grid_used, int *cache_used) {
    BbMatKernel kern = block == 256   ? bb_mat_bs<256>(spw)
                       : block == 512 ? bb_mat_bs<512>(spw)
                                      : bb_mat_bs<1024>(spw);
    const void *fn = reinterpret_cast<const void *>(kern);
    size_t dyn = 0;
    int per = 0;
    hipError_t e = cache_shape(fn, block, cache, &per, &dyn);
    if (e != hipSuccess) return e;
    *cache_used = per;
    const int G = persistent_grid(fn, block, grid, dyn);
    *grid_used = G;
    if (G < 1) return hipErrorInvalidConfiguration;
    MatSolve A;
    A.M = M;
    A.q = q;
    A.gamma = gamma;
    A.g = g;
    A.z[0] = reinterpret_cast<GG *>(zbuf);
    A.z[1] = reinterpret_cast<GG *>(zbuf) + M.nc;
    A.part = part;
    A.sync = sync;
    A.ctrl = ctrl;
    A.tol = tol;
    A.max_iter = max_iter;
    A.bb = bb;
    A.cache = per * (block / kWave);
    void *args[] = {&A};
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(block), args, dyn, s);
}

hipError_t launch_cg_mat(const MatView &M, const double *gamma, double *zbuf, double *p,
                         double *x, double *part, GridSync *sync, CgCtrl *ctrl, double tol,
                         int max_iter, int spw, int cache, int block, int grid, hipStream_t s,
                         int *grid_used, int *cache_used) {
    CgMatKernel kern = block == 256   ? cg_mat_bs<256>(spw)
                       : block == 512 ? cg_mat_bs<512>(spw)
                                      : cg_mat_bs<1024>(spw);
    const void *fn = reinterpret_cast<const void *>(kern);
    size_t dyn = 0;
    int per = 0;
    hipError_t e = cache_shape(fn, block, cache, &per, &dyn);
    if (e != hipSuccess) return e;
    *cache_used = per;
    const int G = persistent_grid(fn, block, grid, dyn);
    *grid_used = G;
    if (G < 1) return hipErrorInvalidConfiguration;
    MatCg A;
    A.M = M;
    A.gamma = gamma;
    A.z[0] = reinterpret_cast<RWS *>(zbuf);
    A.z[1] = reinterpret_cast<RWS *>(zbuf) + M.nc;
    A.p = p;
    A.x = x;
    A.part = part;
    A.sync = sync;
    A.ctrl = ctrl;
    A.tol = tol;
    A.max_iter = max_iter;
    A.cache = per * (block / kWave);
    void *args[] = {&A};
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(block), args, dyn, s);
}

}  // namespace sc

using namespace sc;

extern "C" size_t sc_matrix_bytes(int32_t count, int64_t nnz) {
    return matrix_bytes(count, nnz);
}

extern "C" int sc_assemble_matrix(const sc_particles *p, sc_contacts *c, void *stream) {
    if (!p || !c || p->n < 0 || c->count < 0 || c->count > c->capacity) return SC_ERR_INVALID;
    c->mat_ready = 0;
    Plan pl;
    if (!carve_plan(c->plan, c->plan_bytes, p->n, c->capacity, pl)) return SC_ERR_INVALID;
    MatBufs mb;
    if (!carve_matrix(c->mat, c->mat_bytes, c->count, c->nnz, mb)) return SC_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nc = c->count;
    if (nc > 0) {
        const ChainView C = chain_view(p, c, pl, nullptr);
        const int per = kBlock / kWave;  // slices per workgroup
        k_row_lengths<<<grid_for(nc), kBlock, 0, s>>>(C, mb.len);
        k_slice_sums<<<(mb.ns + per - 1) / per, kBlock, 0, s>>>(nc, mb.ns, mb.len, mb.soff,
                                                              mb.swid);
        scan_exclusive(mb.soff, mb.soff, mb.ns, mb.scan_tmp, s);
        k_assemble<<<(mb.ns + per - 1) / per, kBlock, 0, s>>>(C, mb.ns, mb.len, mb.soff, mb.swid,
                                                            mb.col, mb.val);
    } else {
        SC_HIP_TRY(hipMemsetAsync(mb.soff, 0, sizeof(int32_t), s));
    }
    SC_HIP_TRY(hipStreamSynchronize(s));
    SC_HIP_TRY(hipGetLastError());
    c->mat_ready = 1;
    return SC_OK;
}
