// sc_matrix.hpp -- the assembled M = D^T Mob D (one row per contact) and the
// launchers of the persistent solvers that use it.
#pragma once

#include "sc_chain.hpp"
#include "sc_common.hpp"
#include "sc_sync.hpp"

namespace sc {

// Rows are grouped in slices of kWave consecutive rows; a slice stores its
// entries depth by depth, each depth packed over the rows that reach it.
struct MatView {
    int nc, ns;           // rows, slices
    const int32_t *len;   // [nc] entries per row (the diagonal is entry 0)
    const int32_t *soff;  // [ns+1] first entry of each slice; soff[ns] = nnz
    const int32_t *swid;  // [ns] longest row of each slice
    const int32_t *col;   // [nnz] contact index of each entry
    const double *val;    // [nnz]
};

struct MatBufs {
    int ns;
    int32_t *len, *soff, *swid, *col;
    double *val;
    int32_t *scan_tmp;
};

inline int slices(int32_t nc) { return (nc + kWave - 1) / kWave; }

size_t matrix_bytes(int32_t nc, int64_t nnz);
bool carve_matrix(void *base, size_t bytes, int32_t nc, int64_t nnz, MatBufs &m);
MatView mat_view(int32_t nc, const MatBufs &m);

// BBPGD on the assembled matrix: one persistent launch. gamma holds gamma_0
// on entry and the last iterate on exit, g receives M gamma + q; zbuf is
// scratch of 4 nc doubles; spw = slices each wave works on at once (1, 2 or
// 4); cache = LDS entries of M per wave (0 = as many as fit, < 0 = none).
// Returns the launch's HIP error code; the grid and cache actually used are
// stored.
hipError_t launch_bbpgd_mat(const MatView &M, const double *q, double *gamma, double *g,
                            double *zbuf, double *part, GridSync *sync, SolveCtrl *ctrl,
                            double tol, int max_iter, int bb, int spw, int cache, int block,
                            int grid, hipStream_t s, int *grid_used, int *cache_used);

// Masked CG (Chronopoulos-Gear) on M_AA with A = {gamma > 0}. zbuf holds 8 nc
// doubles: records (r, w, s, pad) of buffer 0 carry the masked right-hand side
// in r and zeros elsewhere on entry; p and x are zero on entry and x receives
// the solution.
hipError_t launch_cg_mat(const MatView &M, const double *gamma, double *zbuf, double *p,
                         double *x, double *part, GridSync *sync, CgCtrl *ctrl, double tol,
                         int max_iter, int spw, int cache, int block, int grid, hipStream_t s,
                         int *grid_used, int *cache_used);

}  // namespace sc
