// sc_batch_build.hpp -- close pairs, contact frames, q, incidence lists and
// the assembled M of every suspension of a batch, in one sequence of
// launches with no host synchronisation (so that it can be captured in a HIP
// graph together with the solves).
//
// The suspensions share one index space of particles/ranks (suspension k
// owns [pbase_k, pbase_k + n_k)), one of search cells, one of contact slots
// (its capacity) and one of matrix slices (ceil(capacity / 64)); each writes
// its outputs, with local indices, into its own buffers. Sizes that depend
// on the positions (contacts, slices, nonzeros) stay on the device.
#pragma once

#include <vector>

#include "sc_build_dev.hpp"
#include "sc_common.hpp"
#include "sc_matrix.hpp"
#include "sc_plan.hpp"

namespace sc {

// One suspension: inputs, search grid (fixed when the batch is planned),
// outputs and its offsets in the shared index spaces.
struct BuildInst {
    Parts P;
    Grid g;
    double ext;             // largest R + h the grid was sized for
    const double *u_nc;
    double dt;
    Plan pl;                // carved for (n, capacity)
    int32_t *ci, *cj;
    double *phi, *q, *frame;
    MatBufs mb;             // carved for (capacity, nnz capacity)
    int cap;
    long long nnz_cap;
    int pbase, cbase, ncell, lbase, sbase;
};

// Written by the build, per suspension.
struct BuildOut {
    int status;             // SC_OK, SC_ERR_NONFINITE, SC_ERR_BOX or SC_ERR_CAPACITY
    int nc, ns;             // contacts, slices of M
    int flags[kFlagCount];
    long long nnz;
};

struct BatchBuild {
    int count = 0;
    int N = 0, C = 0, L = 0, S = 0;   // particles, cells, contact slots, slice slots
    BuildInst *inst = nullptr;        // [count]
    BuildOut *out = nullptr;          // [count]
    int *pbase = nullptr, *lbase = nullptr, *sbase = nullptr;  // [count + 1] each
    int *cell_of = nullptr, *members = nullptr, *cell_r = nullptr, *deg = nullptr,
        *fill = nullptr, *lane_cnt = nullptr, *slots = nullptr, *cell_start = nullptr,
        *cell_fill = nullptr, *scan_tmp = nullptr;
    double *prec = nullptr, *hl = nullptr;
    unsigned long long *ext_bits = nullptr;  // [count], used when planning
};

// Device bytes of the build's tables and shared scratch for these suspensions
// (each item: particles p, contacts c with c.capacity rows and c.nnz the
// nonzero capacity of c.mat).
size_t batch_build_bytes(int32_t count, const sc_batch_item *items);

// Carves the tables and scratch, measures each suspension's particle extent
// (one synchronisation), fixes the search grids and uploads the tables.
// Returns SC_OK, SC_ERR_INVALID (a buffer too small or missing),
// SC_ERR_NONFINITE (bad particle data), SC_ERR_BOX or SC_ERR_HIP.
int batch_build_plan(int32_t count, const sc_batch_item *items, Carver &cv, hipStream_t s,
                     BatchBuild &b, std::vector<BuildInst> &host);

// Enqueues the build of every suspension (no synchronisation, no memset).
int batch_build_enqueue(const BatchBuild &b, hipStream_t s);

}  // namespace sc
