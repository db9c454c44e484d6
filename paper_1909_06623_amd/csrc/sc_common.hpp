// sc_common.hpp -- device helpers and host plumbing shared by the library's
// HIP translation units (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sc_api.h"

namespace sc {

constexpr int kBlock = 256;            // threads per workgroup (4 waves)
constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kMaxReduceBlocks = 1024; // partial-sum slots of grid reductions
constexpr int kPartHalf = 4 * kMaxReduceBlocks;  // doubles per half of the partials buffer

// ------------------------------------------------------------------ host

#define SC_HIP_TRY(expr)                                                    \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess) return SC_ERR_HIP;                            \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over the caller's workspace (no device allocation).
struct Carver {
    char *base;
    size_t size;
    size_t used = 0;
    bool ok = true;
    template <class T>
    T *take(size_t count) {
        size_t off = align_up(used, 256);
        size_t bytes = align_up(count * sizeof(T), 256);
        if (off + bytes > size) {
            ok = false;
            return nullptr;
        }
        used = off + bytes;
        return reinterpret_cast<T *>(base + off);
    }
};

inline int grid_for(long long n, int block = kBlock) {
    long long g = (n + block - 1) / block;
    return g < 1 ? 1 : static_cast<int>(g);
}

// Workspace sizing, one place: every entry point carves from the front.
size_t contacts_ws_bytes(int32_t n, int32_t cap);
size_t solve_ws_bytes(int32_t n, int32_t cap);
size_t adjoint_ws_bytes(int32_t n, int32_t cap);
size_t cell_budget(int32_t n);

// Host resources a thread keeps between calls (sc_release frees them): the
// solve's timing events (sc_solve.hip) and the general-mobility solves'
// pinned control-block slots (sc_mobsolve.hip).
void release_solve_host();
// The calling thread's two timing events (created on first use, destroyed by
// sc_release); false if they cannot be created.
bool thread_events(hipEvent_t *t0, hipEvent_t *t1);
void release_mob_host();

// sc_solve_lcp on a given workspace (defined in sc_solve.hip); `timed`
// records HIP events around the persistent kernel (st->kernel_ms), else no
// event is created and kernel_ms is 0.
int solve_lcp_on(const sc_particles *p, const sc_contacts *c, const sc_solve_opts *opts,
                 double *gamma, double *g, double *f_c, double *u_c, sc_stats *st, void *ws,
                 size_t ws_bytes, void *stream, bool timed);
// sc_solve_lcp's argument checks without the workspace (no device call):
// SC_OK or SC_ERR_INVALID.
int check_solve_args(const sc_particles *p, const sc_contacts *c, const sc_solve_opts *opts,
                     const double *gamma, const double *g, const sc_stats *st);

// Device-wide exclusive scan of n int32 values: out[k] = sum_{m<k} in[m] and
// out[n] = total. `tmp` needs scan_tmp_ints(n) ints. in may equal out.
int scan_tmp_ints(int n);
void scan_exclusive(const int *in, int *out, int n, int *tmp,
                    hipStream_t stream);

// ------------------------------------------------------------------ device

struct V3 {
    double x, y, z;
};

// Global-memory view of a generic pointer into device memory. Where the
// compiler cannot prove a pointer's address space (a pointer picked from a
// dynamically indexed array, a select between buffers) it emits flat
// accesses, and a flat access also counts against the LDS counter: every
// wait for an LDS read would then wait for the outstanding gathers and
// stores too. Accesses through this view are global loads and stores.
// (Records are read member by member: a class object cannot be copied out
// of another address space.)
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p) {
    return (__attribute__((address_space(1))) T *)(reinterpret_cast<uintptr_t>(p));
}
template <class T>
__device__ __forceinline__ T ld_global(const T *p) {
    return *gmem(p);
}

__device__ __forceinline__ V3 v3(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ V3 load3(const double *p) { return {p[0], p[1], p[2]}; }
__device__ __forceinline__ void store3(double *p, V3 a) {
    p[0] = a.x; p[1] = a.y; p[2] = a.z;
}
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Column-major SoA frame access: frame[row * cap + l].
__device__ __forceinline__ V3 frame3(const double *frame, long long cap, int row, long long l) {
    return {frame[(row + 0) * cap + l], frame[(row + 1) * cap + l], frame[(row + 2) * cap + l]};
}

// Dry mobility block: U = a_perp F + (a_par - a_perp)(p.F) p, same for W.
__device__ __forceinline__ void mobility_apply(V3 p, const double *m, V3 f, V3 t,
                                               V3 &u, V3 &w) {
    double a_par = m[0], a_perp = m[1], b_par = m[2], b_perp = m[3];
    u = a_perp * f + ((a_par - a_perp) * dot(p, f)) * p;
    w = b_perp * t + ((b_par - b_perp) * dot(p, t)) * p;
}

// Wave-level sum in a fixed butterfly order (deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

// Block-level sum of NV values; result valid in thread 0. Fixed order.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[kBlock / kWave]) {
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k][wid] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < kBlock / kWave; ++w) s += lds[k][w];
            v[k] = s;
        }
    }
}

}  // namespace sc
