// sc_scan.hip -- device-wide exclusive prefix sum of int32 counts, used to
// turn per-cell and per-particle counts into CSR offsets. Three passes:
// per-tile totals, one workgroup scanning the tile totals, per-tile rescan.
#include "sc_common.hpp"

namespace sc {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kPerThread = 4;
constexpr int kTile = kScanThreads * kPerThread;

// Inclusive wave scan (Hillis-Steele over 64 lanes).
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        int t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over the workgroup; returns the
// thread's exclusive prefix and writes the workgroup total to *total.
__device__ int block_excl_scan(int v, int *total) {
    __shared__ int wsum[kScanThreads / kWave + 1];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    int incl = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        int t = lane < kScanThreads / kWave ? wsum[lane] : 0;
        int ti = wave_incl_scan(t);
        if (lane < kScanThreads / kWave) wsum[lane] = ti - t;  // exclusive
        if (lane == kScanThreads / kWave - 1) wsum[kScanThreads / kWave] = ti;
    }
    __syncthreads();
    int res = wsum[wid] + incl - v;
    if (total) *total = wsum[kScanThreads / kWave];
    __syncthreads();
    return res;
}

__global__ void __launch_bounds__(kScanThreads)
tile_totals(const int *in, int n, int *tile_sum) {
    const long long base = static_cast<long long>(blockIdx.x) * kTile;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        long long idx = base + static_cast<long long>(k) * kScanThreads + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    int total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of ntiles totals in place; writes the grand
// total to *grand.
__global__ void __launch_bounds__(kScanThreads)
scan_tiles(int *tile_sum, int ntiles, int *grand) {
    int carry = 0;
    for (int base = 0; base < ntiles; base += kScanThreads) {
        int idx = base + threadIdx.x;
        int v = idx < ntiles ? tile_sum[idx] : 0;
        int total;
        int ex = block_excl_scan(v, &total);
        if (idx < ntiles) tile_sum[idx] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) *grand = carry;
}

__global__ void __launch_bounds__(kScanThreads)
tile_rescan(const int *in, int *out, int n, const int *tile_off) {
    // Each thread owns kPerThread consecutive items so that the output order
    // is a plain left-to-right prefix.
    const long long base = static_cast<long long>(blockIdx.x) * kTile
                           + static_cast<long long>(threadIdx.x) * kPerThread;
    int v[kPerThread];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        long long idx = base + k;
        v[k] = idx < n ? in[idx] : 0;
        s += v[k];
    }
    int ex = block_excl_scan(s, nullptr) + tile_off[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
        long long idx = base + k;
        if (idx < n) out[idx] = ex;
        ex += v[k];
    }
}

}  // namespace

int scan_tmp_ints(int n) { return (n + kTile - 1) / kTile + 1; }

void scan_exclusive(const int *in, int *out, int n, int *tmp, hipStream_t stream) {
    int ntiles = (n + kTile - 1) / kTile;
    if (ntiles == 0) {
        (void)hipMemsetAsync(out, 0, sizeof(int), stream);
        return;
    }
    // tile_totals reads items in strided order; the sum per tile is the same.
    tile_totals<<<ntiles, kScanThreads, 0, stream>>>(in, n, tmp);
    scan_tiles<<<1, kScanThreads, 0, stream>>>(tmp, ntiles, out + n);
    tile_rescan<<<ntiles, kScanThreads, 0, stream>>>(in, out, n, tmp);
}

}  // namespace sc
