// sc_chain_lds.hpp -- the static per-incidence data of pass A (sc_chain.hpp)
// held in LDS for the whole of a persistent solve on the matrix-free chain.
#pragma once

#include <algorithm>

#include "sc_chain.hpp"
#include "sc_common.hpp"
#include "sc_plan.hpp"

namespace sc {

extern __shared__ double sc_lds_dyn[];

// The chain's static per-incidence data in LDS. Pass A runs every product
// over the same incidences of the same ranks, so a workgroup copies their
// ranges, codes and signed D columns (52 bytes per incidence) once per solve
// and reads them from LDS; incidences past inc_cap are read from global
// memory. Only the (gamma, g) gather and the U store remain per product.
struct ChainLds {
    const int *ptr;  // inc_ptr of rank k at ptr[k - kb] (LDS, or global with kb = 0)
    double *dpm;     // [inc_cap][6]
    int *code;       // [inc_cap]
    int kb, e0, cap;
};

inline size_t chain_lds_bytes(int rank_cap, int inc_cap) {
    return align_up(4 * static_cast<size_t>(rank_cap), 8) + 52 * static_cast<size_t>(inc_cap);
}

__device__ __forceinline__ ChainLds chain_lds_fill(const ChainView &C, int rank_cap, int inc_cap,
                                                   int k0, int k1) {
    ChainLds L;
    int *ptr = reinterpret_cast<int *>(sc_lds_dyn);
    L.dpm = reinterpret_cast<double *>(sc_lds_dyn) + (rank_cap + 1) / 2;
    L.code = reinterpret_cast<int *>(L.dpm + 6 * static_cast<long long>(inc_cap));
    L.e0 = C.inc_ptr[k0];
    const int ne = min(C.inc_ptr[k1] - L.e0, inc_cap);
    L.cap = ne;
    if (rank_cap > 0) {
        for (int k = k0 + static_cast<int>(threadIdx.x); k <= k1; k += blockDim.x)
            ptr[k - k0] = C.inc_ptr[k];
        L.ptr = ptr;
        L.kb = k0;
    } else {  // the ranges do not fit: read them from global memory
        L.ptr = C.inc_ptr;
        L.kb = 0;
    }
    for (int i = threadIdx.x; i < ne; i += blockDim.x) {
        L.code[i] = C.inc[L.e0 + i];
        const double *d = C.dpm + 6 * static_cast<long long>(L.e0 + i);
#pragma unroll
        for (int a = 0; a < 6; ++a) L.dpm[6 * i + a] = d[a];
    }
    __syncthreads();
    return L;
}

// pass_a (sc_chain.hpp) on the LDS copy.
template <int LPP, int BS, class W>
__device__ __forceinline__ void pass_a_lds(const ChainView &C, const ChainLds &L, int k0, int k1,
                                           W weight) {
    constexpr int PER = BS / LPP;
    const int sub = threadIdx.x / LPP, lane = threadIdx.x % LPP;
    for (int base = k0; base < k1; base += PER) {
        const int k = base + sub;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, a5 = 0.0;
        if (k < k1) {
            const int e1 = L.ptr[k - L.kb + 1];
            for (int e = L.ptr[k - L.kb] + lane; e < e1; e += LPP) {
                const int i = e - L.e0;
                const bool in = i < L.cap;
                const double *d = in ? L.dpm + 6 * i : C.dpm + 6 * static_cast<long long>(e);
                const double w = weight(in ? L.code[i] : C.inc[e], e);
                a0 += w * d[0];
                a1 += w * d[1];
                a2 += w * d[2];
                a3 += w * d[3];
                a4 += w * d[4];
                a5 += w * d[5];
            }
        }
#pragma unroll
        for (int off = LPP / 2; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off, kWave);
            a1 += __shfl_xor(a1, off, kWave);
            a2 += __shfl_xor(a2, off, kWave);
            a3 += __shfl_xor(a3, off, kWave);
            a4 += __shfl_xor(a4, off, kWave);
            a5 += __shfl_xor(a5, off, kWave);
        }
        if (k < k1 && lane == 0) {
            V3 u, w;
            plan_mobility(C.pdat + 8 * static_cast<long long>(k), v3(a0, a1, a2), v3(a3, a4, a5),
                          u, w);
            double *Uk = C.U + 8 * static_cast<long long>(k);
            Uk[0] = u.x; Uk[1] = u.y; Uk[2] = u.z;
            Uk[3] = w.x; Uk[4] = w.y; Uk[5] = w.z;
        }
    }
}

// Dynamic LDS a persistent chain kernel asks for: all of kChainLdsBytes
// unless the copy is turned off (lds_entries_per_wave = -1).
constexpr size_t kChainLdsBytes = 144 * 1024;
inline size_t chain_lds_dyn(int req) { return req < 0 ? 0 : kChainLdsBytes; }

// The copy for n ranks and nc contacts on G workgroups of `block` threads
// within `dyn` bytes: the ranges of ceil(n / G) + 1 ranks if they fit (else
// they are read from global memory), then as many incidences as fit, at most
// req per wave if req > 0.
struct ChainLdsPlan {
    int rank_cap, inc_cap, per_wave;
};

inline ChainLdsPlan chain_lds_plan(long long n, long long nc, int G, int block, int req,
                                   size_t dyn) {
    ChainLdsPlan P{};
    const long long waves = block / kWave;
    const long long rank_cap = (n + G - 1) / G + 1;
    P.rank_cap =
        req >= 0 && chain_lds_bytes(static_cast<int>(std::min(rank_cap, 1LL << 30)), 0) <= dyn
            ? static_cast<int>(rank_cap)
            : 0;
    long long room =
        (static_cast<long long>(dyn) - static_cast<long long>(chain_lds_bytes(P.rank_cap, 0))) /
        52;
    if (req > 0) room = std::min(room, req * waves);
    P.inc_cap = static_cast<int>(std::max(0LL, std::min(room, 2LL * nc)));
    P.per_wave = static_cast<int>(P.inc_cap / waves);
    return P;
}

}  // namespace sc
