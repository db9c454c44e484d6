// sc_sync.hpp -- grid-wide barrier for persistent (cooperative) kernels on
// multi-XCD CDNA parts.
//
// Each XCD has its own L2; making one workgroup's stores visible to another
// XCD takes an L2 write-back there and an invalidate on the reader's side.
// A write-back in every workgroup costs ~25 ns per workgroup (serialised in
// the L2), so the release half works per XCD: every workgroup waits for its
// own stores to reach L2 and bumps its XCD's counter; the last arrival on an
// XCD writes back that L2 once and then bumps a top counter; the last of
// those publishes the new generation, which every workgroup polls (all
// XCDs' data is in memory by then). The acquire half (an agent-scope
// invalidate of L1 and L2) is done by every workgroup: measured on gfx950,
// a group-scope invalidate does not drop stale L1 lines of the other CUs. Workgroups are grouped by the hardware XCC_ID register, counted
// at kernel start. Counters only ever increase (the last
// arrival of generation g on a group of m members reads g*m - 1, modulo
// 2^32), so no reset has to be ordered against the next barrier.
//
// Every spin is bounded: on a timeout the barrier raises `err` and returns,
// and callers leave their loop, so the grid always drains.
#pragma once

#include "sc_common.hpp"

namespace sc {

constexpr int kMaxXcc = 16;

struct alignas(256) GridSync {
    unsigned xcnt[kMaxXcc][32];  // arrivals per XCD (one 128-byte line each)
    unsigned xmem[kMaxXcc][32];  // workgroups per XCD
    unsigned top[32];            // XCD arrivals
    unsigned gen[32];            // global generation
    unsigned init[32];           // start-up arrivals
    unsigned err[32];            // timeout flag
    unsigned limit[32];          // polls before a wait gives up (0: 2^21)
};

__device__ __forceinline__ unsigned xcc_id() {
    // HW_REG_XCC_ID (hwreg 20), bits [3:0]
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & (kMaxXcc - 1);
}

__device__ __forceinline__ unsigned ld_relaxed(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns false on timeout (the flag is raised for everybody).
__device__ __forceinline__ bool spin_until(unsigned *word, unsigned target, GridSync *s) {
    unsigned polls = 0;
    const unsigned lim = ld_relaxed(&s->limit[0]);
    const unsigned cap = lim ? lim : (1u << 21);
    while (ld_relaxed(word) != target) {
        if (++polls > cap) {
            __hip_atomic_fetch_or(&s->err[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if (ld_relaxed(&s->err[0])) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

struct GridBarrier {
    GridSync *s;
    unsigned xcc, members, nxcc, gen;

    // Collective start-up (all workgroups): count workgroups per XCD. The
    // sync block must be zeroed before the launch.
    __device__ void init(GridSync *sync) {
        __shared__ unsigned sh[3];
        s = sync;
        gen = 0;
        if (threadIdx.x == 0) {
            const unsigned x = xcc_id();
            __hip_atomic_fetch_add(&s->xmem[x][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&s->init[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            spin_until(&s->init[0], gridDim.x, s);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            unsigned nx = 0;
            for (int k = 0; k < kMaxXcc; ++k) nx += ld_relaxed(&s->xmem[k][0]) ? 1u : 0u;
            sh[0] = x;
            sh[1] = ld_relaxed(&s->xmem[x][0]);
            sh[2] = nx;
        }
        __syncthreads();
        xcc = sh[0];
        members = sh[1];
        nxcc = sh[2];
        __syncthreads();
    }

    // Full barrier with release/acquire semantics for all global memory.
    // Returns false if the grid timed out.
    __device__ bool sync() {
        __shared__ int ok;
        // every wave waits for its own stores to be acknowledged by L2, so
        // the XCD's single write-back below covers them
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const unsigned target = gen + 1;
        if (threadIdx.x == 0) {
            bool good = true;
            const unsigned a = __hip_atomic_fetch_add(&s->xcnt[xcc][0], 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            if (a == target * members - 1u) {
                // last on this XCD: publish its L2, meet the other XCDs
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                const unsigned t = __hip_atomic_fetch_add(&s->top[0], 1u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                if (t == target * nxcc - 1u) {
                    __hip_atomic_store(&s->gen[0], target, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    good = spin_until(&s->gen[0], target, s);
                }
            } else {
                good = spin_until(&s->gen[0], target, s);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            ok = good ? 1 : 0;
        }
        __syncthreads();
        gen = target;
        return ok != 0;
    }
};

// Returns false on timeout: waits until the monotonic counter has reached
// `target` (modulo 2^32; a member is never more than one barrier ahead).
__device__ __forceinline__ bool spin_reach(unsigned *word, unsigned target, unsigned *err) {
    unsigned polls = 0;
    while (static_cast<int>(ld_relaxed(word) - target) < 0) {
        if (++polls > (1u << 21)) {
            __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if (ld_relaxed(err)) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

// Barrier of a team of workgroups that share one XCD (and so one L2): each
// member waits for its stores to reach L2, bumps the team's counter and waits
// until every member has; the acquire invalidates the member's caches. No L2
// write-back is needed inside one XCD. A team of one is a workgroup barrier.
struct alignas(256) TeamSync {
    unsigned cnt[32];   // arrivals, monotonic
    unsigned item[32];  // work item handed to the team by its leader
};

struct TeamBarrier {
    TeamSync *s;
    unsigned *err;
    unsigned members, gen;

    __device__ bool sync() {
        __shared__ int ok;
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (members <= 1) return true;
        ++gen;
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(&s->cnt[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool good = spin_reach(&s->cnt[0], gen * members, err);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            ok = good ? 1 : 0;
        }
        __syncthreads();
        return ok != 0;
    }
};

}  // namespace sc
