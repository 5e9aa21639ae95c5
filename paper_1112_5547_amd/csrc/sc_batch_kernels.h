// sc_batch_kernels.h -- the batch kernels: one launch per step over the
// work items (member, tile, march chunk) of many lattices, and one persistent
// launch per epoch with a grid barrier between steps, templated on the policy
// and the block shape.  Instantiated per policy next to the step kernels
// (sc_step_<policy>.hip); the batch engine reaches them through
// batch_fns<P>.
#pragma once

#include "sc_steps.h"

namespace sc {

// ---------------------------------------------------------------------------
// Batched forms: one launch per step over the work items of many lattices,
// or one persistent launch per epoch with a grid barrier between steps.
// ---------------------------------------------------------------------------

template <class PR, int NT, int TX19, int TY19>
struct BatchTiles {
    using T9 = TileStep<9, PR, NT, 1>;
    using T19 = TileStep<19, PR, TX19, TY19>;
    static_assert(TX19 * TY19 == NT, "both lattice types use the block size");
    static constexpr int LDS_ELEMS =
        T9::LDS_ELEMS > T19::LDS_ELEMS ? T9::LDS_ELEMS : T19::LDS_ELEMS;
    __device__ static __forceinline__ void run(const BatchDesc& d, const WorkItem& w, int k,
                               typename PR::A* lds) {
        const int parity = d.base_parity ^ (k & 1);
        if (d.Q == 9)
            T9::run(d.sp[parity], w.tile_x, w.tile_y, w.chunk, lds);
        else
            T19::run(d.sp[parity], w.tile_x, w.tile_y, w.chunk, lds);
    }
};

template <class PR>
struct BatchWaves {
    static constexpr int value = PR::shifted ? 3 : 2;
};

template <class PR, int NT, int TX19, int TY19>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(BatchWaves<PR>::value)))
k_batch_step(const BatchDesc* __restrict__ desc, const WorkItem* __restrict__ work, int nwork,
             int k) {
    using BT = BatchTiles<PR, NT, TX19, TY19>;
    __shared__ typename PR::A lds[BT::LDS_ELEMS];
    const int it = (int)blockIdx.x;
    if (it >= nwork) return;
    const WorkItem w = work[it];
    const BatchDesc& d = desc[w.member];
    if (k >= d.steps) return;
    BT::run(d, w, k, lds);
}

__device__ __forceinline__ unsigned ld_acquire(unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier for co-resident blocks; returns false if the wait hit
// the spin limit or another block already reported a timeout (all blocks
// then leave the kernel, so every wave terminates).  Arrival is two-level:
// a block counts in at its group's counter, the last of a group at the
// top-level counter, and the last group's last block opens the next
// generation.  Every wave first waits for its own global stores to complete
// at the L2; one agent-scope release by the arriving thread then writes the
// L2 (shared by the CUs of the XCD) back for the whole block, and one
// agent-scope acquire after the wait invalidates the caches the block reads
// through.
__device__ inline bool grid_barrier(unsigned* sync, unsigned nblocks, unsigned& gen, int* s_flag,
                                    unsigned spin_limit) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        int ok = 1;
        const unsigned g = gen;
        const unsigned grp = blockIdx.x / kBarrierGroup;
        const unsigned ngrp = (nblocks + kBarrierGroup - 1) / kBarrierGroup;
        const unsigned gsize = min((unsigned)kBarrierGroup, nblocks - grp * kBarrierGroup);
        unsigned* gc = &sync[SYNC_GRP + grp * kSyncLine];
        bool opened = false;
        if (__hip_atomic_fetch_add(gc, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
            gsize - 1) {
            // no block of the group arrives again before the generation moves
            __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(&sync[SYNC_COUNT], 1u, __ATOMIC_ACQ_REL,
                                       __HIP_MEMORY_SCOPE_AGENT) == ngrp - 1) {
                __hip_atomic_store(&sync[SYNC_COUNT], 0u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&sync[SYNC_GEN], g + 1, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
                opened = true;
            }
        }
        if (!opened) {
            unsigned spins = 0;
            while (ld_acquire(&sync[SYNC_GEN]) == g) {
                if (ld_acquire(&sync[SYNC_TIMEOUT]) != 0u || ++spins > spin_limit) {
                    __hip_atomic_store(&sync[SYNC_TIMEOUT], 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        gen = g + 1;
        *s_flag = ok;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return *s_flag != 0;
}

template <class PR, int NT, int TX19, int TY19>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(BatchWaves<PR>::value)))
k_batch_persistent(const BatchDesc* __restrict__ desc, const WorkItem* __restrict__ work,
                   int nwork, int ksteps, unsigned* sync, unsigned spin_limit) {
    using BT = BatchTiles<PR, NT, TX19, TY19>;
    __shared__ typename PR::A lds[BT::LDS_ELEMS];
    __shared__ int s_item;
    __shared__ int s_flag;
    unsigned gen = 0;
    for (int k = 0; k < ksteps; ++k) {
        unsigned* ctr = &sync[SYNC_CTR + k];
        if (threadIdx.x == 0)
            s_item = (int)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        int it = s_item;
        while (it < nwork) {
            // the next claim is in flight while this item runs
            int next = 0;
            if (threadIdx.x == 0)
                next = (int)__hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            const WorkItem w = work[it];
            const BatchDesc& d = desc[w.member];
            if (k < d.steps) BT::run(d, w, k, lds);
            // every wave is done with this item's LDS ring and has read s_item
            __syncthreads();
            if (threadIdx.x == 0) s_item = next;
            __syncthreads();
            it = s_item;
        }
        if (k + 1 < ksteps && !grid_barrier(sync, gridDim.x, gen, &s_flag, spin_limit)) return;
    }
}

template <class PR>
bool batch_fns(int nt, int tx19, int ty19, BatchStepFn* sf, BatchPersFn* pf) {
#define SC_CFG(NT_, X_, Y_)                                          \
    if (nt == NT_ && tx19 == X_ && ty19 == Y_) {                     \
        *sf = k_batch_step<PR, NT_, X_, Y_>;                         \
        *pf = k_batch_persistent<PR, NT_, X_, Y_>;                   \
        return true;                                                 \
    }
    SC_CFG(256, 64, 4)
    SC_CFG(256, 32, 8)
    SC_CFG(256, 16, 16)
    SC_CFG(128, 32, 4)
    SC_CFG(512, 64, 8)
    SC_CFG(512, 32, 16)
#undef SC_CFG
    return false;
}

#define SC_DECLARE_BATCH(P) extern template bool batch_fns<P>(int, int, int, BatchStepFn*, BatchPersFn*);
SC_POLICIES(SC_DECLARE_BATCH)
#undef SC_DECLARE_BATCH

}  // namespace sc
