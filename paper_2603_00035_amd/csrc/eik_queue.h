// eik_queue.h -- device work queue shared by the queue-scheduled kernels.
//
// A queue of tile indices in a ring of slots (workspace memory). A tile is
// never visited by two waves at once: its state goes idle -> queued ->
// running -> idle, and a tile flagged while running is marked and queued
// again when its visit ends. `pending` counts the tiles queued or running; a
// wave waiting for work leaves when it drops to zero (then nothing can be
// flagged any more), when the visit budget is spent, or when a wait exceeds
// its poll limit (reported as a failure). All queue operations are done by
// lane 0 of a wave.
#pragma once

#include "eik_internal.h"

namespace eik {

__device__ __forceinline__ uint32_t q_load(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Append tile u. The ring holds more slots than tiles plus waves, so a slot is
// normally empty when its ticket comes round again; the compare-and-swap makes
// that a checked fact (a full slot is waited for, with the same bound).
__device__ __forceinline__ void q_put(const WorkQueue &q, int u)
{
    const uint32_t pos = atomicAdd(&q.ctl[kQTail], 1u);
    for (uint32_t spins = 0; atomicCAS(&q.ring[pos & q.mask], 0u, (uint32_t)(u + 1)) != 0u; ++spins) {
        if (q_load(&q.ctl[kQStop])) return;
        if (spins >= q.spin_limit) {
            atomicExch(&q.ctl[kQFail], 1u);
            atomicExch(&q.ctl[kQStop], 1u);
            return;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

// Flag tile u (lane 0 only).
__device__ __forceinline__ void q_flag(const WorkQueue &q, int u)
{
    for (int tries = 0; tries < 64; ++tries) {
        const uint32_t s = atomicCAS(&q.state[u], kTileIdle, kTileQueued);
        if (s == kTileIdle) {
            atomicAdd(&q.ctl[kQPending], 1u);
            q_put(q, u);
            return;
        }
        if (s == kTileQueued || s == kTileAgain) return;
        const uint32_t r = atomicCAS(&q.state[u], kTileRunning, kTileAgain);
        if (r == kTileRunning || r == kTileAgain || r == kTileQueued) return;
        // the visit ended in between (state idle again): retry
    }
    atomicExch(&q.ctl[kQFail], 1u);
    atomicExch(&q.ctl[kQStop], 1u);
}

// End of a visit of tile t (lane 0 only): queue it again if it did not settle
// or was flagged meanwhile, else mark it idle.
__device__ __forceinline__ void q_done(const WorkQueue &q, int t, bool settled)
{
    if (settled && atomicCAS(&q.state[t], kTileRunning, kTileIdle) == kTileRunning) {
        atomicSub(&q.ctl[kQPending], 1u);
        return;
    }
    atomicExch(&q.state[t], kTileQueued); // still counted as pending
    q_put(q, t);
}

// Next tile for this wave (lane 0 only), or -1 to leave.
__device__ __forceinline__ int q_take(const WorkQueue &q)
{
    if (q_load(&q.ctl[kQStop])) return -1;
    const uint32_t pos = atomicAdd(&q.ctl[kQHead], 1u);
    uint32_t *slot = &q.ring[pos & q.mask];
    for (uint32_t spins = 0;; ++spins) {
        const uint32_t v = q_load(slot);
        if (v) {
            __hip_atomic_store(slot, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicExch(&q.state[v - 1], kTileRunning);
            if ((int32_t)atomicSub(&q.ctl[kQBudget], 1u) <= 0) { // visit budget spent
                atomicExch(&q.ctl[kQStop], 1u);
                return -1;
            }
            atomicAdd(&q.ctl[kQVisits], 1u);
            return (int)v - 1;
        }
        if (q_load(&q.ctl[kQPending]) == 0 || q_load(&q.ctl[kQStop])) return -1;
        if (spins >= q.spin_limit) {
            atomicExch(&q.ctl[kQFail], 1u);
            atomicExch(&q.ctl[kQStop], 1u);
            return -1;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

} // namespace eik
