// Device side of the work-queue traversals: the blocked 4-state schedule
// (queue_bmf_kernel, phg_kernels.hip) and the level schedule of the
// vector-ALU kernels (phg_kernels_vs.hip).  Work items run in one launch per
// pass; an item waits on completion marks of the items whose outputs it
// reads, so outputs that cross items are written and read with the
// device-scope coherence bit: MI355X's 8 XCDs each have their own L2, and an
// ordinary load can return a line another XCD has since rewritten.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "phg_internal.h"

namespace phg {
namespace queue {

#define PHG_AS1 __attribute__((address_space(1)))

// A generic pointer taken in the global address space.
template <typename T>
__device__ __forceinline__ PHG_AS1 T* as1(T* p) {
    return (PHG_AS1 T*)p;
}

constexpr int kScDevice = 16;                // buffer cache policy: sc1 (device scope)
constexpr int kRsrcFlags = 0x00020000;       // buffer descriptor word 3 (raw 32-bit data)

// Device-coherent load / store of base[idx] (T of 4, 8 or 16 bytes) through a
// buffer descriptor over base[0, count); base is wave-uniform.
template <typename T>
__device__ __forceinline__ T ld(const PHG_AS1 T* base, uint32_t idx, uint32_t count) {
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<PHG_AS1 T*>(base), 0,
                                                      static_cast<int>(count * sizeof(T)), kRsrcFlags);
    const uint32_t off = idx * static_cast<uint32_t>(sizeof(T));
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, kScDevice));
    } else if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, kScDevice));
    } else {
        static_assert(sizeof(T) == 16, "4-, 8- or 16-byte elements");
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kScDevice));
    }
}
template <typename T>
__device__ __forceinline__ void st(PHG_AS1 T* base, uint32_t idx, uint32_t count, T v) {
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(base, 0, static_cast<int>(count * sizeof(T)), kRsrcFlags);
    const uint32_t off = idx * static_cast<uint32_t>(sizeof(T));
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, off, 0, kScDevice);
    } else if constexpr (sizeof(T) == 8) {
        typedef unsigned int U2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), rs, off, 0, kScDevice);
    } else {
        static_assert(sizeof(T) == 16, "4-, 8- or 16-byte elements");
        typedef unsigned int U4 __attribute__((ext_vector_type(4)));
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, v), rs, off, 0, kScDevice);
    }
}

// The evaluation's epoch: advanced by its P(t) launch, constant during the
// traversal launches, so an ordinary (scalar) load.
__device__ __forceinline__ uint32_t epoch(const QueueArgs& q) {
    return as1(q.ctr)[kQueueEpoch];
}

// Start of an evaluation (one thread of its P(t) launch): a new epoch for the
// marks, no fault yet.
__device__ __forceinline__ void new_evaluation(uint32_t* ctr) {
    __hip_atomic_fetch_add(&ctr[kQueueEpoch], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_exchange(&ctr[kQueueFault], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wave: each lane polls mark m (m < 0: none) until every mark equals
// target.  Bounded: past q.wait_ticks of the constant clock the wave sets the
// fault word and returns; once that word is set every waiting wave returns at
// its next poll (lane 63 watches it).  The caller synchronises its workgroup
// afterwards.
__device__ __forceinline__ void wait_marks(const QueueArgs& q, int m, uint32_t target, uint32_t n_marks, int lane) {
    const PHG_AS1 uint32_t* done = as1(q.done);
    const PHG_AS1 uint32_t* ctr = as1(q.ctr);
    const uint64_t t_start = wall_clock64();
    for (;;) {
        const bool ok = m < 0 || ld(done, static_cast<uint32_t>(m), n_marks) == target;
        const bool quit = lane == 63 && ld(ctr, kQueueFault, kQueueWords) != 0u;
        if (__builtin_amdgcn_ballot_w64(!ok) == 0 || __builtin_amdgcn_ballot_w64(quit) != 0) return;
        if (static_cast<uint64_t>(wall_clock64()) - t_start > q.wait_ticks) {
            if (lane == 0) st(as1(q.ctr), kQueueFault, kQueueWords, 1u);
            return;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// This wave's stores have completed at device scope (vmcnt(0)); every wave
// of the item runs it, then the workgroup synchronises and one thread sets
// the item's mark.
__device__ __forceinline__ void stores_complete() { __builtin_amdgcn_s_waitcnt(0x0F70); }
__device__ __forceinline__ void set_mark(const QueueArgs& q, uint32_t idx, uint32_t target, uint32_t n_marks) {
    st(as1(q.done), idx, n_marks, target);
}

#undef PHG_AS1

}  // namespace queue
}  // namespace phg
