// Device-side candidate pool: a concurrent hash set of int8 keys with full
// key comparison.  Table entries are 64-bit: 0 = empty; otherwise the high
// word is a 31-bit hash tag with bit 31 set and the low word is the key
// index, 0xFFFFFFFF while the inserting lane is still writing the key, and
// 0xFFFFFFFE when the pool ran out of key storage (the call then fails).
// Every lane runs its own bounded probe loop; a lane that wins an empty
// slot finishes the insert in the same loop iteration, so lanes of one
// wave never wait on each other.  The lanes of a wave that win a slot in
// the same iteration take consecutive key indices from one counter update
// (a single atomic per wave instead of one per new key).
#pragma once

#include <hip/hip_runtime.h>

#include "graver_internal.h"

namespace graver {

constexpr uint32_t kIdxBusy = 0xFFFFFFFFu;
constexpr uint32_t kIdxDead = 0xFFFFFFFEu;
constexpr int kMaxProbeIters = 1 << 22;

__device__ __forceinline__ uint64_t hash_mix(uint64_t h, uint64_t w) {
  h ^= w;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  return h;
}
__device__ __forceinline__ uint64_t hash_final(uint64_t h) {
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  return h;
}

// Hash of a key row held as 64-bit words (stride/8 words, zero padded).
__device__ __forceinline__ uint64_t hash_key_words(const uint64_t* w, int nwords) {
  uint64_t h = 0x9E3779B97F4A7C15ull;
  int i = 0;
  for (; i + 4 <= nwords; i += 4) {  // four independent loads in flight
    uint64_t a = w[i], b = w[i + 1], c = w[i + 2], d = w[i + 3];
    h = hash_mix(hash_mix(hash_mix(hash_mix(h, a), b), c), d);
  }
  for (; i < nwords; ++i) h = hash_mix(h, w[i]);
  return hash_final(h);
}

__device__ __forceinline__ uint64_t ld_acquire(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Insert the key (stride bytes at `key`, 8-byte aligned, any address space
// readable by the lane) with hash h.  Returns 1 new, 0 duplicate, -1 pool
// full, -2 probe limit.
__device__ inline int pool_insert(const PoolDev& P, const uint64_t* key, uint64_t h) {
  const uint32_t tag = (uint32_t)(h >> 32) | 0x80000000u;
  const int nwords = P.stride / 8;
  uint64_t slot = h & P.tmask;
  const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  for (int it = 0; it < kMaxProbeIters; ++it) {
    uint64_t e = ld_acquire(&P.table[slot]);
    bool won = false;
    if (e == 0) {
      uint64_t busy = ((uint64_t)tag << 32) | kIdxBusy;
      uint64_t expected = 0;
      won = __hip_atomic_compare_exchange_strong(&P.table[slot], &expected, busy, __ATOMIC_ACQ_REL,
                                                 __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the lanes (still probing) that claimed a slot in this iteration
    const uint64_t wm = __ballot(won);
    if (wm) {
      const uint32_t leader = (uint32_t)__builtin_ctzll(wm);
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&P.count[0], (uint32_t)__popcll(wm));
      base = __shfl(base, (int)leader, 64);
      if (won) {
        const uint32_t idx =
            base + __builtin_amdgcn_mbcnt_hi((uint32_t)(wm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)wm, 0u));
        if (idx >= P.cap) {
          atomicOr(&P.count[1], 1u);
          __hip_atomic_store(&P.table[slot], ((uint64_t)tag << 32) | kIdxDead, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
          return -1;
        }
        uint64_t* dst = reinterpret_cast<uint64_t*>(P.keys + (size_t)idx * P.stride);
        for (int i = 0; i < nwords; ++i) dst[i] = key[i];
        __threadfence();
        __hip_atomic_store(&P.table[slot], ((uint64_t)tag << 32) | idx, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
        return 1;
      }
    }
    if (e == 0) continue;  // lost the race: look at the same slot again
    if ((uint32_t)(e >> 32) == tag) {
      uint32_t idx = (uint32_t)e;
      if (idx == kIdxBusy) continue;  // being written by another lane: re-read
      if (idx != kIdxDead) {
        const uint64_t* other = reinterpret_cast<const uint64_t*>(P.keys + (size_t)idx * P.stride);
        bool same = true;
        for (int i = 0; i < nwords; ++i) {
          uint64_t ow = __hip_atomic_load(const_cast<uint64_t*>(other + i), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
          if (ow != key[i]) {
            same = false;
            break;
          }
        }
        if (same) return 0;
      }
    }
    slot = (slot + 1) & P.tmask;
  }
  atomicOr(&P.count[2], 1u);
  return -2;
}

}  // namespace graver
