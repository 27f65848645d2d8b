// xcd.hpp -- launch helpers for the chip's layout: workgroups are dealt to
// the accelerator complex dies (XCDs, each with its own L2) in turn, and the
// lanes of one atomic instruction that hit one address are served one after
// another.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ftc {

constexpr int kXCD = 8;  // XCDs; workgroup b runs on XCD b % kXCD

inline int32_t round_up_xcd(int64_t b) { return (int32_t)((b + kXCD - 1) / kXCD * kXCD); }

// A wave-uniform grid-stride walk over [0, n) in which the workgroups of
// each XCD take one contiguous eighth of the range (rounded to whole
// wavefronts), so that neighbouring items, which share mesh records and
// bitmap words, meet in one L2.  `group` numbers the workgroups of the
// walk from 0 and `ngroup` counts them (a multiple of kXCD, so that group
// and blockIdx.x agree modulo kXCD when the walk's first workgroup is a
// multiple of kXCD).  Every lane of a wavefront takes the same number of
// steps; items past the end come with ok = false.
struct XcdWalk {
  int64_t base, end, step;
  int lane;
  __device__ XcdWalk(int64_t n, int64_t group, int64_t ngroup) {
    const int64_t per = ((n + kXCD - 1) / kXCD + 63) / 64 * 64;
    const int64_t lo = min((int64_t)(group % kXCD) * per, n);
    end = min(lo + per, n);
    lane = threadIdx.x & 63;
    base = lo + (group / kXCD) * blockDim.x + (threadIdx.x - lane);
    step = (ngroup / kXCD) * blockDim.x;
  }
  template <class Body>
  __device__ __forceinline__ void run(Body body) const {
    for (int64_t b = base; b < end; b += step) {
      const int64_t x = b + lane;
      body(x, x < end);
    }
  }
};

// LDS a wavefront lends wave_count_add: a 128-slot hash of keys, the count
// and the counter's old value per slot.
constexpr int kCountSlots = 128;
struct CountLDS {
  int32_t key[kCountSlots], cnt[kCountSlots], base[kCountSlots];
};

// atomicAdd(&ctr[key], 1) for every lane with act: a lane gets the
// counter's old value plus its rank among the lanes with the same key, i.e.
// a distinct index per lane as with one atomic each (in another order among
// equal keys).  Lanes of one atomic instruction that hit the same address
// are served one after another, so the lanes are grouped by key first: each
// claims its key's slot in an LDS hash (open addressing, at most 64 keys in
// 128 slots) and takes its rank there by an LDS atomic; then the first lane
// of each group adds the group's size to the counter, all groups in one
// atomic instruction.  Called by all 64 lanes, with L owned by the
// wavefront.
__device__ inline int32_t wave_count_add(int32_t* ctr, int32_t key, bool act, CountLDS& L) {
  const int lane = threadIdx.x & 63;
  L.key[lane] = -1;
  L.key[lane + 64] = -1;
  L.cnt[lane] = 0;
  L.cnt[lane + 64] = 0;
  __builtin_amdgcn_wave_barrier();
  int slot = 0, rank = 0;
  if (act) {
    int s = (int)(((uint32_t)key * 2654435761u) >> 25);
    for (int p = 0; p < kCountSlots; ++p) {
      const int32_t prev = atomicCAS(&L.key[s], -1, key);
      if (prev == -1 || prev == key) break;
      s = (s + 1) & (kCountSlots - 1);
    }
    slot = s;
    rank = atomicAdd(&L.cnt[slot], 1);
  }
  __builtin_amdgcn_wave_barrier();
  if (act && rank == 0) L.base[slot] = atomicAdd(&ctr[key], L.cnt[slot]);
  __builtin_amdgcn_wave_barrier();
  return act ? L.base[slot] + rank : 0;
}

// Sets bit `bit` of word `word` of a bitmap for every lane with act.  The
// lanes are grouped by word (register work), each group's bits are gathered
// in acc (64 words of LDS owned by this wavefront) and the lowest lane of
// each group ORs them into the bitmap, all groups in one atomic
// instruction.  Called by all 64 lanes.
__device__ inline void wave_set_bits(uint32_t* bitmap, int64_t word, int bit, bool act, uint32_t* acc) {
  const int lane = threadIdx.x & 63;
  const int32_t wlo = (int32_t)word, whi = (int32_t)(word >> 32);
  uint64_t pend = __ballot(act);
  int leader_of = lane;
  bool lead = false;
  while (pend) {
    const int leader = __builtin_ctzll(pend);
    const int32_t klo = __builtin_amdgcn_readlane(wlo, leader), khi = __builtin_amdgcn_readlane(whi, leader);
    const uint64_t same = __ballot(wlo == klo && whi == khi) & pend;
    if ((same >> lane) & 1ull) leader_of = leader;
    if (lane == leader) lead = true;
    pend &= ~same;
  }
  acc[lane] = 0u;
  __builtin_amdgcn_wave_barrier();
  if (act) atomicOr(&acc[leader_of], 1u << bit);
  __builtin_amdgcn_wave_barrier();
  const uint32_t m = acc[lane];
  if (lead) atomicOr(&bitmap[word], m);
}

}  // namespace ftc
