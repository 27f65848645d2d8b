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
  __device__ void run(Body body) const {
    for (int64_t b = base; b < end; b += step) {
      const int64_t x = b + lane;
      body(x, x < end);
    }
  }
};

// atomicAdd(&ctr[key], 1) for every lane with act: a lane gets the
// counter's old value plus the number of lanes below it with the same key,
// i.e. a distinct index per lane as with one atomic each (in another order
// among equal keys).  Lanes of one atomic instruction that hit the same
// address are served one after another, so the wavefront first groups its
// lanes by key (register work only) and then issues a single atomic
// instruction in which the lowest lane of each group adds the group's size.
// Called by all 64 lanes.
__device__ inline int32_t wave_count_add(int32_t* ctr, int32_t key, bool act) {
  const int lane = threadIdx.x & 63;
  uint64_t pend = __ballot(act);
  int leader_of = lane, below = 0, cnt = 0;
  while (pend) {
    const int leader = __builtin_ctzll(pend);
    const int32_t k = __builtin_amdgcn_readlane(key, leader);
    const uint64_t same = __ballot(key == k) & pend;
    if ((same >> lane) & 1ull) {
      leader_of = leader;
      below = __popcll(same & ((1ull << lane) - 1ull));
    }
    if (lane == leader) cnt = __popcll(same);
    pend &= ~same;
  }
  int32_t old = 0;
  if (cnt > 0) old = atomicAdd(&ctr[key], cnt);
  return __shfl(old, leader_of, 64) + below;
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
