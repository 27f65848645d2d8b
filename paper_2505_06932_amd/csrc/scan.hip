// scan.hip -- device-wide exclusive prefix sums in two passes (block totals;
// block-local scan plus the sum of the earlier blocks' totals, which each
// block reads itself) and small fill kernels.  Used for every count ->
// offset conversion of the library.
#include <algorithm>

#include "dpp.hpp"
#include "ftc_ws.hpp"

namespace ftc {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;  // kThreads * kItems == kScanBlock
static_assert(kThreads * kItems == kScanBlock, "scan block");

struct LoadI32 {
  const int32_t* p;
  __device__ int32_t operator()(int64_t i) const { return p[i]; }
};
struct LoadPop {
  const uint32_t* p;
  __device__ int32_t operator()(int64_t i) const { return __popc(p[i]); }
};

struct LoadBandPop {
  BandWords B;
  __device__ int32_t operator()(int64_t i) const { return __popc(B.word(i)); }
};
struct WordsPlain {
  const uint32_t* p;
  __device__ uint32_t word(int64_t i) const { return p[i]; }
};


// Exclusive scan of one value per thread over the block; returns the block
// total in *total.  blockDim.x must be a multiple of 64 and <= 1024.
__device__ inline int32_t block_excl_scan(int32_t v, int32_t* total) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t wtot;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int32_t inc = wave_incl_scan_dpp(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    int32_t s = lane < nw ? wsum[lane] : 0;
    int32_t si = wave_incl_scan_dpp(s);
    if (lane < nw) wsum[lane] = si - s;
    if (lane == nw - 1) wtot = si;
  }
  __syncthreads();
  int32_t r = inc - v + wsum[wid];
  *total = wtot;
  __syncthreads();
  return r;
}

// Tiles of kScanBlock entries move between global memory and the threads
// through LDS: global accesses are lane-consecutive (entry q * kThreads +
// t of the tile for thread t), the scan works on kItems consecutive entries
// per thread (entries t * kItems + q).  One padding word per 32 spreads a
// thread's consecutive entries over the LDS banks.
constexpr int kTilePad = kScanBlock + kScanBlock / 32;
__device__ inline int tile_ix(int i) { return i + (i >> 5); }

// First pass: the total of each block of kScanBlock inputs (the order of
// the loads does not matter here).
template <class L>
__device__ inline void totals_one(L load, int64_t n, int64_t b, int32_t* slot) {
  const int64_t tile = b * kScanBlock;
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const int64_t i = tile + q * kThreads + threadIdx.x;
    if (i < n) s += load(i);
  }
  int32_t total;
  block_excl_scan(s, &total);
  if (threadIdx.x == 0) *slot = total;
}

// Sum of tmp[0, nb) over the block (every thread gets it).
__device__ inline int32_t block_sum_prefix(const int32_t* tmp, int64_t nb) {
  int32_t s = 0;
  for (int64_t q = threadIdx.x; q < nb; q += blockDim.x) s += tmp[q];
  int32_t total;
  block_excl_scan(s, &total);
  return total;
}

// Second pass for block b of nblocks: the local scan plus the totals of the
// blocks before it; the last block also writes the grand total to out[n]
// and *total_out.  In place is allowed (out == input): the block reads all
// of its tile before any thread writes.
template <class L>
__device__ inline void apply_one(L load, int64_t n, const int32_t* tmp, int32_t* out, int32_t* total_out, int64_t b,
                                 int64_t nblocks) {
  __shared__ int32_t st[kTilePad];
  const int32_t prefix = block_sum_prefix(tmp, b);
  const int64_t tile = b * kScanBlock;
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const int i = q * kThreads + threadIdx.x;
    st[tile_ix(i)] = tile + i < n ? load(tile + i) : 0;
  }
  __syncthreads();
  int32_t v[kItems];
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    v[q] = st[tile_ix(threadIdx.x * kItems + q)];
    s += v[q];
  }
  int32_t total;
  int32_t run = block_excl_scan(s, &total) + prefix;  // its barriers end every read of st
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    st[tile_ix(threadIdx.x * kItems + q)] = run;
    run += v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const int i = q * kThreads + threadIdx.x;
    if (tile + i < n) out[tile + i] = st[tile_ix(i)];
  }
  if (b == nblocks - 1 && threadIdx.x == 0) {
    out[n] = prefix + total;
    if (total_out) *total_out = prefix + total;
  }
}

template <class L>
__global__ __launch_bounds__(kThreads) void k_block_totals(L load, int64_t n, int32_t* tmp) {
  totals_one(load, n, blockIdx.x, tmp + blockIdx.x);
}

template <class L>
__global__ __launch_bounds__(kThreads) void k_block_apply(L load, int64_t n, const int32_t* tmp, int32_t* out,
                                                          int32_t* total_out, int64_t nb) {
  apply_one(load, n, tmp, out, total_out, blockIdx.x, nb);
}

// Up to kMaxSeg independent arrays in one pair of launches: the blocks of
// segment q are [b0[q], b0[q + 1]), and its block totals sit at the same
// positions of tmp.
struct MultiSeg {
  ScanSeg seg[kMaxSeg];
  int64_t b0[kMaxSeg + 1];
  int nseg;
};

__device__ inline int seg_of(const MultiSeg& M, int64_t b) {
  int q = 0;
  while (q + 1 < M.nseg && b >= M.b0[q + 1]) ++q;
  return q;
}

__global__ __launch_bounds__(kThreads) void k_block_totals_multi(MultiSeg M, int32_t* tmp) {
  const int q = seg_of(M, blockIdx.x);
  totals_one(LoadI32{M.seg[q].in}, M.seg[q].n, blockIdx.x - M.b0[q], tmp + blockIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_block_apply_multi(MultiSeg M, const int32_t* tmp) {
  const int q = seg_of(M, blockIdx.x);
  const int64_t b = blockIdx.x - M.b0[q];
  apply_one(LoadI32{M.seg[q].in}, M.seg[q].n, tmp + M.b0[q], M.seg[q].out, M.seg[q].total, b,
            M.b0[q + 1] - M.b0[q]);
  if (M.seg[q].clear) {
    // the block's tile, read in full by apply_one before its barriers
    const int64_t tile = b * kScanBlock;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const int64_t x = tile + i * kThreads + threadIdx.x;
      if (x < M.seg[q].n) M.seg[q].clear[x] = 0;
    }
  }
}

// Second pass of the popcount scan that also lists the set bits: every set
// bit b of word w becomes entry out[w] + (rank of b in w) of `ids`, with the
// value 32 w + b (entries at or past `cap` latch a capacity error).
template <class WL>
__global__ __launch_bounds__(kThreads) void k_block_apply_emit(WL words, int64_t n, const int32_t* tmp, int32_t* out,
                                                               int32_t* total_out, int64_t nb, int32_t* ids,
                                                               int32_t cap, int32_t* counters) {
  __shared__ uint32_t st[kTilePad];
  const int64_t b = blockIdx.x;
  const int32_t prefix = block_sum_prefix(tmp, b);
  const int64_t tile = b * kScanBlock;
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const int i = q * kThreads + threadIdx.x;
    st[tile_ix(i)] = tile + i < n ? words.word(tile + i) : 0u;
  }
  __syncthreads();
  const int64_t base = tile + (int64_t)threadIdx.x * kItems;
  uint32_t wv[kItems];
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    wv[q] = st[tile_ix(threadIdx.x * kItems + q)];
    s += __popc(wv[q]);
  }
  int32_t total;
  int32_t run = block_excl_scan(s, &total) + prefix;  // its barriers end every read of st
  bool over = false;
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    st[tile_ix(threadIdx.x * kItems + q)] = (uint32_t)run;
    uint32_t bits = wv[q];
    while (bits) {
      const int bit = __ffs(bits) - 1;
      if (run < cap)
        ids[run] = (int32_t)((base + q) * 32 + bit);
      else
        over = true;
      ++run;
      bits &= bits - 1u;
    }
  }
  if (over) atomicOr(&counters[C_ERR], ERR_CAPACITY);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const int i = q * kThreads + threadIdx.x;
    if (tile + i < n) out[tile + i] = (int32_t)st[tile_ix(i)];
  }
  if (b == nb - 1 && threadIdx.x == 0) {
    out[n] = prefix + total;
    if (total_out) *total_out = prefix + total;
  }
}

template <class L>
hipError_t scan_impl(L load, int32_t* out, int64_t n, int32_t* tmp, int32_t* total_out, hipStream_t s) {
  if (n < 0 || n > kScanMax) return hipErrorInvalidValue;
  const int64_t nb = std::max<int64_t>((n + kScanBlock - 1) / kScanBlock, 1);
  hipLaunchKernelGGL(k_block_totals<L>, dim3((unsigned)nb), dim3(kThreads), 0, s, load, n, tmp);
  hipLaunchKernelGGL(k_block_apply<L>, dim3((unsigned)nb), dim3(kThreads), 0, s, load, n, (const int32_t*)tmp, out,
                     total_out, nb);
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

hipError_t scan_exclusive(int32_t* data, int64_t n, int32_t* tmp, int32_t* total_out, hipStream_t s) {
  return scan_impl(LoadI32{data}, data, n, tmp, total_out, s);
}

hipError_t scan_popcount(const uint32_t* words, int32_t* out, int64_t n, int32_t* tmp, int32_t* total_out,
                         hipStream_t s) {
  return scan_impl(LoadPop{words}, out, n, tmp, total_out, s);
}

hipError_t scan_popcount_emit(const uint32_t* words, int32_t* out, int64_t n, int32_t* tmp, int32_t* total_out,
                              int32_t* ids, int32_t cap, int32_t* counters, hipStream_t s) {
  if (n < 0 || n > kScanMax) return hipErrorInvalidValue;
  const int64_t nb = std::max<int64_t>((n + kScanBlock - 1) / kScanBlock, 1);
  hipLaunchKernelGGL(k_block_totals<LoadPop>, dim3((unsigned)nb), dim3(kThreads), 0, s, LoadPop{words}, n, tmp);
  hipLaunchKernelGGL(k_block_apply_emit<WordsPlain>, dim3((unsigned)nb), dim3(kThreads), 0, s, WordsPlain{words}, n,
                     (const int32_t*)tmp, out, total_out, nb, ids, cap, counters);
  return hipGetLastError();
}

hipError_t scan_band_emit(const uint32_t* bitmap, int64_t nwords, int64_t ncell, int64_t sy, int64_t sz, int32_t* out,
                          int32_t* tmp, int32_t* total_out, int32_t* ids, int32_t cap, int32_t* counters,
                          hipStream_t s) {
  if (nwords < 0 || nwords > kScanMax) return hipErrorInvalidValue;
  const BandWords B{bitmap, nwords, ncell, sy, sz};
  const int64_t nb = std::max<int64_t>((nwords + kScanBlock - 1) / kScanBlock, 1);
  hipLaunchKernelGGL(k_block_totals<LoadBandPop>, dim3((unsigned)nb), dim3(kThreads), 0, s, LoadBandPop{B}, nwords,
                     tmp);
  hipLaunchKernelGGL(k_block_apply_emit<BandWords>, dim3((unsigned)nb), dim3(kThreads), 0, s, B, nwords,
                     (const int32_t*)tmp, out, total_out, nb, ids, cap, counters);
  return hipGetLastError();
}

hipError_t scan_exclusive_multi(const ScanSeg* segs, int nseg, int32_t* tmp, hipStream_t s) {
  if (nseg < 1 || nseg > kMaxSeg) return hipErrorInvalidValue;
  MultiSeg M{};
  M.nseg = nseg;
  M.b0[0] = 0;
  for (int q = 0; q < nseg; ++q) {
    if (segs[q].n < 0 || segs[q].n > kScanMax) return hipErrorInvalidValue;
    M.seg[q] = segs[q];
    M.b0[q + 1] = M.b0[q] + std::max<int64_t>((segs[q].n + kScanBlock - 1) / kScanBlock, 1);
  }
  for (int q = nseg; q < kMaxSeg; ++q) M.b0[q + 1] = M.b0[nseg];
  const int64_t nb = M.b0[nseg];
  if (nb > kScanMaxBlocks) {
    for (int q = 0; q < nseg; ++q) {
      hipError_t e = scan_impl(LoadI32{segs[q].in}, segs[q].out, segs[q].n, tmp, segs[q].total, s);
      if (e == hipSuccess && segs[q].clear) e = fill_i32(segs[q].clear, segs[q].n, 0, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipLaunchKernelGGL(k_block_totals_multi, dim3((unsigned)nb), dim3(kThreads), 0, s, M, tmp);
  hipLaunchKernelGGL(k_block_apply_multi, dim3((unsigned)nb), dim3(kThreads), 0, s, M, (const int32_t*)tmp);
  return hipGetLastError();
}

hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_blocks(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace ftc
