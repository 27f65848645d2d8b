// scan.hip -- device-wide exclusive prefix sums (three passes: block totals,
// scan of the totals in one block, block-local scan plus offset) and small
// fill kernels.  Used for every count -> offset conversion of the library.
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

// Inclusive scan across one wavefront of 64 lanes.
__device__ inline int32_t wave_incl_scan(int32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int32_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive scan of one value per thread over the block; returns the block
// total in *total.  blockDim.x must be a multiple of 64 and <= 1024.
__device__ inline int32_t block_excl_scan(int32_t v, int32_t* total) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t wtot;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int32_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    int32_t s = lane < nw ? wsum[lane] : 0;
    int32_t si = wave_incl_scan(s);
    if (lane < nw) wsum[lane] = si - s;
    if (lane == nw - 1) wtot = si;
  }
  __syncthreads();
  int32_t r = inc - v + wsum[wid];
  *total = wtot;
  __syncthreads();
  return r;
}

template <class L>
__global__ __launch_bounds__(kThreads) void k_block_totals(L load, int64_t n, int32_t* tmp) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kItems;
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q)
    if (base + q < n) s += load(base + q);
  int32_t total;
  block_excl_scan(s, &total);
  if (threadIdx.x == 0) tmp[blockIdx.x] = total;
}

// One block of 1024 threads scans up to kScanMaxBlocks block totals in place.
__global__ __launch_bounds__(1024) void k_scan_totals(int32_t* tmp, int64_t nb, int32_t* grand, int32_t* grand2) {
  constexpr int per = (int)(kScanMaxBlocks / 1024);
  const int64_t base = (int64_t)threadIdx.x * per;
  int32_t v[per];
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    v[q] = (base + q < nb) ? tmp[base + q] : 0;
    s += v[q];
  }
  int32_t total;
  int32_t run = block_excl_scan(s, &total);
#pragma unroll
  for (int q = 0; q < per; ++q) {
    if (base + q < nb) tmp[base + q] = run;
    run += v[q];
  }
  if (threadIdx.x == 0) {
    if (grand) *grand = total;
    if (grand2) *grand2 = total;
  }
}

template <class L>
__global__ __launch_bounds__(kThreads) void k_block_apply(L load, int64_t n, const int32_t* tmp, int32_t* out) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kItems;
  int32_t v[kItems];
  int32_t s = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    v[q] = (base + q < n) ? load(base + q) : 0;
    s += v[q];
  }
  int32_t total;
  int32_t run = block_excl_scan(s, &total) + tmp[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
}

template <class L>
hipError_t scan_impl(L load, int32_t* out, int64_t n, int32_t* tmp, int32_t* total_out, hipStream_t s) {
  if (n < 0 || n > kScanMax) return hipErrorInvalidValue;
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_block_totals<L>, dim3((unsigned)nb), dim3(kThreads), 0, s, load, n, tmp);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, s, tmp, nb, out + n, total_out);
  hipLaunchKernelGGL(k_block_apply<L>, dim3((unsigned)nb), dim3(kThreads), 0, s, load, n, (const int32_t*)tmp,
                     out);
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

hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_blocks(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace ftc
