// Exclusive scans of int32 counts on the device, for the kernels that build
// index arrays with many workgroups (the device graph build, the replay
// program of large schedules).  Each translation unit that includes this
// header gets its own copy of the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "fs_internal.h"

namespace fs {
namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;   // elements per thread

// Block-wide exclusive scan of one value per thread (NT threads); sh holds
// NT/64 + 1 words.  Every thread must call it.
template <int NT>
__device__ uint32_t scan_block(uint32_t v, uint32_t *sh, uint32_t &total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  if (wid == 0) {
    const uint32_t w = lane < NW ? sh[lane] : 0u;
    uint32_t s = w;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < NW) sh[lane] = s - w;
    if (lane == NW - 1) sh[NW] = s;
  }
  __syncthreads();
  const uint32_t res = sh[wid] + x - v;
  total = sh[NW];
  __syncthreads();
  return res;
}

// pass 1: the sum of each block of kScanThreads * kScanItems elements, and
// the largest element into *max_out when given (one atomicMax per wave)
__global__ __launch_bounds__(kScanThreads) void scan_partial_kernel(const int32_t *in, uint32_t m, uint32_t *sums,
                                                                    int32_t *max_out) {
  __shared__ uint32_t sh[kScanThreads / 64 + 1];
  const uint64_t base = ((uint64_t)blockIdx.x * kScanThreads + threadIdx.x) * kScanItems;
  uint32_t v = 0;
  int32_t mx = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < m) {
      v += (uint32_t)in[base + i];
      mx = max(mx, in[base + i]);
    }
  uint32_t total = 0;
  (void)scan_block<kScanThreads>(v, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
  if (max_out) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0 && mx > 0) atomicMax(max_out, mx);
  }
}

// pass 2, one workgroup: exclusive scan of the nb block sums in place; the
// grand total to *total_out when given
__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(uint32_t *sums, uint32_t nb, int32_t *total_out) {
  __shared__ uint32_t sh[kScanThreads / 64 + 1];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < nb; b0 += kScanThreads) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t v = b < nb ? sums[b] : 0u;
    uint32_t total = 0;
    const uint32_t ex = scan_block<kScanThreads>(v, sh, total);
    if (b < nb) sums[b] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total_out) *total_out = (int32_t)carry;
}

// pass 3: out[i] = sum of in[0..i), out[m] = total.  in and out may be the
// same array (each thread reads its elements before writing them).
__global__ __launch_bounds__(kScanThreads) void scan_final_kernel(const int32_t *in, uint32_t m, const uint32_t *sums,
                                                                  int32_t *out) {
  __shared__ uint32_t sh[kScanThreads / 64 + 1];
  const uint64_t base = ((uint64_t)blockIdx.x * kScanThreads + threadIdx.x) * kScanItems;
  uint32_t v[kScanItems], s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < m ? (uint32_t)in[base + i] : 0u;
    s += v[i];
  }
  uint32_t total = 0;
  uint32_t run = sums[blockIdx.x] + scan_block<kScanThreads>(s, sh, total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < m) out[base + i] = (int32_t)run;
    run += v[i];
  }
  if (base < m && base + kScanItems >= m) out[m] = (int32_t)run;   // the thread holding the last element
}

// One workgroup for short arrays: chunks of kScanThreads * kScanOneItems in
// order with a running carry; out[m] = total, the largest element into
// *max_out when given.  in and out may be the same array.  Every thread of a
// kScanThreads workgroup calls it; sh holds kScanThreads / 64 + 1 words.
constexpr int kScanOneItems = 16;

__device__ void scan_one_block(const int32_t *in, uint32_t m, int32_t *out, int32_t *max_out, uint32_t *sh) {
  constexpr uint32_t kChunk = kScanThreads * kScanOneItems;
  uint32_t carry = 0;
  int32_t mx = 0;
  for (uint32_t c0 = 0; c0 < m; c0 += kChunk) {
    const uint32_t base = c0 + threadIdx.x * kScanOneItems;
    uint32_t v[kScanOneItems], s = 0;
#pragma unroll
    for (int i = 0; i < kScanOneItems; ++i) v[i] = base + i < m ? (uint32_t)in[base + i] : 0u;
#pragma unroll
    for (int i = 0; i < kScanOneItems; ++i) {
      s += v[i];
      mx = max(mx, (int32_t)v[i]);
    }
    uint32_t total = 0;
    uint32_t run = carry + scan_block<kScanThreads>(s, sh, total);
#pragma unroll
    for (int i = 0; i < kScanOneItems; ++i) {
      if (base + i < m) out[base + i] = (int32_t)run;
      run += v[i];
    }
    carry += total;
  }
  if (threadIdx.x == 0) out[m] = (int32_t)carry;
  if (max_out) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0 && mx > 0) atomicMax(max_out, mx);
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_one_kernel(const int32_t *in, uint32_t m, int32_t *out,
                                                                int32_t *max_out) {
  __shared__ uint32_t sh[kScanThreads / 64 + 1];
  scan_one_block(in, m, out, max_out, sh);
}

constexpr uint32_t kScanOneMax = 1u << 16;   // longest array given to scan_one_kernel

// Block sums needed to scan m elements.
inline uint32_t scan_sums_for(uint64_t m) {
  const uint64_t per = (uint64_t)kScanThreads * kScanItems;
  return (uint32_t)std::max<uint64_t>(1, (m + per - 1) / per);
}

// out[0..m] from in[0..m) (m >= 1); sums holds scan_sums_for(m) words.
// With max_out, the largest element (of non-negative counts) is also
// combined into *max_out by atomicMax.  Short arrays take one launch.
inline fs_status scan_i32(const int32_t *in, uint32_t m, uint32_t *sums, int32_t *out, hipStream_t s,
                          int32_t *max_out = nullptr) {
  if (m <= kScanOneMax) {
    hipLaunchKernelGGL(scan_one_kernel, dim3(1), dim3(kScanThreads), 0, s, in, m, out, max_out);
  } else {
    const uint32_t nb = scan_sums_for(m);
    hipLaunchKernelGGL(scan_partial_kernel, dim3(nb), dim3(kScanThreads), 0, s, in, m, sums, max_out);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanThreads), 0, s, sums, nb, (int32_t *)nullptr);
    hipLaunchKernelGGL(scan_final_kernel, dim3(nb), dim3(kScanThreads), 0, s, in, m, sums, out);
  }
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string("scan launch: ") + hipGetErrorString(e));
}

}  // namespace
}  // namespace fs
