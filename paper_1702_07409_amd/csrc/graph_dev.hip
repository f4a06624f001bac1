// Device construction of the seeded LDGM graph (§2.2: an object's graph is
// regenerated from its seed and parameters whenever it is needed).
//
// Every coded row draws from its own counter-based stream, so rows are built
// in parallel, one per thread: the degree by a threshold search, the
// neighbours by Floyd's sampling, sorted ascending.  Rows of more than
// kSegMax neighbours (the Robust Soliton tail) are sampled by a workgroup
// each, with a k-bit LDS bitmap for the membership test, which also yields
// the sorted order.  The CSC comes from per-column counting and a sort of
// each (short) column; the encode segments are placed by a stable counting
// sort over their lengths.  Every array equals the host construction's
// (graph_host.cpp) element for element.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "fs_internal.h"

namespace fs {
namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPurposeGraph = 1;
constexpr int kThreads = 1024;       // rows per block of the counting passes
constexpr int kSampleThreads = 256;  // rows per block of the light sampler
constexpr int kScanItems = 4;        // elements per thread of the scans

// SplitMix64 output function (Steele, Lea & Flood 2014; Stafford's Mix13
// constants), the row streams of the host construction.
__device__ __forceinline__ uint64_t mix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ uint64_t row_key(uint64_t seed, uint64_t stripe_key, uint64_t row) {
  uint64_t h = mix(seed + kGolden);
  h = mix(h ^ kPurposeGraph);
  h = mix(h ^ stripe_key);
  return mix(h ^ row);
}

__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t i) { return mix(key + (i + 1) * kGolden); }

// Floyd's step s of a row of degree d over k inputs: the candidate v, or r
// when v is taken already.
__device__ __forceinline__ uint32_t floyd_candidate(uint64_t key, uint32_t k, uint32_t d, uint32_t s,
                                                    uint32_t &r_out) {
  const uint64_t r = (uint64_t)(k - d) + s;
  r_out = (uint32_t)r;
  return (uint32_t)(((draw(key, s + 1) >> 32) * (r + 1)) >> 32);
}

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

// ---------------------------------------------------------------------------
// degrees
// ---------------------------------------------------------------------------
// d_j = 1 + (number of thresholds <= the row's first draw >> 11); T is
// ascending and its last entry is 2^53, above every draw.
__global__ __launch_bounds__(256) void degree_kernel(DevGraphJob J) {
  const uint32_t j = blockIdx.x * 256u + threadIdx.x;
  if (j >= J.n) return;
  const uint64_t v0 = draw(row_key(J.seed, J.stripe_key, j), 0) >> 11;
  uint32_t lo = 0, hi = J.D;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (J.T[mid] <= v0) lo = mid + 1;
    else hi = mid;
  }
  J.deg[j] = (int32_t)(lo + 1);
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts: out[0..m] (out[m] = total), three passes
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void scan_partial_kernel(const int32_t *in, uint32_t m, uint32_t *sums) {
  __shared__ uint32_t sh[kThreads / 64 + 1];
  const uint64_t base = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) * kScanItems;
  uint32_t v = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < m) v += (uint32_t)in[base + i];
  uint32_t total = 0;
  (void)scan_block<kThreads>(v, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// one workgroup: exclusive scan of the block sums in place (nb of them)
__global__ __launch_bounds__(kThreads) void scan_sums_kernel(uint32_t *sums, uint32_t nb, int32_t *total_out) {
  __shared__ uint32_t sh[kThreads / 64 + 1];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < nb; b0 += kThreads) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t v = b < nb ? sums[b] : 0u;
    uint32_t total = 0;
    const uint32_t ex = scan_block<kThreads>(v, sh, total);
    if (b < nb) sums[b] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total_out) *total_out = (int32_t)carry;
}

__global__ __launch_bounds__(kThreads) void scan_final_kernel(const int32_t *in, uint32_t m, const uint32_t *sums,
                                                              int32_t *out) {
  __shared__ uint32_t sh[kThreads / 64 + 1];
  const uint64_t base = ((uint64_t)blockIdx.x * kThreads + threadIdx.x) * kScanItems;
  uint32_t v[kScanItems], s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < m ? (uint32_t)in[base + i] : 0u;
    s += v[i];
  }
  uint32_t total = 0;
  uint32_t run = sums[blockIdx.x] + scan_block<kThreads>(s, sh, total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < m) out[base + i] = (int32_t)run;
    run += v[i];
  }
  if (base < m && base + kScanItems >= m) out[m] = (int32_t)run;   // the thread holding the last element
}

// ---------------------------------------------------------------------------
// encode segments and heavy rows: a stable counting sort over lengths
// ---------------------------------------------------------------------------
// Segment buckets: b = 64 - length, so that the longest come first (bucket 0
// holds the full kSegMax-edge pieces).  Per block of kThreads rows: the
// segment count of each bucket, and the rows of more than kSegMax edges.
__global__ __launch_bounds__(kThreads) void seg_count_kernel(DevGraphJob J) {
  __shared__ uint32_t hist[kSegMax + 1];   // [64] = heavy rows
  if (threadIdx.x <= kSegMax) hist[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
  if (j < J.n) {
    const uint32_t d = (uint32_t)J.deg[j];
    if (d / kSegMax) atomicAdd(&hist[0], d / kSegMax);
    if (d % kSegMax) atomicAdd(&hist[kSegMax - d % kSegMax], 1u);
    if (d > kSegMax) atomicAdd(&hist[kSegMax], 1u);
    atomicMax(J.scalars + kScalarMaxDeg, (int32_t)d);
    atomicAdd(J.edges, (unsigned long long)d);
  }
  __syncthreads();
  if (threadIdx.x <= kSegMax) J.blk_hist[(uint64_t)blockIdx.x * (kSegMax + 1) + threadIdx.x] = hist[threadIdx.x];
}

// One workgroup: per bucket, the exclusive prefix over blocks plus the
// bucket's start (buckets in order 0..63); the heavy rows likewise.
__global__ __launch_bounds__(kThreads) void seg_scan_kernel(DevGraphJob J, uint32_t nblk) {
  __shared__ uint32_t tot[kSegMax + 1];
  __shared__ uint32_t start[kSegMax + 1];
  const uint32_t b = threadIdx.x;
  if (b <= kSegMax) {
    uint32_t run = 0;
    for (uint32_t blk = 0; blk < nblk; ++blk) {
      uint32_t *p = J.blk_hist + (uint64_t)blk * (kSegMax + 1) + b;
      const uint32_t c = *p;
      *p = run;
      run += c;
    }
    tot[b] = run;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (uint32_t q = 0; q < kSegMax; ++q) {
      start[q] = run;
      run += tot[q];
    }
    start[kSegMax] = 0;
    J.scalars[kScalarSegs] = (int32_t)run;
    J.scalars[kScalarHeavy] = (int32_t)tot[kSegMax];
  }
  __syncthreads();
  if (b <= kSegMax)
    for (uint32_t blk = 0; blk < nblk; ++blk) J.blk_hist[(uint64_t)blk * (kSegMax + 1) + b] += start[b];
}

// Each row's segments at their sorted positions: full pieces in bucket 0
// (row order, then piece order), the remainder in its length's bucket (row
// order).  Ranks within a block: a block scan for the full pieces; for the
// remainders, lanes of equal length are found by ballots over the length's
// six bits, and waves are ordered through per-(wave, bucket) counts.
__global__ __launch_bounds__(kThreads) void seg_place_kernel(DevGraphJob J) {
  __shared__ uint32_t sh[kThreads / 64 + 1];
  __shared__ uint32_t wcnt[kThreads / 64][kSegMax + 1];   // [.][64]: heavy rows
  constexpr int NW = kThreads / 64;
  const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool live = j < J.n;
  const uint32_t d = live ? (uint32_t)J.deg[j] : 0u;
  const uint32_t full = d / kSegMax, rest = d % kSegMax;
  const uint32_t *off = J.blk_hist + (uint64_t)blockIdx.x * (kSegMax + 1);
  uint32_t total = 0;
  const uint32_t full_rank = scan_block<kThreads>(full, sh, total);
  for (int i = threadIdx.x; i < NW * (kSegMax + 1); i += kThreads) (&wcnt[0][0])[i] = 0;
  __syncthreads();
  // lanes sharing this lane's remainder length (rest == 0: no remainder)
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t same = __ballot(live && rest != 0);
  if (!(live && rest != 0)) same = 0;
#pragma unroll
  for (int bit = 0; bit < 6; ++bit) {
    const uint64_t ones = __ballot(live && rest != 0 && ((rest >> bit) & 1u));
    same &= ((rest >> bit) & 1u) ? ones : ~ones;
  }
  const uint64_t heavy_mask = __ballot(live && d > kSegMax);
  const uint32_t b = kSegMax - rest;   // bucket of the remainder
  if (live && rest != 0 && (same & lt) == 0) wcnt[wid][b] = (uint32_t)__popcll(same);
  if (lane == 0) wcnt[wid][kSegMax] = (uint32_t)__popcll(heavy_mask);
  __syncthreads();
  if (!live) return;
  const bool split = d > kSegMax;
  const int32_t e0 = J.row_ptr[j];
  for (uint32_t s = 0; s < full; ++s) {
    const uint32_t at = off[0] + full_rank + s;
    J.seg_row[at] = (int32_t)j;
    J.seg_len[at] = (int32_t)kSegMax;
    J.seg_beg[at] = e0 + (int32_t)(s * kSegMax);
    J.seg_atomic[at] = split ? 1 : 0;
  }
  if (rest) {
    uint32_t before = 0;
    for (int w = 0; w < wid; ++w) before += wcnt[w][b];
    const uint32_t at = off[b] + before + (uint32_t)__popcll(same & lt);
    J.seg_row[at] = (int32_t)j;
    J.seg_len[at] = (int32_t)rest;
    J.seg_beg[at] = e0 + (int32_t)(full * kSegMax);
    J.seg_atomic[at] = split ? 1 : 0;
  }
  if (split) {
    uint32_t before = 0;
    for (int w = 0; w < wid; ++w) before += wcnt[w][kSegMax];
    J.heavy[off[kSegMax] + before + (uint32_t)__popcll(heavy_mask & lt)] = (int32_t)j;
  }
}

__global__ __launch_bounds__(256) void seg_copy_kernel(DevGraphJob J, uint32_t nseg) {
  const uint32_t s = blockIdx.x * 256u + threadIdx.x;
  if (s >= nseg) return;
  const int32_t *src = J.col + J.seg_beg[s];
  int32_t *dst = J.seg_col + J.seg_ptr[s];
  const int32_t len = J.seg_len[s];
  for (int32_t i = 0; i < len; ++i) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// neighbours
// ---------------------------------------------------------------------------
// Rows of at most kSegMax neighbours: one thread each, the picks in LDS
// (slot-major, so that neighbouring threads use neighbouring banks), the
// membership test by a scan of the picks so far, then an insertion sort.
__global__ __launch_bounds__(kSampleThreads) void sample_light_kernel(DevGraphJob J) {
  __shared__ int32_t picks[kSegMax][kSampleThreads];
  const uint32_t j = blockIdx.x * kSampleThreads + threadIdx.x;
  if (j >= J.n) return;
  const uint32_t d = (uint32_t)J.deg[j];
  if (d > kSegMax) return;
  const uint64_t key = row_key(J.seed, J.stripe_key, j);
  const int t = threadIdx.x;
  for (uint32_t s = 0; s < d; ++s) {
    uint32_t r;
    const uint32_t v = floyd_candidate(key, J.k, d, s, r);
    bool taken = false;
    for (uint32_t q = 0; q < s; ++q) taken |= picks[q][t] == (int32_t)v;
    picks[s][t] = (int32_t)(taken ? r : v);
  }
  for (uint32_t a = 1; a < d; ++a) {
    const int32_t x = picks[a][t];
    uint32_t q = a;
    while (q > 0 && picks[q - 1][t] > x) {
      picks[q][t] = picks[q - 1][t];
      --q;
    }
    picks[q][t] = x;
  }
  int32_t *out = J.col + J.row_ptr[j];
  for (uint32_t s = 0; s < d; ++s) out[s] = picks[s][t];
}

// Rows of more than kSegMax neighbours: a workgroup each.  Thread 0 runs
// Floyd's steps against a k-bit LDS bitmap; the set bits, in order, are the
// sorted row.
__global__ __launch_bounds__(kThreads) void sample_heavy_kernel(DevGraphJob J) {
  extern __shared__ uint32_t bits[];   // ceil(k / 32) words
  __shared__ uint32_t sh[kThreads / 64 + 1];
  const uint32_t j = (uint32_t)J.heavy[blockIdx.x];
  const uint32_t d = (uint32_t)J.deg[j];
  const uint32_t words = (J.k + 31) / 32;
  for (uint32_t w = threadIdx.x; w < words; w += kThreads) bits[w] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint64_t key = row_key(J.seed, J.stripe_key, j);
    for (uint32_t s = 0; s < d; ++s) {
      uint32_t r;
      const uint32_t v = floyd_candidate(key, J.k, d, s, r);
      const bool taken = (bits[v >> 5] >> (v & 31)) & 1u;
      const uint32_t pick = taken ? r : v;
      bits[pick >> 5] |= 1u << (pick & 31);
    }
  }
  __syncthreads();
  int32_t *out = J.col + J.row_ptr[j];
  uint32_t base = 0;
  for (uint32_t w0 = 0; w0 < words; w0 += kThreads) {
    const uint32_t w = w0 + threadIdx.x;
    uint32_t m = w < words ? bits[w] : 0u;
    uint32_t total = 0;
    uint32_t at = base + scan_block<kThreads>((uint32_t)__popc(m), sh, total);
    while (m) {
      const uint32_t bit = (uint32_t)__ffs(m) - 1;
      out[at++] = (int32_t)(w * 32 + bit);
      m &= m - 1;
    }
    base += total;
  }
}

// ---------------------------------------------------------------------------
// transpose
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void col_count_kernel(DevGraphJob J) {
  const uint32_t j = blockIdx.x * 256u + threadIdx.x;
  if (j >= J.n) return;
  for (int32_t e = J.row_ptr[j]; e < J.row_ptr[j + 1]; ++e) atomicAdd(&J.ccnt[J.col[e]], 1);
}

__global__ __launch_bounds__(256) void col_fill_kernel(DevGraphJob J) {
  const uint32_t j = blockIdx.x * 256u + threadIdx.x;
  if (j >= J.n) return;
  for (int32_t e = J.row_ptr[j]; e < J.row_ptr[j + 1]; ++e) {
    const int32_t i = J.col[e];
    const int32_t at = atomicAdd(&J.cfill[i], 1);
    J.rowidx[J.col_ptr[i] + at] = (int32_t)j;
  }
}

// rows of one column ascending (insertion sort), and the largest column
__global__ __launch_bounds__(256) void col_sort_kernel(DevGraphJob J) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= J.k) return;
  int32_t *r = J.rowidx + J.col_ptr[i];
  const int32_t c = J.col_ptr[i + 1] - J.col_ptr[i];
  for (int32_t a = 1; a < c; ++a) {
    const int32_t x = r[a];
    int32_t q = a;
    while (q > 0 && r[q - 1] > x) {
      r[q] = r[q - 1];
      --q;
    }
    r[q] = x;
  }
  atomicMax(J.scalars + kScalarMaxCdeg, c);
}

fs_status hip_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

fs_status scan_launch(const int32_t *in, uint32_t m, uint32_t *sums, int32_t *out, hipStream_t s) {
  const uint32_t per = kThreads * kScanItems;
  const uint32_t nb = std::max<uint32_t>(1, (m + per - 1) / per);
  hipLaunchKernelGGL(scan_partial_kernel, dim3(nb), dim3(kThreads), 0, s, in, m, sums);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kThreads), 0, s, sums, nb, (int32_t *)nullptr);
  hipLaunchKernelGGL(scan_final_kernel, dim3(nb), dim3(kThreads), 0, s, in, m, sums, out);
  return hip_ok(hipGetLastError(), "graph scan launch");
}

}  // namespace

void dev_graph_carve(Carver &cv, DevGraphJob &J, uint32_t k, uint32_t n, uint32_t D) {
  const uint32_t nblk = (n + kThreads - 1) / kThreads;
  const uint32_t per = kThreads * kScanItems;
  J.T = cv.take<uint64_t>(D);
  J.deg = cv.take<int32_t>(n);
  J.row_ptr = cv.take<int32_t>((size_t)n + 1);
  J.blk_hist = cv.take<uint32_t>((size_t)nblk * (kSegMax + 1));
  J.scalars = cv.take<int32_t>(kScalarCount);
  J.edges = cv.take<unsigned long long>(1);
  J.sums = cv.take<uint32_t>((std::max(n, k) + per - 1) / per + 1);
  J.ccnt = cv.take<int32_t>(k);
  J.cfill = cv.take<int32_t>(k);
}

void dev_graph_carve_rows(Carver &cv, DevGraphJob &J, uint32_t k, uint32_t n, uint32_t nseg) {
  const uint32_t per = kThreads * kScanItems;
  J.seg_len = cv.take<int32_t>(nseg);
  J.seg_beg = cv.take<int32_t>(nseg);
  J.sums = cv.take<uint32_t>((std::max(std::max(n, k), nseg) + per - 1) / per + 1);
}

fs_status launch_dev_graph_degrees(const DevGraphJob &J, hipStream_t s) {
  if (J.n == 0) return FS_OK;
  hipLaunchKernelGGL(degree_kernel, dim3((J.n + 255) / 256), dim3(256), 0, s, J);
  // row_ptr (into the image) from the degrees; the last entry is nnz
  fs_status st = scan_launch(J.deg, J.n, J.sums, J.row_ptr, s);
  if (st != FS_OK) return st;
  const uint32_t nblk = (J.n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(seg_count_kernel, dim3(nblk), dim3(kThreads), 0, s, J);
  hipLaunchKernelGGL(seg_scan_kernel, dim3(1), dim3(kThreads), 0, s, J, nblk);
  return hip_ok(hipGetLastError(), "graph degree launch");
}

fs_status launch_dev_graph_rows(const DevGraphJob &J, uint32_t nseg, uint32_t nheavy, hipStream_t s) {
  const uint32_t nblk = (J.n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(seg_place_kernel, dim3(nblk), dim3(kThreads), 0, s, J);
  hipLaunchKernelGGL(sample_light_kernel, dim3((J.n + kSampleThreads - 1) / kSampleThreads), dim3(kSampleThreads),
                     0, s, J);
  if (nheavy) {
    const size_t lds = (size_t)((J.k + 31) / 32) * 4;
    static bool done[64] = {false};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev >= 0 && dev < 64 && !done[dev] && lds > 65536) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&sample_heavy_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                device_info(dev).max_lds_per_block - 1024);
      done[dev] = true;
    }
    hipLaunchKernelGGL(sample_heavy_kernel, dim3(nheavy), dim3(kThreads), lds, s, J);
  }
  fs_status st = scan_launch(J.seg_len, nseg, J.sums, J.seg_ptr, s);
  if (st != FS_OK) return st;
  if (nseg) hipLaunchKernelGGL(seg_copy_kernel, dim3((nseg + 255) / 256), dim3(256), 0, s, J, nseg);
  st = hip_ok(hipMemsetAsync(J.ccnt, 0, sizeof(int32_t) * J.k, s), "graph clear");
  if (st == FS_OK) st = hip_ok(hipMemsetAsync(J.cfill, 0, sizeof(int32_t) * J.k, s), "graph clear");
  if (st != FS_OK) return st;
  if (J.n) hipLaunchKernelGGL(col_count_kernel, dim3((J.n + 255) / 256), dim3(256), 0, s, J);
  st = scan_launch(J.ccnt, J.k, J.sums, J.col_ptr, s);
  if (st != FS_OK) return st;
  if (J.n) hipLaunchKernelGGL(col_fill_kernel, dim3((J.n + 255) / 256), dim3(256), 0, s, J);
  hipLaunchKernelGGL(col_sort_kernel, dim3((J.k + 255) / 256), dim3(256), 0, s, J);
  return hip_ok(hipGetLastError(), "graph rows launch");
}

}  // namespace fs
