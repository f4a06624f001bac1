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
#include "scan.h"

namespace fs {
namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPurposeGraph = 1;
constexpr int kThreads = 1024;       // rows per block of the counting passes
constexpr int kSampleThreads = 256;  // rows per block of the light sampler

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
// Floyd's steps s0 .. s0 + 63 of a row of degree d, one per lane of a wave
// (live: the step exists), given whether each lane's candidate v was picked
// by an earlier batch (taken).  A lane falls back to its r when v was picked
// before it: by an earlier batch, or by an earlier lane, either as that
// lane's v (then v was picked before whatever that lane did) or as that
// lane's r (only when that lane fell back; r = k - d + s, so the lane is
// found from v).  The first two are independent of the other lanes'
// outcomes; the third is followed to its fixed point, at most one round per
// link of a chain of fallbacks.  Returns the lane's pick.
__device__ __forceinline__ uint32_t floyd_wave(uint32_t v, uint32_t r, bool live, bool taken, uint32_t k,
                                               uint32_t d, uint32_t s0) {
  const int lane = threadIdx.x & 63;
  const int nlive = (int)min(64u, d - s0);
  bool dup = live && taken;
  for (int q = 0; q < nlive - 1; ++q) {
    const uint32_t vq = (uint32_t)__builtin_amdgcn_readlane((int)v, q);
    dup |= live && lane > q && v == vq;
  }
  const int64_t idx = (int64_t)v - ((int64_t)k - (int64_t)d + (int64_t)s0);
  const bool in_range = live && idx >= 0 && idx < lane;
  const uint32_t at = in_range ? (uint32_t)idx : 0u;
  for (;;) {
    const uint64_t mask = __ballot(dup);
    const bool nd = dup || (in_range && ((mask >> at) & 1ull));
    if (__ballot(nd != dup) == 0ull) break;
    dup = nd;
  }
  return dup ? r : v;
}

// Rows of at most kLightMax neighbours: one thread each, the picks in LDS
// (slot-major, so that neighbouring threads use neighbouring banks), the
// membership test by a scan of the picks so far, then an insertion sort.
constexpr uint32_t kLightMax = 16;

__global__ __launch_bounds__(kSampleThreads) void sample_light_kernel(DevGraphJob J) {
  __shared__ int32_t picks[kLightMax][kSampleThreads];
  const uint32_t j = blockIdx.x * kSampleThreads + threadIdx.x;
  if (j >= J.n) return;
  const uint32_t d = (uint32_t)J.deg[j];
  if (d > kLightMax) return;
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

// Rows of kLightMax + 1 .. kSegMax neighbours: one wave each, lane s taking
// Floyd's step s (floyd_wave).  A lane's place in the sorted row is the
// number of picks below its own.
__global__ __launch_bounds__(256) void sample_medium_kernel(DevGraphJob J) {
  const int lane = threadIdx.x & 63;
  const uint32_t j = blockIdx.x * 4u + (threadIdx.x >> 6);
  if (j >= J.n) return;
  const uint32_t d = (uint32_t)J.deg[j];
  if (d <= kLightMax || d > kSegMax) return;
  const uint64_t key = row_key(J.seed, J.stripe_key, j);
  const bool live = (uint32_t)lane < d;
  uint32_t r = 0, v = 0;
  if (live) v = floyd_candidate(key, J.k, d, (uint32_t)lane, r);
  const uint32_t pick = floyd_wave(v, r, live, false, J.k, d, 0);
  uint32_t below = 0;
  for (int q = 0; q < (int)d; ++q) below += (uint32_t)__builtin_amdgcn_readlane((int)pick, q) < pick ? 1u : 0u;
  if (live) J.col[J.row_ptr[j] + below] = (int32_t)pick;
}

// Rows of more than kSegMax neighbours: a workgroup each.  Wave 0 runs
// Floyd's steps against a k-bit LDS bitmap, 64 steps at a time (floyd_wave:
// each lane tests its candidate against the bitmap of earlier batches, then
// against the lanes before it).  A fallback r is never taken (every earlier
// pick is at most the previous step's r).  The set bits, read in order, are
// the sorted row.
__global__ __launch_bounds__(kThreads) void sample_heavy_kernel(DevGraphJob J) {
  extern __shared__ uint32_t bits[];   // ceil(k / 32) words
  __shared__ uint32_t sh[kThreads / 64 + 1];
  const uint32_t j = (uint32_t)J.heavy[blockIdx.x];
  const uint32_t d = (uint32_t)J.deg[j];
  const uint32_t words = (J.k + 31) / 32;
  for (uint32_t w = threadIdx.x; w < words; w += kThreads) bits[w] = 0;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const uint64_t key = row_key(J.seed, J.stripe_key, j);
    for (uint32_t s0 = 0; s0 < d; s0 += 64) {
      const uint32_t s = s0 + lane;
      const bool live = s < d;
      uint32_t r = 0, v = 0;
      if (live) v = floyd_candidate(key, J.k, d, s, r);
      const bool taken = live && ((bits[v >> 5] >> (v & 31)) & 1u);
      const uint32_t pick = floyd_wave(v, r, live, taken, J.k, d, s0);
      if (live) atomicOr(&bits[pick >> 5], 1u << (pick & 31));
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
// One thread per encode segment (at most kSegMax edges), so that a row of
// thousands of neighbours does not serialise its atomics in one thread.
__global__ __launch_bounds__(256) void col_count_kernel(DevGraphJob J, uint32_t nseg) {
  const uint32_t s = blockIdx.x * 256u + threadIdx.x;
  if (s >= nseg) return;
  const int32_t e0 = J.seg_beg[s], e1 = e0 + J.seg_len[s];
  for (int32_t e = e0; e < e1; ++e) atomicAdd(&J.ccnt[J.col[e]], 1);
}

__global__ __launch_bounds__(256) void col_fill_kernel(DevGraphJob J, uint32_t nseg) {
  const uint32_t s = blockIdx.x * 256u + threadIdx.x;
  if (s >= nseg) return;
  const int32_t j = J.seg_row[s];
  const int32_t e0 = J.seg_beg[s], e1 = e0 + J.seg_len[s];
  for (int32_t e = e0; e < e1; ++e) {
    const int32_t i = J.col[e];
    const int32_t at = atomicAdd(&J.cfill[i], 1);
    J.rowidx[J.col_ptr[i] + at] = j;
  }
}

// rows of one column ascending, and the largest column: a column of at most
// 64 rows is sorted in LDS (slot-major), a longer one in place
__global__ __launch_bounds__(256) void col_sort_kernel(DevGraphJob J) {
  __shared__ int32_t buf[64][256];
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= J.k) return;
  const int t = threadIdx.x;
  int32_t *r = J.rowidx + J.col_ptr[i];
  const int32_t c = J.col_ptr[i + 1] - J.col_ptr[i];
  atomicMax(J.scalars + kScalarMaxCdeg, c);
  if (c <= 64) {
    for (int32_t a = 0; a < c; ++a) buf[a][t] = r[a];
    for (int32_t a = 1; a < c; ++a) {
      const int32_t x = buf[a][t];
      int32_t q = a;
      while (q > 0 && buf[q - 1][t] > x) {
        buf[q][t] = buf[q - 1][t];
        --q;
      }
      buf[q][t] = x;
    }
    for (int32_t a = 0; a < c; ++a) r[a] = buf[a][t];
    return;
  }
  for (int32_t a = 1; a < c; ++a) {
    const int32_t x = r[a];
    int32_t q = a;
    while (q > 0 && r[q - 1] > x) {
      r[q] = r[q - 1];
      --q;
    }
    r[q] = x;
  }
}

fs_status hip_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

void dev_graph_carve(Carver &cv, DevGraphJob &J, uint32_t k, uint32_t n, uint32_t D) {
  const uint32_t nblk = (n + kThreads - 1) / kThreads;
  J.T = cv.take<uint64_t>(D);
  J.deg = cv.take<int32_t>(n);
  J.row_ptr = cv.take<int32_t>((size_t)n + 1);
  J.blk_hist = cv.take<uint32_t>((size_t)nblk * (kSegMax + 1));
  J.scalars = cv.take<int32_t>(kScalarCount);
  J.edges = cv.take<unsigned long long>(1);
  J.sums = cv.take<uint32_t>(scan_sums_for(std::max(n, k)) + 1);
  J.ccnt = cv.take<int32_t>(k);
  J.cfill = cv.take<int32_t>(k);
}

void dev_graph_carve_rows(Carver &cv, DevGraphJob &J, uint32_t k, uint32_t n, uint32_t nseg) {
  J.seg_len = cv.take<int32_t>(nseg);
  J.seg_beg = cv.take<int32_t>(nseg);
  J.sums = cv.take<uint32_t>(scan_sums_for(std::max(std::max(n, k), nseg)) + 1);
}

fs_status launch_dev_graph_degrees(const DevGraphJob &J, hipStream_t s) {
  if (J.n == 0) return FS_OK;
  hipLaunchKernelGGL(degree_kernel, dim3((J.n + 255) / 256), dim3(256), 0, s, J);
  // row_ptr (into the image) from the degrees; the last entry is nnz
  fs_status st = scan_i32(J.deg, J.n, J.sums, J.row_ptr, s);
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
  hipLaunchKernelGGL(sample_medium_kernel, dim3((J.n + 3) / 4), dim3(256), 0, s, J);
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
  fs_status st = scan_i32(J.seg_len, nseg, J.sums, J.seg_ptr, s);
  if (st != FS_OK) return st;
  if (nseg) hipLaunchKernelGGL(seg_copy_kernel, dim3((nseg + 255) / 256), dim3(256), 0, s, J, nseg);
  st = hip_ok(hipMemsetAsync(J.ccnt, 0, sizeof(int32_t) * J.k, s), "graph clear");
  if (st == FS_OK) st = hip_ok(hipMemsetAsync(J.cfill, 0, sizeof(int32_t) * J.k, s), "graph clear");
  if (st != FS_OK) return st;
  if (nseg) hipLaunchKernelGGL(col_count_kernel, dim3((nseg + 255) / 256), dim3(256), 0, s, J, nseg);
  st = scan_i32(J.ccnt, J.k, J.sums, J.col_ptr, s);
  if (st != FS_OK) return st;
  if (nseg) hipLaunchKernelGGL(col_fill_kernel, dim3((nseg + 255) / 256), dim3(256), 0, s, J, nseg);
  hipLaunchKernelGGL(col_sort_kernel, dim3((J.k + 255) / 256), dim3(256), 0, s, J);
  return hip_ok(hipGetLastError(), "graph rows launch");
}

}  // namespace fs
