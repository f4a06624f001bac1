// HIP kernels of libfs for gfx950 (CDNA4, wave64).
//
//   gather_kernel   out[r] = (out[r] ^) XOR_{e in row r} src[idx[e]]  - encode,
//                   repair, and the delta pass of update.  Items are (byte
//                   slice, tile of rows), slice-major; each lane moves 16-byte
//                   chunks, so a row's lanes read contiguous bytes of each
//                   neighbour block.  Workgroup ids are renumbered so that each
//                   XCD walks a contiguous range of slices: the k x W bytes of
//                   one slice of every input block then stay in that XCD's L2
//                   while all rows of the slice gather from it.
//   peel_kernel     one workgroup per stripe; level-synchronous peeling with
//                   a worklist frontier; state in LDS when it fits.
//   replay_kernel   one workgroup per byte slice owns the slice through every
//                   level of the schedule (a barrier between levels).
//   small planning kernels for repair and update.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "fs_internal.h"
#include "scan.h"

namespace fs {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

namespace {

constexpr int kPlanThreads = 1024;

__device__ __forceinline__ v4u ld16(const uint8_t *p) { return *reinterpret_cast<const v4u *>(p); }

// a load of data read once (marked to leave the caches first)
__device__ __forceinline__ v4u ld16_once(const uint8_t *p) {
  return __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));
}

template <bool NT>
__device__ __forceinline__ void st16(uint8_t *p, v4u v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, reinterpret_cast<v4u *>(p));
  else
    *reinterpret_cast<v4u *>(p) = v;
}

// Workgroups are dispatched round-robin over the 8 XCDs (id % 8).  Renumber
// so that XCD x owns the contiguous virtual ids [start_x, start_x + count_x).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nwg) {
  const uint32_t xcd = b & 7u, local = b >> 3;
  const uint32_t per = nwg >> 3, rem = nwg & 7u;
  return xcd * per + min(xcd, rem) + local;
}

// Block-wide exclusive scan of one uint32 per thread.  sh needs NT/64 + 1
// words.  Every thread must call it.
template <int NT>
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
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
// gather-XOR
// ---------------------------------------------------------------------------
constexpr int kGatherThreads = 256;
constexpr int kStageCap = 2048;   // edges of one row tile staged in LDS

// XOR of the sources of one row into acc.  Neighbour ids come from idx (LDS
// when the tile's edge list was staged, else global); loads are issued in
// batches of U = 4 neighbours x CH chunks before any is consumed.  (Eight
// neighbours in flight measured 5-10 % slower for one and two chunks on
// finite-degree and Robust Soliton stripes: the extra loads in flight
// thrash the L2 more than they hide latency.)
template <int CH, uint32_t STEP, class IdxPtr>
__device__ __forceinline__ void gather_row(v4u (&acc)[CH], const bool (&valid)[CH], IdxPtr idx, int e,
                                           const int e1, const uint8_t *src, const uint64_t stride) {
  constexpr int U = 4;
  const v4u zero = {0u, 0u, 0u, 0u};
  for (; e < e1; e += U) {
    const int cnt = e1 - e;
    const uint8_t *p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) p[u] = src + (uint64_t)(u < cnt ? idx[e + u] : 0) * stride;
    v4u v[U][CH];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < CH; ++c) v[u][c] = (valid[c] && u < cnt) ? ld16(p[u] + c * STEP) : zero;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      v4u x = v[0][c];
#pragma unroll
      for (int u = 1; u < U; ++u) x ^= v[u][c];
      acc[c] ^= x;
    }
  }
}

// One (slice, tile) item of a gather job.  All threads of the workgroup call
// it with the same arguments (it contains barriers).  ntiles is the tile
// count the item index was decomposed with, nrows the live row count.
template <int LPR, int CH, bool NT>
__device__ __forceinline__ void gather_item(const GatherJob &j, uint32_t nrows, uint32_t ntiles, uint64_t item,
                                            int32_t *s_ptr, int32_t *s_idx) {
  constexpr uint32_t RPB = kGatherThreads / LPR;   // rows per tile
  constexpr uint32_t STEP = LPR * 16;              // bytes between a lane's chunks
  constexpr uint32_t W = STEP * CH;                // slice bytes
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid % LPR;
  const uint32_t sub = tid / LPR;
  const bool contiguous = j.csr_map == nullptr;
  // tiles of one slice are consecutive items, so neighbouring workgroups share a slice
  const uint32_t slice = (uint32_t)(item / ntiles);
  const uint32_t tile = (uint32_t)(item % ntiles);
  const uint32_t r0 = tile * RPB;
  if (r0 >= nrows) return;
  const uint32_t r = r0 + sub;
  // stage the tile's edge list (rows r0 .. r0+RPB-1 are contiguous in CSR)
  bool staged = false;
  if (contiguous) {
    const uint32_t rend = min(r0 + RPB, nrows);
    const int ebase = j.ptr[r0];
    const int ecount = j.ptr[rend] - ebase;
    staged = ecount <= kStageCap;
    __syncthreads();   // the previous item's readers are done with the LDS copy
    if (staged) {
      for (int i = (int)tid; i < ecount; i += kGatherThreads) s_idx[i] = j.idx[ebase + i];
      for (uint32_t i = tid; i <= rend - r0; i += kGatherThreads) s_ptr[i] = j.ptr[r0 + i] - ebase;
    }
    __syncthreads();
  }
  if (r >= nrows) return;
  const uint32_t jr = contiguous ? r : j.csr_map[r];
  if (jr >= j.csr_rows) return;
  const uint32_t ob = j.out_map ? (uint32_t)j.out_map[r] : jr;
  const uint64_t off0 = (uint64_t)slice * W + lane * 16u;
  uint8_t *out = j.dst + (uint64_t)ob * j.dst_stride + off0;
  bool valid[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) valid[c] = off0 + (uint64_t)c * STEP < j.t;
  v4u acc[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) acc[c] = v4u{0u, 0u, 0u, 0u};
  if (j.row_ok && j.row_ok[r] == 0) {
#pragma unroll
    for (int c = 0; c < CH; ++c)
      if (valid[c]) st16<NT>(out + c * STEP, acc[c]);
    return;
  }
  if (j.accumulate) {
#pragma unroll
    for (int c = 0; c < CH; ++c)
      if (valid[c]) acc[c] = ld16(out + c * STEP);
  }
  const uint8_t *src = j.src + off0;
  if (staged)
    gather_row<CH, STEP>(acc, valid, s_idx, s_ptr[sub], s_ptr[sub + 1], src, j.src_stride);
  else
    gather_row<CH, STEP>(acc, valid, j.idx, j.ptr[jr], j.ptr[jr + 1], src, j.src_stride);
  if (j.seg_atomic && j.seg_atomic[r]) {
    // one of several segments of a long row: XOR into the zeroed row
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (!valid[c]) continue;
      unsigned long long *q = reinterpret_cast<unsigned long long *>(out + c * STEP);
      atomicXor(q, ((unsigned long long)acc[c].y << 32) | acc[c].x);
      atomicXor(q + 1, ((unsigned long long)acc[c].w << 32) | acc[c].z);
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < CH; ++c)
    if (valid[c]) st16<NT>(out + c * STEP, acc[c]);
}

__device__ __forceinline__ uint32_t live_rows(const GatherJob &j) {
  uint32_t nrows = j.nrows;
  if (j.nrows_dev) nrows = min(nrows, (uint32_t)max(*j.nrows_dev, 0));
  return nrows;
}

template <int LPR, int CH, bool NT>
__global__ __launch_bounds__(kGatherThreads) void gather_kernel(GatherJob j, uint32_t nslices,
                                                                 uint32_t remap) {
  constexpr uint32_t RPB = kGatherThreads / LPR;
  __shared__ int32_t s_ptr[RPB + 1];
  __shared__ int32_t s_idx[kStageCap];
  if (j.skip_flag && *j.skip_flag) return;
  const uint32_t nrows = live_rows(j);
  const uint32_t ntiles = (nrows + RPB - 1) / RPB;
  const uint64_t nitems = (uint64_t)ntiles * nslices;
  const uint32_t vb = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  for (uint64_t item = vb; item < nitems; item += gridDim.x)
    gather_item<LPR, CH, NT>(j, nrows, ntiles, item, s_ptr, s_idx);
}

// Persistent gather over the items of many jobs (a batch): the item space is
// the concatenation of every job's (slice, tile) items (prefix[] holds the
// running counts, computed with each job's row-count bound).  It is cut into
// 8 contiguous partitions, one per XCD, each with its own counter: the
// workgroups of an XCD (hardware places workgroup b on XCD b % 8) claim small
// chunks of consecutive items from their partition, so the items in flight on
// an XCD stay close together (same job, same slice: the slice's input slab
// stays in that XCD's L2) while uneven stripes still balance dynamically.  A
// workgroup whose partition is used up moves on to the next partitions.
// counters[x * kCounterStride] must start at the first item of partition x
// (reset kernel); each counter has a 256-byte line of its own, so the claims
// of different XCDs do not queue on one L2 channel.
constexpr uint32_t kXcds = 8;

template <int LPR, int CH, bool NT>
__global__ __launch_bounds__(kGatherThreads) void gather_batch_kernel(const GatherJob *jobs,
                                                                       const unsigned long long *prefix,
                                                                       uint32_t njobs,
                                                                       unsigned long long *counters,
                                                                       uint32_t chunk) {
  constexpr uint32_t RPB = kGatherThreads / LPR;
  __shared__ int32_t s_ptr[RPB + 1];
  __shared__ int32_t s_idx[kStageCap];
  __shared__ unsigned long long s_next;
  const unsigned long long total = prefix[njobs];
  uint32_t jb = 0, jcur = 0xffffffffu;
  GatherJob j{};
  uint32_t nrows = 0, ntiles = 1;
  bool skip = false;
  for (uint32_t pass = 0; pass < kXcds; ++pass) {
    const uint32_t part = (blockIdx.x + pass) % kXcds;
    const unsigned long long hi = total * (part + 1) / kXcds;
    for (;;) {
      __syncthreads();   // everyone has read s_next
      if (threadIdx.x == 0) s_next = atomicAdd(&counters[part * kCounterStride], (unsigned long long)chunk);
      __syncthreads();
      const unsigned long long base = s_next;
      if (base >= hi) break;
      const unsigned long long end = min(base + chunk, hi);
      for (unsigned long long item = base; item < end; ++item) {
        if (jcur == 0xffffffffu || item < prefix[jb]) {
          uint32_t lo = 0, hj = njobs;
          while (hj - lo > 1) {
            const uint32_t mid = (lo + hj) / 2;
            if (prefix[mid] <= item) lo = mid; else hj = mid;
          }
          jb = lo;
        }
        while (jb + 1 < njobs && prefix[jb + 1] <= item) ++jb;
        if (jb != jcur) {
          j = jobs[jb];
          jcur = jb;
          skip = j.skip_flag && *j.skip_flag;
          nrows = live_rows(j);
          ntiles = (nrows + RPB - 1) / RPB;   // live rows, as batch_start_kernel counted them
        }
        if (!skip) gather_item<LPR, CH, NT>(j, nrows, ntiles, item - prefix[jb], s_ptr, s_idx);
      }
    }
  }
}

// Start of a batched gather (a kernel, so it can sit in a graph): every
// job's (slice, tile) item count from its live rows (jobs sized on the
// device count only their live tiles; skipped jobs none) into prefix, then
// partition x's counter at total * x / 8.  One workgroup, 1024 jobs a pass.
__global__ __launch_bounds__(1024) void batch_start_kernel(const GatherJob *jobs, unsigned long long *prefix,
                                                          uint32_t njobs, unsigned long long *counters, uint32_t rpb,
                                                          uint32_t w) {
  __shared__ unsigned long long wsum[16];
  __shared__ unsigned long long s_carry;
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (threadIdx.x == 0) {
    s_carry = 0;
    prefix[0] = 0;
  }
  __syncthreads();
  for (uint32_t b0 = 0; b0 < njobs; b0 += 1024) {
    const uint32_t i = b0 + threadIdx.x;
    unsigned long long v = 0;
    if (i < njobs) {
      const GatherJob &j = jobs[i];
      uint32_t rows = live_rows(j);
      if (j.skip_flag && *j.skip_flag) rows = 0;
      v = (unsigned long long)((j.t + w - 1) / w) * ((rows + rpb - 1) / rpb);
    }
    unsigned long long x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long y = __shfl_up(x, o, 64);
      if ((int)lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long run = s_carry;
      for (int q = 0; q < 16; ++q) {
        const unsigned long long t = wsum[q];
        wsum[q] = run;
        run += t;
      }
      s_carry = run;
    }
    __syncthreads();
    if (i < njobs) prefix[i + 1] = wsum[wid] + x;
    __syncthreads();
  }
  if (threadIdx.x < kXcds) counters[threadIdx.x * kCounterStride] = prefix[njobs] * threadIdx.x / kXcds;
}

__global__ __launch_bounds__(256) void zero_rows_kernel(uint8_t *dst, const int32_t *rows, uint32_t nrows,
                                                        uint64_t t, uint32_t chunks) {
  const uint32_t r = blockIdx.x / chunks, ch = blockIdx.x % chunks;
  if (r >= nrows) return;
  const uint64_t off = (uint64_t)ch * 4096 + threadIdx.x * 16u;
  if (off < t) *reinterpret_cast<v4u *>(dst + (uint64_t)rows[r] * t + off) = v4u{0u, 0u, 0u, 0u};
}

// ---------------------------------------------------------------------------
// LDS-slab encode
// ---------------------------------------------------------------------------
// One workgroup per CU walks byte slices of W = 16 LPS bytes.  For each slice
// the k x W bytes of every input block are copied into LDS once; every encode
// segment then XORs its neighbours from LDS and writes its part of the slice.
// The gather reads a neighbour through the caches once per edge; here each
// input byte is read from memory once per slice and the edges read LDS.  The
// next slice's inputs are loaded into registers while the current one is
// computed.  k LPS <= kSlabEntries, so every thread holds at most M entries.
constexpr int kSlabThreads = 1024;
constexpr uint32_t kSlabEntries = 8192;                  // 16-byte entries: 128 KiB
constexpr int kSlabPerThread = kSlabEntries / kSlabThreads;

template <int LPS>
__global__ __launch_bounds__(kSlabThreads) void slab_encode_kernel(GatherJob j, uint32_t k, uint32_t nslices) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  v4u *slab = reinterpret_cast<v4u *>(smem);
  constexpr uint32_t NS = kSlabThreads / LPS;
  constexpr uint32_t W = 16u * LPS;
  constexpr int M = kSlabPerThread;
  const uint32_t lane = threadIdx.x % LPS, grp = threadIdx.x / LPS;
  const uint32_t nseg = j.nrows;
  const v4u zero = {0u, 0u, 0u, 0u};
  v4u pre[M];
  auto issue = [&](uint32_t slice) {
    const uint64_t off = (uint64_t)slice * W + lane * 16u;
    const bool live = off < j.t;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const uint32_t i = grp + (uint32_t)m * NS;
      pre[m] = (live && i < k) ? ld16(j.src + (uint64_t)i * j.src_stride + off) : zero;
    }
  };
  uint32_t slice = xcd_remap(blockIdx.x, gridDim.x);
  if (slice < nslices) issue(slice);
  while (slice < nslices) {
    const uint64_t off = (uint64_t)slice * W + lane * 16u;
    const bool live = off < j.t;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const uint32_t i = grp + (uint32_t)m * NS;
      if (i < k) slab[i * LPS + lane] = pre[m];
    }
    __syncthreads();
    const uint32_t next = slice + gridDim.x;
    if (next < nslices) issue(next);
    if (live) {
      for (uint32_t r = grp; r < nseg; r += NS) {
        const int e1 = j.ptr[r + 1];
        int e = j.ptr[r];
        v4u acc = zero;
        for (; e + 4 <= e1; e += 4) {
          const uint32_t a = (uint32_t)j.idx[e], b = (uint32_t)j.idx[e + 1];
          const uint32_t c = (uint32_t)j.idx[e + 2], d = (uint32_t)j.idx[e + 3];
          acc ^= (slab[a * LPS + lane] ^ slab[b * LPS + lane]) ^ (slab[c * LPS + lane] ^ slab[d * LPS + lane]);
        }
        for (; e < e1; ++e) acc ^= slab[(uint32_t)j.idx[e] * LPS + lane];
        uint8_t *out = j.dst + (uint64_t)j.out_map[r] * j.dst_stride + off;
        if (j.seg_atomic && j.seg_atomic[r]) {
          unsigned long long *q = reinterpret_cast<unsigned long long *>(out);
          atomicXor(q, ((unsigned long long)acc.y << 32) | acc.x);
          atomicXor(q + 1, ((unsigned long long)acc.w << 32) | acc.z);
        } else {
          // plain stores: the slices of one 128-byte line are written by
          // neighbouring workgroups of one XCD and merge in its L2
          *reinterpret_cast<v4u *>(out) = acc;
        }
      }
    }
    __syncthreads();   // the slab is rewritten for the next slice
    slice = next;
  }
}

// Lanes per slab row for k inputs (0: the slab does not apply).  Slices
// narrower than 256 bytes (k > 512) read memory in pieces too short to
// keep up with the gather, which wins there (the finite-degree k = 4096
// stripe: 0.25 ms with 32-byte slices against 0.157 ms for the gather).
int slab_lanes(uint32_t k) {
  for (int lps = 64; lps >= 16; lps /= 2)
    if ((uint64_t)k * lps <= kSlabEntries) return lps;
  return 0;
}

template <int LPS>
hipError_t run_slab_encode(const GatherJob &j, uint32_t nslices, int grid, int dev, hipStream_t s) {
  static bool done[64] = {false};
  const int bytes = (int)(kSlabEntries * 16);
  if (dev >= 0 && dev < 64 && !done[dev]) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&slab_encode_kernel<LPS>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    done[dev] = true;
  }
  hipLaunchKernelGGL(slab_encode_kernel<LPS>, dim3(grid), dim3(kSlabThreads), bytes, s, j, j.slab_k, nslices);
  return hipGetLastError();
}

// The slab encode for an encode job when it applies: k fits the slab and
// the slices are enough to give every CU one.
bool try_slab_encode(const GatherJob &j, const fs_tune &tune, hipStream_t s, hipError_t &e) {
  if (!tune.encode_slab || j.slab_k == 0 || j.accumulate || j.csr_map || j.nrows_dev || j.row_ok || j.skip_flag)
    return false;
  const int lps = slab_lanes(j.slab_k);
  if (lps == 0) return false;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cu = device_info(dev).cu_count;
  if ((int)device_info(dev).max_lds_per_block < (int)(kSlabEntries * 16)) return false;
  const uint32_t w = 16u * (uint32_t)lps;
  const uint64_t nslices = (j.t + w - 1) / w;
  if (nslices < (uint64_t)cu || nslices > 0xffffffffull) return false;
  const int grid = cu;
  fs_launch_info &rec = launch_record();
  rec.gather_kind = 2;
  rec.gather_lanes_per_row = (uint32_t)lps;
  rec.gather_chunks = 1;
  rec.gather_slice_bytes = w;
  switch (lps) {
    case 64: e = run_slab_encode<64>(j, (uint32_t)nslices, grid, dev, s); break;
    case 32: e = run_slab_encode<32>(j, (uint32_t)nslices, grid, dev, s); break;
    default: e = run_slab_encode<16>(j, (uint32_t)nslices, grid, dev, s); break;
  }
  return true;
}

template <int LPR, int CH, bool NT>
hipError_t run_gather(const GatherJob &j, uint32_t remap, hipStream_t s, int cu_count) {
  constexpr uint32_t RPB = kGatherThreads / LPR;
  constexpr uint32_t W = LPR * 16 * CH;
  const uint32_t nslices = (uint32_t)((j.t + W - 1) / W);
  const uint64_t ntiles = (j.nrows + RPB - 1) / RPB;
  uint64_t nitems = ntiles * nslices;
  // device-sized jobs use a bounded grid that strides over the live items
  const uint64_t cap = j.nrows_dev ? (uint64_t)cu_count * 8 : (uint64_t)1 << 30;
  uint64_t grid = nitems < cap ? nitems : cap;
  fs_launch_info &rec = launch_record();
  rec.gather_kind = 1;
  rec.gather_lanes_per_row = LPR;
  rec.gather_chunks = CH;
  rec.gather_slice_bytes = W;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((gather_kernel<LPR, CH, NT>), dim3((uint32_t)grid), dim3(kGatherThreads), 0, s,
                     j, nslices, remap);
  return hipGetLastError();
}

template <int LPR, int CH>
hipError_t run_gather_nt(const GatherJob &j, const fs_tune &t, hipStream_t s, int cu) {
  return t.nt_store ? run_gather<LPR, CH, true>(j, t.xcd_remap, s, cu)
                    : run_gather<LPR, CH, false>(j, t.xcd_remap, s, cu);
}

// ---------------------------------------------------------------------------
// level-synchronous peeling schedule
// ---------------------------------------------------------------------------
constexpr int kPeelThreads = 1024;
constexpr int kPeelBatch = 8;   // column entries loaded before any is applied
constexpr unsigned long long kCountOne = 1ull << 40;   // acc = count << 40 | sum of ids
constexpr unsigned long long kSumMask = kCountOne - 1;
// Erased rows start with a count far above any degree (2^23): removing all
// their inputs never brings it near 2, so they never enter a frontier and the
// propagation step needs no erasure test.
constexpr unsigned long long kErasedAcc = 1ull << 63;
// The same state packed in 32 bits (count << 24 | sum of ids) when degrees
// are at most 127 and every sum of ids stays below 2^24: erased rows start at
// count 255 and never come down to 128.
constexpr uint32_t kCountOne32 = 1u << 24;
constexpr uint32_t kSumMask32 = kCountOne32 - 1u;
constexpr uint32_t kErasedAcc32 = 255u << 24;

__device__ __forceinline__ uint32_t words_of(uint32_t k) { return (k + 31) / 32; }

struct PeelState {
  unsigned long long *acc, *best;
  uint32_t *acc32;    // packed row state (kPeelLdsRows32, kPeelLdsRows32B, kPeelLds16)
  uint32_t *best32;   // decoding row per input as degree << 24 | row (kPeelLdsRows32B), else null
  int32_t *fa, *fb, *dl;
  uint16_t *fa16, *fb16, *dl16, *ridx;   // kPeelLds16: 16-bit frontiers, list and column rows
  uint32_t *mask, *decm;
  int32_t *cptr;      // column pointers (LDS copy, or the graph's)
  uint16_t *deg;      // row degrees (LDS variants only)
};

// Wave 0 lists the set bits of mask (one k-bit set) in ascending order: each
// lane owns a contiguous run of words; a wave prefix sum places its ids.
// clear: also clear the words and OR them into decm; flist: list the
// complement of decm instead (the unrecovered inputs).
template <bool FLIST>
__device__ __forceinline__ uint32_t wave0_list(const PeelState &S, const PeelJob &J, uint32_t kw,
                                               uint32_t base) {
  const uint32_t lane = threadIdx.x;   // caller guarantees wave 0
  const uint32_t wpl = (kw + 63) / 64;
  const uint32_t w0 = min(kw, lane * wpl), w1 = min(kw, w0 + wpl);
  const uint32_t k = J.k;
  uint32_t cnt = 0;
  for (uint32_t w = w0; w < w1; ++w) {
    uint32_t m = FLIST ? ~S.decm[w] : S.mask[w];
    if (FLIST && w == kw - 1 && (k & 31)) m &= (1u << (k & 31)) - 1u;
    cnt += __popc(m);
  }
  uint32_t incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if ((int)lane >= o) incl += y;
  }
  const uint32_t total = __shfl(incl, 63, 64);
  uint32_t pos = base + incl - cnt;
  for (uint32_t w = w0; w < w1; ++w) {
    uint32_t m;
    if (FLIST) {
      m = ~S.decm[w];
      if (w == kw - 1 && (k & 31)) m &= (1u << (k & 31)) - 1u;
    } else {
      m = S.mask[w];
      if (!m) continue;
      S.mask[w] = 0;
      S.decm[w] |= m;
    }
    while (m) {
      const uint32_t f = w * 32 + __builtin_ctz(m);
      J.dp_f[pos] = (int32_t)f;
      if (FLIST) {
        J.dp_g[pos] = -1;
      } else {
        J.dp_g[pos] = S.best32 ? (int32_t)(S.best32[f] & 0xffffffu) : (int32_t)(uint32_t)(S.best[f] & 0xffffffffull);
        J.recovered[f] = 1;
      }
      ++pos;
      m &= m - 1;
    }
  }
  return total;
}

// Where the peel keeps its state: kPeelLds all of it in LDS, kPeelLdsRows
// only the per-row counters (the one array every edge updates atomically;
// for stripes whose full state does not fit), kPeelLdsRows32 the counters
// packed in 32 bits (for stripes whose 64-bit counters do not fit either),
// kPeelGlobal none of it.  kPeelLdsRows32B keeps, beside the packed
// counters, the decoding row of each input (32 bits: degree << 24 | row) and
// the input masks in LDS, so that a level's atomics stay on the CU (for
// stripes too large for kPeelLds16, such as the k = 10246 code).
// kPeelLds16 keeps everything in LDS in compact form (k, n <= 65535, degrees
// <= 127): packed 32-bit counters, 16-bit frontiers and input list, and the
// graph's column lists as 16-bit row ids, so a level touches no global
// memory but the schedule it writes.
constexpr int kPeelGlobal = 0, kPeelLdsRows = 1, kPeelLds = 2, kPeelLdsRows32 = 3, kPeelLds16 = 4,
              kPeelLdsRows32B = 5;

// LDS of kPeelLdsRows32B: counters (n), best rows (k), input masks (2 x k bits)
__host__ __device__ inline size_t peel_rows32b_bytes(uint32_t k, uint32_t n) {
  return 4ull * n + 4ull * k + 8ull * ((k + 31) / 32);
}

__host__ __device__ inline size_t peel_lds16_bytes(uint32_t k, uint32_t n, uint64_t nnz) {
  const size_t kw = (k + 31) / 32;
  size_t b = 8ull * k;                                  // best
  b += 4ull * n + 8ull * kw + 4ull * (k + 1);           // acc32, mask, decm, cptr
  b += 2ull * n + 2ull * n + 2ull * k + 2ull * n;       // fa16, fb16, dl16, deg
  return b + 2ull * nnz;                                // ridx
}

template <int MODE>
__device__ __forceinline__ void peel_body(const PeelJob &J) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int s_nA, s_nB, s_nD;
  if (J.skip_flag && *J.skip_flag) return;
  const uint32_t k = J.k, n = J.n, kw = words_of(k);
  const int tid = threadIdx.x;
  const int wid = tid >> 6;
  constexpr bool PACKED = MODE == kPeelLdsRows32 || MODE == kPeelLds16 || MODE == kPeelLdsRows32B;   // 32-bit counters
  constexpr bool BEST32 = MODE == kPeelLdsRows32B;                         // 32-bit best rows in LDS
  constexpr bool ALL = MODE == kPeelLds || MODE == kPeelLds16;             // degrees, column pointers in LDS
  constexpr bool SHORT = MODE == kPeelLds16;                               // 16-bit lists
  PeelState S;
  if constexpr (MODE == kPeelLds16) {
    unsigned char *p = smem;
    S.best = reinterpret_cast<unsigned long long *>(p); p += 8ull * k;
    S.acc32 = reinterpret_cast<uint32_t *>(p); p += 4ull * n;
    S.mask = reinterpret_cast<uint32_t *>(p); p += 4ull * kw;
    S.decm = reinterpret_cast<uint32_t *>(p); p += 4ull * kw;
    S.cptr = reinterpret_cast<int32_t *>(p); p += 4ull * (k + 1);
    S.fa16 = reinterpret_cast<uint16_t *>(p); p += 2ull * n;
    S.fb16 = reinterpret_cast<uint16_t *>(p); p += 2ull * n;
    S.dl16 = reinterpret_cast<uint16_t *>(p); p += 2ull * k;
    S.deg = reinterpret_cast<uint16_t *>(p); p += 2ull * n;
    S.ridx = reinterpret_cast<uint16_t *>(p);
    S.acc = nullptr; S.fa = S.fb = S.dl = nullptr;
    S.best32 = nullptr;
  } else if constexpr (MODE == kPeelLdsRows32B) {
    unsigned char *p = smem;
    S.acc32 = reinterpret_cast<uint32_t *>(p); p += 4ull * n;
    S.best32 = reinterpret_cast<uint32_t *>(p); p += 4ull * k;
    S.mask = reinterpret_cast<uint32_t *>(p); p += 4ull * kw;
    S.decm = reinterpret_cast<uint32_t *>(p);
    S.acc = nullptr; S.best = nullptr;
    S.fa = J.front_a; S.fb = J.front_b; S.dl = J.dlist;
    S.fa16 = S.fb16 = S.dl16 = S.ridx = nullptr;
    S.cptr = const_cast<int32_t *>(J.col_ptr);
    S.deg = nullptr;
  } else if constexpr (MODE == kPeelLds) {
    unsigned char *p = smem;
    S.acc = reinterpret_cast<unsigned long long *>(p); p += 8ull * n;
    S.best = reinterpret_cast<unsigned long long *>(p); p += 8ull * k;
    S.fa = reinterpret_cast<int32_t *>(p); p += 4ull * n;
    S.fb = reinterpret_cast<int32_t *>(p); p += 4ull * n;
    S.dl = reinterpret_cast<int32_t *>(p); p += 4ull * k;
    S.mask = reinterpret_cast<uint32_t *>(p); p += 4ull * kw;
    S.decm = reinterpret_cast<uint32_t *>(p); p += 4ull * kw;
    S.cptr = reinterpret_cast<int32_t *>(p); p += 4ull * (k + 1);
    S.deg = reinterpret_cast<uint16_t *>(p);
    S.best32 = nullptr;
  } else {
    S.acc = MODE == kPeelLdsRows ? reinterpret_cast<unsigned long long *>(smem) : J.acc;
    S.acc32 = MODE == kPeelLdsRows32 ? reinterpret_cast<uint32_t *>(smem) : nullptr;
    S.best = J.best; S.fa = J.front_a; S.fb = J.front_b; S.dl = J.dlist;
    S.mask = J.mask; S.decm = J.decmask;
    S.cptr = const_cast<int32_t *>(J.col_ptr);
    S.deg = nullptr;
    S.best32 = nullptr;
  }
  for (uint32_t f = tid; f < k; f += kPeelThreads) {
    if constexpr (BEST32)
      S.best32[f] = ~0u;
    else
      S.best[f] = ~0ull;
    J.recovered[f] = 0;
  }
  for (uint32_t w = tid; w < kw; w += kPeelThreads) {
    S.mask[w] = 0;
    S.decm[w] = 0;
  }
  if constexpr (ALL) {
    for (uint32_t i = tid; i <= k; i += kPeelThreads) S.cptr[i] = J.col_ptr[i];
  }
  if constexpr (SHORT) {
    for (uint64_t e = tid; e < J.nnz; e += kPeelThreads) S.ridx[e] = (uint16_t)J.rowidx[e];
  }
  if (tid == 0) {
    s_nA = 0;
    s_nB = 0;
    s_nD = 0;
    J.level_ptr[0] = 0;
  }
  __syncthreads();
  if (!ALL && J.acc_ready) {
    // the row states were made by the init kernels: take them over (packed
    // when the counters are 32-bit) and list the rows of one unknown
    for (uint32_t g = tid; g < n; g += kPeelThreads) {
      const unsigned long long a0 = J.acc[g];
      const bool erased_row = (a0 & kErasedAcc) != 0;
      if constexpr (PACKED)
        S.acc32[g] = erased_row ? (kErasedAcc32 + (uint32_t)(a0 & kSumMask32))
                                : ((uint32_t)(a0 >> 40) << 24 | (uint32_t)(a0 & kSumMask32));
      else if constexpr (MODE == kPeelLdsRows)
        S.acc[g] = a0;
      if (!erased_row && (a0 >> 40) == 1ull) S.fa[atomicAdd(&s_nA, 1)] = (int32_t)g;
    }
  }
  for (uint32_t g = tid; g < n && !(!ALL && J.acc_ready); g += kPeelThreads) {
    const int d = J.row_ptr[g + 1] - J.row_ptr[g];
    if constexpr (ALL) S.deg[g] = (uint16_t)d;
    if (J.erased[g]) {
      if constexpr (PACKED)
        S.acc32[g] = kErasedAcc32;
      else
        S.acc[g] = kErasedAcc;
      continue;
    }
    if constexpr (PACKED)
      S.acc32[g] = (uint32_t)d << 24;
    else
      S.acc[g] = (unsigned long long)d << 40;
    if (d == 1) {
      if constexpr (SHORT)
        S.fa16[atomicAdd(&s_nA, 1)] = (uint16_t)g;
      else
        S.fa[atomicAdd(&s_nA, 1)] = (int32_t)g;
    }
  }
  __syncthreads();
  // sums of neighbour ids, accumulated by input over the CSC: the work per
  // thread follows the column degrees, which stay small even when a few rows
  // have huge degree
  for (uint32_t i = tid; i < k && !(!ALL && J.acc_ready); i += kPeelThreads) {
    const int c1 = S.cptr[i + 1];
    for (int e = S.cptr[i]; e < c1; e += kPeelBatch) {
      int32_t h[kPeelBatch];
#pragma unroll
      for (int u = 0; u < kPeelBatch; ++u) {
        if constexpr (SHORT)
          h[u] = e + u < c1 ? (int32_t)S.ridx[e + u] : -1;
        else
          h[u] = e + u < c1 ? J.rowidx[e + u] : -1;
      }
#pragma unroll
      for (int u = 0; u < kPeelBatch; ++u) {
        if (h[u] < 0) continue;
        if constexpr (PACKED)
          atomicAdd(&S.acc32[h[u]], i);
        else
          atomicAdd(&S.acc[h[u]], (unsigned long long)i);
      }
    }
  }
  __syncthreads();

  int32_t *cur = S.fa, *nxt = S.fb;
  uint16_t *cur16 = S.fa16, *nxt16 = S.fb16;
  uint32_t level = 0, npairs = 0;
  while (true) {
    const int nA = s_nA;
    if (nA == 0 || (J.maxit != 0 && level == J.maxit)) break;
    // every surviving row of residual weight 1 names its last unknown input;
    // keep the namer of least (original degree, row)
    for (int q = tid; q < nA; q += kPeelThreads) {
      int32_t g;
      if constexpr (SHORT)
        g = (int32_t)cur16[q];
      else
        g = cur[q];
      uint32_t f;
      if constexpr (PACKED) {
        const uint32_t a = S.acc32[g];
        if ((a >> 24) != 1u) continue;
        f = a & kSumMask32;
      } else {
        const unsigned long long a = S.acc[g];
        if ((a >> 40) != 1ull) continue;
        f = (uint32_t)(a & kSumMask);
      }
      uint32_t d;
      if constexpr (ALL)
        d = S.deg[g];
      else
        d = (uint32_t)(J.row_ptr[g + 1] - J.row_ptr[g]);
      if constexpr (BEST32)
        atomicMin(&S.best32[f], (d << 24) | (uint32_t)g);
      else
        atomicMin(&S.best[f], ((unsigned long long)d << 32) | (uint32_t)g);
      const uint32_t bit = 1u << (f & 31);
      const uint32_t old = atomicOr(&S.mask[f >> 5], bit);
      if (!(old & bit)) {
        if constexpr (SHORT)
          S.dl16[atomicAdd(&s_nD, 1)] = (uint16_t)f;
        else
          S.dl[atomicAdd(&s_nD, 1)] = (int32_t)f;
      }
    }
    __syncthreads();
    const int nD = s_nD;
    if (nD == 0) break;
    if (wid == 0) {
      // list the level's inputs in ascending order with their decoding rows
      wave0_list<false>(S, J, kw, npairs);
    } else {
      // remove the decoded inputs from every row they touch; a row whose
      // residual weight drops to 1 joins the next frontier
      for (int q = tid - 64; q < nD; q += kPeelThreads - 64) {
        uint32_t f;
        if constexpr (SHORT)
          f = S.dl16[q];
        else
          f = (uint32_t)S.dl[q];
        const unsigned long long dec = 0ull - (kCountOne | f);
        const uint32_t dec32 = 0u - (kCountOne32 | f);
        const int c1 = S.cptr[f + 1];
        for (int e = S.cptr[f]; e < c1; e += kPeelBatch) {
          // the column's row ids are loaded together, then applied
          int32_t h[kPeelBatch];
#pragma unroll
          for (int u = 0; u < kPeelBatch; ++u) {
            if constexpr (SHORT)
              h[u] = e + u < c1 ? (int32_t)S.ridx[e + u] : -1;
            else
              h[u] = e + u < c1 ? J.rowidx[e + u] : -1;
          }
#pragma unroll
          for (int u = 0; u < kPeelBatch; ++u) {
            if (h[u] < 0) continue;
            bool two;
            if constexpr (PACKED)
              two = (atomicAdd(&S.acc32[h[u]], dec32) >> 24) == 2u;
            else
              two = (atomicAdd(&S.acc[h[u]], dec) >> 40) == 2ull;
            if (two) {
              if constexpr (SHORT)
                nxt16[atomicAdd(&s_nB, 1)] = (uint16_t)h[u];
              else
                nxt[atomicAdd(&s_nB, 1)] = h[u];
            }
          }
        }
      }
    }
    npairs += (uint32_t)nD;
    ++level;
    __syncthreads();
    if (tid == 0) {
      J.level_ptr[level] = (int32_t)npairs;
      s_nA = s_nB;
      s_nB = 0;
      s_nD = 0;
    }
    int32_t *tmp = cur;
    cur = nxt;
    nxt = tmp;
    uint16_t *tmp16 = cur16;
    cur16 = nxt16;
    nxt16 = tmp16;
    __syncthreads();
  }
  // the unrecovered inputs follow the schedule, ascending, with row -1
  if (wid == 0) wave0_list<true>(S, J, kw, npairs);
  if (tid == 0) {
    J.status[0] = npairs == k ? 1 : 0;
    J.status[1] = (int32_t)(k - npairs);
    J.status[2] = (int32_t)level;
    if (J.status_out) {
      J.status_out[0] = npairs == k ? 1 : 0;
      J.status_out[1] = (int32_t)(k - npairs);
      J.status_out[2] = (int32_t)level;
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(kPeelThreads) void peel_kernel(PeelJob J) {
  peel_body<MODE>(J);
}

// one workgroup per stripe of a batch
template <int MODE>
__global__ __launch_bounds__(kPeelThreads) void peel_batch_kernel(const PeelJob *jobs) {
  peel_body<MODE>(jobs[blockIdx.x]);
}

// ---------------------------------------------------------------------------
// replay program and schedule replay
// ---------------------------------------------------------------------------
constexpr int kReplayThreads = 1024;

// Flatten the schedule into a replay program: for pair p (schedule order) the
// inputs of its decoding row other than f, at pidx[poff[p] .. poff[p+1]);
// gsrc[f] is the decoding row of f (-1 for unrecovered inputs).  Pairs that
// do not fit the graph are dropped; meta = {nR, L, entries, usable}.
// Loads are hoisted in groups of G pairs so each thread keeps several
// dependent chains (row -> row pointer -> neighbour ids) in flight (G = 4
// where the registers are capped at 64 per lane, so that nothing spills).
template <int G = 8>
__device__ __forceinline__ void prog_body(const ProgJob &P) {
  __shared__ uint32_t scan_sh[kPlanThreads / 64 + 1];
  const int tid = threadIdx.x;
  const int k = (int)P.k;
  // the dependency-slab form is unusable until prog_lookahead_kernel says otherwise
  if (tid == 0 && P.la_meta) P.la_meta[0] = 0;
  if (P.skip_flag && *P.skip_flag) {
    if (tid == 0) P.meta[3] = 0;
    return;
  }
  const int L = min(max(P.status[2], 0), k);
  const int nR = min(max(k - P.status[1], 0), k);
  // inputs without a decoding row stay at -1, rows decoding nothing too (the
  // scan below orders these writes before the ones of the pairs)
  for (int f = tid; f < k; f += kPlanThreads) P.gsrc[f] = -1;
  for (uint32_t g = tid; g < P.n; g += kPlanThreads) P.finv[g] = -1;
  const int cpt = (nR + kPlanThreads - 1) / kPlanThreads;
  const int p0 = min(nR, tid * cpt), p1 = min(nR, p0 + cpt);
  uint32_t cnt = 0;
  for (int b = p0; b < p1; b += G) {
    int32_t f[G], g[G], r0[G], r1[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      f[u] = b + u < p1 ? P.dp_f[b + u] : -1;
      g[u] = b + u < p1 ? P.dp_g[b + u] : -1;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const bool ok = (uint32_t)f[u] < P.k && (uint32_t)g[u] < P.n;
      r0[u] = ok ? P.row_ptr[g[u]] : 0;
      r1[u] = ok ? P.row_ptr[g[u] + 1] : 1;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) cnt += (uint32_t)(r1[u] - r0[u] - 1);
  }
  uint32_t total;
  uint32_t o = block_exclusive_scan<kPlanThreads>(cnt, scan_sh, total);   // has barriers
  const bool fits = total <= P.pidx_cap;
  for (int b = p0; b < p1; b += G) {
    int32_t f[G], g[G], r0[G], r1[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      f[u] = b + u < p1 ? P.dp_f[b + u] : -1;
      g[u] = b + u < p1 ? P.dp_g[b + u] : -1;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const bool ok = (uint32_t)f[u] < P.k && (uint32_t)g[u] < P.n;
      r0[u] = ok ? P.row_ptr[g[u]] : 0;
      r1[u] = ok ? P.row_ptr[g[u] + 1] : 1;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (b + u >= p1) break;
      P.poff[b + u] = (int32_t)o;
      const uint32_t end = o + (uint32_t)(r1[u] - r0[u] - 1);
      if ((uint32_t)f[u] < P.k && (uint32_t)g[u] < P.n) {
        P.gsrc[f[u]] = g[u];
        P.finv[g[u]] = f[u];
      }
      for (int e = r0[u]; e < r1[u] && o < end; e += G) {
        int32_t cv[G];
#pragma unroll
        for (int v = 0; v < G; ++v) cv[v] = e + v < r1[u] ? P.col[e + v] : f[u];
#pragma unroll
        for (int v = 0; v < G; ++v) {
          if (cv[v] != f[u] && o < end) {
            if (fits) P.pidx[o] = cv[v];
            ++o;
          }
        }
      }
      o = end;
    }
  }
  __syncthreads();
  // decoding rows in ascending order with their inputs: the slab loads then
  // walk the coded blocks in address order
  const uint32_t rpt = (P.n + kPlanThreads - 1) / kPlanThreads;
  const uint32_t g0 = min(P.n, (uint32_t)tid * rpt), g1 = min(P.n, g0 + rpt);
  uint32_t used = 0;
  for (uint32_t g = g0; g < g1; ++g) used += P.finv[g] >= 0;
  uint32_t nused;
  uint32_t pos = block_exclusive_scan<kPlanThreads>(used, scan_sh, nused);
  for (uint32_t g = g0; g < g1; ++g) {
    const int32_t f = P.finv[g];
    if (f >= 0 && pos < P.k) {
      P.gl[pos] = (int32_t)g;
      P.fl[pos] = f;
      ++pos;
    }
  }
  if (tid == 0) {
    P.poff[nR] = (int32_t)total;
    P.meta[0] = nR;
    P.meta[1] = L;
    P.meta[2] = (int32_t)total;
    P.meta[3] = fits && nused == (uint32_t)nR ? 1 : 0;
  }
}

__global__ __launch_bounds__(kPlanThreads) void prog_build_kernel(ProgJob P) { prog_body(P); }

// The same program built by many workgroups, for large schedules (one
// workgroup walks every pair and row in turn and is bound by its memory
// latency there):
//   1. decoding maps cleared, each pair's count of other inputs into poff;
//   2. poff scanned in place (entries past the pairs are 0);
//   3. per pair, its other inputs copied to pidx, gsrc and finv set;
//   4. the decoding rows listed ascending (gl, fl) by one workgroup with a
//      running count, and meta.
// The result is prog_body's, entry for entry.
__device__ __forceinline__ int prog_pairs(const ProgJob &P) {
  return min(max((int)P.k - P.status[1], 0), (int)P.k);
}

__global__ __launch_bounds__(256) void prog_wide_count_kernel(ProgJob P) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  // the dependency-slab form is unusable until prog_lookahead_kernel says otherwise
  if (i == 0 && P.la_meta) P.la_meta[0] = 0;
  if (P.skip_flag && *P.skip_flag) return;
  if (i < P.k) P.gsrc[i] = -1;
  if (i < P.n) P.finv[i] = -1;
  if (i < P.k) {
    int32_t cnt = 0;
    if ((int)i < prog_pairs(P)) {
      const int32_t f = P.dp_f[i], g = P.dp_g[i];
      if ((uint32_t)f < P.k && (uint32_t)g < P.n) cnt = P.row_ptr[g + 1] - P.row_ptr[g] - 1;
    }
    P.poff[i] = cnt;
  }
}

__global__ __launch_bounds__(256) void prog_wide_fill_kernel(ProgJob P) {
  if (P.skip_flag && *P.skip_flag) return;
  const int p = (int)(blockIdx.x * 256u + threadIdx.x);
  const int nR = prog_pairs(P);
  if (p >= nR) return;
  const int32_t f = P.dp_f[p], g = P.dp_g[p];
  if (!((uint32_t)f < P.k && (uint32_t)g < P.n)) return;
  P.gsrc[f] = g;
  P.finv[g] = f;
  if ((uint32_t)P.poff[nR] > P.pidx_cap) return;   // does not fit: the program is marked unusable
  int32_t o = P.poff[p];
  const int32_t end = P.poff[p + 1];
  const int e1 = P.row_ptr[g + 1];
  // the row's entries eight at a time, loaded before any is stored (the
  // longest rows set the launch's time)
  for (int e = P.row_ptr[g]; e < e1 && o < end; e += 8) {
    int32_t c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = e + u < e1 ? P.col[e + u] : f;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (c[u] != f && o < end) P.pidx[o++] = c[u];
  }
}

// The decoding rows ascending (gl, fl) in one workgroup: chunks of 16 rows
// per thread with a running count, then meta.
constexpr int kRowsItems = 16;

__global__ __launch_bounds__(1024) void prog_wide_rows_kernel(ProgJob P) {
  __shared__ uint32_t sh[1024 / 64 + 1];
  if (P.skip_flag && *P.skip_flag) {
    if (threadIdx.x == 0) P.meta[3] = 0;
    return;
  }
  constexpr uint32_t kChunk = 1024u * kRowsItems;
  uint32_t carry = 0;
  for (uint32_t c0 = 0; c0 < P.n; c0 += kChunk) {
    const uint32_t base = c0 + threadIdx.x * kRowsItems;
    int32_t f[kRowsItems];
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < kRowsItems; ++i) {
      f[i] = base + i < P.n ? P.finv[base + i] : -1;
      cnt += f[i] >= 0 ? 1u : 0u;
    }
    uint32_t total = 0;
    uint32_t pos = carry + scan_block<1024>(cnt, sh, total);
#pragma unroll
    for (int i = 0; i < kRowsItems; ++i) {
      if (f[i] < 0) continue;
      if (pos < P.k) {
        P.gl[pos] = (int32_t)(base + i);
        P.fl[pos] = f[i];
      }
      ++pos;
    }
    carry += total;
  }
  if (threadIdx.x == 0) {
    const int nR = prog_pairs(P);
    const int L = min(max(P.status[2], 0), (int)P.k);
    const uint32_t total = (uint32_t)P.poff[nR];
    P.poff[nR] = (int32_t)total;
    P.meta[0] = nR;
    P.meta[1] = L;
    P.meta[2] = (int32_t)total;
    P.meta[3] = total <= P.pidx_cap && carry == (uint32_t)nR ? 1 : 0;
  }
}

fs_status launch_prog_wide(const ProgJob &P, hipStream_t s) {
  const uint32_t span = std::max(P.k, P.n);
  hipLaunchKernelGGL(prog_wide_count_kernel, dim3((span + 255) / 256), dim3(256), 0, s, P);
  const fs_status st = scan_i32(P.poff, P.k, P.psums, P.poff, s);
  if (st != FS_OK) return st;
  hipLaunchKernelGGL(prog_wide_fill_kernel, dim3((P.k + 255) / 256), dim3(256), 0, s, P);
  hipLaunchKernelGGL(prog_wide_rows_kernel, dim3(1), dim3(1024), 0, s, P);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? FS_OK : fail(FS_ERR_HIP, std::string("program launch: ") + hipGetErrorString(e));
}

__global__ __launch_bounds__(kPlanThreads) void prog_batch_kernel(const ProgJob *jobs) { prog_body(jobs[blockIdx.x]); }

// A decode plan in one launch: the peel, then (after a barrier, reading the
// schedule the same workgroup just wrote) the replay program.  The plan of
// one stripe usually runs beside the payload kernels of another, so its
// registers are capped at 64 per lane (a few spill to scratch): that lets its
// one workgroup share a CU with the replay's workgroups instead of holding
// them back.  On the 4096 x 64 KiB stripe an overlapped encode + decode step
// went from 0.447 to 0.414 ms.
template <int MODE>
__global__ __launch_bounds__(kPeelThreads) __attribute__((amdgpu_waves_per_eu(8)))
void plan_kernel(PeelJob J, ProgJob P) {
  peel_body<MODE>(J);
  __syncthreads();
  prog_body<4>(P);
}

// Dependency-slab form of a replay program (one workgroup, after
// prog_body).  Every input that some pair reads (a dependency) gets its own
// slot, numbered in decode order, in an LDS slab that the lookahead replay
// keeps for the whole slice; the pair records then name slots only.  Per
// pair q: {f, g, entries offset, 1 + slot of f (0: nobody reads f)}; la_idx
// holds the slots of the pair's other inputs; la_meta = {usable, slots,
// largest level}.  A schedule whose pairs read an input no pair decodes, or
// whose level pointers do not run from 0 to nR, is marked unusable.
__global__ __launch_bounds__(kPlanThreads) void prog_lookahead_kernel(ProgJob P) {
  __shared__ uint32_t scan_sh[kPlanThreads / 64 + 1];
  __shared__ int s_bad, s_max;
  const int tid = threadIdx.x;
  const int k = (int)P.k;
  if ((P.skip_flag && *P.skip_flag) || !P.meta[3]) {
    if (tid == 0) P.la_meta[0] = 0;
    return;
  }
  const int nR = P.meta[0], L = P.meta[1];
  if (tid == 0) {
    s_bad = 0;
    s_max = 0;
  }
  __syncthreads();
  int mx = 0;
  for (int l = tid; l <= L; l += kPlanThreads) {
    const int v = P.level_ptr[l];
    if (v < 0 || v > nR || (l == 0 && v != 0) || (l == L && v != nR) || (l < L && v > P.level_ptr[l + 1]))
      atomicOr(&s_bad, 1);
    else if (l < L)
      mx = max(mx, P.level_ptr[l + 1] - v);
  }
  if (mx) atomicMax(&s_max, mx);
  for (int i = tid; i < k; i += kPlanThreads) P.la_slot[i] = 0;
  __syncthreads();
  if (s_bad) {
    if (tid == 0) P.la_meta[0] = 0;
    return;
  }
  // mark the dependencies
  for (int o = tid; o < P.meta[2]; o += kPlanThreads) {
    const int i = P.pidx[o];
    if ((uint32_t)i < (uint32_t)k) P.la_slot[i] = 1;
  }
  __syncthreads();
  // number them in decode order (a contiguous run of pairs per thread)
  const int cpt = (nR + kPlanThreads - 1) / kPlanThreads;
  const int p0 = min(nR, tid * cpt), p1 = min(nR, p0 + cpt);
  uint32_t cnt = 0;
  for (int q = p0; q < p1; ++q) cnt += P.la_slot[P.dp_f[q]] != 0;
  uint32_t marked;
  uint32_t run = block_exclusive_scan<kPlanThreads>(cnt, scan_sh, marked);
  for (int q = p0; q < p1; ++q) {
    P.la_pre[q] = (int32_t)run;
    run += P.la_slot[P.dp_f[q]] != 0;
  }
  __syncthreads();
  for (int q = tid; q < nR; q += kPlanThreads) {
    const int f = P.dp_f[q];
    if (P.la_slot[f]) P.la_slot[f] = 2 + P.la_pre[q];   // 2 + slot until every pair is numbered
  }
  __syncthreads();
  int bad = 0;
  for (int o = tid; o < P.meta[2]; o += kPlanThreads) {
    const int i = P.pidx[o];
    const int v = (uint32_t)i < (uint32_t)k ? P.la_slot[i] : 0;
    if (v < 2) bad = 1;   // read but never decoded
    P.la_idx[o] = v - 2;
  }
  for (int q = tid; q < nR; q += kPlanThreads) {
    const int f = P.dp_f[q];
    int32_t *rec = P.la_pair + 4 * (size_t)q;
    rec[0] = f;
    rec[1] = P.dp_g[q];
    rec[2] = P.poff[q];
    rec[3] = P.la_slot[f] ? P.la_slot[f] - 1 : 0;
  }
  if (bad) atomicOr(&s_bad, 1);
  __syncthreads();
  if (tid == 0) {
    P.la_meta[0] = s_bad ? 0 : 1;
    P.la_meta[1] = (int32_t)marked;
    P.la_meta[2] = s_max;
  }
}

// One workgroup per CU walks byte slices of T = 16 LPS bytes.  For each slice
// the k x T slab of x lives in LDS: x_f starts as c_{g(f)} (zero for the
// unrecovered inputs), each level XORs in the other inputs of f's decoding
// row from the slab, and the finished slab is written out.  The loads of the
// next slice's c_{g(f)} are issued before the level phase of the current one
// and held in registers (barriers only wait for LDS traffic), so HBM stays
// busy while the levels run.  The replay program is copied to LDS as 16-bit
// indices when it fits, else read from global memory.
template <int LPS, int M, class IT>
__device__ __forceinline__ void replay_slices(const ReplayJob &J, v4u *slab, const int32_t *gl, const int32_t *fl,
                                              const IT *lp, const IT *pf, const IT *poff, const IT *pidx,
                                              int L, int nR, uint32_t nslices, uint32_t vb) {
  constexpr int NS = kReplayThreads / LPS;
  const uint32_t lane = threadIdx.x % LPS, sym = threadIdx.x / LPS;
  const uint32_t k = J.k;
  const v4u zero = {0u, 0u, 0u, 0u};
  // unrecovered inputs stay zero in every slice: clear the slab once, the
  // slices only rewrite the recovered entries
  for (uint32_t f = sym; f < k; f += NS) slab[f * LPS + lane] = zero;
  __syncthreads();
  // (coded row, input) pairs of this thread, rows ascending across lanes
  int32_t gm[M], fm[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int q = (int)sym + m * NS;
    gm[m] = q < nR ? gl[q] : -1;
    fm[m] = q < nR ? fl[q] : -1;
    if ((uint32_t)fm[m] >= k || (uint32_t)gm[m] >= J.n) gm[m] = fm[m] = -1;
  }
  v4u pre[M];
  auto issue = [&](uint32_t slice) {
    const uint64_t off = (uint64_t)slice * (LPS * 16) + lane * 16u;
    const bool live = off < J.t;
#pragma unroll
    for (int m = 0; m < M; ++m)
      pre[m] = (live && gm[m] >= 0) ? ld16(J.c + (uint64_t)gm[m] * J.t + off) : zero;
  };
  uint32_t slice = vb;
  if (slice < nslices) issue(slice);
  while (slice < nslices) {
    const uint64_t off = (uint64_t)slice * (LPS * 16) + lane * 16u;
    const bool live = off < J.t;
#pragma unroll
    for (int m = 0; m < M; ++m)
      if (fm[m] >= 0) slab[(uint32_t)fm[m] * LPS + lane] = pre[m];
    __syncthreads();
    const uint32_t next = slice + gridDim.x;
    if (next < nslices) issue(next);
    for (int l = 0; l < L; ++l) {
      const int q1 = min((int)lp[l + 1], nR);
      for (int q = max((int)lp[l], 0) + (int)sym; q < q1; q += NS) {
        const uint32_t f = (uint32_t)pf[q];
        if (f >= k) continue;
        const int o0 = (int)poff[q], o1 = (int)poff[q + 1];
        v4u acc = slab[f * LPS + lane];
        int o = o0;
        for (; o + 2 <= o1; o += 2) {
          const uint32_t i0 = (uint32_t)pidx[o], i1 = (uint32_t)pidx[o + 1];
          acc ^= slab[i0 * LPS + lane] ^ slab[i1 * LPS + lane];
        }
        if (o < o1) acc ^= slab[(uint32_t)pidx[o] * LPS + lane];
        slab[f * LPS + lane] = acc;
      }
      __syncthreads();
    }
    // plain stores: the slices of one 128-byte line are written by
    // neighbouring workgroups of one XCD and merge in its L2
    if (live)
      for (uint32_t f = sym; f < k; f += NS) st16<false>(J.x + (uint64_t)f * J.t + off, slab[f * LPS + lane]);
    __syncthreads();
    slice = next;
  }
}

template <int LPS, int M>
__global__ __launch_bounds__(kReplayThreads) void replay_lds_kernel(ReplayJob J, ProgJob P, uint32_t nslices,
                                                                   uint32_t lds_bytes, uint32_t prog_lds) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  if (J.skip_flag && *J.skip_flag) return;
  if (!P.meta[3]) return;
  const uint32_t k = J.k;
  const int nR = P.meta[0], L = P.meta[1], total = P.meta[2];
  v4u *slab = reinterpret_cast<v4u *>(smem);
  const size_t slab_bytes = (size_t)k * LPS * 16;
  const size_t prog16 = 2ull * ((size_t)(L + 1) + (size_t)nR + (size_t)(nR + 1) + (size_t)total);
  const uint32_t vb = xcd_remap(blockIdx.x, gridDim.x);
  // level pointers are clamped to [0, nR] so a foreign schedule stays in bounds
  if (prog_lds && k <= 65535 && total <= 65535 && slab_bytes + prog16 <= lds_bytes) {
    uint16_t *q = reinterpret_cast<uint16_t *>(smem + slab_bytes);
    uint16_t *lp = q; q += L + 1;
    uint16_t *pf = q; q += nR;
    uint16_t *poff = q; q += nR + 1;
    uint16_t *pidx = q;
    for (int i = threadIdx.x; i <= L; i += kReplayThreads) lp[i] = (uint16_t)min(max(J.level_ptr[i], 0), nR);
    for (int i = threadIdx.x; i < nR; i += kReplayThreads) pf[i] = (uint16_t)min((uint32_t)J.dp_f[i], 65535u);
    for (int i = threadIdx.x; i <= nR; i += kReplayThreads) poff[i] = (uint16_t)P.poff[i];
    for (int i = threadIdx.x; i < total; i += kReplayThreads) pidx[i] = (uint16_t)P.pidx[i];
    __syncthreads();
    replay_slices<LPS, M, uint16_t>(J, slab, P.gl, P.fl, lp, pf, poff, pidx, L, nR, nslices, vb);
  } else {
    replay_slices<LPS, M, int32_t>(J, slab, P.gl, P.fl, J.level_ptr, J.dp_f, P.poff, P.pidx, L, nR, nslices, vb);
  }
}

// Wide-slice replay for large k: one workgroup per W = 16 LPS byte slice
// keeps x in global memory (full-line accesses; re-reads of x hit L2 or the
// infinity cache) and walks the levels with a barrier between them.  The
// program (pairs, decoding rows, other inputs) sits in LDS as 16-bit indices
// when it fits, so a level costs one round trip to memory: every load of a
// pair (its coded block and the other inputs) is issued before any is used.
template <int LPS, class IT, int MP = (LPS >= 32 ? 4 : 2)>
__device__ __forceinline__ void replay_wide_slices(const ReplayJob &J, const IT *lp, const IT *pf, const IT *pg,
                                                   const IT *poff, const IT *pidx, int L, int nR,
                                                   uint32_t nslices, uint32_t vb, uint32_t stride) {
  constexpr int NS = kReplayThreads / LPS;
  // MP: pairs per thread whose coded block is prefetched; PD: how many
  // levels ahead (two levels ahead measured no faster than one)
  constexpr int PD = 1;
  // Each coded block is read once, so its loads are non-temporal: the caches
  // keep the decoded inputs that later pairs read instead (replay of the
  // 4096 x 64 KiB stripe: 0.208 -> 0.182 ms).  Marking decoded inputs that
  // no later pair reads non-temporal as well measured no faster.
  constexpr uint32_t W = LPS * 16;
  const uint32_t lane = threadIdx.x % LPS, sym = threadIdx.x / LPS;
  const uint32_t k = J.k;
  const v4u zero = {0u, 0u, 0u, 0u};
  for (uint32_t slice = vb; slice < nslices; slice += stride) {
    const uint64_t off = (uint64_t)slice * W + lane * 16u;
    const bool live = off < J.t;
    // coded blocks of the first MP pairs of a level are loaded PD levels
    // before it runs (c is never written here); cb[d] holds level l + d
    v4u cb[PD][MP];
    auto prefetch = [&](int l, v4u (&dst)[MP]) {
      const int q0 = max((int)lp[l], 0), q1 = min((int)lp[l + 1], nR);
#pragma unroll
      for (int m = 0; m < MP; ++m) {
        const int q = q0 + (int)sym + m * NS;
        const uint32_t g = q < q1 ? (uint32_t)pg[q] : 0xffffffffu;
        dst[m] = (live && g < J.n) ? ld16_once(J.c + (uint64_t)g * J.t + off) : zero;
      }
    };
#pragma unroll
    for (int d = 0; d < PD; ++d)
      if (d < L) prefetch(d, cb[d]);
    for (int l = 0; l < L; ++l) {
      const int q0 = max((int)lp[l], 0), q1 = min((int)lp[l + 1], nR);
      v4u cur[MP];
#pragma unroll
      for (int m = 0; m < MP; ++m) cur[m] = cb[0][m];
#pragma unroll
      for (int d = 0; d + 1 < PD; ++d)
#pragma unroll
        for (int m = 0; m < MP; ++m) cb[d][m] = cb[d + 1][m];
      if (l + PD < L) prefetch(l + PD, cb[PD - 1]);
#pragma unroll
      for (int m = 0; m < MP; ++m) {
        const int q = q0 + (int)sym + m * NS;
        if (q >= q1 || !live) continue;
        const uint32_t f = (uint32_t)pf[q], g = (uint32_t)pg[q];
        if (f >= k || g >= J.n) continue;
        const int o1 = (int)poff[q + 1];
        v4u acc = cur[m];
        int o = (int)poff[q];
        for (; o + 4 <= o1; o += 4) {
          const v4u a = ld16(J.x + (uint64_t)pidx[o] * J.t + off);
          const v4u b = ld16(J.x + (uint64_t)pidx[o + 1] * J.t + off);
          const v4u c = ld16(J.x + (uint64_t)pidx[o + 2] * J.t + off);
          const v4u d = ld16(J.x + (uint64_t)pidx[o + 3] * J.t + off);
          acc ^= (a ^ b) ^ (c ^ d);
        }
        for (; o < o1; ++o) acc ^= ld16(J.x + (uint64_t)pidx[o] * J.t + off);
        *reinterpret_cast<v4u *>(J.x + (uint64_t)f * J.t + off) = acc;
      }
      // pairs beyond MP per thread (very large levels) load their block here
      for (int q = q0 + (int)sym + MP * NS; q < q1; q += NS) {
        const uint32_t f = (uint32_t)pf[q], g = (uint32_t)pg[q];
        if (!live || f >= k || g >= J.n) continue;
        v4u acc = ld16_once(J.c + (uint64_t)g * J.t + off);
        const int o1 = (int)poff[q + 1];
        for (int o = (int)poff[q]; o < o1; ++o) acc ^= ld16(J.x + (uint64_t)pidx[o] * J.t + off);
        *reinterpret_cast<v4u *>(J.x + (uint64_t)f * J.t + off) = acc;
      }
      __syncthreads();
    }
    if (live) {
      for (int q = nR + (int)sym; q < (int)k; q += NS) {
        const int32_t f = J.dp_f[q];
        if ((uint32_t)f < k) st16<false>(J.x + (uint64_t)f * J.t + off, zero);
      }
    }
  }
}

template <int LPS, int MP = (LPS >= 32 ? 4 : 2)>
__device__ __forceinline__ void replay_wide_body(const ReplayJob &J, const ProgJob &P, uint32_t nslices,
                                                 uint32_t lds_bytes, uint32_t prog_lds, uint32_t vb,
                                                 uint32_t stride) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  if (J.skip_flag && *J.skip_flag) return;
  if (!P.meta[3]) return;
  const uint32_t k = J.k;
  const int nR = P.meta[0], L = P.meta[1], total = P.meta[2];
  const size_t prog16 = 2ull * ((size_t)(L + 1) + 2ull * nR + (size_t)(nR + 1) + (size_t)total);
  if (prog_lds && k <= 65535 && J.n <= 65535 && total <= 65535 && prog16 <= lds_bytes) {
    uint16_t *q = reinterpret_cast<uint16_t *>(smem);
    uint16_t *lp = q; q += L + 1;
    uint16_t *pf = q; q += nR;
    uint16_t *pg = q; q += nR;
    uint16_t *poff = q; q += nR + 1;
    uint16_t *pidx = q;
    for (int i = threadIdx.x; i <= L; i += kReplayThreads) lp[i] = (uint16_t)min(max(J.level_ptr[i], 0), nR);
    for (int i = threadIdx.x; i < nR; i += kReplayThreads) {
      pf[i] = (uint16_t)min((uint32_t)J.dp_f[i], 65535u);
      pg[i] = (uint16_t)min((uint32_t)J.dp_g[i], 65535u);
    }
    for (int i = threadIdx.x; i <= nR; i += kReplayThreads) poff[i] = (uint16_t)P.poff[i];
    for (int i = threadIdx.x; i < total; i += kReplayThreads) pidx[i] = (uint16_t)P.pidx[i];
    __syncthreads();
    replay_wide_slices<LPS, uint16_t, MP>(J, lp, pf, pg, poff, pidx, L, nR, nslices, vb, stride);
  } else {
    replay_wide_slices<LPS, int32_t, MP>(J, J.level_ptr, J.dp_f, J.dp_g, P.poff, P.pidx, L, nR, nslices, vb,
                                         stride);
  }
}

// Narrow slices (LPS <= 16) run two workgroups per CU: registers are capped
// for 8 waves per SIMD, so a level's pairs fit one round of the two groups.
template <int LPS>
__global__ __launch_bounds__(kReplayThreads) __attribute__((amdgpu_waves_per_eu(LPS <= 16 ? 8 : 1)))
void replay_wide_kernel(ReplayJob J, ProgJob P, uint32_t nslices, uint32_t lds_bytes, uint32_t prog_lds) {
  replay_wide_body<LPS>(J, P, nslices, lds_bytes, prog_lds, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// The same for narrow slices when the program's LDS leaves one workgroup per
// CU anyway: the registers of four waves per SIMD, and four pairs per thread
// prefetched a level ahead (levels of up to 4 x 1024 / LPS pairs load no
// coded block inside the level).
template <int LPS>
__global__ __launch_bounds__(kReplayThreads) __attribute__((amdgpu_waves_per_eu(4)))
void replay_wide_one_kernel(ReplayJob J, ProgJob P, uint32_t nslices, uint32_t lds_bytes, uint32_t prog_lds) {
  replay_wide_body<LPS, 4>(J, P, nslices, lds_bytes, prog_lds, xcd_remap(blockIdx.x, gridDim.x), gridDim.x);
}

// Lookahead replay with a dependency slab.  One workgroup per CU walks byte
// slices of W = 16 lps bytes.  Every decoded input that a later pair reads
// keeps its slice in an LDS slab slot for the whole slice, so a level
// reads LDS only: x_f = c_g ^ (slab entries of g's other inputs), stored to
// x and, when read later, to f's slot.  The coded blocks are the only loads;
// each thread holds one pair per level and loads c_g PD steps ahead (steps
// run level by level and continue into the workgroup's next slice), so a
// level never waits on a round trip of its own.  Loads and stores go through
// buffer resources: an absent operand has an offset past the end, which
// reads zero and drops the store, so every step issues the same memory
// instructions and the compiler keeps the later loads in flight.  lps is the
// widest of 8, 4, 2, 1 whose slab fits LDS beside the 16-bit program; pairs
// past 1024 / lps in a level load their block when they run.
typedef __amdgpu_buffer_rsrc_t bufrsrc;
constexpr uint32_t kBufOob = 0x80000000u;   // offsets at or past this read zero

__device__ __forceinline__ bufrsrc make_rsrc(const uint8_t *p, uint64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(p), (short)0,
                                           (int)(uint32_t)min<uint64_t>(bytes, (uint64_t)kBufOob - 1), 0x00020000);
}

__device__ __forceinline__ v4u bld16(bufrsrc r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
}

__device__ __forceinline__ void bst16(bufrsrc r, uint32_t off, v4u v) {
  __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, 0);
}

// byte offset of (block b, byte off) as a buffer offset; past the end reads
// zero and drops stores
__device__ __forceinline__ uint32_t boff(uint32_t b, uint64_t t, uint32_t off) {
  const uint64_t o = (uint64_t)b * t + off;
  return o < kBufOob ? (uint32_t)o : kBufOob;
}

// 16-bit program in LDS: lp[L+1], pf[nR], pg[nR], po[nR+1], ps[nR], pidx[total]
__host__ __device__ inline size_t replay_la_prog_bytes(size_t L, size_t nR, size_t total) {
  return ((2 * ((L + 1) + 4 * nR + 1 + total)) + 15) & ~size_t(15);
}

template <int PD>
__global__ __launch_bounds__(kReplayThreads) void replay_la_kernel(ReplayJob J, ProgJob P, uint32_t lds_bytes) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  if (J.skip_flag && *J.skip_flag) return;
  if (!P.meta[3]) return;
  const int nR = P.meta[0], L = P.meta[1], total = P.meta[2];
  const uint32_t k = J.k;
  const uint64_t t = J.t;
  const uint32_t vb = xcd_remap(blockIdx.x, gridDim.x), stride = gridDim.x;
  const size_t progb = replay_la_prog_bytes(L, nR, total);
  const int nslots = P.la_meta[1];
  const bool usable = P.la_meta[0] && total <= 65535 && nslots >= 0 && nslots <= nR;
  uint32_t lsh = 4;
  for (uint32_t c = 3; c <= 3; --c)
    if (usable && progb + (size_t)nslots * (16u << c) <= lds_bytes) {
      lsh = c;
      break;
    }
  const uint32_t lps = 1u << lsh, W = 16u * lps;
  const uint32_t nslices = lsh < 4 ? (uint32_t)((t + W - 1) / W) : 0u;
  const uint32_t nmine = vb < nslices ? (nslices - 1 - vb) / stride + 1 : 0u;
  if (lsh == 4 || (uint64_t)nmine * (uint64_t)max(L, 1) >= (1ull << 31)) {
    const uint32_t ns8 = (uint32_t)((t + 127) / 128);
    replay_wide_body<8>(J, P, ns8, lds_bytes, 1u, vb, stride);
    return;
  }
  uint16_t *q16 = reinterpret_cast<uint16_t *>(smem);
  uint16_t *lp = q16; q16 += L + 1;
  uint16_t *pf = q16; q16 += nR;
  uint16_t *pg = q16; q16 += nR;
  uint16_t *po = q16; q16 += nR + 1;
  uint16_t *ps = q16; q16 += nR;
  uint16_t *pidx = q16;
  for (int i = threadIdx.x; i <= L; i += kReplayThreads) lp[i] = (uint16_t)min(max(J.level_ptr[i], 0), nR);
  for (int i = threadIdx.x; i < nR; i += kReplayThreads) {
    const int32_t *rec = P.la_pair + 4 * (size_t)i;
    pf[i] = (uint16_t)rec[0];
    pg[i] = (uint16_t)rec[1];
    po[i] = (uint16_t)rec[2];
    ps[i] = (uint16_t)rec[3];
  }
  if (threadIdx.x == 0) po[nR] = (uint16_t)total;
  for (int i = threadIdx.x; i < total; i += kReplayThreads) pidx[i] = (uint16_t)P.la_idx[i];
  v4u *slab = reinterpret_cast<v4u *>(smem + progb);
  __syncthreads();

  const uint32_t lane = threadIdx.x & (lps - 1), sym = threadIdx.x >> lsh;
  const int NS = (int)(kReplayThreads >> lsh);
  const v4u zero = {0u, 0u, 0u, 0u};
  const bufrsrc rc = make_rsrc(J.c, (uint64_t)J.n * J.t);
  const bufrsrc rx = make_rsrc(J.x, (uint64_t)J.k * J.t);
  const uint32_t steps = nmine * (uint32_t)L;
  // inputs no pair decodes are zero in every slice
  auto zero_fill = [&](uint32_t off) {
    if (off < t)
      for (int q = nR + (int)sym; q < (int)k; q += NS) {
        const int32_t f = J.dp_f[q];
        if ((uint32_t)f < k) bst16(rx, boff((uint32_t)f, t, off), zero);
      }
  };
  if (L == 0) {
    for (uint32_t s = vb; s < nslices; s += stride) zero_fill(s * W + lane * 16u);
    return;
  }
  // coded block of this thread's pair at step j (zero when there is none)
  auto load_step = [&](uint32_t j) -> v4u {
    const uint32_t jj = min(j, steps - 1);
    const uint32_t sl = vb + stride * (jj / (uint32_t)L), l = jj % (uint32_t)L;
    const uint32_t off = sl * W + lane * 16u;
    const int q = (int)lp[l] + (int)sym;
    const bool valid = j < steps && off < t && q < (int)lp[l + 1];
    return bld16(rc, valid ? boff(pg[valid ? q : 0], t, off) : kBufOob);
  };
  v4u C[PD];
#pragma unroll
  for (int d = 0; d < PD; ++d) C[d] = load_step((uint32_t)d);
  for (uint32_t j0 = 0; j0 < steps; j0 += PD) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const uint32_t j = j0 + (uint32_t)d;
      const v4u cur = C[d];
      C[d] = load_step(j + PD);
      const uint32_t jj = min(j, steps - 1);
      const uint32_t sl = vb + stride * (jj / (uint32_t)L), l = jj % (uint32_t)L;
      const uint32_t off = sl * W + lane * 16u;
      const bool run = j < steps;
      const bool live = run && off < t;
      const int q0 = lp[l], q1 = lp[l + 1];
      const int q = q0 + (int)sym;
      const bool valid = live && q < q1;
      v4u acc = cur;
      const int qv = valid ? q : 0;
      if (valid) {
        const int o1 = po[qv + 1];
        for (int o = po[qv]; o < o1; ++o) acc ^= slab[((uint32_t)pidx[o] << lsh) + lane];
      }
      const uint32_t f = pf[qv];
      bst16(rx, valid && f < k ? boff(f, t, off) : kBufOob, acc);
      const uint32_t s1 = ps[qv];
      if (valid && s1) slab[((s1 - 1u) << lsh) + lane] = acc;
      // pairs past one per thread: their block is loaded here
      if (live)
        for (int qq = q + NS; qq < q1; qq += NS) {
          v4u a2 = bld16(rc, boff(pg[qq], t, off));
          for (int o = po[qq]; o < po[qq + 1]; ++o) a2 ^= slab[((uint32_t)pidx[o] << lsh) + lane];
          const uint32_t f2 = pf[qq];
          bst16(rx, f2 < k ? boff(f2, t, off) : kBufOob, a2);
          if (ps[qq]) slab[(((uint32_t)ps[qq] - 1u) << lsh) + lane] = a2;
        }
      if (run && l == 0) zero_fill(off);
      __syncthreads();
    }
  }
}

// Replays of a batch: stripe i owns workgroups [wg_prefix[i], wg_prefix[i+1])
// which stride over its slices.
template <int LPS>
__global__ __launch_bounds__(kReplayThreads) void replay_batch_kernel(const ReplayJob *rj, const ProgJob *pj,
                                                                     const uint32_t *wg_prefix, uint32_t nitems,
                                                                     uint32_t lds_bytes, uint32_t prog_lds) {
  const uint32_t b = blockIdx.x;
  uint32_t lo = 0, hi = nitems;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (wg_prefix[mid] <= b) lo = mid; else hi = mid;
  }
  const ReplayJob &J = rj[lo];
  const uint32_t w = 16u * LPS;
  const uint32_t nslices = (uint32_t)((J.t + w - 1) / w);
  replay_wide_body<LPS>(J, pj[lo], nslices, lds_bytes, prog_lds, b - wg_prefix[lo], wg_prefix[lo + 1] - wg_prefix[lo]);
}

// Fallback for slabs too large for LDS: one workgroup per byte slice reads
// and writes x in global memory, a barrier between levels.
template <int LPS>
__global__ __launch_bounds__(kReplayThreads) void replay_kernel(ReplayJob J) {
  constexpr uint32_t W = LPS * 16;
  constexpr uint32_t NS = kReplayThreads / LPS;
  if (J.skip_flag && *J.skip_flag) return;
  const uint32_t slice = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t lane = threadIdx.x % LPS, sym = threadIdx.x / LPS;
  const uint64_t off = (uint64_t)slice * W + lane * 16u;
  const bool live = off < J.t;
  const int k = (int)J.k;
  // the schedule comes from the peel kernel; indices are still clamped so a
  // foreign schedule cannot address outside x or c
  const int L = min(max(J.status[2], 0), k);
  for (int l = 0; l < L; ++l) {
    const int p1 = min(J.level_ptr[l + 1], k);
    for (int p = max(J.level_ptr[l], 0) + (int)sym; p < p1; p += (int)NS) {
      const int32_t f = J.dp_f[p], g = J.dp_g[p];
      if (!live || (uint32_t)f >= J.k || (uint32_t)g >= J.n) continue;
      v4u acc = ld16(J.c + (uint64_t)g * J.t + off);
      for (int e = J.row_ptr[g]; e < J.row_ptr[g + 1]; ++e) {
        const int32_t i = J.col[e];
        if (i != f) acc ^= ld16(J.x + (uint64_t)i * J.t + off);
      }
      *reinterpret_cast<v4u *>(J.x + (uint64_t)f * J.t + off) = acc;
    }
    __syncthreads();
  }
  const int nR = min(max(k - J.status[1], 0), k);
  if (live) {
    for (int p = nR + (int)sym; p < k; p += (int)NS) {
      const int32_t f = J.dp_f[p];
      if ((uint32_t)f < J.k) st16<true>(J.x + (uint64_t)f * J.t + off, v4u{0u, 0u, 0u, 0u});
    }
  }
}

// ---------------------------------------------------------------------------
// repair and update planning
// ---------------------------------------------------------------------------

__device__ __forceinline__ void repair_prep_body(const RepairPrepJob &J, int default_ok) {
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const uint32_t nw = (J.n + 31) / 32;
  if (tid == 0) s_bad = 0;
  for (uint32_t w = tid; w < nw; w += kPlanThreads) J.seen[w] = 0;
  if (J.erased2)
    for (uint32_t g = tid; g < J.n; g += kPlanThreads) J.erased2[g] = J.erased ? (J.erased[g] ? 1 : 0) : 0;
  __syncthreads();
  for (uint32_t m = tid; m < J.n_lost; m += kPlanThreads) {
    const uint32_t j = J.lost[m];
    if (j >= J.n) {
      atomicOr(&s_bad, 1);
      continue;
    }
    const uint32_t bit = 1u << (j & 31);
    if (atomicOr(&J.seen[j >> 5], bit) & bit) atomicOr(&s_bad, 1);
    if (J.erased2) J.erased2[j] = 1;
  }
  __syncthreads();
  const int bad = s_bad;
  for (uint32_t m = tid; m < J.n_lost; m += kPlanThreads) J.repaired[m] = (!bad && default_ok) ? 1 : 0;
  if (tid == 0) {
    J.flag[0] = bad ? FS_ERR_INVALID : 0;
    J.status[0] = bad ? 0 : 1;
    J.status[1] = bad ? (int32_t)J.n_lost : 0;
    J.status[2] = bad ? FS_ERR_INVALID : 0;
  }
  if (!J.sptr) return;
  // the lost rows' edges, row after row, cut into pieces of at most kSegMax
  // edges (the ids are valid and distinct here, or the gather is skipped).
  // A row of at most kSegMax edges is copied by its thread; longer rows by
  // the whole workgroup, which also zeroes them (their pieces XOR into them).
  __shared__ uint32_t sh[kPlanThreads / 64 + 1];
  __shared__ uint32_t s_heavy[kPlanThreads];
  __shared__ uint32_t s_nheavy;
  uint32_t carry = 0, ecarry = 0;
  for (uint32_t m0 = 0; !bad && m0 < J.n_lost; m0 += kPlanThreads) {
    const uint32_t m = m0 + tid;
    int32_t e0 = 0, e1 = 0;
    if (m < J.n_lost) {
      const uint32_t j = J.lost[m];
      e0 = J.row_ptr[j];
      e1 = J.row_ptr[j + 1];
    }
    const uint32_t d = (uint32_t)(e1 - e0);
    const uint32_t pieces = m < J.n_lost ? max(1u, (d + kSegMax - 1) / kSegMax) : 0u;
    uint32_t total = 0, etotal = 0;
    const uint32_t first = carry + scan_block<kPlanThreads>(pieces, sh, total);
    const uint32_t off = ecarry + scan_block<kPlanThreads>(d, sh, etotal);
    if (tid == 0) s_nheavy = 0;
    if (m < J.n_lost) {
      J.roff[m] = (int32_t)off;
      for (uint32_t p = 0; p < pieces; ++p) {
        const uint32_t sg = first + p;
        if (sg >= J.seg_cap) break;
        J.sptr[sg] = (int32_t)(off + p * kSegMax);
        J.sout[sg] = (int32_t)J.lost[m];
        J.satomic[sg] = pieces > 1 ? 1 : 0;
      }
      if (d <= kSegMax)
        for (uint32_t e = 0; e < d; ++e) J.sidx[off + e] = J.col[e0 + (int32_t)e];
    }
    __syncthreads();
    if (m < J.n_lost && d > kSegMax) s_heavy[atomicAdd(&s_nheavy, 1u)] = m;
    __syncthreads();
    const uint32_t nh = s_nheavy;
    for (uint32_t h = 0; h < nh; ++h) {
      const uint32_t mh = s_heavy[h], j = J.lost[mh];
      const int32_t h0 = J.row_ptr[j], hd = J.row_ptr[j + 1] - h0;
      int32_t *dst = J.sidx + J.roff[mh];
      for (int32_t e = (int32_t)tid; e < hd; e += kPlanThreads) dst[e] = J.col[h0 + e];
      uint8_t *row = J.c + (uint64_t)j * J.t;
      for (uint64_t o = (uint64_t)tid * 16; o < J.t; o += (uint64_t)kPlanThreads * 16)
        *reinterpret_cast<v4u *>(row + o) = v4u{0u, 0u, 0u, 0u};
    }
    __syncthreads();
    carry += total;
    ecarry += etotal;
  }
  if (tid == 0) {
    const uint32_t ns = min(carry, J.seg_cap);
    *J.nseg = bad ? 0 : (int32_t)ns;
    J.sptr[ns] = (int32_t)ecarry;
  }
}

__global__ __launch_bounds__(kPlanThreads) void repair_prep_kernel(RepairPrepJob J, int default_ok) {
  repair_prep_body(J, default_ok);
}

__global__ __launch_bounds__(kPlanThreads) void repair_prep_batch_kernel(const RepairPrepJob *jobs) {
  repair_prep_body(jobs[blockIdx.x], jobs[blockIdx.x].erased2 ? 0 : 1);
}

__global__ __launch_bounds__(256) void extend_prep_kernel(ExtendPrepJob J) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= J.n) return;
  if (i < J.n - J.n_old) J.ids[i] = J.n_old + i;
  if (J.erased_full) J.erased_full[i] = (i < J.n_old && J.erased && J.erased[i]) ? 1 : 0;
}

__global__ __launch_bounds__(kPlanThreads) void repair_check_kernel(RepairCheckJob J) {
  __shared__ int s_fail;
  const int tid = threadIdx.x;
  if (J.flag[0]) return;
  if (tid == 0) s_fail = 0;
  __syncthreads();
  for (uint32_t m = tid; m < J.n_lost; m += kPlanThreads) {
    const uint32_t j = J.lost[m];
    int ok = 1;
    for (int e = J.row_ptr[j]; e < J.row_ptr[j + 1]; ++e) ok &= J.recovered[J.col[e]] ? 1 : 0;
    J.repaired[m] = (uint8_t)ok;
    if (!ok) atomicAdd(&s_fail, 1);
  }
  __syncthreads();
  if (tid == 0) {
    J.status[0] = s_fail == 0 ? 1 : 0;
    J.status[1] = s_fail;
    J.status[2] = 0;
  }
}

__device__ __forceinline__ void update_plan_body(const UpdatePlanJob &J) {
  __shared__ uint32_t scan_sh[kPlanThreads / 64 + 1];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const uint32_t kw = (J.k + 31) / 32;
  if (tid == 0) s_bad = 0;
  for (uint32_t w = tid; w < kw; w += kPlanThreads) J.seen[w] = 0;
  for (uint32_t h = tid; h < J.n; h += kPlanThreads) J.cnt[h] = 0;
  __syncthreads();
  for (uint32_t u = tid; u < J.n_ids; u += kPlanThreads) {
    const uint32_t i = J.ids[u];
    if (i >= J.k) {
      atomicOr(&s_bad, 1);
      continue;
    }
    const uint32_t bit = 1u << (i & 31);
    if (atomicOr(&J.seen[i >> 5], bit) & bit) atomicOr(&s_bad, 1);
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0) {
      J.flag[0] = FS_ERR_INVALID;
      J.n_aff[0] = 0;
      J.status[0] = 0;
      J.status[1] = 0;
      J.status[2] = FS_ERR_INVALID;
    }
    return;
  }
  // pairs (row h, id u) counted per row
  for (uint32_t u = tid; u < J.n_ids; u += kPlanThreads) {
    const uint32_t i = J.ids[u];
    for (int e = J.col_ptr[i]; e < J.col_ptr[i + 1]; ++e) atomicAdd(&J.cnt[J.rowidx[e]], 1);
  }
  __syncthreads();
  // compact affected rows ascending, with prefix sums of their pair counts
  const uint32_t cpt = (J.n + kPlanThreads - 1) / kPlanThreads;
  const uint32_t h0 = min(J.n, (uint32_t)tid * cpt), h1 = min(J.n, h0 + cpt);
  uint32_t rows = 0, pairs = 0;
  for (uint32_t h = h0; h < h1; ++h) {
    const int c = J.cnt[h];
    rows += c > 0;
    pairs += (uint32_t)c;
  }
  uint32_t trows, tpairs;
  uint32_t a = block_exclusive_scan<kPlanThreads>(rows, scan_sh, trows);
  uint32_t p = block_exclusive_scan<kPlanThreads>(pairs, scan_sh, tpairs);
  for (uint32_t h = h0; h < h1; ++h) {
    const int c = J.cnt[h];
    if (c > 0) {
      J.arow[a] = (int32_t)h;
      J.aptr[a] = (int32_t)p;
      J.cnt[h] = (int32_t)p;      // becomes the fill cursor of row h
      ++a;
      p += (uint32_t)c;
    }
  }
  __syncthreads();
  for (uint32_t u = tid; u < J.n_ids; u += kPlanThreads) {
    const uint32_t i = J.ids[u];
    for (int e = J.col_ptr[i]; e < J.col_ptr[i + 1]; ++e) {
      const int slot = atomicAdd(&J.cnt[J.rowidx[e]], 1);
      J.asrc[slot] = (int32_t)u;
    }
  }
  if (tid == 0) {
    J.aptr[trows] = (int32_t)tpairs;
    J.n_aff[0] = (int32_t)trows;
    J.flag[0] = 0;
    J.status[0] = (int32_t)trows;
    J.status[1] = (int32_t)tpairs;
    J.status[2] = 0;
  }
}

__global__ __launch_bounds__(kPlanThreads) void update_plan_kernel(UpdatePlanJob J) { update_plan_body(J); }

__global__ __launch_bounds__(kPlanThreads) void update_plan_batch_kernel(const UpdatePlanJob *jobs) {
  update_plan_body(jobs[blockIdx.x]);
}

constexpr int kDeltaThreads = 256;

__global__ __launch_bounds__(kDeltaThreads) void update_delta_kernel(UpdateDeltaJob J, uint32_t nslices) {
  if (J.flag[0]) return;
  const uint32_t u = blockIdx.x / nslices, s = blockIdx.x % nslices;
  const uint64_t off = (uint64_t)s * (kDeltaThreads * 16) + threadIdx.x * 16u;
  if (u >= J.n_ids || off >= J.t) return;
  uint8_t *xi = J.x + (uint64_t)J.ids[u] * J.t + off;
  const v4u nv = ld16(J.new_blocks + (uint64_t)u * J.t + off);
  const v4u ov = ld16(xi);
  *reinterpret_cast<v4u *>(J.delta + (uint64_t)u * J.t + off) = ov ^ nv;
  *reinterpret_cast<v4u *>(xi) = nv;
}

// delta pass of a batch of updates: job i owns workgroups [prefix[i], prefix[i+1])
__global__ __launch_bounds__(kDeltaThreads) void update_delta_batch_kernel(const UpdateDeltaJob *jobs,
                                                                           const uint32_t *prefix, uint32_t njobs) {
  const uint32_t b = blockIdx.x;
  uint32_t lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (prefix[mid] <= b) lo = mid; else hi = mid;
  }
  const UpdateDeltaJob &J = jobs[lo];
  if (J.flag[0]) return;
  const uint32_t nslices = (uint32_t)((J.t + kDeltaThreads * 16 - 1) / (kDeltaThreads * 16));
  const uint32_t local = b - prefix[lo];
  const uint32_t u = local / nslices, sl = local % nslices;
  const uint64_t off = (uint64_t)sl * (kDeltaThreads * 16) + threadIdx.x * 16u;
  if (u >= J.n_ids || off >= J.t) return;
  uint8_t *xi = J.x + (uint64_t)J.ids[u] * J.t + off;
  const v4u nv = ld16(J.new_blocks + (uint64_t)u * J.t + off);
  const v4u ov = ld16(xi);
  *reinterpret_cast<v4u *>(J.delta + (uint64_t)u * J.t + off) = ov ^ nv;
  *reinterpret_cast<v4u *>(xi) = nv;
}

// zero the listed blocks of a batch: entry i is (base, t, row)
__global__ __launch_bounds__(256) void zero_batch_kernel(const ZeroEntry *rows, uint32_t nrows, uint32_t chunks) {
  const uint32_t r = blockIdx.x / chunks, ch = blockIdx.x % chunks;
  if (r >= nrows) return;
  const ZeroEntry z = rows[r];
  const uint64_t off = (uint64_t)ch * 4096 + threadIdx.x * 16u;
  if (off < z.t) *reinterpret_cast<v4u *>(z.base + (uint64_t)z.row * z.t + off) = v4u{0u, 0u, 0u, 0u};
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static fs_status hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define FS_TRY_LAUNCH(name, job, s)                                                     \
  do {                                                                                  \
    hipLaunchKernelGGL(name##_kernel, dim3(1), dim3(kPlanThreads), 0, s, job);          \
    fs_status _st = hip_check(hipGetLastError(), #name " launch");                      \
    if (_st != FS_OK) return _st;                                                       \
  } while (0)

#define FS_HIP_TRY(e, what)                     \
  do {                                          \
    fs_status _st = hip_check((e), (what));     \
    if (_st != FS_OK) return _st;               \
  } while (0)

fs_status launch_gather(const GatherJob &job, const fs_tune &tune, hipStream_t s) {
  hipError_t e;
  if (try_slab_encode(job, tune, s, e)) return hip_check(e, "slab encode launch");
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cu = device_info(dev).cu_count;
  switch (tune.lanes_per_row * 10 + tune.chunks) {
    case 81: e = run_gather_nt<8, 1>(job, tune, s, cu); break;
    case 82: e = run_gather_nt<8, 2>(job, tune, s, cu); break;
    case 84: e = run_gather_nt<8, 4>(job, tune, s, cu); break;
    case 161: e = run_gather_nt<16, 1>(job, tune, s, cu); break;
    case 162: e = run_gather_nt<16, 2>(job, tune, s, cu); break;
    case 164: e = run_gather_nt<16, 4>(job, tune, s, cu); break;
    case 321: e = run_gather_nt<32, 1>(job, tune, s, cu); break;
    case 322: e = run_gather_nt<32, 2>(job, tune, s, cu); break;
    case 324: e = run_gather_nt<32, 4>(job, tune, s, cu); break;
    case 641: e = run_gather_nt<64, 1>(job, tune, s, cu); break;
    case 642: e = run_gather_nt<64, 2>(job, tune, s, cu); break;
    case 644: e = run_gather_nt<64, 4>(job, tune, s, cu); break;
    case 1281: e = run_gather_nt<128, 1>(job, tune, s, cu); break;
    case 1282: e = run_gather_nt<128, 2>(job, tune, s, cu); break;
    case 2561: e = run_gather_nt<256, 1>(job, tune, s, cu); break;
    case 2562: e = run_gather_nt<256, 2>(job, tune, s, cu); break;
    default: return fail(FS_ERR_INVALID, "unsupported gather tuning");
  }
  return hip_check(e, "gather launch");
}

fs_status launch_zero_rows(uint8_t *dst, const int32_t *rows, uint32_t nrows, uint64_t t, hipStream_t s) {
  const uint32_t chunks = (uint32_t)((t + 4095) / 4096);
  const uint64_t grid = (uint64_t)nrows * chunks;
  if (grid == 0) return FS_OK;
  hipLaunchKernelGGL(zero_rows_kernel, dim3((uint32_t)grid), dim3(256), 0, s, dst, rows, nrows, t, chunks);
  return hip_check(hipGetLastError(), "zero rows launch");
}

size_t peel_lds_bytes(uint32_t k, uint32_t n) {
  const size_t kw = (k + 31) / 32;
  return 8ull * n + 8ull * k + 4ull * n + 4ull * n + 4ull * k + 8ull * kw + 4ull * (k + 1) + 2ull * n;
}

void peel_carve(Carver &cv, PeelJob &j) {
  const size_t kw = (j.k + 31) / 32;
  j.acc = cv.take<unsigned long long>(j.n);
  j.best = cv.take<unsigned long long>(j.k);
  j.front_a = cv.take<int32_t>(j.n);
  j.front_b = cv.take<int32_t>(j.n);
  j.dlist = cv.take<int32_t>(j.k);
  j.mask = cv.take<uint32_t>(kw);
  j.decmask = cv.take<uint32_t>(kw);
}

size_t peel_ws_bytes(uint32_t k, uint32_t n) {
  Carver cv(nullptr);
  PeelJob j{};
  j.k = k;
  j.n = n;
  peel_carve(cv, j);
  return cv.size();
}

static void set_max_lds(const void *fn, int dev, int bytes, bool *done) {
  if (dev >= 0 && dev < 64 && !done[dev]) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    done[dev] = true;
  }
}

int peel_mode(uint32_t k, uint32_t n, uint32_t max_deg) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const size_t budget = (size_t)device_info(dev).max_lds_per_block - 64;
  if (max_deg < 65536 && peel_lds_bytes(k, n) <= budget) return kPeelLds;
  if (8ull * n <= budget) return kPeelLdsRows;
  if (4ull * n <= budget && max_deg <= 127 && (uint64_t)max_deg * (k ? k - 1 : 0) < (1ull << 24))
    return peel_rows32b_bytes(k, n) <= budget && n < (1u << 24) ? kPeelLdsRows32B : kPeelLdsRows32;
  return kPeelGlobal;
}

// the compact all-LDS peel applies: 16-bit ids, packed counters, and its
// state with the column lists fits LDS beside the static arrays
static bool peel16_ok(const PeelJob &job, uint32_t max_deg, int budget) {
  return job.nnz > 0 && job.k <= 65535 && job.n <= 65535 && max_deg <= 127 &&
         (uint64_t)max_deg * (job.k ? job.k - 1 : 0) < (1ull << 24) &&
         peel_lds16_bytes(job.k, job.n, job.nnz) + 256 <= (size_t)budget;
}

fs_status launch_plan(const PeelJob &job, const ProgJob &prog, hipStream_t s, uint32_t max_deg) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int budget = device_info(dev).max_lds_per_block;
  if (peel16_ok(job, max_deg, budget)) {
    static bool done[64] = {false};
    set_max_lds(reinterpret_cast<const void *>(&plan_kernel<kPeelLds16>), dev, budget - 256, done);
    hipLaunchKernelGGL(plan_kernel<kPeelLds16>, dim3(1), dim3(kPeelThreads),
                       peel_lds16_bytes(job.k, job.n, job.nnz), s, job, prog);
  } else if (peel_mode(job.k, job.n, max_deg) == kPeelLds) {
    static bool done[64] = {false};
    set_max_lds(reinterpret_cast<const void *>(&plan_kernel<kPeelLds>), dev, budget - 256, done);
    hipLaunchKernelGGL(plan_kernel<kPeelLds>, dim3(1), dim3(kPeelThreads), peel_lds_bytes(job.k, job.n), s, job,
                       prog);
  } else {
    const fs_status st = launch_peel(job, s, max_deg);
    return st != FS_OK ? st : launch_prog(prog, s);
  }
  const fs_status st = hip_check(hipGetLastError(), "decode plan launch");
  return st != FS_OK ? st : launch_prog_lookahead(prog, s);
}

// Initial row states for the peels whose rows live in global memory or in
// LDS rows only: count << 40 | sum of the row's input ids (erased rows
// flagged), by one thread per row and then one per column (the column
// degrees stay small even when a few rows have huge degree).  One
// workgroup took about 0.05 ms for this on the k = 10246 code.
__global__ __launch_bounds__(256) void peel_init_rows_kernel(PeelJob J) {
  const uint32_t g = blockIdx.x * 256u + threadIdx.x;
  if (g >= J.n) return;
  const int d = J.row_ptr[g + 1] - J.row_ptr[g];
  J.acc[g] = J.erased[g] ? kErasedAcc : ((unsigned long long)d << 40);
}

// rows of bounded degree: the sum of the row's ids read from the CSR, eight
// entries at a time, in the same launch
__global__ __launch_bounds__(256) void peel_init_rowsum_kernel(PeelJob J) {
  const uint32_t g = blockIdx.x * 256u + threadIdx.x;
  if (g >= J.n) return;
  const int e0 = J.row_ptr[g], e1 = J.row_ptr[g + 1];
  unsigned long long sum = 0;
  for (int e = e0; e < e1; e += 8) {
    int32_t c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = e + u < e1 ? J.col[e + u] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += (uint32_t)c[u];
  }
  J.acc[g] = (J.erased[g] ? kErasedAcc : ((unsigned long long)(e1 - e0) << 40)) + sum;
}

__global__ __launch_bounds__(256) void peel_init_cols_kernel(PeelJob J) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= J.k) return;
  const int c1 = J.col_ptr[i + 1];
  for (int e = J.col_ptr[i]; e < c1; ++e) atomicAdd(&J.acc[J.rowidx[e]], (unsigned long long)i);
}

fs_status launch_peel(const PeelJob &job_in, hipStream_t s, uint32_t max_deg) {
  PeelJob job = job_in;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const size_t lds = peel_lds_bytes(job.k, job.n);
  const size_t static_lds = 64;
  const int budget = device_info(dev).max_lds_per_block;
  const int mode = peel_mode(job.k, job.n, max_deg);
  if (peel16_ok(job, max_deg, budget)) {
    static bool done[64] = {false};
    set_max_lds(reinterpret_cast<const void *>(&peel_kernel<kPeelLds16>), dev, budget - 256, done);
    hipLaunchKernelGGL(peel_kernel<kPeelLds16>, dim3(1), dim3(kPeelThreads), peel_lds16_bytes(job.k, job.n, job.nnz),
                       s, job);
  } else if (mode == kPeelLds) {
    static bool done[64] = {false};
    set_max_lds(reinterpret_cast<const void *>(&peel_kernel<kPeelLds>), dev, budget - (int)static_lds, done);
    hipLaunchKernelGGL(peel_kernel<kPeelLds>, dim3(1), dim3(kPeelThreads), lds, s, job);
  } else {
    if (!job.acc) return fail(FS_ERR_WORKSPACE, "peel state needs the workspace");
    if (max_deg <= 128) {
      if (job.n) hipLaunchKernelGGL(peel_init_rowsum_kernel, dim3((job.n + 255) / 256), dim3(256), 0, s, job);
    } else {
      if (job.n) hipLaunchKernelGGL(peel_init_rows_kernel, dim3((job.n + 255) / 256), dim3(256), 0, s, job);
      if (job.k) hipLaunchKernelGGL(peel_init_cols_kernel, dim3((job.k + 255) / 256), dim3(256), 0, s, job);
    }
    job.acc_ready = 1;
    if (mode == kPeelLdsRows) {
      static bool done[64] = {false};
      set_max_lds(reinterpret_cast<const void *>(&peel_kernel<kPeelLdsRows>), dev, budget - (int)static_lds, done);
      hipLaunchKernelGGL(peel_kernel<kPeelLdsRows>, dim3(1), dim3(kPeelThreads), 8ull * job.n, s, job);
    } else if (mode == kPeelLdsRows32B) {
      static bool done[64] = {false};
      set_max_lds(reinterpret_cast<const void *>(&peel_kernel<kPeelLdsRows32B>), dev, budget - (int)static_lds, done);
      hipLaunchKernelGGL(peel_kernel<kPeelLdsRows32B>, dim3(1), dim3(kPeelThreads), peel_rows32b_bytes(job.k, job.n),
                         s, job);
    } else if (mode == kPeelLdsRows32) {
      static bool done[64] = {false};
      set_max_lds(reinterpret_cast<const void *>(&peel_kernel<kPeelLdsRows32>), dev, budget - (int)static_lds, done);
      hipLaunchKernelGGL(peel_kernel<kPeelLdsRows32>, dim3(1), dim3(kPeelThreads), 4ull * job.n, s, job);
    } else {
      hipLaunchKernelGGL(peel_kernel<kPeelGlobal>, dim3(1), dim3(kPeelThreads), 0, s, job);
    }
  }
  return hip_check(hipGetLastError(), "peel launch");
}

void prog_carve(Carver &cv, ProgJob &p, uint64_t nnz) {
  p.gsrc = cv.take<int32_t>(p.k);
  p.finv = cv.take<int32_t>(p.n ? p.n : 1);
  p.gl = cv.take<int32_t>(p.k);
  p.fl = cv.take<int32_t>(p.k);
  p.poff = cv.take<int32_t>((size_t)p.k + 1);
  p.pidx = cv.take<int32_t>(nnz ? nnz : 1);
  p.meta = cv.take<int32_t>(4);
  p.psums = cv.take<uint32_t>(std::max(scan_sums_for((uint64_t)p.k + 1), (p.n + 1023u) / 1024u) + 2);
  p.pidx_cap = (uint32_t)(nnz ? nnz : 1);
  if (p.k <= 65535 && p.n <= 65535) {
    p.la_slot = cv.take<int32_t>(p.k);
    p.la_pre = cv.take<int32_t>((size_t)p.k + 1);
    p.la_idx = cv.take<int32_t>(nnz ? nnz : 1);
    p.la_pair = cv.take<int32_t>(4ull * p.k);
    p.la_meta = cv.take<int32_t>(4);
  } else {
    p.la_slot = p.la_pre = p.la_idx = p.la_pair = p.la_meta = nullptr;
  }
}

bool prog_has_lookahead(const ProgJob &p) {
  return p.k <= 65535 && p.n <= 65535 && p.la_meta != nullptr && p.la_pair != nullptr;
}

// LDS layout of the slab replay: the widest row slice (16 LPS bytes, LPS in
// 64..8) whose k x 16 LPS slab leaves room for a typical 16-bit program;
// 0 = k too large for a slab of 128-byte rows.
int replay_lanes(uint32_t k) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const size_t budget = (size_t)device_info(dev).max_lds_per_block;
  for (int lps = 64; lps >= 8; lps /= 2)
    if ((size_t)k * 16 * lps + 24576 <= budget) return lps;
  return 0;
}

template <int LPS, int M>
static hipError_t run_replay_lds(const ReplayJob &job, const ProgJob &prog, uint32_t nslices, uint32_t grid,
                                 int budget, int dev, hipStream_t s) {
  static bool done[64] = {false};
  set_max_lds(reinterpret_cast<const void *>(&replay_lds_kernel<LPS, M>), dev, budget, done);
  fs_launch_info &rec = launch_record();
  rec.replay_kind = 1;
  rec.replay_slice_bytes = 16u * LPS;
  rec.replay_workgroups = grid;
  hipLaunchKernelGGL((replay_lds_kernel<LPS, M>), dim3(grid), dim3(kReplayThreads), budget, s, job, prog,
                     nslices, (uint32_t)budget, tune_snapshot().replay_prog_global ? 0u : 1u);
  return hipGetLastError();
}

template <int LPS>
static hipError_t run_replay_wide(const ReplayJob &job, const ProgJob &prog, int budget, int dev, int cu,
                                  hipStream_t s) {
  static bool done[64] = {false};
  set_max_lds(reinterpret_cast<const void *>(&replay_wide_kernel<LPS>), dev, budget, done);
  const uint32_t w = 16u * LPS;
  const uint32_t nslices = (uint32_t)((job.t + w - 1) / w);
  const uint32_t grid = std::min<uint32_t>(nslices, (uint32_t)cu * 2);
  // LDS for the 16-bit program: its largest possible size (the kernel checks
  // the actual one), so that two workgroups share a CU when it is small
  const int lds = (int)std::min<size_t>((size_t)budget, replay_prog_lds_bound(job.k, prog.pidx_cap));
  fs_launch_info &rec = launch_record();
  rec.replay_kind = 2;
  rec.replay_slice_bytes = w;
  rec.replay_workgroups = grid;
  const uint32_t prog_lds = tune_snapshot().replay_prog_global ? 0u : 1u;
  if (LPS <= 4 && 2 * lds > budget) {
    static bool done_one[64] = {false};
    set_max_lds(reinterpret_cast<const void *>(&replay_wide_one_kernel<LPS <= 4 ? LPS : 4>), dev, budget, done_one);
    hipLaunchKernelGGL(replay_wide_one_kernel<LPS <= 4 ? LPS : 4>, dim3(grid), dim3(kReplayThreads), lds, s, job,
                       prog, nslices, (uint32_t)lds, prog_lds);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(replay_wide_kernel<LPS>, dim3(grid), dim3(kReplayThreads), lds, s, job, prog, nslices,
                     (uint32_t)lds, prog_lds);
  return hipGetLastError();
}

template <int LPS>
static hipError_t run_replay_lds_m(const ReplayJob &job, const ProgJob &prog, uint32_t mneed, uint32_t nslices,
                                   uint32_t grid, int budget, int dev, hipStream_t s) {
  if (mneed <= 4) return run_replay_lds<LPS, 4>(job, prog, nslices, grid, budget, dev, s);
  if (mneed <= 8) return run_replay_lds<LPS, 8>(job, prog, nslices, grid, budget, dev, s);
  return run_replay_lds<LPS, 16>(job, prog, nslices, grid, budget, dev, s);
}

// Schedules of this many inputs or more build their replay program with
// many workgroups (prog_wide_*): on the k = 10246 code one workgroup took
// 0.137 ms.
constexpr uint32_t kProgWideMinK = 4096;

fs_status launch_prog(const ProgJob &prog, hipStream_t s) {
  if (prog.k >= kProgWideMinK) {
    const fs_status st = launch_prog_wide(prog, s);
    if (st != FS_OK) return st;
  } else {
    FS_TRY_LAUNCH(prog_build, prog, s);
  }
  return launch_prog_lookahead(prog, s);
}

fs_status launch_prog_lookahead(const ProgJob &prog, hipStream_t s) {
  if (!prog_has_lookahead(prog) || !tune_snapshot().replay_lookahead || tune_snapshot().replay_prog_global)
    return FS_OK;
  hipLaunchKernelGGL(prog_lookahead_kernel, dim3(1), dim3(kPlanThreads), 0, s, prog);
  return hip_check(hipGetLastError(), "lookahead program launch");
}

// Lookahead replay: one workgroup per CU with the whole LDS (program and
// dependency slab), coded blocks loaded eight steps ahead.
template <int PD>
static hipError_t run_replay_la(const ReplayJob &job, const ProgJob &prog, int budget, int dev, int cu,
                                hipStream_t s) {
  static bool done[64] = {false};
  set_max_lds(reinterpret_cast<const void *>(&replay_la_kernel<PD>), dev, budget, done);
  fs_launch_info &rec = launch_record();
  rec.replay_kind = 3;
  rec.replay_slice_bytes = 0;  // chosen in the kernel from the slab it fits
  rec.replay_workgroups = (uint32_t)cu;
  hipLaunchKernelGGL(replay_la_kernel<PD>, dim3(cu), dim3(kReplayThreads), budget, s, job, prog, (uint32_t)budget);
  return hipGetLastError();
}

static bool use_lookahead(const ReplayJob &job, const ProgJob &prog) {
  const fs_tune tu = tune_snapshot();
  return tu.replay_lookahead && !tu.replay_prog_global && prog_has_lookahead(prog) &&
         (uint64_t)job.n * job.t < kBufOob && (uint64_t)job.k * job.t < kBufOob;
}

fs_status launch_replay(const ReplayJob &job, const ProgJob *prog, hipStream_t s) {
  if (prog) {
    const fs_status st = launch_prog(*prog, s);
    if (st != FS_OK) return st;
  }
  return launch_replay_prog(job, prog, s);
}

fs_status launch_replay_prog(const ReplayJob &job, const ProgJob *prog, hipStream_t s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cu = device_info(dev).cu_count;
  const int budget = device_info(dev).max_lds_per_block;
  if (!prog) {
    // no workspace for a program: the plain global-memory replay
    fs_launch_info &rec = launch_record();
    rec.replay_kind = 4;
    if (job.t >= 256ull * 512) {
      const uint32_t ns = (uint32_t)((job.t + 255) / 256);
      rec.replay_slice_bytes = 256;
      rec.replay_workgroups = ns;
      hipLaunchKernelGGL(replay_kernel<16>, dim3(ns), dim3(kReplayThreads), 0, s, job);
    } else {
      const uint32_t ns = (uint32_t)((job.t + 63) / 64);
      rec.replay_slice_bytes = 64;
      rec.replay_workgroups = ns;
      hipLaunchKernelGGL(replay_kernel<4>, dim3(ns), dim3(kReplayThreads), 0, s, job);
    }
    return hip_check(hipGetLastError(), "replay launch");
  }
  const int lps = replay_lanes(job.k);
  hipError_t e;
  if (lps) {
    // small k: the k x 16 LPS slab of a slice lives in LDS
    const uint32_t mneed = (job.k + (kReplayThreads / lps) - 1) / (kReplayThreads / lps);
    const uint32_t w = 16u * (uint32_t)lps;
    const uint32_t nslices = (uint32_t)((job.t + w - 1) / w);
    const uint32_t grid = std::min<uint32_t>(nslices, (uint32_t)cu);
    switch (lps) {
      case 64: e = run_replay_lds_m<64>(job, *prog, mneed, nslices, grid, budget, dev, s); break;
      case 32: e = run_replay_lds_m<32>(job, *prog, mneed, nslices, grid, budget, dev, s); break;
      case 16: e = run_replay_lds_m<16>(job, *prog, mneed, nslices, grid, budget, dev, s); break;
      default: e = run_replay_lds_m<8>(job, *prog, mneed, nslices, grid, budget, dev, s); break;
    }
  } else if (use_lookahead(job, *prog)) {
    e = run_replay_la<8>(job, *prog, budget, dev, cu, s);
  } else {
    // large k: wide slices in global memory, about two workgroups per CU.
    // Blocks too short for that take the widest of 128, 64, 32 or 16 bytes
    // that still gives three quarters of the workgroups that fit at once (one
    // or two per CU, by the program's LDS) a slice: one round of workgroups
    // beats two rounds of narrower ones.  Successive slices share an XCD, so
    // their 128-byte lines meet in one L2.
    const uint64_t per = (job.t + 2ull * cu - 1) / (2ull * cu);
    const uint64_t lds_w = std::max<uint64_t>(
        1, std::min<uint64_t>((uint64_t)budget, replay_prog_lds_bound(job.k, prog->pidx_cap)));
    const uint64_t fit = std::min<uint64_t>(2, std::max<uint64_t>(1, (uint64_t)budget / lds_w));
    const uint64_t want = (3ull * (uint64_t)cu * fit) / 4;
    auto slices = [&](uint64_t w) { return (job.t + w - 1) / w; };
    if (per >= 1024)
      e = run_replay_wide<64>(job, *prog, budget, dev, cu, s);
    else if (per >= 512)
      e = run_replay_wide<32>(job, *prog, budget, dev, cu, s);
    else if (per >= 256)
      e = run_replay_wide<16>(job, *prog, budget, dev, cu, s);
    else if (per >= 128 || slices(128) >= want)
      e = run_replay_wide<8>(job, *prog, budget, dev, cu, s);
    else if (slices(64) >= want)
      e = run_replay_wide<4>(job, *prog, budget, dev, cu, s);
    else if (slices(32) >= want)
      e = run_replay_wide<2>(job, *prog, budget, dev, cu, s);
    else
      e = run_replay_wide<1>(job, *prog, budget, dev, cu, s);
  }
  return hip_check(e, "replay launch");
}

fs_status launch_repair_prep(const RepairPrepJob &job, hipStream_t s) {
  const int default_ok = job.erased2 ? 0 : 1;
  hipLaunchKernelGGL(repair_prep_kernel, dim3(1), dim3(kPlanThreads), 0, s, job, default_ok);
  return hip_check(hipGetLastError(), "repair prep launch");
}

fs_status launch_extend_prep(const ExtendPrepJob &job, hipStream_t s) {
  if (job.n == 0) return FS_OK;
  hipLaunchKernelGGL(extend_prep_kernel, dim3((job.n + 255) / 256), dim3(256), 0, s, job);
  return hip_check(hipGetLastError(), "extend prep launch");
}

fs_status launch_repair_check(const RepairCheckJob &job, hipStream_t s) {
  hipLaunchKernelGGL(repair_check_kernel, dim3(1), dim3(kPlanThreads), 0, s, job);
  return hip_check(hipGetLastError(), "repair check launch");
}

fs_status launch_update_plan(const UpdatePlanJob &job, hipStream_t s) {
  hipLaunchKernelGGL(update_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, job);
  return hip_check(hipGetLastError(), "update plan launch");
}

fs_status launch_update_delta(const UpdateDeltaJob &job, hipStream_t s) {
  const uint32_t nslices = (uint32_t)((job.t + kDeltaThreads * 16 - 1) / (kDeltaThreads * 16));
  const uint64_t grid = (uint64_t)nslices * job.n_ids;
  if (grid == 0) return FS_OK;
  hipLaunchKernelGGL(update_delta_kernel, dim3((uint32_t)grid), dim3(kDeltaThreads), 0, s, job, nslices);
  return hip_check(hipGetLastError(), "update delta launch");
}

}  // namespace fs

// ---------------------------------------------------------------------------
// batched launchers
// ---------------------------------------------------------------------------
namespace fs {

template <int LPR, int CH>
static hipError_t run_gather_batch(const GatherJob *jobs, unsigned long long *prefix, uint32_t njobs,
                                   unsigned long long *counter, bool nt, uint32_t grid, uint32_t chunk,
                                   hipStream_t s) {
  hipLaunchKernelGGL(batch_start_kernel, dim3(1), dim3(1024), 0, s, jobs, prefix, njobs, counter,
                     (uint32_t)(kGatherThreads / LPR), (uint32_t)(16 * LPR * CH));
  if (nt)
    hipLaunchKernelGGL((gather_batch_kernel<LPR, CH, true>), dim3(grid), dim3(kGatherThreads), 0, s, jobs, prefix,
                       njobs, counter, chunk);
  else
    hipLaunchKernelGGL((gather_batch_kernel<LPR, CH, false>), dim3(grid), dim3(kGatherThreads), 0, s, jobs, prefix,
                       njobs, counter, chunk);
  return hipGetLastError();
}

fs_status launch_gather_batch(const GatherJob *d_jobs, unsigned long long *d_prefix, uint32_t njobs,
                              unsigned long long *d_counter, const fs_tune &tune, uint32_t grid,
                              uint64_t total_items, hipStream_t s) {
  if (njobs == 0 || grid == 0) return FS_OK;
  // small chunks keep the items in flight on an XCD close together
  const uint32_t chunk = tune.claim_chunk ? tune.claim_chunk
                                          : (uint32_t)std::min<uint64_t>(
                                                16, std::max<uint64_t>(2, total_items / ((uint64_t)grid * 64)));
  const bool nt = tune.nt_store != 0;
  hipError_t e;
  switch (tune.lanes_per_row * 10 + tune.chunks) {
    case 81: e = run_gather_batch<8, 1>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 82: e = run_gather_batch<8, 2>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 84: e = run_gather_batch<8, 4>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 161: e = run_gather_batch<16, 1>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 162: e = run_gather_batch<16, 2>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 164: e = run_gather_batch<16, 4>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 321: e = run_gather_batch<32, 1>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 322: e = run_gather_batch<32, 2>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 324: e = run_gather_batch<32, 4>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 641: e = run_gather_batch<64, 1>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 642: e = run_gather_batch<64, 2>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 644: e = run_gather_batch<64, 4>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 1281: e = run_gather_batch<128, 1>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 1282: e = run_gather_batch<128, 2>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 2561: e = run_gather_batch<256, 1>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    case 2562: e = run_gather_batch<256, 2>(d_jobs, d_prefix, njobs, d_counter, nt, grid, chunk, s); break;
    default: return fail(FS_ERR_INVALID, "unsupported gather tuning");
  }
  return hip_check(e, "batched gather launch");
}

fs_status launch_peel_batch(const PeelJob *d_jobs, uint32_t njobs, int mode, size_t lds_bytes, hipStream_t s) {
  if (njobs == 0) return FS_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (mode == kPeelLds) {
    static bool done[64] = {false};
    set_max_lds(reinterpret_cast<const void *>(&peel_batch_kernel<kPeelLds>), dev,
                device_info(dev).max_lds_per_block - 64, done);
    hipLaunchKernelGGL(peel_batch_kernel<kPeelLds>, dim3(njobs), dim3(kPeelThreads), lds_bytes, s, d_jobs);
  } else if (mode == kPeelLdsRows) {
    static bool done[64] = {false};
    set_max_lds(reinterpret_cast<const void *>(&peel_batch_kernel<kPeelLdsRows>), dev,
                device_info(dev).max_lds_per_block - 64, done);
    hipLaunchKernelGGL(peel_batch_kernel<kPeelLdsRows>, dim3(njobs), dim3(kPeelThreads), lds_bytes, s, d_jobs);
  } else if (mode == kPeelLdsRows32) {
    static bool done[64] = {false};
    set_max_lds(reinterpret_cast<const void *>(&peel_batch_kernel<kPeelLdsRows32>), dev,
                device_info(dev).max_lds_per_block - 64, done);
    hipLaunchKernelGGL(peel_batch_kernel<kPeelLdsRows32>, dim3(njobs), dim3(kPeelThreads), lds_bytes, s, d_jobs);
  } else {
    hipLaunchKernelGGL(peel_batch_kernel<kPeelGlobal>, dim3(njobs), dim3(kPeelThreads), 0, s, d_jobs);
  }
  return hip_check(hipGetLastError(), "batched peel launch");
}

fs_status launch_prog_batch(const ProgJob *d_jobs, uint32_t njobs, hipStream_t s) {
  if (njobs == 0) return FS_OK;
  hipLaunchKernelGGL(prog_batch_kernel, dim3(njobs), dim3(kPlanThreads), 0, s, d_jobs);
  return hip_check(hipGetLastError(), "batched program launch");
}

size_t replay_prog_lds_bound(uint32_t k, uint32_t pidx_cap) {
  const uint64_t bound = 2ull * (2ull * (k + 1) + 2ull * k + pidx_cap) + 256;
  return (size_t)((bound + 255) & ~255ull);
}

fs_status launch_replay_batch(const ReplayJob *d_rj, const ProgJob *d_pj, const uint32_t *d_wg_prefix,
                              uint32_t nitems, uint32_t total_wg, size_t prog_lds, hipStream_t s) {
  if (nitems == 0 || total_wg == 0) return FS_OK;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int budget = device_info(dev).max_lds_per_block;
  static bool done[64] = {false};
  set_max_lds(reinterpret_cast<const void *>(&replay_batch_kernel<kBatchReplayLanes>), dev, budget, done);
  const int lds = (int)std::min<size_t>((size_t)budget, prog_lds);
  hipLaunchKernelGGL(replay_batch_kernel<kBatchReplayLanes>, dim3(total_wg), dim3(kReplayThreads), lds, s, d_rj,
                     d_pj, d_wg_prefix, nitems, (uint32_t)lds, tune_snapshot().replay_prog_global ? 0u : 1u);
  return hip_check(hipGetLastError(), "batched replay launch");
}

fs_status launch_repair_prep_batch(const RepairPrepJob *d_jobs, uint32_t njobs, hipStream_t s) {
  if (njobs == 0) return FS_OK;
  hipLaunchKernelGGL(repair_prep_batch_kernel, dim3(njobs), dim3(kPlanThreads), 0, s, d_jobs);
  return hip_check(hipGetLastError(), "batched repair prep launch");
}

fs_status launch_update_plan_batch(const UpdatePlanJob *d_jobs, uint32_t njobs, hipStream_t s) {
  if (njobs == 0) return FS_OK;
  hipLaunchKernelGGL(update_plan_batch_kernel, dim3(njobs), dim3(kPlanThreads), 0, s, d_jobs);
  return hip_check(hipGetLastError(), "batched update plan launch");
}

fs_status launch_update_delta_batch(const UpdateDeltaJob *d_jobs, const uint32_t *d_prefix, uint32_t njobs,
                                    uint32_t total_wg, hipStream_t s) {
  if (njobs == 0 || total_wg == 0) return FS_OK;
  hipLaunchKernelGGL(update_delta_batch_kernel, dim3(total_wg), dim3(kDeltaThreads), 0, s, d_jobs, d_prefix, njobs);
  return hip_check(hipGetLastError(), "batched update delta launch");
}

void prepare_batch_kernels() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int budget = device_info(dev).max_lds_per_block;
  static bool d1[64] = {false}, d2[64] = {false}, d3[64] = {false}, d4[64] = {false};
  set_max_lds(reinterpret_cast<const void *>(&peel_batch_kernel<kPeelLds>), dev, budget - 64, d1);
  set_max_lds(reinterpret_cast<const void *>(&replay_batch_kernel<kBatchReplayLanes>), dev, budget, d2);
  set_max_lds(reinterpret_cast<const void *>(&peel_batch_kernel<kPeelLdsRows>), dev, budget - 64, d3);
  set_max_lds(reinterpret_cast<const void *>(&peel_batch_kernel<kPeelLdsRows32>), dev, budget - 64, d4);
}

fs_status launch_zero_batch(const ZeroEntry *d_rows, uint32_t nrows, uint64_t max_t, hipStream_t s) {
  const uint32_t chunks = (uint32_t)((max_t + 4095) / 4096);
  const uint64_t grid = (uint64_t)nrows * chunks;
  if (grid == 0) return FS_OK;
  hipLaunchKernelGGL(zero_batch_kernel, dim3((uint32_t)grid), dim3(256), 0, s, d_rows, nrows, chunks);
  return hip_check(hipGetLastError(), "batched zero launch");
}

}  // namespace fs
