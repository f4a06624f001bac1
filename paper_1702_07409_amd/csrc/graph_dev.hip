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
constexpr int kThreads = 1024;       // threads of the workgroup-wide kernels
constexpr int kRowBlk = 256;         // rows per block of the segment passes

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
// degrees, encode segments and heavy rows: a stable counting sort over lengths
// ---------------------------------------------------------------------------
// d_j = 1 + (number of thresholds <= the row's first draw >> 11); T is
// ascending and its last entry is 2^53, above every draw.
//
// Segment buckets: b = 64 - length, so that the longest come first (bucket 0
// holds the full kSegMax-edge pieces).  Per block of kRowBlk rows: the
// segment count of each bucket and the rows of more than kSegMax edges
// (blk_hist, bucket-major: [b * blocks + block]), the largest degree and the
// sum of the degrees.
__global__ __launch_bounds__(kRowBlk) void degree_kernel(DevGraphJob J) {
  __shared__ uint32_t hist[kSegMax + 1];   // [64] = heavy rows
  __shared__ uint32_t wmax[kRowBlk / 64], wsum[kRowBlk / 64];
  if (threadIdx.x <= kSegMax) hist[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t j = blockIdx.x * kRowBlk + threadIdx.x;
  uint32_t d = 0;
  if (j < J.n) {
    const uint64_t v0 = draw(row_key(J.seed, J.stripe_key, j), 0) >> 11;
    uint32_t lo = 0, hi = J.D;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (J.T[mid] <= v0) lo = mid + 1;
      else hi = mid;
    }
    d = lo + 1;
    J.deg[j] = (int32_t)d;
    if (d / kSegMax) atomicAdd(&hist[0], d / kSegMax);
    if (d % kSegMax) atomicAdd(&hist[kSegMax - d % kSegMax], 1u);
    if (d > kSegMax) atomicAdd(&hist[kSegMax], 1u);
  }
  // a block's degrees sum to at most 256 * 2^20
  uint32_t mx = d, sum = d;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    sum += (uint32_t)__shfl_xor((int)sum, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    wmax[threadIdx.x >> 6] = mx;
    wsum[threadIdx.x >> 6] = sum;
  }
  __syncthreads();
  if (threadIdx.x <= kSegMax) J.blk_hist[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = hist[threadIdx.x];
  if (threadIdx.x == 0) {
    uint32_t m = 0, t = 0;
    for (int w = 0; w < kRowBlk / 64; ++w) {
      m = max(m, wmax[w]);
      t += wsum[w];
    }
    J.blk_max[blockIdx.x] = m;
    J.blk_sum[blockIdx.x] = t;
  }
}

// One workgroup: per bucket, the exclusive prefix over blocks plus the
// bucket's start (buckets in order 0..63); the heavy rows likewise.  A wave
// scans its buckets' block counts 64 at a time, the loads of all its buckets
// issued together (also row_ptr from the degrees when scan_rows).  Also the
// scalars: the largest degree, the edge count,
// the segment and heavy-row counts (the others cleared for the later
// passes), and per bucket its first segment and first edge, from which a
// segment's offset follows (every segment of bucket b has 64 - b edges).
constexpr uint32_t kScanWaves = kThreads / 64;
constexpr uint32_t kBucketsPerWave = (kSegMax + kScanWaves) / kScanWaves;   // ceil(65 / waves)

static_assert(kThreads == kScanThreads, "seg_scan_kernel runs the one-workgroup scan");

__global__ __launch_bounds__(kThreads) void seg_scan_kernel(DevGraphJob J, uint32_t nblk, uint32_t scan_rows) {
  __shared__ uint32_t sh[kThreads / 64 + 1];
  __shared__ uint32_t tot[kSegMax + 1];
  __shared__ uint32_t start[kSegMax + 1];
  __shared__ uint32_t red_max[kScanWaves];
  __shared__ unsigned long long red_sum[kScanWaves];
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t run[kBucketsPerWave] = {};
  for (uint32_t c0 = 0; c0 < nblk; c0 += 64) {
    const uint32_t blk = c0 + lane;
    uint32_t c[kBucketsPerWave];
#pragma unroll
    for (uint32_t q = 0; q < kBucketsPerWave; ++q) {
      const uint32_t b = wid + q * kScanWaves;
      c[q] = (b <= kSegMax && blk < nblk) ? J.blk_hist[(uint64_t)b * nblk + blk] : 0u;
    }
#pragma unroll
    for (uint32_t q = 0; q < kBucketsPerWave; ++q) {
      const uint32_t b = wid + q * kScanWaves;
      uint32_t x = c[q];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if ((int)lane >= o) x += y;
      }
      if (b <= kSegMax && blk < nblk) J.blk_hist[(uint64_t)b * nblk + blk] = run[q] + x - c[q];
      run[q] += (uint32_t)__shfl((int)x, 63, 64);
    }
  }
#pragma unroll
  for (uint32_t q = 0; q < kBucketsPerWave; ++q) {
    const uint32_t b = wid + q * kScanWaves;
    if (b <= kSegMax && lane == 0) tot[b] = run[q];
  }
  uint32_t mx = 0;
  unsigned long long sum = 0;
  for (uint32_t blk = threadIdx.x; blk < nblk; blk += kThreads) {
    mx = max(mx, J.blk_max[blk]);
    sum += J.blk_sum[blk];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, o, 64));
    sum += (unsigned long long)__shfl_xor((long long)sum, o, 64);
  }
  if (lane == 0) {
    red_max[wid] = mx;
    red_sum[wid] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0, edge = 0;
    for (uint32_t q = 0; q < kSegMax; ++q) {
      start[q] = acc;
      J.bucket[q] = (int32_t)acc;
      J.bucket[kSegMax + 1 + q] = (int32_t)edge;
      acc += tot[q];
      edge += tot[q] * (kSegMax - q);   // below 2^31: the host rejects larger graphs
    }
    start[kSegMax] = 0;
    uint32_t m = 0;
    unsigned long long e = 0;
    for (uint32_t w = 0; w < kScanWaves; ++w) {
      m = max(m, red_max[w]);
      e += red_sum[w];
    }
    J.scalars[kScalarMaxDeg] = (int32_t)m;
    J.scalars[kScalarSegs] = (int32_t)acc;
    J.scalars[kScalarHeavy] = (int32_t)tot[kSegMax];
    J.scalars[kScalarMaxCdeg] = 0;
    J.scalars[kScalarMidCols] = 0;
    J.scalars[kScalarLongCols] = 0;
    *J.edges = e;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < (kSegMax + 1) * nblk; i += kThreads) J.blk_hist[i] += start[i / nblk];
  // row_ptr from the degrees (short row counts; longer ones take the
  // three-pass scan before this kernel)
  if (scan_rows) scan_one_block(J.deg, J.n, J.row_ptr, nullptr, sh);
}

// Each row's segments at their sorted positions: full pieces in bucket 0
// (row order, then piece order), the remainder in its length's bucket (row
// order).  Ranks within a block: a block scan for the full pieces; for the
// remainders, lanes of equal length are found by ballots over the length's
// six bits, and waves are ordered through per-(wave, bucket) counts.  A row
// of several full pieces has them written by its whole wave.  A segment's
// first edge in seg_col follows from its bucket's first segment and edge.
// The heavy rows also go after the scalars, for one copy to the host.  The
// kernel also copies row_ptr into the image and clears the column counters.
__global__ __launch_bounds__(kRowBlk) void seg_place_kernel(DevGraphJob J) {
  __shared__ uint32_t sh[kRowBlk / 64 + 1];
  __shared__ uint32_t wcnt[kRowBlk / 64][kSegMax + 1];   // [.][64]: heavy rows
  constexpr int NW = kRowBlk / 64;
  const uint32_t j = blockIdx.x * kRowBlk + threadIdx.x;
  for (uint32_t i = j; i < J.k; i += gridDim.x * kRowBlk) {
    J.ccnt[i] = 0;
    J.cfill[i] = 0;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool live = j < J.n;
  const uint32_t d = live ? (uint32_t)J.deg[j] : 0u;
  const int32_t e0 = live ? J.row_src[j] : 0;
  if (live) J.row_ptr[j] = e0;
  if (j + 1 == J.n) J.row_ptr[J.n] = J.row_src[J.n];
  const uint32_t full = d / kSegMax, rest = d % kSegMax;
  const uint32_t nblk = gridDim.x;
  auto off = [&](uint32_t bucket) { return J.blk_hist[(uint64_t)bucket * nblk + blockIdx.x]; };
  uint32_t total = 0;
  const uint32_t full_rank = scan_block<kRowBlk>(full, sh, total);
  for (int i = threadIdx.x; i < NW * (kSegMax + 1); i += kRowBlk) (&wcnt[0][0])[i] = 0;
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
  const bool split = d > kSegMax;
  const uint32_t off0 = off(0);   // bucket 0 starts at segment 0 and edge 0
  if (j == 0) J.seg_ptr[J.scalars[kScalarSegs]] = J.row_src[J.n];
  if (full == 1) {
    const uint32_t at = off0 + full_rank;
    J.seg_row[at] = (int32_t)j;
    J.seg_len[at] = (int32_t)kSegMax;
    J.seg_beg[at] = e0;
    J.seg_ptr[at] = (int32_t)(at * kSegMax);
    J.seg_atomic[at] = split ? 1 : 0;
  }
  // rows of two or more full pieces (all split), one at a time by the wave
  for (uint64_t many = __ballot(full > 1); many; many &= many - 1) {
    const int src = __ffsll((long long)many) - 1;
    const uint32_t f = (uint32_t)__shfl((int)full, src, 64);
    const uint32_t r0 = off0 + (uint32_t)__shfl((int)full_rank, src, 64);
    const int32_t row = __shfl((int)j, src, 64), beg = __shfl(e0, src, 64);
    for (uint32_t s = lane; s < f; s += 64) {
      J.seg_row[r0 + s] = row;
      J.seg_len[r0 + s] = (int32_t)kSegMax;
      J.seg_beg[r0 + s] = beg + (int32_t)(s * kSegMax);
      J.seg_ptr[r0 + s] = (int32_t)((r0 + s) * kSegMax);
      J.seg_atomic[r0 + s] = 1;
    }
  }
  if (live && rest) {
    uint32_t before = 0;
    for (int w = 0; w < wid; ++w) before += wcnt[w][b];
    const uint32_t at = off(b) + before + (uint32_t)__popcll(same & lt);
    J.seg_row[at] = (int32_t)j;
    J.seg_len[at] = (int32_t)rest;
    J.seg_beg[at] = e0 + (int32_t)(full * kSegMax);
    J.seg_ptr[at] = J.bucket[kSegMax + 1 + b] + (int32_t)((at - (uint32_t)J.bucket[b]) * rest);
    J.seg_atomic[at] = split ? 1 : 0;
  }
  if (split) {
    uint32_t before = 0;
    for (int w = 0; w < wid; ++w) before += wcnt[w][kSegMax];
    const uint32_t at = off(kSegMax) + before + (uint32_t)__popcll(heavy_mask & lt);
    J.heavy[at] = (int32_t)j;
    J.scalars[kScalarWords + at] = (int32_t)j;
  }
}

// segment s into seg_col: one wave (at most kSegMax edges), a lane per edge
__device__ __forceinline__ void seg_copy(const DevGraphJob &J, uint32_t s, int lane) {
  if (lane < J.seg_len[s]) J.seg_col[J.seg_ptr[s] + lane] = J.col[J.seg_beg[s] + lane];
}

// ---------------------------------------------------------------------------
// neighbours (each pick also counted in its column, ccnt)
// ---------------------------------------------------------------------------
// Floyd's steps of a row of degree d, one per lane of a group of lanes
// (gm: the group's lanes, gbase: its first lane; live: the step exists; base
// = k - d, so that a lane's fallback is r = base + its step).  A lane falls
// back to its r when its candidate v was picked before it: by an earlier
// lane, either as that lane's v (then v was in the set before whatever that
// lane did) or as that lane's r (only when that lane fell back; the lane is
// found from v as v - base).  Equal candidates are found by one ballot per
// bit of v (nbits = bits of k - 1); the fallback chains are followed to their
// fixed point, at most one round per link.  Returns the lane's pick.
__device__ __forceinline__ uint32_t floyd_group(uint32_t v, uint32_t r, bool live, uint32_t base, int nbits,
                                                uint64_t gm, int gbase) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (lane ? (~0ull >> (64 - lane)) : 0ull) & gm;
  uint64_t same = __ballot(live) & gm;
  for (int bit = 0; bit < nbits; ++bit) {
    const bool one = (v >> bit) & 1u;
    const uint64_t ones = __ballot(live && one);
    same &= one ? ones : ~ones;
  }
  bool dup = live && (same & lt) != 0;
  const bool in_range = live && v >= base && v - base < (uint32_t)(lane - gbase);
  const uint32_t at = in_range ? (uint32_t)gbase + (v - base) : 0u;
  for (;;) {
    const uint64_t mask = __ballot(dup);
    const bool nd = dup || (in_range && ((mask >> at) & 1ull));
    if (__ballot(nd != dup) == 0ull) break;
    dup = nd;
  }
  return dup ? r : v;
}

// Number of live lanes of the group whose x is below this lane's (x <
// 2^nbits): bits from the top, keeping the lanes that agree so far.
__device__ __forceinline__ uint32_t group_rank(uint32_t x, bool live, int nbits, uint64_t gm) {
  uint64_t agree = __ballot(live) & gm, below = 0;
  for (int bit = nbits - 1; bit >= 0; --bit) {
    const bool one = (x >> bit) & 1u;
    const uint64_t ones = __ballot(live && one);
    if (one) below |= agree & ~ones;
    agree &= one ? ones : ~ones;
  }
  return (uint32_t)__popcll(below);
}

__device__ __forceinline__ int bits_for(uint32_t k) { return k > 1 ? 32 - __clz((int)(k - 1)) : 1; }

// Rows of at most kSegMax neighbours, four rows per wave: rows of at most
// kLightMax neighbours take a group of 16 lanes each, lane s taking Floyd's
// step s (floyd_group); then each longer row of the four takes the whole
// wave.  A lane's place in the sorted row is the number of picks below its
// own.
constexpr uint32_t kLightMax = 16;

__device__ __forceinline__ void sample_rows_wave(const DevGraphJob &J, uint32_t wave) {
  const int lane = threadIdx.x & 63;
  const uint32_t j0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(wave * 4u));
  if (j0 >= J.n) return;
  const int nbits = bits_for(J.k);
  const int g = lane >> 4;
  const uint32_t j = j0 + (uint32_t)g;
  const uint32_t d = j < J.n ? (uint32_t)J.deg[j] : 0u;
  {
    const uint32_t step = (uint32_t)(lane & 15);
    const bool live = d <= kLightMax && step < d;
    uint32_t r = 0, v = 0;
    if (live) v = floyd_candidate(row_key(J.seed, J.stripe_key, j), J.k, d, step, r);
    const uint64_t gm = 0xFFFFull << (16 * g);
    const uint32_t pick = floyd_group(v, r, live, J.k - min(d, J.k), nbits, gm, 16 * g);
    const uint32_t below = group_rank(pick, live, nbits, gm);
    if (live) {
      J.col[J.row_ptr[j] + below] = (int32_t)pick;
      atomicAdd(&J.ccnt[pick], 1);
    }
  }
  for (uint64_t med = __ballot((lane & 15) == 0 && d > kLightMax && d <= kSegMax); med; med &= med - 1) {
    const int src = __ffsll((long long)med) - 1;
    const uint32_t jm = j0 + (uint32_t)(src >> 4);
    const uint32_t dm = (uint32_t)__builtin_amdgcn_readlane((int)d, src);
    const bool live = (uint32_t)lane < dm;
    uint32_t r = 0, v = 0;
    if (live) v = floyd_candidate(row_key(J.seed, J.stripe_key, jm), J.k, dm, (uint32_t)lane, r);
    const uint32_t pick = floyd_group(v, r, live, J.k - dm, nbits, ~0ull, 0);
    const uint32_t below = group_rank(pick, live, nbits, ~0ull);
    if (live) {
      J.col[J.row_ptr[jm] + below] = (int32_t)pick;
      atomicAdd(&J.ccnt[pick], 1);
    }
  }
}

// Rows of more than kSegMax neighbours: a workgroup each, kThreads of
// Floyd's steps at a time against a k-bit LDS bitmap of the earlier batches'
// picks.  Within a batch a lane falls back when its candidate was picked
// before it (as for floyd_wave): equal candidates meet in an LDS hash table
// that keeps the first lane of each, and the fallback chains are followed to
// their fixed point through per-lane flags.  A fallback r is never taken
// (every earlier pick is at most the previous step's r).  The set bits, read
// in order, are the sorted row.
constexpr int kHashBits = 11;
constexpr uint32_t kHash = 1u << kHashBits;   // twice the lanes of a batch
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr size_t kHeavyStaticLds = 20u << 10;   // above what the kernel declares statically

__device__ void sample_heavy_block(const DevGraphJob &J, uint32_t h_index) {
  extern __shared__ uint32_t bits[];   // ceil(k / 32) words
  __shared__ uint32_t sh[kThreads / 64 + 1];
  __shared__ uint32_t hkey[kHash], hlane[kHash];
  __shared__ uint8_t fell[kThreads];
  const uint32_t t = threadIdx.x;
  const uint32_t j = (uint32_t)J.heavy[h_index];
  const uint32_t d = (uint32_t)J.deg[j];
  const uint32_t words = (J.k + 31) / 32;
  for (uint32_t w = t; w < words; w += kThreads) bits[w] = 0;
  for (uint32_t h = t; h < kHash; h += kThreads) {
    hkey[h] = kEmpty;
    hlane[h] = kEmpty;
  }
  __syncthreads();
  const uint64_t key = row_key(J.seed, J.stripe_key, j);
  for (uint32_t s0 = 0; s0 < d; s0 += kThreads) {
    const bool live = s0 + t < d;
    uint32_t r = 0, v = 0;
    if (live) v = floyd_candidate(key, J.k, d, s0 + t, r);
    bool dup = live && ((bits[v >> 5] >> (v & 31)) & 1u);
    const bool insert = live && !dup;
    uint32_t h = (v * 0x9E3779B1u) >> (32 - kHashBits);
    if (insert) {
      for (;;) {
        const uint32_t old = atomicCAS(&hkey[h], kEmpty, v);
        if (old == kEmpty || old == v) break;
        h = (h + 1) & (kHash - 1);
      }
      atomicMin(&hlane[h], t);
    }
    __syncthreads();
    if (insert) dup = hlane[h] < t;
    const uint32_t base = J.k - d + s0;
    const bool in_range = live && v >= base && v - base < t;
    const uint32_t q = in_range ? v - base : 0u;
    fell[t] = dup ? 1 : 0;
    __syncthreads();
    // flags only turn on, so a flag read while it is being set is harmless;
    // a round in which nothing changes has read the settled flags
    for (;;) {
      int changed = 0;
      if (in_range && !dup && fell[q]) {
        dup = true;
        fell[t] = 1;
        changed = 1;
      }
      if (!__syncthreads_or(changed)) break;
    }
    const uint32_t pick = dup ? r : v;
    if (live) atomicOr(&bits[pick >> 5], 1u << (pick & 31));
    if (insert) {
      hkey[h] = kEmpty;
      hlane[h] = kEmpty;
    }
    __syncthreads();
  }
  int32_t *out = J.col + J.row_ptr[j];
  uint32_t done = 0;
  for (uint32_t w0 = 0; w0 < words; w0 += kThreads) {
    const uint32_t w = w0 + t;
    uint32_t m = w < words ? bits[w] : 0u;
    uint32_t total = 0;
    uint32_t at = done + scan_block<kThreads>((uint32_t)__popc(m), sh, total);
    while (m) {
      const uint32_t bit = (uint32_t)__ffs(m) - 1;
      out[at++] = (int32_t)(w * 32 + bit);
      atomicAdd(&J.ccnt[w * 32 + bit], 1);
      m &= m - 1;
    }
    done += total;
  }
}

// One launch for all rows: the first nheavy workgroups take the heavy rows
// (the longest work, so they start first), the rest four rows per wave.
__global__ __launch_bounds__(kThreads) void sample_kernel(DevGraphJob J, uint32_t nheavy) {
  if (blockIdx.x < nheavy) {
    sample_heavy_block(J, blockIdx.x);
    return;
  }
  sample_rows_wave(J, (blockIdx.x - nheavy) * (kThreads / 64) + (threadIdx.x >> 6));
}

// ---------------------------------------------------------------------------
// transpose
// ---------------------------------------------------------------------------
// The samplers count each column's rows; each edge is then placed in its
// column by a fill cursor (one thread per edge, the row found by a binary
// search of row_ptr), which leaves a column's rows in arbitrary order in
// `unsorted`; each column is then sorted into rowidx by the kernel that fits
// its length.
// the row holding edge e: the last j with row_ptr[j] <= e
__device__ __forceinline__ uint32_t row_of(const int32_t *row_ptr, uint32_t n, uint32_t e) {
  uint32_t lo = 0, hi = n;   // row_ptr[lo] <= e < row_ptr[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if ((uint32_t)row_ptr[mid] <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void col_fill_kernel(DevGraphJob J) {
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  if (e >= J.nnz) return;
  const int32_t i = J.col[e];
  const int32_t at = atomicAdd(&J.cfill[i], 1);
  J.unsorted[J.col_ptr[i] + at] = (int32_t)row_of(J.row_ptr, J.n, e);
}

// Columns of at most 64 rows: one wave each, a lane per entry, placed by
// its rank among the column's (distinct) rows.  Longer columns are listed
// for the two kernels below: up to kMidCol rows from the front of col_list,
// more from its back.
constexpr int32_t kMidCol = 1024;

// The waves after the first k copy the encode segments (seg_copy).
__global__ __launch_bounds__(256) void col_sort_kernel(DevGraphJob J, uint32_t nseg) {
  const int lane = threadIdx.x & 63;
  const uint32_t i = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4u + (threadIdx.x >> 6)));
  if (i >= J.k) {
    if (i - J.k < nseg) seg_copy(J, i - J.k, lane);
    return;
  }
  const int32_t b = __builtin_amdgcn_readfirstlane(J.col_ptr[i]);
  const int32_t c = __builtin_amdgcn_readfirstlane(J.col_ptr[i + 1]) - b;
  if (c <= 64) {
    const bool live = lane < c;
    const uint32_t v = live ? (uint32_t)J.unsorted[b + lane] : 0u;
    const uint32_t below = group_rank(v, live, bits_for(J.n), ~0ull);
    if (live) J.rowidx[b + (int32_t)below] = (int32_t)v;
  } else if (lane == 0) {
    if (c <= kMidCol) J.col_list[atomicAdd(J.scalars + kScalarMidCols, 1)] = (int32_t)i;
    else J.col_list[J.k - 1 - (uint32_t)atomicAdd(J.scalars + kScalarLongCols, 1)] = (int32_t)i;
  }
}

// Columns of more than 64 rows, a workgroup each.  Up to kMidCol rows: an
// entry's place is the number of entries below it (a column's rows are
// distinct).  Longer: a bitmap over kLongRows rows at a time, its set bits
// read in order.  The counts of both lists come from col_sort_kernel.
constexpr uint32_t kLongWords = 15360;   // under 64 KiB with the scan words
constexpr uint32_t kLongRows = kLongWords * 32;
constexpr uint32_t kBigThreads = 256;

__global__ __launch_bounds__(kBigThreads) void col_sort_big_kernel(DevGraphJob J) {
  __shared__ uint32_t bits[kLongWords];   // a mid column uses the first kMidCol words
  __shared__ uint32_t sh[kBigThreads / 64 + 1];
  const uint32_t nmid = (uint32_t)J.scalars[kScalarMidCols];
  const uint32_t nlong = (uint32_t)J.scalars[kScalarLongCols];
  const uint32_t t = threadIdx.x;
  for (uint32_t x = blockIdx.x; x < nmid + nlong; x += gridDim.x) {
    const uint32_t i = (uint32_t)J.col_list[x < nmid ? x : J.k - 1 - (x - nmid)];
    const int32_t b = J.col_ptr[i], c = J.col_ptr[i + 1] - b;
    if (x < nmid) {
      int32_t *buf = reinterpret_cast<int32_t *>(bits);
      for (int32_t a = (int32_t)t; a < c; a += kBigThreads) buf[a] = J.unsorted[b + a];
      __syncthreads();
      for (int32_t a = (int32_t)t; a < c; a += kBigThreads) {
        const int32_t v = buf[a];
        int32_t below = 0;
        for (int32_t q = 0; q < c; ++q) below += buf[q] < v ? 1 : 0;
        J.rowidx[b + below] = v;
      }
      __syncthreads();
      continue;
    }
    uint32_t done = 0;
    for (uint32_t lo = 0; lo < J.n; lo += kLongRows) {
      const uint32_t span = min(J.n - lo, kLongRows), words = (span + 31) / 32;
      for (uint32_t w = t; w < words; w += kBigThreads) bits[w] = 0;
      __syncthreads();
      for (int32_t a = (int32_t)t; a < c; a += kBigThreads) {
        const uint32_t rr = (uint32_t)J.unsorted[b + a] - lo;
        if (rr < span) atomicOr(&bits[rr >> 5], 1u << (rr & 31));
      }
      __syncthreads();
      for (uint32_t w0 = 0; w0 < words; w0 += kBigThreads) {
        const uint32_t w = w0 + t;
        uint32_t m = w < words ? bits[w] : 0u;
        uint32_t total = 0;
        uint32_t at = done + scan_block<kBigThreads>((uint32_t)__popc(m), sh, total);
        while (m) {
          const uint32_t bit = (uint32_t)__ffs(m) - 1;
          J.rowidx[b + (int32_t)at++] = (int32_t)(lo + w * 32 + bit);
          m &= m - 1;
        }
        done += total;
      }
      __syncthreads();
    }
  }
}

fs_status hip_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

void dev_graph_carve(Carver &cv, DevGraphJob &J, uint32_t k, uint32_t n) {
  const uint32_t nblk = (n + kRowBlk - 1) / kRowBlk;
  J.deg = cv.take<int32_t>(n);
  J.row_ptr = cv.take<int32_t>((size_t)n + 1);
  J.blk_hist = cv.take<uint32_t>((size_t)nblk * (kSegMax + 1));
  // the scalars, the edge count in their last two words, then room for the
  // heavy-row list
  J.scalars = cv.take<int32_t>(kScalarWords + (size_t)n);
  J.edges = reinterpret_cast<unsigned long long *>(J.scalars + kScalarCount);
  J.blk_max = cv.take<uint32_t>(nblk);
  J.blk_sum = cv.take<uint32_t>(nblk);
  J.bucket = cv.take<int32_t>(2 * (kSegMax + 1));
  J.sums = cv.take<uint32_t>(scan_sums_for(std::max(n, k)) + 1);
  J.ccnt = cv.take<int32_t>(k);
  J.cfill = cv.take<int32_t>(k);
}

void dev_graph_carve_rows(Carver &cv, DevGraphJob &J, uint32_t k, uint32_t n, uint32_t nseg, uint64_t nnz) {
  J.seg_len = cv.take<int32_t>(nseg);
  J.unsorted = cv.take<int32_t>(nnz);
  J.col_list = cv.take<int32_t>(k);
  J.seg_beg = cv.take<int32_t>(nseg);
  J.sums = cv.take<uint32_t>(scan_sums_for(std::max(n, k)) + 1);
}

fs_status launch_dev_graph_degrees(const DevGraphJob &J, hipStream_t s) {
  if (J.n == 0) return FS_OK;
  const uint32_t nblk = (J.n + kRowBlk - 1) / kRowBlk;
  hipLaunchKernelGGL(degree_kernel, dim3(nblk), dim3(kRowBlk), 0, s, J);
  // row_ptr from the degrees (the last entry is nnz): in the bucket scan's
  // workgroup when the rows are few
  const uint32_t scan_rows = J.n <= kScanOneMax ? 1u : 0u;
  if (!scan_rows) {
    const fs_status st = scan_i32(J.deg, J.n, J.sums, J.row_ptr, s);
    if (st != FS_OK) return st;
  }
  hipLaunchKernelGGL(seg_scan_kernel, dim3(1), dim3(kThreads), 0, s, J, nblk, scan_rows);
  return hip_ok(hipGetLastError(), "graph degree launch");
}

fs_status launch_dev_graph_rows(const DevGraphJob &J, uint32_t nseg, uint32_t nheavy, hipStream_t s) {
  const uint32_t nblk = (J.n + kRowBlk - 1) / kRowBlk;
  hipLaunchKernelGGL(seg_place_kernel, dim3(nblk), dim3(kRowBlk), 0, s, J);
  // the heavy rows' bitmap in dynamic LDS (every workgroup gets it)
  const size_t lds = (size_t)((J.k + 31) / 32) * 4;
  static bool done[64] = {false};
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) return fail(FS_ERR_INVALID, "device index out of range");
  const size_t cap = (size_t)device_info(dev).max_lds_per_block - kHeavyStaticLds;
  if (lds > cap) return fail(FS_ERR_UNSUPPORTED, "k too large for the heavy-row bitmap in LDS");
  if (!done[dev]) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&sample_kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap);
    if (e != hipSuccess) return hip_ok(e, "row sampler LDS");
    done[dev] = true;
  }
  const uint32_t row_blocks = (J.n + 4 * (kThreads / 64) - 1) / (4 * (kThreads / 64));
  hipLaunchKernelGGL(sample_kernel, dim3(nheavy + row_blocks), dim3(kThreads), lds, s, J, nheavy);
  fs_status st = scan_i32(J.ccnt, J.k, J.sums, J.col_ptr, s, J.scalars + kScalarMaxCdeg);
  if (st != FS_OK) return st;
  hipLaunchKernelGGL(col_fill_kernel, dim3((uint32_t)((J.nnz + 255) / 256)), dim3(256), 0, s, J);
  hipLaunchKernelGGL(col_sort_kernel, dim3((uint32_t)(((uint64_t)J.k + nseg + 3) / 4)), dim3(256), 0, s, J, nseg);
  // the longer columns' kernels read their counts on the device
  hipLaunchKernelGGL(col_sort_big_kernel, dim3(std::min<uint32_t>(J.k, 1024)), dim3(kBigThreads), 0, s, J);
  return hip_ok(hipGetLastError(), "graph rows launch");
}

}  // namespace fs
