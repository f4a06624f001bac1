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

#include "fs_internal.h"

namespace fs {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ v4u ld16(const uint8_t *p) { return *reinterpret_cast<const v4u *>(p); }

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

template <int LPR, int CH, bool NT>
__global__ __launch_bounds__(kGatherThreads) void gather_kernel(GatherJob j, uint32_t nslices,
                                                                 uint32_t remap) {
  constexpr uint32_t RPB = kGatherThreads / LPR;   // rows per tile
  constexpr uint32_t STEP = LPR * 16;              // bytes between a lane's chunks
  constexpr uint32_t W = STEP * CH;                // slice bytes
  if (j.skip_flag && *j.skip_flag) return;
  uint32_t nrows = j.nrows;
  if (j.nrows_dev) nrows = min(nrows, (uint32_t)max(*j.nrows_dev, 0));
  const uint32_t ntiles = (nrows + RPB - 1) / RPB;
  const uint64_t nitems = (uint64_t)ntiles * nslices;
  const uint32_t vb = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const uint32_t lane = threadIdx.x % LPR;
  const uint32_t sub = threadIdx.x / LPR;
  for (uint64_t item = vb; item < nitems; item += gridDim.x) {
    const uint32_t slice = (uint32_t)(item / ntiles);
    const uint32_t tile = (uint32_t)(item % ntiles);
    const uint32_t r = tile * RPB + sub;
    if (r >= nrows) continue;
    const uint32_t jr = j.csr_map ? j.csr_map[r] : r;
    if (jr >= j.csr_rows) continue;
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
      continue;
    }
    if (j.accumulate) {
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (valid[c]) acc[c] = ld16(out + c * STEP);
    }
    const uint8_t *src = j.src + off0;
    int e = j.ptr[jr];
    const int e1 = j.ptr[jr + 1];
    for (; e + 4 <= e1; e += 4) {
      const uint8_t *p0 = src + (uint64_t)j.idx[e] * j.src_stride;
      const uint8_t *p1 = src + (uint64_t)j.idx[e + 1] * j.src_stride;
      const uint8_t *p2 = src + (uint64_t)j.idx[e + 2] * j.src_stride;
      const uint8_t *p3 = src + (uint64_t)j.idx[e + 3] * j.src_stride;
      v4u v0[CH], v1[CH], v2[CH], v3[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        if (valid[c]) {
          v0[c] = ld16(p0 + c * STEP);
          v1[c] = ld16(p1 + c * STEP);
          v2[c] = ld16(p2 + c * STEP);
          v3[c] = ld16(p3 + c * STEP);
        }
      }
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (valid[c]) acc[c] ^= (v0[c] ^ v1[c]) ^ (v2[c] ^ v3[c]);
    }
    for (; e < e1; ++e) {
      const uint8_t *p0 = src + (uint64_t)j.idx[e] * j.src_stride;
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (valid[c]) acc[c] ^= ld16(p0 + c * STEP);
    }
#pragma unroll
    for (int c = 0; c < CH; ++c)
      if (valid[c]) st16<NT>(out + c * STEP, acc[c]);
  }
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
constexpr unsigned long long kCountOne = 1ull << 40;   // acc = count << 40 | sum of ids
constexpr unsigned long long kSumMask = kCountOne - 1;

struct PeelState {
  unsigned long long *acc, *best;
  int32_t *fa, *fb, *dl;
  uint32_t *mask, *decm;
};

__device__ __forceinline__ uint32_t words_of(uint32_t k) { return (k + 31) / 32; }

template <bool LDS>
__global__ __launch_bounds__(kPeelThreads) void peel_kernel(PeelJob J) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ uint32_t scan_sh[kPeelThreads / 64 + 1];
  __shared__ int s_nA, s_nB, s_nD;
  if (J.skip_flag && *J.skip_flag) return;
  const uint32_t k = J.k, n = J.n, kw = words_of(k);
  const int tid = threadIdx.x;
  PeelState S;
  if constexpr (LDS) {
    unsigned char *p = smem;
    S.acc = reinterpret_cast<unsigned long long *>(p); p += 8ull * n;
    S.best = reinterpret_cast<unsigned long long *>(p); p += 8ull * k;
    S.fa = reinterpret_cast<int32_t *>(p); p += 4ull * n;
    S.fb = reinterpret_cast<int32_t *>(p); p += 4ull * n;
    S.dl = reinterpret_cast<int32_t *>(p); p += 4ull * k;
    S.mask = reinterpret_cast<uint32_t *>(p); p += 4ull * kw;
    S.decm = reinterpret_cast<uint32_t *>(p);
  } else {
    S.acc = J.acc; S.best = J.best; S.fa = J.front_a; S.fb = J.front_b; S.dl = J.dlist;
    S.mask = J.mask; S.decm = J.decmask;
  }
  for (uint32_t f = tid; f < k; f += kPeelThreads) {
    S.best[f] = ~0ull;
    J.recovered[f] = 0;
  }
  for (uint32_t w = tid; w < kw; w += kPeelThreads) {
    S.mask[w] = 0;
    S.decm[w] = 0;
  }
  if (tid == 0) {
    s_nA = 0;
    s_nB = 0;
    s_nD = 0;
    J.level_ptr[0] = 0;
  }
  __syncthreads();
  for (uint32_t g = tid; g < n; g += kPeelThreads) {
    if (J.erased[g]) {
      S.acc[g] = 0;
      continue;
    }
    const int e0 = J.row_ptr[g], e1 = J.row_ptr[g + 1];
    unsigned long long sum = 0;
    for (int e = e0; e < e1; ++e) sum += (unsigned)J.col[e];
    S.acc[g] = ((unsigned long long)(e1 - e0) << 40) | sum;
    if (e1 - e0 == 1) S.fa[atomicAdd(&s_nA, 1)] = (int32_t)g;
  }
  __syncthreads();

  // words of the k-bit masks handled by this thread (contiguous, ascending)
  const uint32_t wpt = (kw + kPeelThreads - 1) / kPeelThreads;
  const uint32_t w0 = min(kw, (uint32_t)tid * wpt), w1 = min(kw, w0 + wpt);
  int32_t *cur = S.fa, *nxt = S.fb;
  uint32_t level = 0, npairs = 0;
  while (true) {
    const int nA = s_nA;
    if (nA == 0 || (J.maxit != 0 && level == J.maxit)) break;
    // every surviving row of residual weight 1 names its last unknown input;
    // keep the namer of least (original degree, row)
    for (int q = tid; q < nA; q += kPeelThreads) {
      const int32_t g = cur[q];
      const unsigned long long a = S.acc[g];
      if ((a >> 40) != 1ull) continue;
      const uint32_t f = (uint32_t)(a & kSumMask);
      const uint32_t d = (uint32_t)(J.row_ptr[g + 1] - J.row_ptr[g]);
      atomicMin(&S.best[f], ((unsigned long long)d << 32) | (uint32_t)g);
      const uint32_t bit = 1u << (f & 31);
      const uint32_t old = atomicOr(&S.mask[f >> 5], bit);
      if (!(old & bit)) S.dl[atomicAdd(&s_nD, 1)] = (int32_t)f;
    }
    __syncthreads();
    const int nD = s_nD;
    if (nD == 0) break;
    // list the level's inputs in ascending order
    uint32_t cnt = 0;
    for (uint32_t w = w0; w < w1; ++w) cnt += __popc(S.mask[w]);
    uint32_t total;
    uint32_t pos = npairs + block_exclusive_scan<kPeelThreads>(cnt, scan_sh, total);
    for (uint32_t w = w0; w < w1; ++w) {
      uint32_t m = S.mask[w];
      if (!m) continue;
      S.mask[w] = 0;
      S.decm[w] |= m;
      while (m) {
        const uint32_t f = w * 32 + __builtin_ctz(m);
        J.dp_f[pos] = (int32_t)f;
        J.dp_g[pos] = (int32_t)(uint32_t)(S.best[f] & 0xffffffffull);
        J.recovered[f] = 1;
        ++pos;
        m &= m - 1;
      }
    }
    // remove the decoded inputs from every surviving row they touch; a row
    // whose residual weight drops to 1 joins the next frontier
    for (int q = tid; q < nD; q += kPeelThreads) {
      const uint32_t f = (uint32_t)S.dl[q];
      const unsigned long long dec = 0ull - (kCountOne | f);
      for (int e = J.col_ptr[f]; e < J.col_ptr[f + 1]; ++e) {
        const int32_t h = J.rowidx[e];
        if (J.erased[h]) continue;
        const unsigned long long old = atomicAdd(&S.acc[h], dec);
        if ((old >> 40) == 2ull) nxt[atomicAdd(&s_nB, 1)] = h;
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
    __syncthreads();
  }
  // the unrecovered inputs follow the schedule, ascending, with row -1
  uint32_t cnt = 0;
  for (uint32_t w = w0; w < w1; ++w) {
    uint32_t um = ~S.decm[w];
    if (w == kw - 1 && (k & 31)) um &= (1u << (k & 31)) - 1u;
    cnt += __popc(um);
  }
  uint32_t total;
  uint32_t pos = npairs + block_exclusive_scan<kPeelThreads>(cnt, scan_sh, total);
  for (uint32_t w = w0; w < w1; ++w) {
    uint32_t um = ~S.decm[w];
    if (w == kw - 1 && (k & 31)) um &= (1u << (k & 31)) - 1u;
    while (um) {
      const uint32_t f = w * 32 + __builtin_ctz(um);
      J.dp_f[pos] = (int32_t)f;
      J.dp_g[pos] = -1;
      ++pos;
      um &= um - 1;
    }
  }
  if (tid == 0) {
    J.status[0] = npairs == k ? 1 : 0;
    J.status[1] = (int32_t)(k - npairs);
    J.status[2] = (int32_t)level;
  }
}

// ---------------------------------------------------------------------------
// schedule replay
// ---------------------------------------------------------------------------
constexpr int kReplayThreads = 1024;

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
constexpr int kPlanThreads = 1024;

__global__ __launch_bounds__(kPlanThreads) void repair_prep_kernel(RepairPrepJob J, int default_ok) {
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

__global__ __launch_bounds__(kPlanThreads) void update_plan_kernel(UpdatePlanJob J) {
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

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static fs_status hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

fs_status launch_gather(const GatherJob &job, const fs_tune &tune, hipStream_t s) {
  int dev = 0;
  hipGetDevice(&dev);
  const int cu = device_info(dev).cu_count;
  hipError_t e;
  switch (tune.lanes_per_row * 10 + tune.chunks) {
    case 161: e = run_gather_nt<16, 1>(job, tune, s, cu); break;
    case 162: e = run_gather_nt<16, 2>(job, tune, s, cu); break;
    case 164: e = run_gather_nt<16, 4>(job, tune, s, cu); break;
    case 321: e = run_gather_nt<32, 1>(job, tune, s, cu); break;
    case 322: e = run_gather_nt<32, 2>(job, tune, s, cu); break;
    case 324: e = run_gather_nt<32, 4>(job, tune, s, cu); break;
    case 641: e = run_gather_nt<64, 1>(job, tune, s, cu); break;
    case 642: e = run_gather_nt<64, 2>(job, tune, s, cu); break;
    case 644: e = run_gather_nt<64, 4>(job, tune, s, cu); break;
    default: return fail(FS_ERR_INVALID, "unsupported gather tuning");
  }
  return hip_check(e, "gather launch");
}

size_t peel_lds_bytes(uint32_t k, uint32_t n) {
  const size_t kw = (k + 31) / 32;
  return 8ull * n + 8ull * k + 4ull * n + 4ull * n + 4ull * k + 8ull * kw;
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

fs_status launch_peel(const PeelJob &job, hipStream_t s) {
  int dev = 0;
  hipGetDevice(&dev);
  const size_t lds = peel_lds_bytes(job.k, job.n);
  const size_t static_lds = 4 * (kPeelThreads / 64 + 1) + 16;
  if (lds + static_lds <= (size_t)device_info(dev).max_lds_per_block) {
    static bool attr_set[64] = {false};
    if (dev < 64 && !attr_set[dev]) {
      hipFuncSetAttribute(reinterpret_cast<const void *>(&peel_kernel<true>),
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          device_info(dev).max_lds_per_block - (int)static_lds);
      attr_set[dev] = true;
    }
    hipLaunchKernelGGL(peel_kernel<true>, dim3(1), dim3(kPeelThreads), lds, s, job);
  } else {
    if (!job.acc) return fail(FS_ERR_WORKSPACE, "peel state needs the workspace");
    hipLaunchKernelGGL(peel_kernel<false>, dim3(1), dim3(kPeelThreads), 0, s, job);
  }
  return hip_check(hipGetLastError(), "peel launch");
}

fs_status launch_replay(const ReplayJob &job, hipStream_t s) {
  // 16 lanes (256 B) per symbol on wide blocks; 4 lanes (64 B) when that
  // would leave fewer than ~2 workgroups per CU
  if (job.t >= 256ull * 512) {
    const uint32_t ns = (uint32_t)((job.t + 255) / 256);
    hipLaunchKernelGGL(replay_kernel<16>, dim3(ns), dim3(kReplayThreads), 0, s, job);
  } else {
    const uint32_t ns = (uint32_t)((job.t + 63) / 64);
    hipLaunchKernelGGL(replay_kernel<4>, dim3(ns), dim3(kReplayThreads), 0, s, job);
  }
  return hip_check(hipGetLastError(), "replay launch");
}

fs_status launch_repair_prep(const RepairPrepJob &job, hipStream_t s) {
  const int default_ok = job.erased2 ? 0 : 1;
  hipLaunchKernelGGL(repair_prep_kernel, dim3(1), dim3(kPlanThreads), 0, s, job, default_ok);
  return hip_check(hipGetLastError(), "repair prep launch");
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
