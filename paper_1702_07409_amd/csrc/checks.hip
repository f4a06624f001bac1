// Check #2 / check #3 generation (CGA) and local-group repair for gfx950.
//
//   cga_setup_kernel   columns of B (the inputs of each coded block) and of
//                      L (the identity) as bitsets, and their weights
//   cga_rows_kernel    rows of B as bitsets (the columns holding each input)
//   cga_kernel         one workgroup runs the sweeps in the exact order of
//                      the algorithm: for column j it finds, among i = cursor
//                      .. n-1 (i != j) in parallel, the first i with
//                      2 w(b_j) > w(b_i) and w(b_j ^ b_i) < w(b_j), applies
//                      it to b_j and l_j, and continues from i + 1.  Column
//                      j is the only one that changes while it is processed,
//                      so this visits the same (j, i) pairs as the sequential
//                      loops and takes the same steps.
//   local_*_kernel     BP over the check #3 groups: level by level, each lost
//                      coded block still unknown takes the first group
//                      holding it whose other members are all known; writes
//                      the XOR lists in level order
//   local_apply_kernel rebuilds the blocks level by level, one workgroup per
//                      16- to 256-byte slice of every block
//
// The bitsets live in a workspace the generation call allocates; the columns
// of the workgroup's current j are copied to LDS.  Reads after a barrier of
// what the same workgroup wrote before it are ordered by that barrier.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "fs_internal.h"

namespace fs {

namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr int kCgaThreads = 1024;
constexpr uint32_t kNoCol = 0xffffffffu;

__global__ __launch_bounds__(256) void cga_setup_kernel(CgaJob J) {
  const uint32_t j = blockIdx.x * 256u + threadIdx.x;
  if (j >= J.n) return;
  uint32_t *b = J.bcol + (size_t)j * J.kw;
  uint32_t *l = J.lcol + (size_t)j * J.nw;
  for (uint32_t q = 0; q < J.kw; ++q) b[q] = 0;
  for (uint32_t q = 0; q < J.nw; ++q) l[q] = 0;
  const int32_t lo = J.row_ptr[j], hi = J.row_ptr[j + 1];
  for (int32_t e = lo; e < hi; ++e) {
    const uint32_t i = (uint32_t)J.col[e];
    b[i >> 5] |= 1u << (i & 31);
  }
  l[j >> 5] |= 1u << (j & 31);
  J.w[j] = (uint32_t)(hi - lo);
}

// Rows of B: R_r holds the columns whose coded block has input r (from the
// graph's column lists), one thread per input.
__global__ __launch_bounds__(256) void cga_rows_kernel(CgaJob J) {
  const uint32_t r = blockIdx.x * 256u + threadIdx.x;
  if (r >= J.k) return;
  uint32_t *row = J.rrow + (size_t)r * J.nw;
  for (uint32_t q = 0; q < J.nw; ++q) row[q] = 0;
  for (int32_t e = J.col_ptr[r]; e < J.col_ptr[r + 1]; ++e) {
    const uint32_t j = (uint32_t)J.rowidx[e];
    row[j >> 5] |= 1u << (j & 31);
  }
}

// The sweeps of Algorithm 4 in their sequential order, on one workgroup.
// For column j the next i (from the cursor on) must satisfy 2 w_j > w_i and
// w(b_j ^ b_i) < w_j; since w(b_j ^ b_i) = w_j + w_i - 2 |b_j & b_i|, the
// second test is w_i < 2 |b_j & b_i|, so only columns sharing an input with
// b_j can pass.  Those are found from the rows of b_j's inputs: per 32
// columns, the OR of those rows' words names the candidates and a count
// over them gives |b_j & b_i|; a block minimum picks the first passing i.
// b_j ^= b_i then also flips column j in the rows of b_i's inputs.
__global__ __launch_bounds__(kCgaThreads) void cga_kernel(CgaJob J) {
  extern __shared__ __align__(16) uint32_t cga_lds[];
  uint32_t *bj = cga_lds;                 // [kw]
  uint32_t *lj = cga_lds + J.kw;          // [nw]
  uint32_t *sj = cga_lds + J.kw + J.nw;   // [max_w] inputs of b_j
  __shared__ uint32_t s_zero, s_best, s_bestw, s_cnt;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t n = J.n, k = J.k, kw = J.kw, nw = J.nw;
  uint32_t sweeps = 0, zero = 0;
  for (;;) {
    __syncthreads();
    if (tid == 0) s_zero = 0;
    __syncthreads();
    uint32_t cnt = 0;
    for (uint32_t j = tid; j < n; j += nt) cnt += J.w[j] == 0 ? 1u : 0u;
    if (cnt) atomicAdd(&s_zero, cnt);
    __syncthreads();
    zero = s_zero;
    if (zero + k >= n || (J.max_sweeps && sweeps == J.max_sweeps)) break;
    bool changed = false;
    for (uint32_t j = 0; j < n; ++j) {
      for (uint32_t q = tid; q < kw; q += nt) bj[q] = J.bcol[(size_t)j * kw + q];
      for (uint32_t q = tid; q < nw; q += nt) lj[q] = J.lcol[(size_t)j * nw + q];
      uint32_t wj = J.w[j];
      uint32_t cursor = 0;
      for (;;) {
        // the inputs of b_j (their order does not matter)
        if (tid == 0) {
          s_cnt = 0;
          s_best = kNoCol;
        }
        __syncthreads();
        for (uint32_t q = tid; q < kw; q += nt) {
          uint32_t x = bj[q];
          if (x) {
            uint32_t at = atomicAdd(&s_cnt, (uint32_t)__popc(x));
            for (; x; x &= x - 1) {
              if (at < J.max_w) sj[at] = 32u * q + (uint32_t)__ffs(x) - 1u;
              ++at;
            }
          }
        }
        __syncthreads();
        const uint32_t m = min(s_cnt, J.max_w);
        // each thread scans its words in increasing order; its first passing
        // column is its smallest
        uint32_t mine = kNoCol, minew = 0;
        for (uint32_t q = (cursor >> 5) + tid; q < nw && mine == kNoCol; q += nt) {
          uint32_t cand = 0;
          for (uint32_t e = 0; e < m; ++e) cand |= J.rrow[(size_t)sj[e] * nw + q];
          if (q == (cursor >> 5)) cand &= ~0u << (cursor & 31);
          if (q == (j >> 5)) cand &= ~(1u << (j & 31));
          for (; cand; cand &= cand - 1) {
            const uint32_t bit = (uint32_t)__ffs(cand) - 1u, i = 32u * q + bit;
            if (i >= n) break;
            const uint32_t wi = J.w[i];
            if (!(2 * wj > wi)) continue;
            uint32_t both = 0;
            for (uint32_t e = 0; e < m; ++e) both += (J.rrow[(size_t)sj[e] * nw + q] >> bit) & 1u;
            if (wi < 2 * both) {
              mine = i;
              minew = wj + wi - 2 * both;
              break;
            }
          }
        }
        if (mine != kNoCol) atomicMin(&s_best, mine);
        __syncthreads();
        const uint32_t found = s_best;
        if (found == kNoCol) break;
        if (mine == found) s_bestw = minew;
        // b_j ^= b_found (flipping column j in the rows of b_found's inputs), l_j ^= l_found
        for (uint32_t q = tid; q < kw; q += nt) {
          const uint32_t x = J.bcol[(size_t)found * kw + q];
          bj[q] ^= x;
          for (uint32_t y = x; y; y &= y - 1) {
            const uint32_t r = 32u * q + (uint32_t)__ffs(y) - 1u;
            J.rrow[(size_t)r * nw + (j >> 5)] ^= 1u << (j & 31);
          }
        }
        for (uint32_t q = tid; q < nw; q += nt) lj[q] ^= J.lcol[(size_t)found * nw + q];
        __syncthreads();
        wj = s_bestw;
        changed = true;
        cursor = found + 1;
      }
      for (uint32_t q = tid; q < kw; q += nt) J.bcol[(size_t)j * kw + q] = bj[q];
      for (uint32_t q = tid; q < nw; q += nt) J.lcol[(size_t)j * nw + q] = lj[q];
      if (tid == 0) J.w[j] = wj;
      __syncthreads();
    }
    ++sweeps;
    if (!changed) {
      // zero columns are unchanged since the count above
      break;
    }
  }
  if (tid == 0) {
    J.meta[0] = (int32_t)sweeps;
    J.meta[1] = (int32_t)zero;
  }
}

// inclusive prefix sums of one value per thread (kCgaThreads threads)
__device__ uint32_t block_inclusive_scan(uint32_t v, uint32_t *sh) {
  const uint32_t tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (uint32_t o = 1; o < kCgaThreads; o <<= 1) {
    const uint32_t add = tid >= o ? sh[tid - o] : 0u;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  return sh[tid];
}

// BP over the check #3 groups, run as a peel over them, in four launches.
//   local_prep_kernel   (one workgroup) checks the lost ids and builds the
//                       bitset of unknown blocks (erased or lost)
//   local_count_kernel  (the device) gives every group (unknown members << 40
//                       | sum of their ids), so a group with one unknown
//                       names it, and lists those groups: the first frontier
//   local_plan_kernel   (one workgroup) runs the levels.  A level takes the
//                       frontier; each lost block still unknown that one of
//                       its groups names keeps the smallest such group index
//                       (the first group in the stored order whose other
//                       members are all known).  After a barrier the blocks
//                       taken become known and every group holding one loses
//                       it; a group left with one unknown joins the next
//                       frontier.  The loop ends at a level that takes none.
//                       The items are then laid out level by level (blocks in
//                       lost order within a level, the unrebuilt ones last
//                       with no sources).  The group counters sit in LDS when
//                       they fit.
//   local_fill_kernel   (the device) writes each item's sources: its group
//                       without the block it rebuilds
constexpr unsigned long long kGrpOne = 1ull << 40;

__device__ __forceinline__ bool local_failed(const LocalPlanJob &J) { return J.flag[0] != 0; }

__global__ __launch_bounds__(kCgaThreads) void local_prep_kernel(LocalPlanJob J) {
  extern __shared__ uint32_t lds[];
  uint32_t *down = lds;                                // [ceil(n / 32)] unknown blocks
  __shared__ uint32_t s_bad;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t nw = (J.n + 31) / 32, m = J.n_lost;
  if (tid == 0) s_bad = 0;
  for (uint32_t w = tid; w < nw; w += nt) down[w] = 0;
  __syncthreads();
  for (uint32_t r = tid; r < m; r += nt) {
    const uint32_t s = J.lost[r];
    if (s >= J.n) {
      atomicOr(&s_bad, 1u);
      continue;
    }
    const uint32_t bit = 1u << (s & 31);
    if (atomicOr(&down[s >> 5], bit) & bit) atomicOr(&s_bad, 1u);
  }
  if (J.erased)
    for (uint32_t s = tid; s < J.n; s += nt)
      if (J.erased[s]) atomicOr(&down[s >> 5], 1u << (s & 31));
  __syncthreads();
  if (s_bad) {
    for (uint32_t r = tid; r < m; r += nt) J.repaired[r] = 0;
    if (tid == 0) {
      J.flag[0] = FS_ERR_INVALID;
      J.status[0] = 0;
      J.status[1] = (int32_t)m;
      J.status[2] = -FS_ERR_INVALID;
    }
    return;
  }
  for (uint32_t w = tid; w < nw; w += nt) J.unk[w] = down[w];
  // lost index of every block, smallest usable group per lost block
  for (uint32_t s = tid; s < J.n; s += nt) {
    J.rof[s] = -1;
    J.best[s] = 0x7fffffff;
  }
  __syncthreads();
  for (uint32_t r = tid; r < m; r += nt) {
    J.chosen[r] = -1;
    J.level[r] = -1;
    J.rof[J.lost[r]] = (int32_t)r;
  }
  if (tid == 0) {
    J.flag[0] = 0;
    J.meta[1] = 0;
  }
}

// one wave per group, its lanes splitting the members
__global__ __launch_bounds__(256) void local_count_kernel(LocalPlanJob J) {
  if (local_failed(J)) return;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t nwv = gridDim.x * 4u;
  for (uint32_t q = blockIdx.x * 4u + (threadIdx.x >> 6); q < J.n_groups; q += nwv) {
    unsigned long long acc = 0;
    for (int32_t e = J.grp_ptr[q] + (int32_t)lane; e < J.grp_ptr[q + 1]; e += 64) {
      const uint32_t u = (uint32_t)J.grp_col[e];
      if ((J.unk[u >> 5] >> (u & 31)) & 1u) acc += kGrpOne | u;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) {
      J.gacc[q] = acc;
      if ((acc >> 40) == 1ull) {
        const uint32_t at = (uint32_t)atomicAdd(&J.meta[1], 1);
        J.fa[2 * at] = (int32_t)q;
        J.fa[2 * at + 1] = (int32_t)(acc & (kGrpOne - 1));
      }
    }
  }
}

template <bool LDSG>
__global__ __launch_bounds__(kCgaThreads) void local_plan_kernel(LocalPlanJob J) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lsm[];
  uint32_t *lds = reinterpret_cast<uint32_t *>(lsm);
  const uint32_t nw = (J.n + 31) / 32, m = J.n_lost, ng = J.n_groups;
  uint32_t *down = lds;                                // [nw] unknown blocks
  uint32_t *took = lds + nw;                           // [nw] taken at this level
  // group counters: LDS copy (8-byte aligned: 2 nw words precede it) or the workspace
  unsigned long long *gacc = LDSG ? reinterpret_cast<unsigned long long *>(lds + 2 * nw) : J.gacc;
  __shared__ uint32_t s_fail, s_nA, s_nB, s_nT;
  __shared__ uint32_t scan_sh[kCgaThreads];
  if (local_failed(J)) return;
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) {
    s_fail = 0;
    s_nA = (uint32_t)J.meta[1];
    s_nB = 0;
    s_nT = 0;
  }
  for (uint32_t w = tid; w < nw; w += nt) {
    down[w] = J.unk[w];
    took[w] = 0;
  }
  if (LDSG)
    for (uint32_t q = tid; q < ng; q += nt) gacc[q] = J.gacc[q];
  __syncthreads();
  int32_t *cur = J.fa, *nxt = J.fb;
  int level = 0;
  for (;;) {
    const uint32_t nA = s_nA;
    // each frontier group offers its unknown block, if that block is lost
    // and still unknown; the block keeps the smallest group index
    for (uint32_t a = tid; a < nA; a += nt) {
      const int32_t q = cur[2 * a];
      const uint32_t u = (uint32_t)cur[2 * a + 1];
      if (u >= J.n || J.rof[u] < 0 || !((down[u >> 5] >> (u & 31)) & 1u)) continue;
      atomicMin(&J.best[u], q);
      const uint32_t bit = 1u << (u & 31);
      if (!(atomicOr(&took[u >> 5], bit) & bit)) atomicAdd(&s_nT, 1u);
    }
    __syncthreads();
    const uint32_t taken = s_nT;
    __syncthreads();   // every thread has read the count before it is reused
    if (taken == 0) break;
    // the blocks taken at this level, listed (J.pos serves as the list until
    // the layout below), then one wave per block: record it, make it known,
    // and remove it from every group holding it, the lanes splitting its
    // groups
    if (tid == 0) s_nT = 0;
    __syncthreads();
    for (uint32_t w = tid; w < nw; w += nt) {
      const uint32_t x = took[w];
      if (!x) continue;
      uint32_t at = atomicAdd(&s_nT, (uint32_t)__popc(x));
      for (uint32_t y = x; y; y &= y - 1) J.pos[at++] = (int32_t)(32u * w + (uint32_t)__ffs(y) - 1u);
      took[w] = 0;
    }
    __syncthreads();
    // a wave takes blocks wave, wave + nwave, ...: up to 64 at a time, one
    // per lane, whose record and group-list bounds load in one round; it
    // then walks them two at a time, the lanes loading both blocks' groups
    // before lowering their counters
    const uint32_t nT = s_nT, lane = tid & 63u, wave = tid >> 6, nwave = nt >> 6;
    for (uint32_t bb = 0; wave + nwave * bb < nT; bb += 64) {
      const uint32_t i = wave + nwave * (bb + lane);
      uint32_t u = 0;
      int32_t a0 = 0, a1 = 0;
      if (i < nT) {
        u = (uint32_t)J.pos[i];
        const int32_t r = J.rof[u];
        a0 = J.sym_ptr[u];
        a1 = J.sym_ptr[u + 1];
        J.chosen[r] = atomicAdd(&J.best[u], 0);
        J.level[r] = level;
        atomicAnd(&down[u >> 5], ~(1u << (u & 31)));
      }
      const uint32_t nb = (uint32_t)__popcll(__ballot(i < nT));   // lanes 0 .. nb-1 hold blocks
      for (uint32_t j = 0; j < nb; j += 2) {
        const uint32_t jb = min(j + 1, nb - 1);
        const uint32_t u0 = (uint32_t)__shfl((int)u, (int)j, 64), u1 = (uint32_t)__shfl((int)u, (int)jb, 64);
        const int32_t f0 = __shfl(a0, (int)j, 64), g0 = __shfl(a1, (int)j, 64);
        const int32_t f1 = __shfl(a0, (int)jb, 64), g1 = j + 1 < nb ? __shfl(a1, (int)jb, 64) : f1;
        const unsigned long long d0 = 0ull - (kGrpOne | u0), d1 = 0ull - (kGrpOne | u1);
        const int32_t span = max(g0 - f0, g1 - f1);
        for (int32_t o = 0; o < span; o += 128) {
          int32_t q[4];
          const int32_t e0 = f0 + o + (int32_t)lane, e1 = f1 + o + (int32_t)lane;
          q[0] = e0 < g0 ? J.sym_grp[e0] : -1;
          q[1] = e0 + 64 < g0 ? J.sym_grp[e0 + 64] : -1;
          q[2] = e1 < g1 ? J.sym_grp[e1] : -1;
          q[3] = e1 + 64 < g1 ? J.sym_grp[e1 + 64] : -1;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (q[v] < 0) continue;
            const unsigned long long dec = v < 2 ? d0 : d1;
            const unsigned long long after = atomicAdd(&gacc[q[v]], dec) + dec;
            if ((after >> 40) == 1ull) {
              const uint32_t at = atomicAdd(&s_nB, 1u);
              nxt[2 * at] = q[v];
              nxt[2 * at + 1] = (int32_t)(after & (kGrpOne - 1));
            }
          }
        }
      }
    }
    ++level;
    __syncthreads();
    if (tid == 0) {
      s_nA = s_nB;
      s_nB = 0;
      s_nT = 0;
    }
    int32_t *tmp = cur;
    cur = nxt;
    nxt = tmp;
    __syncthreads();
  }
  // level order: a contiguous run of lost blocks per thread, one scan per
  // level (the unrebuilt blocks form the last one)
  const uint32_t per = (m + nt - 1) / nt;
  const uint32_t r0 = min(m, tid * per), r1 = min(m, r0 + per);
  uint32_t base = 0;
  for (int l = 0; l <= level; ++l) {
    const int want = l < level ? l : -1;
    uint32_t c = 0;
    for (uint32_t r = r0; r < r1; ++r) c += J.level[r] == want;
    const uint32_t incl = block_inclusive_scan(c, scan_sh);
    const uint32_t tot = scan_sh[nt - 1];
    uint32_t p = base + incl - c;
    for (uint32_t r = r0; r < r1; ++r)
      if (J.level[r] == want) J.pos[r] = (int32_t)p++;
    if (tid == 0) J.lvl_ptr[l] = (int32_t)base;
    base += tot;
    __syncthreads();
  }
  if (tid == 0) J.lvl_ptr[level + 1] = (int32_t)m;
  // sources per item (at the item's place), then their offsets by a scan
  // over item places, each thread rewriting only its own run of places
  uint32_t fail = 0;
  for (uint32_t r = r0; r < r1; ++r) {
    const int32_t g = J.chosen[r];
    J.item_ptr[J.pos[r]] = g >= 0 ? J.grp_ptr[g + 1] - J.grp_ptr[g] - 1 : 0;
    J.item_dst[J.pos[r]] = (int32_t)J.lost[r];
    J.repaired[r] = g >= 0 ? 1 : 0;
    fail += g < 0;
  }
  if (fail) atomicAdd(&s_fail, fail);
  __syncthreads();
  uint32_t c = 0;
  for (uint32_t p = r0; p < r1; ++p) c += (uint32_t)J.item_ptr[p];
  const uint32_t incl = block_inclusive_scan(c, scan_sh);
  uint32_t off = incl - c;
  for (uint32_t p = r0; p < r1; ++p) {
    const uint32_t sz = (uint32_t)J.item_ptr[p];
    J.item_ptr[p] = (int32_t)off;
    off += sz;
  }
  if (tid == nt - 1) J.item_ptr[m] = (int32_t)incl;
  if (tid == 0) {
    J.meta[0] = level;
    J.status[0] = s_fail == 0 ? 1 : 0;
    J.status[1] = (int32_t)s_fail;
    J.status[2] = level;
  }
}

// one wave per lost block rebuilt: its group's members but itself, in
// order, at the item's offset (the ballot of the members kept gives each
// lane its place)
__global__ __launch_bounds__(256) void local_fill_kernel(LocalPlanJob J) {
  if (local_failed(J)) return;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t nwv = gridDim.x * 4u;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (uint32_t r = blockIdx.x * 4u + (threadIdx.x >> 6); r < J.n_lost; r += nwv) {
    const int32_t g = J.chosen[r];
    if (g < 0) continue;
    const int32_t s = (int32_t)J.lost[r];
    int32_t o = J.item_ptr[J.pos[r]];
    const int32_t e1 = J.grp_ptr[g + 1];
    for (int32_t e0 = J.grp_ptr[g]; e0 < e1; e0 += 64) {
      const int32_t e = e0 + (int32_t)lane;
      const int32_t col = e < e1 ? J.grp_col[e] : s;
      const bool keep = col != s;
      const unsigned long long mask = __ballot(keep);
      if (keep) J.item_col[o + (int32_t)__popcll(mask & below)] = col;
      o += (int32_t)__popcll(mask);
    }
  }
}

// One workgroup per slice of 16 LPS bytes of every block walks the levels:
// 256 / LPS items at a time, LPS lanes each, XOR their sources and store the
// result; a barrier between levels orders a level's stores before the next
// level's loads (blocks rebuilt earlier are sources later).
// Slice of workgroup b: workgroups go round-robin over the 8 XCDs (b % 8),
// so XCD x takes the contiguous slices [start_x, start_x + count_x).  The
// slices that share a 128-byte line then meet in one XCD's L2 instead of each
// XCD fetching the whole line for its 16 bytes.
__device__ __forceinline__ uint32_t slice_of_block(uint32_t b, uint32_t nwg) {
  const uint32_t xcd = b & 7u, local = b >> 3;
  const uint32_t per = nwg >> 3, rem = nwg & 7u;
  return xcd * per + min(xcd, rem) + local;
}

template <int LPS>
__global__ __launch_bounds__(256) void local_apply_kernel(LocalPlanJob J, uint8_t *c, uint64_t t, int first) {
  if (J.flag[0]) return;
  constexpr int IPW = 256 / LPS;
  const int levels = J.meta[0];
  const uint32_t lane = threadIdx.x % LPS, it = threadIdx.x / LPS;
  const uint64_t off = (uint64_t)slice_of_block(blockIdx.x, gridDim.x) * (16u * LPS) + lane * 16u;
  const bool live = off < t;
  const v4u zero = {0u, 0u, 0u, 0u};
  for (int l = first; l <= levels; ++l) {
    const int p1 = J.lvl_ptr[l + 1];
    if (live)
      for (int p = J.lvl_ptr[l] + (int)it; p < p1; p += IPW) {
        v4u acc = zero;
        const int e1 = J.item_ptr[p + 1];
        int e = J.item_ptr[p];
        for (; e + 4 <= e1; e += 4) {
          const v4u a0 = *reinterpret_cast<const v4u *>(c + (uint64_t)(uint32_t)J.item_col[e] * t + off);
          const v4u a1 = *reinterpret_cast<const v4u *>(c + (uint64_t)(uint32_t)J.item_col[e + 1] * t + off);
          const v4u a2 = *reinterpret_cast<const v4u *>(c + (uint64_t)(uint32_t)J.item_col[e + 2] * t + off);
          const v4u a3 = *reinterpret_cast<const v4u *>(c + (uint64_t)(uint32_t)J.item_col[e + 3] * t + off);
          acc ^= (a0 ^ a1) ^ (a2 ^ a3);
        }
        for (; e < e1; ++e) acc ^= *reinterpret_cast<const v4u *>(c + (uint64_t)(uint32_t)J.item_col[e] * t + off);
        *reinterpret_cast<v4u *>(c + (uint64_t)(uint32_t)J.item_dst[p] * t + off) = acc;
      }
    __syncthreads();
  }
}

// One level of the rebuild, for blocks too short to give every CU two
// workgroups of 128-byte slices: one workgroup per (item, 1 KiB chunk) of the
// level.  Its four waves take a quarter of the item's sources each, every
// lane 16 bytes of the chunk, eight loads in flight, so every source load is
// a whole 1 KiB run of one block; the four partial XORs meet in LDS.  Levels
// follow each other as launches on the stream.  The level past the last
// rebuilt one holds the blocks no group rebuilds (no sources: they are
// zeroed).
constexpr uint64_t kLevelChunk = 1024;

__global__ __launch_bounds__(256) void local_level_kernel(LocalPlanJob J, uint8_t *c, uint64_t t, int l) {
  __shared__ v4u part[4][64];
  if (J.flag[0] || l > J.meta[0]) return;
  const int p0 = J.lvl_ptr[l], p1 = J.lvl_ptr[l + 1];
  if (p1 <= p0) return;
  const uint64_t nch = (t + kLevelChunk - 1) / kLevelChunk;
  const uint64_t nwork = (uint64_t)(p1 - p0) * nch;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const v4u zero = {0u, 0u, 0u, 0u};
  for (uint64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int p = p0 + (int)(w / nch);
    const uint64_t off = (w % nch) * kLevelChunk + lane * 16u;
    const int b0 = J.item_ptr[p], b1 = J.item_ptr[p + 1];
    const int e1 = b0 + (int)(((int64_t)(b1 - b0) * (wv + 1)) / 4);
    int e = b0 + (int)(((int64_t)(b1 - b0) * wv) / 4);
    v4u acc = zero;
    if (off < t) {
      const uint8_t *src = c + off;
      for (; e + 8 <= e1; e += 8) {
        v4u a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          a[u] = *reinterpret_cast<const v4u *>(src + (uint64_t)(uint32_t)J.item_col[e + u] * t);
        acc ^= ((a[0] ^ a[1]) ^ (a[2] ^ a[3])) ^ ((a[4] ^ a[5]) ^ (a[6] ^ a[7]));
      }
      for (; e < e1; ++e) acc ^= *reinterpret_cast<const v4u *>(src + (uint64_t)(uint32_t)J.item_col[e] * t);
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && off < t)
      *reinterpret_cast<v4u *>(c + (uint64_t)(uint32_t)J.item_dst[p] * t + off) =
          (part[0][lane] ^ part[1][lane]) ^ (part[2][lane] ^ part[3][lane]);
    __syncthreads();   // the parts are read before the next item overwrites them
  }
}

constexpr int kLevelLaunches = 16;   // levels rebuilt by per-level launches

fs_status ck_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

fs_status run_cga(const CgaJob &job, hipStream_t s) {
  if (job.n == 0) return FS_OK;
  hipLaunchKernelGGL(cga_setup_kernel, dim3((job.n + 255) / 256), dim3(256), 0, s, job);
  fs_status st = ck_hip(hipGetLastError(), "check generation setup launch");
  if (st != FS_OK) return st;
  hipLaunchKernelGGL(cga_rows_kernel, dim3((job.k + 255) / 256), dim3(256), 0, s, job);
  st = ck_hip(hipGetLastError(), "check generation rows launch");
  if (st != FS_OK) return st;
  const size_t lds = 4ull * (job.kw + job.nw + job.max_w);
  const void *fn = reinterpret_cast<const void *>(&cga_kernel);
  if (lds > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(cga_kernel, dim3(1), dim3(kCgaThreads), lds, s, job);
  return ck_hip(hipGetLastError(), "check generation launch");
}

fs_status launch_local_plan(const LocalPlanJob &job, hipStream_t s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cu = device_info(dev).cu_count;
  const size_t budget = (size_t)device_info(dev).max_lds_per_block;
  const size_t bits = 4ull * ((job.n + 31) / 32);
  const void *prep = reinterpret_cast<const void *>(&local_prep_kernel);
  if (bits > 32 * 1024) (void)hipFuncSetAttribute(prep, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bits);
  hipLaunchKernelGGL(local_prep_kernel, dim3(1), dim3(kCgaThreads), bits, s, job);
  fs_status st = ck_hip(hipGetLastError(), "local repair check launch");
  if (st != FS_OK) return st;
  const uint32_t cgrid = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>(8ull * (uint64_t)cu, ((uint64_t)job.n_groups + 3) / 4));
  hipLaunchKernelGGL(local_count_kernel, dim3(cgrid), dim3(256), 0, s, job);
  st = ck_hip(hipGetLastError(), "local repair count launch");
  if (st != FS_OK) return st;
  // the group counters go to LDS when they fit beside the two bitsets
  const size_t with_g = 2 * bits + 8ull * job.n_groups;
  if (with_g <= budget) {
    const void *fn = reinterpret_cast<const void *>(&local_plan_kernel<true>);
    if (with_g > 32 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)with_g);
    hipLaunchKernelGGL(local_plan_kernel<true>, dim3(1), dim3(kCgaThreads), with_g, s, job);
  } else {
    const void *fn = reinterpret_cast<const void *>(&local_plan_kernel<false>);
    if (2 * bits > 32 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(2 * bits));
    hipLaunchKernelGGL(local_plan_kernel<false>, dim3(1), dim3(kCgaThreads), 2 * bits, s, job);
  }
  st = ck_hip(hipGetLastError(), "local repair plan launch");
  if (st != FS_OK) return st;
  if (job.n_lost == 0) return FS_OK;
  const uint32_t fgrid = (uint32_t)std::max<uint64_t>(
      1, std::min<uint64_t>(8ull * (uint64_t)cu, ((uint64_t)job.n_lost + 3) / 4));
  hipLaunchKernelGGL(local_fill_kernel, dim3(fgrid), dim3(256), 0, s, job);
  return ck_hip(hipGetLastError(), "local repair fill launch");
}

fs_status launch_local_apply(const LocalPlanJob &plan, uint8_t *c, uint64_t t, hipStream_t s) {
  // the widest slice (16 to 256 bytes) that still gives every CU two workgroups
  int dev = 0;
  (void)hipGetDevice(&dev);
  const uint64_t want = 2ull * (uint64_t)device_info(dev).cu_count;
  int lps = 16;
  while (lps > 1 && (t + 16ull * lps - 1) / (16ull * lps) < want) lps /= 2;
  const uint64_t nslices = (t + 16ull * lps - 1) / (16ull * lps);
  if (nslices == 0) return FS_OK;
  if (nslices > 0x7fffffffull) return fail(FS_ERR_UNSUPPORTED, "block too large for the local repair");
  const dim3 grid((uint32_t)nslices), block(256);
  int first = 0;
  if (lps < 8) {
    // short blocks: the first levels as launches of their own (the levels
    // are known on the device only; launches past the last one return at
    // once), the rest, if any, by the slice walk below
    const uint64_t nch = (t + kLevelChunk - 1) / kLevelChunk;
    const uint64_t units = (uint64_t)plan.n_lost * nch;
    const uint32_t lgrid = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(8ull * (uint64_t)device_info(dev).cu_count, units));
    for (int l = 0; l < kLevelLaunches; ++l) {
      hipLaunchKernelGGL(local_level_kernel, dim3(lgrid), block, 0, s, plan, c, t, l);
      const fs_status st = ck_hip(hipGetLastError(), "local repair level launch");
      if (st != FS_OK) return st;
    }
    first = kLevelLaunches;
  }
  switch (lps) {
    case 16: hipLaunchKernelGGL(local_apply_kernel<16>, grid, block, 0, s, plan, c, t, first); break;
    case 8: hipLaunchKernelGGL(local_apply_kernel<8>, grid, block, 0, s, plan, c, t, first); break;
    case 4: hipLaunchKernelGGL(local_apply_kernel<4>, grid, block, 0, s, plan, c, t, first); break;
    case 2: hipLaunchKernelGGL(local_apply_kernel<2>, grid, block, 0, s, plan, c, t, first); break;
    default: hipLaunchKernelGGL(local_apply_kernel<1>, grid, block, 0, s, plan, c, t, first); break;
  }
  return ck_hip(hipGetLastError(), "local repair launch");
}


}  // namespace fs
