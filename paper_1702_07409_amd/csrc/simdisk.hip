// Disk-failure sweep for gfx950: for every f-subset of s equally striped
// disks, the peeling decode of one graph with the rows of those disks erased,
// reduced to its status {ok, |F|, levels}.
//
// One workgroup runs one failure combination at a time (persistent grid,
// each workgroup a contiguous run of ranks).  No payload is touched: the
// decode is symbolic, so the state of a combination is, per row, the number
// of its neighbours not yet decoded and the XOR of their indices (the last
// unknown input once the count is one), plus two bitsets over the inputs:
// decoded, and decoded at the current level beyond what the claiming lanes
// hold in registers.  It is kept in LDS when it fits:
//
//   kSimDiskByte   counts in bytes, XORs in 16 bits (3 bytes a row); for
//                  k <= 65535 and degrees <= 127
//   kSimDiskXor16  one word a row, count in the high half; degrees <= 32767
//   kSimDiskGlobal two words a row in a per-workgroup slot of the workspace
//
// A level scans every row for a count of one (these are exactly the rows of
// weight one in the level-synchronous schedule: a row that named an input at
// an earlier level has lost that input since), claims each named input once,
// and after a barrier lowers the count of every row on each input claimed at
// this level, with atomics whose result nobody waits for.  The decoded set
// of each level is that of the schedule, so |F| and the level count agree
// with it; which row decodes an input is not needed here and not recorded.
// An erased row carries an offset in its count that keeps it above one.
// With a precode the same workgroup then runs the second BP pass over the
// check equations (8 bytes of state per check) when data blocks are missing.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "fs_internal.h"

namespace fs {

namespace {

constexpr int kBinomN = 65;          // C(a, b) for 0 <= a, b <= 64
constexpr uint32_t kNone = 0xffffffffu;
constexpr int kBatch = 8;            // column edges loaded ahead of the updates
constexpr uint32_t kChunk = 16;      // rows one lane scans at a time
constexpr int kHeld = 4;             // claims a lane keeps in registers

constexpr uint32_t kErasedByte = 128u;        // counts <= 127
constexpr uint32_t kErasedXor16 = 1u << 31;   // counts <= 32767, high half
constexpr uint32_t kErasedGlobal = 1u << 31;

__device__ __forceinline__ uint32_t rows_padded(uint32_t n) { return (n + kChunk - 1) & ~(kChunk - 1); }

// ---- setup: initial per-row state image and the binomial table ------------
//
// rowinfo holds the image the kernel copies into its state at the start of
// every combination (n16 = n rounded up to 16; padding rows are empty):
//   kSimDiskByte   uint8 count[n16], then uint16 xor[n16]
//   kSimDiskXor16  uint32 (count << 16 | xor)[n16]
//   kSimDiskGlobal uint32 count[n16], then uint32 xor[n16]

template <int MODE>
__global__ __launch_bounds__(256) void simdisk_setup_kernel(SimDiskJob J) {
  if (blockIdx.x == gridDim.x - 1) {
    // Pascal's triangle, one row at a time, in LDS
    __shared__ unsigned long long prev[kBinomN], cur[kBinomN];
    const int b = threadIdx.x;
    if (b < kBinomN) prev[b] = (b == 0) ? 1ull : 0ull;
    __syncthreads();
    for (int a = 0; a < kBinomN; ++a) {
      if (b < kBinomN) {
        J.binom[a * kBinomN + b] = prev[b];
        cur[b] = (b == 0) ? 1ull : prev[b - 1] + prev[b];
      }
      __syncthreads();
      if (b < kBinomN) prev[b] = cur[b];
      __syncthreads();
    }
    return;
  }
  const uint32_t h = blockIdx.x * 256u + threadIdx.x;
  const uint32_t n16 = rows_padded(J.n);
  if (h >= n16) return;
  uint32_t deg = 0, acc = 0;
  if (h < J.n) {
    const int32_t lo = J.row_ptr[h], hi = J.row_ptr[h + 1];
    for (int32_t e = lo; e < hi; ++e) acc ^= (uint32_t)J.col[e];
    deg = (uint32_t)(hi - lo);
  }
  uint8_t *img = reinterpret_cast<uint8_t *>(J.rowinfo);
  if (MODE == kSimDiskByte) {
    img[h] = (uint8_t)deg;
    reinterpret_cast<uint16_t *>(img + n16)[h] = (uint16_t)acc;
  } else if (MODE == kSimDiskXor16) {
    J.rowinfo[h] = (deg << 16) | acc;
  } else {
    J.rowinfo[h] = deg;
    J.rowinfo[n16 + h] = acc;
  }
}

// ---- per-mode state access ------------------------------------------------
//
// In LDS every access is plain: LDS is coherent inside the workgroup and the
// barriers order it.  The global fallback is read and written with agent-
// scope atomics, which are served by L2 like the read-modify-writes, so no
// stale L1 line is ever read.

template <int MODE>
struct State {
  uint8_t *base;       // state image (layout of rowinfo)
  uint32_t n16;
  uint32_t *dec;       // decoded inputs
  uint32_t *fresh;     // inputs decoded at the current level

  __device__ __forceinline__ uint32_t ld(const uint32_t *p) const {
    if (MODE == kSimDiskGlobal) return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *p;
  }
  __device__ __forceinline__ void st(uint32_t *p, uint32_t v) const {
    if (MODE == kSimDiskGlobal)
      __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      *p = v;
  }
  __device__ __forceinline__ uint32_t *words() const { return reinterpret_cast<uint32_t *>(base); }
  __device__ __forceinline__ uint16_t *xor16() const { return reinterpret_cast<uint16_t *>(base + n16); }
  __device__ __forceinline__ uint32_t image_words() const {
    return MODE == kSimDiskByte ? 3 * n16 / 4 : MODE == kSimDiskXor16 ? n16 : 2 * n16;
  }
  __device__ __forceinline__ void mark_erased(uint32_t h) const {
    if (MODE == kSimDiskByte) base[h] = (uint8_t)(base[h] + kErasedByte);
    if (MODE == kSimDiskXor16) words()[h] += kErasedXor16;
    if (MODE == kSimDiskGlobal) st(words() + h, ld(words() + h) + kErasedGlobal);
  }
  // rows 16 q .. 16 q + 15 with a count of exactly one, as a bit mask
  __device__ __forceinline__ uint32_t ones(uint32_t q) const {
    uint32_t m = 0;
    if (MODE == kSimDiskByte) {
      const uint4 v = reinterpret_cast<const uint4 *>(base)[q];
      const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // bytes equal to 1: the zero bytes of w ^ 0x01010101, exactly
        const uint32_t x = w4[i] ^ 0x01010101u;
        const uint32_t z = ~(((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x | 0x7f7f7f7fu);   // 0x80 per zero byte
        m |= (((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) | ((z >> 28) & 8u)) << (4 * i);
      }
    } else if (MODE == kSimDiskXor16) {
      const uint4 *p = reinterpret_cast<const uint4 *>(words() + kChunk * q);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint4 v = p[i];
        m |= (uint32_t)((v.x >> 16) == 1u) << (4 * i);
        m |= (uint32_t)((v.y >> 16) == 1u) << (4 * i + 1);
        m |= (uint32_t)((v.z >> 16) == 1u) << (4 * i + 2);
        m |= (uint32_t)((v.w >> 16) == 1u) << (4 * i + 3);
      }
    } else {
#pragma unroll
      for (uint32_t i = 0; i < kChunk; ++i) m |= (uint32_t)(ld(words() + kChunk * q + i) == 1u) << i;
    }
    return m;
  }
  // the last unknown input of a row whose count is one
  __device__ __forceinline__ uint32_t last(uint32_t h) const {
    if (MODE == kSimDiskByte) return xor16()[h];
    if (MODE == kSimDiskXor16) return words()[h] & 0xffffu;
    return ld(words() + n16 + h);
  }
  // input f is decoded: row h has one unknown neighbour less (no return)
  __device__ __forceinline__ void remove(uint32_t h, uint32_t f) const {
    if (MODE == kSimDiskByte) {
      atomicSub(words() + (h >> 2), 1u << (8 * (h & 3)));
      atomicXor(reinterpret_cast<uint32_t *>(xor16()) + (h >> 1), f << (16 * (h & 1)));
    } else if (MODE == kSimDiskXor16) {
      atomicSub(words() + h, 1u << 16);
      atomicXor(words() + h, f);
    } else {
      atomicSub(words() + h, 1u);
      atomicXor(words() + n16 + h, f);
    }
  }
};

// Input f is decoded: every row of its column rowidx[p..hi) loses it.  The
// lane loads kBatch edges ahead of the updates.
template <int MODE>
__device__ __forceinline__ void drop_column(const State<MODE> &S, const int32_t *rowidx, uint32_t f, int32_t p,
                                            int32_t hi) {
  for (; p < hi; p += kBatch) {
    uint32_t rows[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) rows[b] = (p + b < hi) ? (uint32_t)rowidx[p + b] : kNone;
#pragma unroll
    for (int b = 0; b < kBatch; ++b)
      if (rows[b] != kNone) S.remove(rows[b], f);
  }
}

template <int MODE>
__device__ __forceinline__ void fence_for_barrier() {
  if (MODE == kSimDiskGlobal) __threadfence();
}

// Data blocks (inputs below b) not decoded; every thread of the workgroup
// calls it and gets the same count.
template <int MODE>
__device__ __forceinline__ uint32_t missing_data(const State<MODE> &S, uint32_t b, uint32_t *s_miss) {
  const uint32_t tid = threadIdx.x, nt = blockDim.x, bw = (b + 31) / 32;
  __syncthreads();
  if (tid == 0) *s_miss = 0;
  __syncthreads();
  uint32_t miss = 0;
  for (uint32_t w = tid; w < bw; w += nt) {
    uint32_t bits = ~S.ld(S.dec + w);
    if (w == bw - 1 && (b & 31)) bits &= (1u << (b & 31)) - 1u;
    miss += (uint32_t)__popc(bits);
  }
  if (miss) atomicAdd(s_miss, miss);
  __syncthreads();
  return *s_miss;
}

template <int MODE>
__global__ __launch_bounds__(1024) void simdisk_kernel(SimDiskJob J) {
  extern __shared__ __align__(16) uint8_t lds[];
  __shared__ unsigned long long s_rev;
  __shared__ uint32_t s_dec, s_miss;

  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t n = J.n, k = J.k;
  const uint32_t n16 = rows_padded(n), kw = (k + 31) / 32, nq = n16 / kChunk;
  const uint32_t lane = __lane_id();

  State<MODE> S;
  uint8_t *base = (MODE == kSimDiskGlobal) ? J.slots + (size_t)blockIdx.x * J.slot_bytes : lds;
  S.base = base + J.off_w;
  S.n16 = n16;
  S.dec = reinterpret_cast<uint32_t *>(base + J.off_dec);
  S.fresh = reinterpret_cast<uint32_t *>(base + J.off_fresh);
  const uint32_t img_words = S.image_words();

  // A failure combination is kept as a mask with disk d at bit s-1-d: the
  // lexicographic order of the sorted disk lists is then the decreasing
  // order of the masks, and the next combination is the next smaller mask
  // with f bits set.  Each workgroup takes a contiguous run of ranks.
  const unsigned long long all = (J.s == 64) ? ~0ull : ((1ull << J.s) - 1ull);
  const uint64_t per = (J.count + gridDim.x - 1) / gridDim.x;
  const uint64_t r_begin = (uint64_t)blockIdx.x * per;
  const uint64_t r_end = min(J.count, r_begin + per);
  for (uint64_t r = r_begin; r < r_end; ++r) {
    if (tid == 0) {
      unsigned long long rev = s_rev;
      if (r == r_begin) {
        // unrank J.first + r: the f-subsets whose smallest disk is a number
        // C(s - 1 - a, f - 1)
        uint64_t rank = J.first + r;
        uint32_t a = 0;
        rev = 0;
        for (uint32_t p = 0; p < J.f; ++p) {
          for (; a < J.s; ++a) {
            const uint64_t c = J.binom[(J.s - 1 - a) * kBinomN + (J.f - 1 - p)];
            if (rank < c) break;
            rank -= c;
          }
          if (a < J.s) rev |= 1ull << (J.s - 1 - a);
          ++a;
        }
      } else {
        // the next smaller mask with f bits set: the complement (s - f bits)
        // steps to the next larger one with the same count of bits
        const unsigned long long c = ~rev & all;
        const unsigned long long t = c | (c - 1ull);
        const unsigned long long nxt = (t + 1ull) | (((~t & (t + 1ull)) - 1ull) >> (__builtin_ctzll(c) + 1));
        rev = ~nxt & all;
      }
      s_rev = rev;
      s_dec = 0;
    }
    for (uint32_t w = tid; w < kw; w += nt) {
      S.st(S.dec + w, 0u);
      S.st(S.fresh + w, 0u);
    }
    // the initial state is a copy of the image
    uint32_t *img = reinterpret_cast<uint32_t *>(S.base);
    for (uint32_t i = 4 * tid; i < img_words; i += 4 * nt) {
      const uint4 v = *reinterpret_cast<const uint4 *>(J.rowinfo + i);
      if (MODE == kSimDiskGlobal) {
        S.st(img + i, v.x);
        S.st(img + i + 1, v.y);
        S.st(img + i + 2, v.z);
        S.st(img + i + 3, v.w);
      } else {
        *reinterpret_cast<uint4 *>(img + i) = v;
      }
    }
    fence_for_barrier<MODE>();
    __syncthreads();

    // the rows of the failed disks (each row lies on one disk: plain updates)
    const unsigned long long mask = __builtin_bitreverse64(s_rev) >> (64 - J.s);
    for (uint32_t d = 0; d < J.s; ++d) {
      if (!((mask >> d) & 1ull)) continue;
      const uint32_t lo = (uint32_t)((uint64_t)d * n / J.s), hi = (uint32_t)((uint64_t)(d + 1) * n / J.s);
      for (uint32_t h = lo + tid; h < hi; h += nt) S.mark_erased(h);
    }
    fence_for_barrier<MODE>();
    __syncthreads();

    uint32_t decoded = 0, levels = 0;
    while (decoded < k && (J.maxit == 0 || levels < J.maxit)) {
      // every surviving row with one unknown neighbour names it; the first
      // claim of an input decodes it.  The claiming lane keeps up to kHeld
      // of its claims in registers for the update pass; further ones go
      // through the fresh set.
      uint32_t mine = 0;
      uint32_t held[kHeld];
#pragma unroll
      for (int b = 0; b < kHeld; ++b) held[b] = kNone;
      for (uint32_t q = tid; q < nq; q += nt) {
        uint32_t m = S.ones(q);
        while (m) {
          const uint32_t h = kChunk * q + (uint32_t)__builtin_ctz(m);
          m &= m - 1u;
          const uint32_t f = S.last(h);
          const uint32_t bit = 1u << (f & 31);
          if (!(atomicOr(S.dec + (f >> 5), bit) & bit)) {
            if (mine < (uint32_t)kHeld) {
#pragma unroll
              for (int b = kHeld - 1; b > 0; --b) held[b] = held[b - 1];
              held[0] = f;
            } else {
              atomicOr(S.fresh + (f >> 5), bit);
            }
            ++mine;
          }
        }
      }
      // one LDS atomic per wave for the count
      uint32_t sum = mine;
      for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
      if (lane == 0 && sum) atomicAdd(&s_dec, sum);
      fence_for_barrier<MODE>();
      __syncthreads();
      const uint32_t now = s_dec;
      if (now == decoded) break;
      ++levels;
      // the inputs decoded at this level leave every row on them: first the
      // claims held in registers (their column bounds loaded together), then
      // the fresh set, a word per lane
      int32_t lo[kHeld], hi[kHeld];
#pragma unroll
      for (int b = 0; b < kHeld; ++b) {
        lo[b] = hi[b] = 0;
        if (held[b] != kNone) {
          lo[b] = J.col_ptr[held[b]];
          hi[b] = J.col_ptr[held[b] + 1];
        }
      }
#pragma unroll
      for (int b = 0; b < kHeld; ++b)
        if (held[b] != kNone) drop_column(S, J.rowidx, held[b], lo[b], hi[b]);
      for (uint32_t wi = tid; wi < kw; wi += nt) {
        uint32_t bits = S.ld(S.fresh + wi);
        if (!bits) continue;
        S.st(S.fresh + wi, 0u);
        while (bits) {
          const uint32_t f = 32 * wi + (uint32_t)__builtin_ctz(bits);
          bits &= bits - 1u;
          drop_column(S, J.rowidx, f, J.col_ptr[f], J.col_ptr[f + 1]);
        }
      }
      fence_for_barrier<MODE>();
      __syncthreads();
      decoded = now;
    }
    if (J.pc_m) {
      // precoded: the second BP pass over the checks when data blocks are
      // still missing, then the data blocks missing after both
      uint32_t levels2 = 0;
      uint32_t missing = missing_data(S, J.pc_b, &s_miss);
      if (missing) {
        uint32_t *ccnt = reinterpret_cast<uint32_t *>(base + J.off_chk), *cxs = ccnt + J.pc_m;
        for (uint32_t c = tid; c < J.pc_m; c += nt) {
          uint32_t u = 0, x = 0;
          for (int32_t e = J.chk_ptr[c]; e < J.chk_ptr[c + 1]; ++e) {
            const uint32_t sb = (uint32_t)J.chk_col[e];
            if (!((S.ld(S.dec + (sb >> 5)) >> (sb & 31)) & 1u)) {
              ++u;
              x ^= sb;
            }
          }
          S.st(ccnt + c, u);
          S.st(cxs + c, x);
        }
        if (tid == 0) s_dec = 0;
        fence_for_barrier<MODE>();
        __syncthreads();
        uint32_t prev = 0;
        for (;;) {
          uint32_t mine = 0;
          for (uint32_t c = tid; c < J.pc_m; c += nt) {
            if (S.ld(ccnt + c) != 1u) continue;
            const uint32_t f = S.ld(cxs + c), bit = 1u << (f & 31);
            if (!(atomicOr(S.dec + (f >> 5), bit) & bit)) {
              atomicOr(S.fresh + (f >> 5), bit);
              ++mine;
            }
          }
          for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o, 64);
          if (lane == 0 && mine) atomicAdd(&s_dec, mine);
          fence_for_barrier<MODE>();
          __syncthreads();
          const uint32_t now = s_dec;
          if (now == prev) break;
          ++levels2;
          for (uint32_t wi = tid; wi < kw; wi += nt) {
            uint32_t bits = S.ld(S.fresh + wi);
            if (!bits) continue;
            S.st(S.fresh + wi, 0u);
            while (bits) {
              const uint32_t f = 32 * wi + (uint32_t)__builtin_ctz(bits);
              bits &= bits - 1u;
              for (int32_t e = J.sym_ptr[f]; e < J.sym_ptr[f + 1]; ++e) {
                const uint32_t h = (uint32_t)J.sym_chk[e];
                atomicSub(ccnt + h, 1u);
                atomicXor(cxs + h, f);
              }
            }
          }
          fence_for_barrier<MODE>();
          __syncthreads();
          prev = now;
        }
        missing = missing_data(S, J.pc_b, &s_miss);
      }
      if (tid == 0) {
        int32_t *out = J.result + r * 4;
        out[0] = missing == 0 ? 1 : 0;
        out[1] = (int32_t)missing;
        out[2] = (int32_t)levels;
        out[3] = (int32_t)levels2;
      }
    } else if (tid == 0) {
      int32_t *out = J.result + r * 3;
      out[0] = decoded == k ? 1 : 0;
      out[1] = (int32_t)(k - decoded);
      out[2] = (int32_t)levels;
    }
    // every thread has read s_rev / s_dec before they are reset
    __syncthreads();
  }
}

}  // namespace

SimDiskLayout simdisk_layout(uint32_t k, uint32_t n, uint32_t max_deg, uint32_t checks, size_t max_lds) {
  SimDiskLayout L{};
  auto up = [](size_t v) { return (v + 15) & ~size_t(15); };
  const size_t n16 = ((size_t)n + kChunk - 1) & ~size_t(kChunk - 1), kw = (k + 31) / 32;
  if (k <= 0xffff && max_deg <= 32767) {
    L.mode = max_deg <= 127 ? kSimDiskByte : kSimDiskXor16;
    L.image_bytes = L.mode == kSimDiskByte ? 3 * n16 : 4 * n16;
    L.off_w = 0;
    L.off_dec = up(L.image_bytes);
    L.off_fresh = up(L.off_dec + 4 * kw);
    L.off_chk = up(L.off_fresh + 4 * kw);
    L.bytes = up(L.off_chk + 8ull * checks);
    if (L.bytes <= max_lds) return L;
  }
  // per-workgroup slots in global memory
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  L.mode = kSimDiskGlobal;
  L.image_bytes = 8 * n16;
  L.off_w = 0;
  L.off_dec = al(L.image_bytes);
  L.off_fresh = al(L.off_dec + 4 * kw);
  L.off_chk = al(L.off_fresh + 4 * kw);
  L.bytes = al(L.off_chk + 8ull * checks);
  return L;
}

static fs_status simdisk_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <int MODE>
static fs_status run_simdisk(SimDiskJob j, const SimDiskLayout &L, int cu, hipStream_t s) {
  const uint32_t n16 = (j.n + kChunk - 1) & ~(kChunk - 1);
  hipLaunchKernelGGL(simdisk_setup_kernel<MODE>, dim3((n16 + 255) / 256 + 1), dim3(256), 0, s, j);
  fs_status st = simdisk_hip(hipGetLastError(), "sim disks setup launch");
  if (st != FS_OK || j.count == 0) return st;
  size_t lds = 0;
  int threads = 1024;
  uint64_t grid = 0;
  if (MODE == kSimDiskGlobal) {
    grid = kSimDiskSlots;
  } else {
    lds = L.bytes;
    const void *fn = reinterpret_cast<const void *>(&simdisk_kernel<MODE>);
    if (lds > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    // resident workgroups per size; the most threads per combination that
    // still keeps as many combinations in flight as the chip can hold
    const int sizes[3] = {1024, 512, 256};
    uint64_t slots[3], most = 0;
    for (int i = 0; i < 3; ++i) {
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, sizes[i], lds) != hipSuccess || occ < 1) occ = 1;
      slots[i] = (uint64_t)cu * (uint64_t)occ;
      most = std::max(most, slots[i]);
    }
    const uint64_t want = std::min<uint64_t>(j.count, most);
    for (int i = 0; i < 3; ++i)
      if (slots[i] >= want) {
        threads = sizes[i];
        grid = slots[i];
        break;
      }
  }
  if (grid > j.count) grid = j.count;
  hipLaunchKernelGGL(simdisk_kernel<MODE>, dim3((uint32_t)grid), dim3(threads), lds, s, j);
  return simdisk_hip(hipGetLastError(), "sim disks launch");
}

fs_status launch_simdisk(const SimDiskJob &job_in, const SimDiskLayout &L, hipStream_t s) {
  SimDiskJob job = job_in;
  job.off_w = L.off_w;
  job.off_dec = L.off_dec;
  job.off_fresh = L.off_fresh;
  job.off_chk = L.off_chk;
  job.slot_bytes = L.bytes;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const int cu = device_info(dev).cu_count;
  if (L.mode == kSimDiskByte) return run_simdisk<kSimDiskByte>(job, L, cu, s);
  if (L.mode == kSimDiskXor16) return run_simdisk<kSimDiskXor16>(job, L, cu, s);
  return run_simdisk<kSimDiskGlobal>(job, L, cu, s);
}

}  // namespace fs
