// Array-LDPC precode (check #1) for gfx950: the check sets of Algorithm 2,
// and the second BP pass of the two-stage decode.
//
// The parity encode reuses the gather kernel, one launch per block row of
// checks: row r of L(1) lists the blocks whose XOR is parity block b + r,
// and those lie in the data or in earlier block rows, so a block row reads
// only blocks that are final.
//
// The second pass, after the LDGM decode, is BP over the check equations:
//   precode_peel_kernel    one workgroup; per check the count of unknown
//                          members and the XOR of their indices in LDS; each
//                          level names the last unknown member of every
//                          check at count one, claims it once, and lowers the
//                          counts of the checks on it.  It writes the
//                          (block, check) pairs of each level.
//   precode_level_kernel   replays one level: block = XOR of the other
//                          members of its check, one workgroup per (pair,
//                          1 KiB chunk) of the level
//   precode_replay_kernel  replays the later levels, one workgroup per 1 KiB
//                          byte slice of every block

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "fs_internal.h"

namespace fs {

namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

constexpr int kPcThreads = 1024;
constexpr uint32_t kPcSlice = 1024;   // bytes of every block per replay workgroup
constexpr int kPcReplayThreads = 256;

__global__ __launch_bounds__(kPcThreads) void precode_peel_kernel(PrecodePeelJob J) {
  extern __shared__ __align__(16) uint32_t pc_lds[];
  uint32_t *cnt = pc_lds;              // [m]
  uint32_t *xs = pc_lds + J.m;         // [m]
  uint32_t *known = pc_lds + 2 * J.m;  // [ceil(k / 32)]
  __shared__ uint32_t s_missing, s_tail;
  const uint32_t tid = threadIdx.x, nt = blockDim.x, kw = (J.k + 31) / 32;
  if (tid == 0) {
    s_missing = 0;
    s_tail = 0;
  }
  // the recovered flags as a bitmap: a wave reads 64 consecutive flags and
  // ballots them into two words (blockDim is a multiple of 64)
  for (uint32_t s0 = (tid & ~63u) * 1u; s0 < 32 * kw; s0 += nt) {
    const uint32_t s = s0 + (tid & 63);
    const uint64_t m = __ballot(s < J.k && J.recovered[s] != 0);
    if ((tid & 63) == 0) {
      known[s0 >> 5] = (uint32_t)m;
      if ((s0 >> 5) + 1 < kw) known[(s0 >> 5) + 1] = (uint32_t)(m >> 32);
    }
  }
  __syncthreads();
  uint32_t miss = 0;
  for (uint32_t s = tid; s < J.b; s += nt) miss += ((known[s >> 5] >> (s & 31)) & 1u) ^ 1u;
  if (miss) atomicAdd(&s_missing, miss);
  __syncthreads();
  int levels = 0;
  if (s_missing) {
    // the second pass runs only when data blocks are still missing
    for (uint32_t r = tid; r < J.m; r += nt) {
      uint32_t c = 0, x = 0;
      const int32_t e1 = J.chk_ptr[r + 1];
      // the check's entries eight at a time, loaded before any is tested
      for (int32_t e = J.chk_ptr[r]; e < e1; e += 8) {
        int32_t sv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) sv[u] = e + u < e1 ? J.chk_col[e + u] : -1;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (sv[u] < 0) continue;
          const uint32_t sym = (uint32_t)sv[u];
          if (!((known[sym >> 5] >> (sym & 31)) & 1u)) {
            ++c;
            x ^= sym;
          }
        }
      }
      cnt[r] = c;
      xs[r] = x;
    }
    if (tid == 0) J.level_ptr[0] = 0;
    __syncthreads();
    uint32_t prev = 0;
    for (;;) {
      for (uint32_t r = tid; r < J.m; r += nt) {
        if (cnt[r] != 1u) continue;
        const uint32_t f = xs[r], bit = 1u << (f & 31);
        if (atomicOr(&known[f >> 5], bit) & bit) continue;
        const uint32_t at = atomicAdd(&s_tail, 1u);
        J.pair_sym[at] = (int32_t)f;
        J.pair_chk[at] = (int32_t)r;
      }
      __syncthreads();
      const uint32_t now = s_tail;
      if (now == prev) break;
      ++levels;
      if (tid == 0) J.level_ptr[levels] = (int32_t)now;
      for (uint32_t i = prev + tid; i < now; i += nt) {
        const uint32_t f = (uint32_t)J.pair_sym[i];
        for (int32_t e = J.sym_ptr[f]; e < J.sym_ptr[f + 1]; ++e) {
          const uint32_t h = (uint32_t)J.sym_chk[e];
          atomicSub(&cnt[h], 1u);
          atomicXor(&xs[h], f);
        }
      }
      __syncthreads();
      prev = now;
    }
  }
  const uint32_t pairs = s_tail;
  for (uint32_t i = tid; i < pairs; i += nt) J.recovered[J.pair_sym[i]] = 1;
  __syncthreads();
  if (tid == 0) s_missing = 0;
  __syncthreads();
  miss = 0;
  for (uint32_t s = tid; s < J.b; s += nt) miss += ((known[s >> 5] >> (s & 31)) & 1u) ^ 1u;
  if (miss) atomicAdd(&s_missing, miss);
  __syncthreads();
  if (tid == 0) {
    J.status[0] = s_missing == 0 ? 1 : 0;
    J.status[1] = (int32_t)s_missing;
    J.status[2] = J.status1[2];
    J.status[3] = levels;
    J.meta[0] = levels;
    J.meta[1] = (int32_t)pairs;
  }
}

__global__ __launch_bounds__(kPcReplayThreads) void precode_replay_kernel(PrecodeReplayJob J, int first) {
  const int levels = J.meta[0];
  if (levels <= first) return;
  const uint64_t off0 = (uint64_t)blockIdx.x * kPcSlice;
  if (off0 >= J.t) return;
  const uint32_t chunks = (uint32_t)(min<uint64_t>(kPcSlice, J.t - off0) / 16);
  for (int l = first; l < levels; ++l) {
    const int lo = J.level_ptr[l], hi = J.level_ptr[l + 1];
    const uint32_t items = (uint32_t)(hi - lo) * chunks;
    for (uint32_t it = threadIdx.x; it < items; it += kPcReplayThreads) {
      const int q = lo + (int)(it / chunks);
      const uint64_t off = off0 + 16ull * (it % chunks);
      const uint32_t f = (uint32_t)J.pair_sym[q];
      const int32_t r = J.pair_chk[q];
      v4u acc = {0u, 0u, 0u, 0u};
      for (int32_t e = J.chk_ptr[r]; e < J.chk_ptr[r + 1]; ++e) {
        const uint32_t s = (uint32_t)J.chk_col[e];
        if (s != f) acc ^= *reinterpret_cast<const v4u *>(J.x + (uint64_t)s * J.t + off);
      }
      *reinterpret_cast<v4u *>(J.x + (uint64_t)f * J.t + off) = acc;
    }
    // the next level reads blocks this workgroup wrote
    __syncthreads();
  }
}

// One level of the second pass as a launch of its own: one workgroup per
// (pair, 1 KiB chunk) of the level.  Its four waves take a quarter of the
// check's members each, every lane 16 bytes of the chunk, eight loads in
// flight; the four partial XORs meet in LDS.  The per-slice walk above
// takes the levels past the ones launched this way.
constexpr int kPcLevelLaunches = 4;

__global__ __launch_bounds__(kPcReplayThreads) void precode_level_kernel(PrecodeReplayJob J, int l) {
  __shared__ v4u part[4][64];
  if (l >= J.meta[0]) return;
  const int lo = J.level_ptr[l], hi = J.level_ptr[l + 1];
  if (hi <= lo) return;
  const uint64_t nch = (J.t + kPcSlice - 1) / kPcSlice;
  const uint64_t nwork = (uint64_t)(hi - lo) * nch;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const v4u zero = {0u, 0u, 0u, 0u};
  for (uint64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
    const int q = lo + (int)(w / nch);
    const uint64_t off = (w % nch) * kPcSlice + lane * 16u;
    const uint32_t f = (uint32_t)J.pair_sym[q];
    const int32_t r = J.pair_chk[q];
    const int32_t b0 = J.chk_ptr[r], b1 = J.chk_ptr[r + 1];
    const int32_t e1 = b0 + (int32_t)(((int64_t)(b1 - b0) * (wv + 1)) / 4);
    int32_t e = b0 + (int32_t)(((int64_t)(b1 - b0) * wv) / 4);
    v4u acc = zero;
    if (off < J.t) {
      const uint8_t *src = J.x + off;
      for (; e + 8 <= e1; e += 8) {
        uint32_t sv[8];
        v4u a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) sv[u] = (uint32_t)J.chk_col[e + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = sv[u] != f ? *reinterpret_cast<const v4u *>(src + (uint64_t)sv[u] * J.t) : zero;
        acc ^= ((a[0] ^ a[1]) ^ (a[2] ^ a[3])) ^ ((a[4] ^ a[5]) ^ (a[6] ^ a[7]));
      }
      for (; e < e1; ++e) {
        const uint32_t sv = (uint32_t)J.chk_col[e];
        if (sv != f) acc ^= *reinterpret_cast<const v4u *>(src + (uint64_t)sv * J.t);
      }
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && off < J.t)
      *reinterpret_cast<v4u *>(J.x + (uint64_t)f * J.t + off) =
          (part[0][lane] ^ part[1][lane]) ^ (part[2][lane] ^ part[3][lane]);
    __syncthreads();   // the parts are read before the next pair overwrites them
  }
}

fs_status pc_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

uint32_t largest_prime_factor(uint32_t k) {
  uint32_t best = 1, x = k;
  for (uint32_t d = 2; (uint64_t)d * d <= x; ++d)
    while (x % d == 0) {
      best = d;
      x /= d;
    }
  return x > 1 ? std::max(best, x) : best;
}

// L(1) of Algorithm 2 for an array code with largest prime factor p of k,
// k' = k / p and j' = k' - b / p.  The k blocks form k' block columns of p;
// block row j < j' of the array code's check matrix holds p x p powers of the
// cyclic shift at block columns j .. c_j (c_j = j + k' - j'), the power at
// block column c being s = (j' - 1 - j)(c - c_j) mod p.  Check i + j p thus
// meets block c p + (i + s) mod p of each block column c < c_j, and its own
// parity block b + j p + i in the identity block at c_j.
fs_status build_precode_host(uint32_t b, uint32_t k, fs_precode &pc) {
  if (k < 2 || b == 0 || b >= k) return fail(FS_ERR_INVALID, "need 0 < b < k");
  const uint32_t p = largest_prime_factor(k);
  if (b % p) return fail(FS_ERR_INVALID, "b must be a multiple of the largest prime factor of k (" +
                                             std::to_string(p) + ")");
  const uint32_t kp = k / p, jp = kp - b / p;
  if (jp < 1 || jp >= kp) return fail(FS_ERR_INVALID, "need 1 <= j' < k'");
  pc.b = b;
  pc.k = k;
  pc.p = p;
  pc.kp = kp;
  pc.jp = jp;
  pc.m = k - b;
  const uint32_t w = kp - jp;
  pc.enc_ptr.assign(pc.m + 1, 0);
  pc.enc_col.assign((size_t)pc.m * w, 0);
  for (uint32_t j = 0; j < jp; ++j) {
    const uint32_t cj = j + w;
    for (uint32_t c = j; c < cj; ++c) {
      // shift of block (j, c): (j' - 1 - j)(c - c_j) mod p, with c - c_j < 0
      const uint64_t s = ((uint64_t)(jp - 1 - j) * (uint64_t)(cj - c)) % p;
      const uint32_t shift = (uint32_t)((p - s) % p);
      for (uint32_t i = 0; i < p; ++i)   // columns ascend with c, so each row stays sorted
        pc.enc_col[(size_t)(i + j * p) * w + (c - j)] = (int32_t)(c * p + (i + shift) % p);
    }
  }
  for (uint32_t r = 0; r < pc.m; ++r) pc.enc_ptr[r + 1] = (int32_t)((r + 1) * w);
  // check members: the row plus its parity block (which is the largest)
  pc.chk_ptr.assign(pc.m + 1, 0);
  pc.chk_col.clear();
  pc.chk_col.reserve((size_t)pc.m * (w + 1));
  for (uint32_t r = 0; r < pc.m; ++r) {
    for (uint32_t e = 0; e < w; ++e) pc.chk_col.push_back(pc.enc_col[(size_t)r * w + e]);
    pc.chk_col.push_back((int32_t)(b + r));
    pc.chk_ptr[r + 1] = (int32_t)pc.chk_col.size();
  }
  for (int32_t v : pc.enc_col)
    if (v < 0 || (uint32_t)v >= k) return fail(FS_ERR_INVALID, "check index out of range");
  // the checks of every block, in increasing check order
  pc.sym_ptr.assign(k + 1, 0);
  for (int32_t v : pc.chk_col) ++pc.sym_ptr[v + 1];
  for (uint32_t s = 0; s < k; ++s) pc.sym_ptr[s + 1] += pc.sym_ptr[s];
  pc.sym_chk.assign(pc.chk_col.size(), 0);
  std::vector<int32_t> fill(pc.sym_ptr.begin(), pc.sym_ptr.end() - 1);
  for (uint32_t r = 0; r < pc.m; ++r)
    for (int32_t e = pc.chk_ptr[r]; e < pc.chk_ptr[r + 1]; ++e) pc.sym_chk[fill[pc.chk_col[e]]++] = (int32_t)r;
  return FS_OK;
}

size_t precode_peel_lds(uint32_t k, uint32_t m) { return 4ull * (2ull * m + (k + 31) / 32); }

// After a two-stage decode for a repair: with every data block back
// (status[0]) the parity blocks count as known, since they are encoded again
// from the data; skip[0] tells that encode to write nothing otherwise, or
// when the repair's ids were rejected (bad[0]).
__global__ __launch_bounds__(256) void parity_known_kernel(const int32_t *status, uint8_t *recovered, uint32_t b,
                                                           uint32_t k, const int32_t *bad, int32_t *skip) {
  const bool all = status[0] != 0 && bad[0] == 0;
  for (uint32_t i = b + blockIdx.x * 256u + threadIdx.x; all && i < k; i += gridDim.x * 256u) recovered[i] = 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) skip[0] = all ? 0 : 1;
}

fs_status launch_parity_known(const int32_t *status, uint8_t *recovered, uint32_t b, uint32_t k, const int32_t *bad,
                              int32_t *skip, hipStream_t s) {
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(64, (k - b + 255) / 256));
  hipLaunchKernelGGL(parity_known_kernel, dim3(grid), dim3(256), 0, s, status, recovered, b, k, bad, skip);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? FS_OK : fail(FS_ERR_HIP, std::string("parity launch: ") + hipGetErrorString(e));
}

fs_status launch_precode_peel(const PrecodePeelJob &job, hipStream_t s) {
  const size_t lds = precode_peel_lds(job.k, job.m);
  const void *fn = reinterpret_cast<const void *>(&precode_peel_kernel);
  if (lds > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(precode_peel_kernel, dim3(1), dim3(kPcThreads), lds, s, job);
  return pc_hip(hipGetLastError(), "precode peel launch");
}

fs_status launch_precode_replay(const PrecodeReplayJob &job, hipStream_t s) {
  const uint64_t slices = (job.t + kPcSlice - 1) / kPcSlice;
  if (slices == 0) return FS_OK;
  if (slices > 0x7fffffffull) return fail(FS_ERR_INVALID, "t too large");
  // the first levels as launches of their own (the level count is known on
  // the device only: launches past the last level return at once), the rest
  // by the slice walk
  int dev = 0;
  (void)hipGetDevice(&dev);
  const uint32_t lgrid = 8u * (uint32_t)device_info(dev).cu_count;
  for (int l = 0; l < kPcLevelLaunches; ++l) {
    hipLaunchKernelGGL(precode_level_kernel, dim3(lgrid), dim3(kPcReplayThreads), 0, s, job, l);
    const fs_status st = pc_hip(hipGetLastError(), "precode level launch");
    if (st != FS_OK) return st;
  }
  hipLaunchKernelGGL(precode_replay_kernel, dim3((uint32_t)slices), dim3(kPcReplayThreads), 0, s, job,
                     kPcLevelLaunches);
  return pc_hip(hipGetLastError(), "precode replay launch");
}

}  // namespace fs
