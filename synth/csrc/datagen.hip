// Seeded payload generator on the GPU (synthetic inputs, not the coding path).
//
// Word w (8 bytes, little endian) of block i of stripe s is draw w of the
// counter-based stream key(seed, purpose, s, i):
//   key(seed, p, a, b) = mix(mix(mix(mix(seed + G) ^ p) ^ a) ^ b)
//   draw w             = mix(key + (w + 1) G),  G = 0x9E3779B97F4A7C15
// with mix the SplitMix64 output function (Steele, Lea & Flood 2014).  The
// same definition is implemented in numpy by synth.gen.payload.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kG = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// each thread writes 16 bytes (two words) of block first + blockIdx.y
__global__ __launch_bounds__(256) void fill_kernel(uint8_t *dst, uint64_t t, uint64_t first, uint64_t seed,
                                                   uint64_t purpose, uint64_t stripe) {
  const uint64_t i = first + blockIdx.y;
  const uint64_t off = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * 16;
  if (off >= t) return;
  uint64_t key = mix(seed + kG);
  key = mix(key ^ purpose);
  key = mix(key ^ stripe);
  key = mix(key ^ i);
  const uint64_t w = off / 8;
  const uint64_t a = mix(key + (w + 1) * kG);
  const uint64_t b = mix(key + (w + 2) * kG);
  uint64_t *p = reinterpret_cast<uint64_t *>(dst + blockIdx.y * t + off);
  p[0] = a;
  p[1] = b;
}

}  // namespace

extern "C" __attribute__((visibility("default"))) int synth_fill(void *dst, uint64_t nblocks, uint64_t t,
                                                                  uint64_t first_block, uint64_t seed,
                                                                  uint64_t purpose, uint64_t stripe,
                                                                  hipStream_t stream) {
  if (!dst || t == 0 || (t & 15) || (reinterpret_cast<uintptr_t>(dst) & 15)) return 1;
  const uint64_t chunks = (t + 4095) / 4096;
  for (uint64_t b0 = 0; b0 < nblocks; b0 += 65535) {
    const uint64_t nb = nblocks - b0 < 65535 ? nblocks - b0 : 65535;
    hipLaunchKernelGGL(fill_kernel, dim3((uint32_t)chunks, (uint32_t)nb), dim3(256), 0, stream,
                       static_cast<uint8_t *>(dst) + b0 * t, t, first_block + b0, seed, purpose, stripe);
    if (hipGetLastError() != hipSuccess) return 2;
  }
  return 0;
}
