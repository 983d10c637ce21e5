// GPU twin of synth/philox.py: fills a device buffer with the seeded synthetic
// values that the NumPy side computes for the same (seed, tensor id, element).
// No part of the contraction method lives here.
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the two value maps:
//   uniform [-1,1): 53 high bits of (w1:w0) of the block at counter
//                   (e_lo, e_hi, 0, 0), scaled by 2^-52, minus 1;
//   normal:         (sum of the twelve words of the blocks at counters
//                   (e_lo, e_hi, d, 0), d = 0,1,2) * 2^-32 - 6.
// Both are exact in binary64; a scale is applied as one binary64 multiply.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = static_cast<uint64_t>(M0) * c.x;
    const uint64_t p1 = static_cast<uint64_t>(M1) * c.z;
    const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
    const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__device__ __forceinline__ double value_at(uint64_t e, uint32_t seed, uint32_t tid, int dist) {
  const uint32_t elo = static_cast<uint32_t>(e), ehi = static_cast<uint32_t>(e >> 32);
  if (dist == 0) {
    const U4 w = philox4x32_10(U4{elo, ehi, 0u, 0u}, seed, tid);
    const uint64_t k = ((static_cast<uint64_t>(w.y) << 32) | w.x) >> 11;
    return static_cast<double>(k) * 0x1p-52 - 1.0;
  }
  uint64_t s = 0;
#pragma unroll
  for (uint32_t d = 0; d < 3; ++d) {
    const U4 w = philox4x32_10(U4{elo, ehi, d, 0u}, seed, tid);
    s += static_cast<uint64_t>(w.x) + w.y + w.z + w.w;
  }
  return static_cast<double>(s) * 0x1p-32 - 6.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T* __restrict__ out, int64_t n, uint64_t first,
                                              uint32_t seed, uint32_t tid, int dist, double scale,
                                              int apply_scale) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    double x = value_at(first + static_cast<uint64_t>(i), seed, tid, dist);
    if (apply_scale) x = x * scale;
    out[i] = static_cast<T>(x);
  }
}

}  // namespace

extern "C" {

// Fill out[0..n) with the values of elements first..first+n-1 of tensor
// (seed, tensor_id).  dtype 0: binary64; 1: binary32 (rounded to nearest even
// from the binary64 value).  dist 0: uniform, 1: normal.  Returns a hipError_t.
int synth_fill(void* out, int64_t n, int64_t first, uint32_t seed, uint32_t tensor_id, int dist,
               double scale, int dtype, void* stream) {
  if (n <= 0) return 0;
  const int apply = scale != 1.0;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536 * 4) blocks = 65536 * 4;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dtype == 0)
    hipLaunchKernelGGL(k_fill<double>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<double*>(out), n, static_cast<uint64_t>(first), seed, tensor_id,
                       dist, scale, apply);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<float*>(out), n, static_cast<uint64_t>(first), seed, tensor_id,
                       dist, scale, apply);
  return static_cast<int>(hipGetLastError());
}

}  // extern "C"
